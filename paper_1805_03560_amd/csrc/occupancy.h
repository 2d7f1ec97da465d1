// Occupancy cap by LDS reservation, host arithmetic only (no HIP dependency).
#pragma once

namespace whmc {

// Bytes of LDS a workgroup must reserve so that at most k of them fit on a compute unit with
// lds_per_cu bytes: the smallest multiple of 2 KiB above lds_per_cu / (k + 1), so k + 1 do not fit.
// It is accepted only if k still fit when each workgroup's allocation (the reservation plus a small
// static array) is rounded up by one allocation granule of up to 2 KiB.  Returns 0 when no such cap
// exists: k outside 2 .. 8, unknown device limits, a reservation larger than one workgroup may
// allocate (lds_per_wg), or too little LDS for k rounded allocations.
inline unsigned lds_reservation(long long lds_per_cu, long long lds_per_wg, int k) {
  constexpr long long kGranule = 2048;
  if (k < 2 || k > 8 || lds_per_cu <= 0 || lds_per_wg <= 0) return 0;
  const long long b = (lds_per_cu / (k + 1) + 1 + kGranule - 1) / kGranule * kGranule;
  if ((b + kGranule) * k > lds_per_cu || b * (k + 1) <= lds_per_cu || b > lds_per_wg) return 0;
  return (unsigned)b;
}

}  // namespace whmc
