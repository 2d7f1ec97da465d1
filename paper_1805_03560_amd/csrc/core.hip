// Context, gauge storage, layout conversion, the hopping-matrix launchers and FP64 BLAS.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "internal.h"
#include "stencil.h"

namespace whmc {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// Scratch of whmc_apply_MdagM_noalloc: a file-scope device array, so that the entry point needs no
// allocation.  Every GPU the library runs on holds its own copy until the process ends.  In host
// code `scratch` names a host-side stand-in, never the device memory: its device address is taken
// once per device with hipGetSymbolAddress (scratch_address) and only that address is used.
constexpr size_t kNoAllocScratch = (size_t)WHMC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

static std::mutex g_scratch_mutex;
static std::map<int, void*> g_scratch_ptr;   // device ordinal -> device address of `scratch`

// device address of `scratch` on the current device `device` (looked up once per device)
static whmc_status scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  auto it = g_scratch_ptr.find(device);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    WHMC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    WHMC_CHECK(p != nullptr, WHMC_EHIP, "hipGetSymbolAddress returned no address for the no-allocation scratch");
    it = g_scratch_ptr.emplace(device, p).first;
  }
  *out = it->second;
  return WHMC_OK;
}

whmc_status workspace(whmc_ctx* c, const std::string& name, size_t bytes, void** out) {
  auto it = c->ws.find(name);
  if (it != c->ws.end() && it->second.second >= bytes) {
    *out = it->second.first;
    return WHMC_OK;
  }
  if (it != c->ws.end()) {
    WHMC_HIP(hipStreamSynchronize(c->stream));
    WHMC_HIP(hipFree(it->second.first));
    c->ws.erase(it);
  }
  void* p = nullptr;
  WHMC_HIP(hipMalloc(&p, bytes > 0 ? bytes : 16));
  c->ws[name] = {p, bytes};
  *out = p;
  return WHMC_OK;
}

// ------------------------------------------------------------------ hop kernels
// out = a x + b H_{par,1-par}^{(dag)} in; NTS: non-temporal output store (apply_H on large lattices,
// where the result is not read back by the next kernel); NORM: FP64 |out|^2 reduction.
template <int DAG, bool XPAY, bool NORM, bool NTS, class Lnk, class SIn, class SX, class SOut>
__global__ __launch_bounds__(kBlock) void k_hop(Geom g, int par, Lnk L, SIn in, SX x, SOut out, double a,
                                                double b, Reduce red, double* norm_out) {
  using R = typename SOut::Real;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  double nrm = 0.0;
  if (i < g.Vh) {
    Spinor<R> acc;
    hop_site<DAG>(g, par, i, L, in, acc);
    if (XPAY) {
      Spinor<R> xv;
      x.load(i, xv);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) acc.c[s][cc] = R(a) * xv.c[s][cc] + R(b) * acc.c[s][cc];
    } else {
      scale(acc, b);
    }
    out.template store<NTS>(i, acc);
    if (NORM) nrm = norm2(acc);
  }
  if (NORM) block_partial<kBlock>(nrm, red.partials, blockIdx.x);
}

template <class Lnk, class S>
static whmc_status launch_hop(whmc_ctx* c, const Lnk& L, int par, int dag, S in, S x, S out, bool xpay, double a,
                              double b, double* norm_out, bool nts) {
  dim3 grid(c->site_blocks()), block(kBlock);
  // the occupancy cap applies to FP64 spinors with 18- or 12-real links only (the low-precision and
  // 8-real kernels carry more arithmetic per byte and need every wave)
  const unsigned lds = std::is_same<S, SpinorF64>::value && !is_8real<Lnk>::value ? c->stencil_lds : 0u;
#define WHMC_L(D, XP, N, NS) hipLaunchKernelGGL((k_hop<D, XP, N, NS, Lnk, S, S, S>), grid, block, lds, \
                                                c->stream, c->g, \
                                                par, L, in, x, out, a, b, c->red, norm_out)
  const bool norm = norm_out != nullptr;
  if (xpay) {
    if (dag) { if (norm) WHMC_L(1, true, true, false); else WHMC_L(1, true, false, false); }
    else     { if (norm) WHMC_L(0, true, true, false); else WHMC_L(0, true, false, false); }
  } else {
    WHMC_CHECK(!norm, WHMC_EARG, "hop: norm only with the xpay form");
    if (dag) { if (nts) WHMC_L(1, false, false, true); else WHMC_L(1, false, false, false); }
    else     { if (nts) WHMC_L(0, false, false, true); else WHMC_L(0, false, false, false); }
  }
#undef WHMC_L
  WHMC_HIP(hipGetLastError());
  if (norm) return finish_sum(c, (int)grid.x, norm_out);
  return WHMC_OK;
}

static SpinorF64 sp64(const void* p, int Vh) { return SpinorF64{(double2*)p, Vh}; }
static SpinorF32 sp32(const void* p, int Vh) { return SpinorF32{(float4*)p, Vh}; }
static SpinorF16 sp16(const void* p, int Vh) {
  return SpinorF16{(uint4*)p, p ? (float*)((uint4*)p + (size_t)3 * Vh) : nullptr, Vh};
}

template <bool NT>
static whmc_status hop_nt(whmc_ctx* c, int prec, int links, int par, int dag, void* out, const void* in,
                          const void* x, double a, double b, double* norm_out, bool nts) {
  const bool xpay = x != nullptr;
  const int Vh = c->Vh;
  if (prec == WHMC_F64) {
    if (links == WHMC_L18)
      return launch_hop(c, LinkF64_18T<NT>{c->U18, Vh}, par, dag, sp64(in, Vh), sp64(x, Vh), sp64(out, Vh), xpay, a,
                        b, norm_out, nts);
    if (links == WHMC_L8)
      return launch_hop(c, LinkF64_8T<NT>{c->U8, Vh}, par, dag, sp64(in, Vh), sp64(x, Vh), sp64(out, Vh), xpay, a, b,
                        norm_out, nts);
    return launch_hop(c, LinkF64_12T<NT>{c->U12, Vh}, par, dag, sp64(in, Vh), sp64(x, Vh), sp64(out, Vh), xpay, a, b,
                      norm_out, nts);
  }
  if (prec == WHMC_F32) {
    if (links == WHMC_L18)
      return launch_hop(c, LinkF32_18T<NT>{c->U32_18, Vh}, par, dag, sp32(in, Vh), sp32(x, Vh), sp32(out, Vh), xpay,
                        a, b, norm_out, nts);
    if (links == WHMC_L8)
      return launch_hop(c, LinkF32_8T<NT>{c->U32_8, Vh}, par, dag, sp32(in, Vh), sp32(x, Vh), sp32(out, Vh), xpay, a,
                        b, norm_out, nts);
    return launch_hop(c, LinkF32_12T<NT>{c->U32_12, Vh}, par, dag, sp32(in, Vh), sp32(x, Vh), sp32(out, Vh), xpay, a,
                      b, norm_out, nts);
  }
  if (links == WHMC_L8)
    return launch_hop(c, LinkF16_8T<NT>{c->U16_8, Vh}, par, dag, sp16(in, Vh), sp16(x, Vh), sp16(out, Vh), xpay, a, b,
                      norm_out, nts);
  return launch_hop(c, LinkF16_12T<NT>{c->U16_12, Vh}, par, dag, sp16(in, Vh), sp16(x, Vh), sp16(out, Vh), xpay, a,
                    b, norm_out, nts);
}

// Full-lattice H in one launch of 2 nb workgroups: each XCD applies both parity blocks of H to the
// sites of its own region.
template <int DAG, bool NTS, class Lnk, class S>
__global__ __launch_bounds__(kBlock) void k_hop_full(Geom g, Lnk L, S in_e, S in_o, S out_e, S out_o) {
  using R = typename S::Real;
  int par;
  const int i = site_block_pair(g, blockIdx.x, gridDim.x >> 1, par) * kBlock + threadIdx.x;
  if (i >= g.Vh) return;
  Spinor<R> acc;
  hop_site<DAG>(g, par, i, L, par ? in_e : in_o, acc);
  (par ? out_o : out_e).template store<NTS>(i, acc);
}

template <class Lnk, class S>
static whmc_status launch_full(whmc_ctx* c, const Lnk& L, int dag, S ie, S io, S oe, S oo, bool nts) {
  dim3 grid(2 * c->stencil_blocks()), block(kBlock);
  const unsigned lds = std::is_same<S, SpinorF64>::value && !is_8real<Lnk>::value ? c->stencil_lds : 0u;
  if (dag) {
    if (nts) hipLaunchKernelGGL((k_hop_full<1, true, Lnk, S>), grid, block, lds, c->stream, c->g, L, ie, io, oe, oo);
    else hipLaunchKernelGGL((k_hop_full<1, false, Lnk, S>), grid, block, lds, c->stream, c->g, L, ie, io, oe, oo);
  } else {
    if (nts) hipLaunchKernelGGL((k_hop_full<0, true, Lnk, S>), grid, block, lds, c->stream, c->g, L, ie, io, oe, oo);
    else hipLaunchKernelGGL((k_hop_full<0, false, Lnk, S>), grid, block, lds, c->stream, c->g, L, ie, io, oe, oo);
  }
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

static size_t half_bytes(int prec, int Vh);

template <bool NT>
static whmc_status hop_full_nt(whmc_ctx* c, int prec, int links, int dag, void* out, const void* in, bool nts) {
  const int Vh = c->Vh;
  const size_t hb = half_bytes(prec, Vh);
  const char* i0 = (const char*)in;
  char* o0 = (char*)out;
  if (prec == WHMC_F64) {
    auto ie = sp64(i0, Vh), io = sp64(i0 + hb, Vh), oe = sp64(o0, Vh), oo = sp64(o0 + hb, Vh);
    if (links == WHMC_L18) return launch_full(c, LinkF64_18T<NT>{c->U18, Vh}, dag, ie, io, oe, oo, nts);
    if (links == WHMC_L8) return launch_full(c, LinkF64_8T<NT>{c->U8, Vh}, dag, ie, io, oe, oo, nts);
    return launch_full(c, LinkF64_12T<NT>{c->U12, Vh}, dag, ie, io, oe, oo, nts);
  }
  if (prec == WHMC_F32) {
    auto ie = sp32(i0, Vh), io = sp32(i0 + hb, Vh), oe = sp32(o0, Vh), oo = sp32(o0 + hb, Vh);
    if (links == WHMC_L18) return launch_full(c, LinkF32_18T<NT>{c->U32_18, Vh}, dag, ie, io, oe, oo, nts);
    if (links == WHMC_L8) return launch_full(c, LinkF32_8T<NT>{c->U32_8, Vh}, dag, ie, io, oe, oo, nts);
    return launch_full(c, LinkF32_12T<NT>{c->U32_12, Vh}, dag, ie, io, oe, oo, nts);
  }
  auto ie = sp16(i0, Vh), io = sp16(i0 + hb, Vh), oe = sp16(o0, Vh), oo = sp16(o0 + hb, Vh);
  if (links == WHMC_L8) return launch_full(c, LinkF16_8T<NT>{c->U16_8, Vh}, dag, ie, io, oe, oo, nts);
  return launch_full(c, LinkF16_12T<NT>{c->U16_12, Vh}, dag, ie, io, oe, oo, nts);
}

whmc_status hop_full(whmc_ctx* c, int prec, int links, int dag, void* out, const void* in) {
  WHMC_TRY(ensure_links(c, prec, links));
  if (prec == WHMC_F16 && links == WHMC_L18) {
    set_error("unsupported precision / link format combination");
    return WHMC_EUNSUP;
  }
  if (c->stream_links(prec, links)) return hop_full_nt<true>(c, prec, links, dag, out, in, true);
  return hop_full_nt<false>(c, prec, links, dag, out, in, false);
}

whmc_status hop(whmc_ctx* c, int prec, int links, int par, int dag, void* out, const void* in, const void* x,
                double a, double b, double* norm_out, bool nt_store) {
  WHMC_TRY(ensure_links(c, prec, links));
  const bool nt = c->stream_links(prec, links);
  if (nt) return hop_nt<true>(c, prec, links, par, dag, out, in, x, a, b, norm_out, nt_store && nt);
  return hop_nt<false>(c, prec, links, par, dag, out, in, x, a, b, norm_out, false);
}

// ------------------------------------------------------------------ gauge field storage
__global__ void k_pack_gauge(Geom g, const double2* __restrict__ Ucan, double2* __restrict__ U18, int unpack) {
  const long long lex = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long V = 2LL * g.Vh;
  if (lex >= V) return;
  int x = (int)(lex % g.L[3]);
  long long r = lex / g.L[3];
  int y = (int)(r % g.L[2]);
  r /= g.L[2];
  int z = (int)(r % g.L[1]);
  int t = (int)(r / g.L[1]);
  const int par = (t + z + y + x) & 1;
  const int cb = (int)(lex >> 1);
  for (int mu = 0; mu < 4; ++mu)
    for (int k = 0; k < 9; ++k) {
      size_t ci = ((size_t)lex * 4 + mu) * 9 + k;
      size_t si = (size_t)(par * 4 + mu) * 9 * g.Vh + aos(k, cb, 9, g.Vh);
      if (unpack) ((double2*)Ucan)[ci] = U18[si];
      else U18[si] = Ucan[ci];
    }
}

// max over links of |U U^dag - 1|_max and |det U - 1|, as ordered bit patterns of doubles >= 0
__global__ void k_unitarity(int n, const double2* __restrict__ U18, int Vh, unsigned long long* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;   // over 8 * Vh links
  double dev = 0.0;
  if (idx < n) {
    const int pm = idx / Vh, i = idx - pm * Vh;
    SU3<double> U;
    for (int k = 0; k < 9; ++k) {
      double2 v = U18[(size_t)pm * 9 * Vh + aos(k, i, 9, Vh)];
      U.e[k / 3][k % 3] = {v.x, v.y};
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        cplx<double> s = {0.0, 0.0};
        for (int k = 0; k < 3; ++k) s = s + cmul(U.e[a][k], conj(U.e[b][k]));
        if (a == b) s.re -= 1.0;
        dev = fmax(dev, fmax(fabs(s.re), fabs(s.im)));
      }
    cplx<double> det = cmul(U.e[0][0], cmul(U.e[1][1], U.e[2][2]) - cmul(U.e[1][2], U.e[2][1])) -
                       cmul(U.e[0][1], cmul(U.e[1][0], U.e[2][2]) - cmul(U.e[1][2], U.e[2][0])) +
                       cmul(U.e[0][2], cmul(U.e[1][0], U.e[2][1]) - cmul(U.e[1][1], U.e[2][0]));
    det.re -= 1.0;
    dev = fmax(dev, sqrt(norm2(det)));
    // fmax drops NaN operands, so a non-finite entry is checked for explicitly and counts as failure
    bool finite = true;
    for (int k = 0; k < 9; ++k) finite = finite && isfinite(U.e[k / 3][k % 3].re) && isfinite(U.e[k / 3][k % 3].im);
    if (!finite) dev = 1e300;
  }
  for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(dev));
}

// derived link formats from the FP64 18-real master, one thread per (parity, mu, cb); the 8-real
// formats also report min over links of n = |U01|^2 + |U02|^2 (ordered bits of a double >= 0)
__global__ void k_derive_links(int n, int Vh, const double2* __restrict__ U18, int fmt, void* dst,
                               unsigned long long* nmin) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  double nn = 1.0;
  if (idx < n) {
  const int pm = idx / Vh, i = idx - pm * Vh;
  double2 v[9];
  for (int k = 0; k < 9; ++k) v[k] = U18[(size_t)pm * 9 * Vh + aos(k, i, 9, Vh)];
  if (fmt >= 4) {  // 8-real: U01, U02, the smaller of U10 / U20, phases (see reconstruct8)
    nn = v[1].x * v[1].x + v[1].y * v[1].y + v[2].x * v[2].x + v[2].y * v[2].y;
    const double t00 = atan2(v[0].y, v[0].x);
    const bool swap = fmt != 6 && (v[6].x * v[6].x + v[6].y * v[6].y < v[3].x * v[3].x + v[3].y * v[3].y);
    const double2 s = swap ? v[6] : v[3];
    const double ts = swap ? atan2(v[3].y, v[3].x) + 8.0 : atan2(v[6].y, v[6].x);
    if (fmt == 4) {
      double2* d = (double2*)dst + (size_t)pm * 4 * Vh;
      d[aos(0, i, 4, Vh)] = v[1];
      d[aos(1, i, 4, Vh)] = v[2];
      d[aos(2, i, 4, Vh)] = s;
      d[aos(3, i, 4, Vh)] = make_double2(t00, ts);
    } else if (fmt == 5) {
      float4* d = (float4*)dst + (size_t)pm * 2 * Vh;
      d[aos(0, i, 2, Vh)] = make_float4((float)v[1].x, (float)v[1].y, (float)v[2].x, (float)v[2].y);
      d[aos(1, i, 2, Vh)] = make_float4((float)s.x, (float)s.y, (float)t00, (float)ts);
    } else {
      const double ipi = 0.31830988618379067;
      uint4* d = (uint4*)dst + (size_t)pm * Vh;
      d[aos(0, i, 1, Vh)] = make_uint4((unsigned)f2h((float)v[1].x) | ((unsigned)f2h((float)v[1].y) << 16),
                                       (unsigned)f2h((float)v[2].x) | ((unsigned)f2h((float)v[2].y) << 16),
                                       (unsigned)f2h((float)s.x) | ((unsigned)f2h((float)s.y) << 16),
                                       (unsigned)f2h((float)(t00 * ipi)) | ((unsigned)f2h((float)(ts * ipi)) << 16));
    }
  } else if (fmt == 0) {  // F64-12
    double2* d = (double2*)dst;
    for (int k = 0; k < 6; ++k) d[(size_t)pm * 6 * Vh + aos(k, i, 6, Vh)] = v[k];
  } else if (fmt == 1) {  // F32-18
    float2* d = (float2*)dst;
    for (int k = 0; k < 9; ++k) d[(size_t)pm * 9 * Vh + aos(k, i, 9, Vh)] = make_float2((float)v[k].x, (float)v[k].y);
  } else if (fmt == 2) {  // F32-12
    float4* d = (float4*)dst;
    for (int k = 0; k < 3; ++k)
      d[(size_t)pm * 3 * Vh + aos(k, i, 3, Vh)] =
          make_float4((float)v[2 * k].x, (float)v[2 * k].y, (float)v[2 * k + 1].x, (float)v[2 * k + 1].y);
  } else {  // F16-12
    uint2* d = (uint2*)dst;
    for (int k = 0; k < 3; ++k) {
      unsigned int w0 = (unsigned)f2h((float)v[2 * k].x) | ((unsigned)f2h((float)v[2 * k].y) << 16);
      unsigned int w1 = (unsigned)f2h((float)v[2 * k + 1].x) | ((unsigned)f2h((float)v[2 * k + 1].y) << 16);
      d[(size_t)pm * 3 * Vh + aos(k, i, 3, Vh)] = make_uint2(w0, w1);
    }
  }
  }
  if (nmin) {
    for (int off = 32; off > 0; off >>= 1) nn = fmin(nn, __shfl_xor(nn, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMin(nmin, (unsigned long long)__double_as_longlong(nn));
  }
}

whmc_status gauge_changed(whmc_ctx* c) {
  for (int k = 0; k < 7; ++k) c->derived_valid[k] = false;
  return WHMC_OK;
}

whmc_status ensure_links(whmc_ctx* c, int prec, int links) {
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded (call whmc_load_gauge first)");
  int fmt = -1;
  size_t bytes = 0;
  void** slot = nullptr;
  const size_t nl = (size_t)8 * c->Vh;
  if (prec == WHMC_F64 && links == WHMC_L18) return WHMC_OK;
  if (prec == WHMC_F64 && links == WHMC_L12) { fmt = 0; bytes = nl * 6 * sizeof(double2); slot = (void**)&c->U12; }
  else if (prec == WHMC_F32 && links == WHMC_L18) { fmt = 1; bytes = nl * 9 * sizeof(float2); slot = (void**)&c->U32_18; }
  else if (prec == WHMC_F32 && links == WHMC_L12) { fmt = 2; bytes = nl * 3 * sizeof(float4); slot = (void**)&c->U32_12; }
  else if (prec == WHMC_F16 && links == WHMC_L12) { fmt = 3; bytes = nl * 3 * sizeof(uint2); slot = (void**)&c->U16_12; }
  else if (prec == WHMC_F64 && links == WHMC_L8) { fmt = 4; bytes = nl * 4 * sizeof(double2); slot = (void**)&c->U8; }
  else if (prec == WHMC_F32 && links == WHMC_L8) { fmt = 5; bytes = nl * 2 * sizeof(float4); slot = (void**)&c->U32_8; }
  else if (prec == WHMC_F16 && links == WHMC_L8) { fmt = 6; bytes = nl * sizeof(uint4); slot = (void**)&c->U16_8; }
  else {
    set_error("unsupported precision / link format combination");
    return WHMC_EUNSUP;
  }
  if (c->derived_valid[fmt]) return WHMC_OK;
  if (*slot == nullptr) WHMC_HIP(hipMalloc(slot, bytes));
  const int n = (int)nl;
  unsigned long long* nmin = nullptr;
  if (fmt >= 4) {
    void* w;
    WHMC_TRY(workspace(c, "derive_nmin", sizeof(unsigned long long), &w));
    nmin = (unsigned long long*)w;
    const double one = 1.0;
    WHMC_HIP(hipMemcpyAsync(nmin, &one, sizeof(one), hipMemcpyHostToDevice, c->stream));
  }
  hipLaunchKernelGGL(k_derive_links, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, c->Vh, c->U18, fmt, *slot,
                     nmin);
  WHMC_HIP(hipGetLastError());
  if (nmin) {
    // the 8-real form needs n = |U01|^2 + |U02|^2 > 0 on every link (reconstruct8); half precision
    // needs it well inside the normal FP16 range
    WHMC_HIP(hipMemcpyAsync(c->host_pinned, nmin, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    WHMC_HIP(hipStreamSynchronize(c->stream));
    const double lim = fmt == 6 ? 1e-6 : 1e-20;
    if (!(c->host_pinned[0] >= lim)) {
      set_error("8-real links: a link has |U01|^2 + |U02|^2 = " + std::to_string(c->host_pinned[0]) + " < " +
                std::to_string(lim) + " (|U00| = 1 to that precision), which the 8-real form cannot represent");
      return WHMC_EUNSUP;
    }
  }
  c->derived_valid[fmt] = true;
  return WHMC_OK;
}

// ------------------------------------------------------------------ spinor layouts
__global__ void k_pack_spinor(Geom g, double2* dst, const double2* src, int parity, int unpack, int nfields) {
  const long long n_sites = parity < 0 ? 2LL * g.Vh : (long long)g.Vh;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_sites * nfields) return;
  const int f = (int)(idx / n_sites);
  const long long s = idx - (long long)f * n_sites;
  int par, cb;
  if (parity < 0) {
    int x = (int)(s % g.L[3]);
    long long r = s / g.L[3];
    int y = (int)(r % g.L[2]);
    r /= g.L[2];
    int z = (int)(r % g.L[1]);
    int t = (int)(r / g.L[1]);
    par = (t + z + y + x) & 1;
    cb = (int)(s >> 1);
  } else {
    par = 0;
    cb = (int)s;
  }
  const size_t field_off = (size_t)f * n_sites * 12;   // same element count in both layouts
  for (int k = 0; k < 12; ++k) {
    size_t ci = field_off + (size_t)s * 12 + k;
    size_t si = field_off + (size_t)par * 12 * g.Vh + aos(k, cb, 12, g.Vh);
    if (unpack) dst[ci] = src[si];
    else dst[si] = src[ci];
  }
}

template <class SD, class SS>
__global__ void k_convert(int Vh, int nhalf, SD d, SS s, size_t dstride_bytes, size_t sstride_bytes) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)Vh * nhalf) return;
  const int f = (int)(idx / Vh), i = (int)(idx - (long long)f * Vh);
  SD dd = d;
  SS ss = s;
  dd.p = (decltype(dd.p))((char*)d.p + f * dstride_bytes);
  ss.p = (decltype(ss.p))((char*)s.p + f * sstride_bytes);
  if constexpr (std::is_same<SD, SpinorF16>::value) dd.scale = (float*)((char*)d.scale + f * dstride_bytes);
  if constexpr (std::is_same<SS, SpinorF16>::value) ss.scale = (float*)((char*)s.scale + f * sstride_bytes);
  using RD = typename SD::Real;
  using RS = typename SS::Real;
  Spinor<RS> a;
  ss.load(i, a);
  Spinor<RD> b;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) b.c[p][cc] = {(RD)a.c[p][cc].re, (RD)a.c[p][cc].im};
  dd.store(i, b);
}

static size_t half_bytes(int prec, int Vh) {
  if (prec == WHMC_F64) return (size_t)Vh * 192;
  if (prec == WHMC_F32) return (size_t)Vh * 96;
  return (size_t)Vh * 52;
}

template <class SD>
static whmc_status convert_from(whmc_ctx* c, SD d, const void* src, int src_prec, int nhalf, size_t db) {
  const long long n = (long long)c->Vh * nhalf;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  const size_t sb = half_bytes(src_prec, c->Vh);
  if (src_prec == WHMC_F64)
    hipLaunchKernelGGL((k_convert<SD, SpinorF64>), grid, block, 0, c->stream, c->Vh, nhalf, d, sp64(src, c->Vh), db, sb);
  else if (src_prec == WHMC_F32)
    hipLaunchKernelGGL((k_convert<SD, SpinorF32>), grid, block, 0, c->stream, c->Vh, nhalf, d, sp32(src, c->Vh), db, sb);
  else
    hipLaunchKernelGGL((k_convert<SD, SpinorF16>), grid, block, 0, c->stream, c->Vh, nhalf, d, sp16(src, c->Vh), db, sb);
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

whmc_status convert_spinor(whmc_ctx* c, void* dst, int dst_prec, const void* src, int src_prec, int nhalf) {
  WHMC_CHECK(dst && src && nhalf >= 1, WHMC_EARG, "convert_spinor: null pointer or nhalf < 1");
  WHMC_CHECK(dst_prec >= 0 && dst_prec <= 2 && src_prec >= 0 && src_prec <= 2, WHMC_EARG, "convert_spinor: bad prec");
  const size_t db = half_bytes(dst_prec, c->Vh);
  if (dst_prec == WHMC_F64) return convert_from(c, sp64(dst, c->Vh), src, src_prec, nhalf, db);
  if (dst_prec == WHMC_F32) return convert_from(c, sp32(dst, c->Vh), src, src_prec, nhalf, db);
  return convert_from(c, sp16(dst, c->Vh), src, src_prec, nhalf, db);
}

// ------------------------------------------------------------------ FP64 BLAS (flat over components)
__global__ void k_axpby(long long n, double2* y, double a, const double2* x, double b) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 xv = x[i], yv = y[i];
  y[i] = make_double2(a * xv.x + b * yv.x, a * xv.y + b * yv.y);
}
// y = gamma_5 x = diag(-1, -1, 1, 1) x on nhalf half fields, site by site
__global__ void k_gamma5(int Vh, int nhalf, double2* y, const double2* x) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)Vh * nhalf) return;
  const int f = (int)(idx / Vh), i = (int)(idx - (long long)f * Vh);
  SpinorF64 X{(double2*)x + (size_t)f * 12 * Vh, Vh}, Y{y + (size_t)f * 12 * Vh, Vh};
  Spinor<double> s;
  X.load(i, s);
  for (int c = 0; c < 3; ++c) {
    s.c[0][c] = -s.c[0][c];
    s.c[1][c] = -s.c[1][c];
  }
  Y.store(i, s);
}
__global__ void k_fill(long long n, unsigned int* p) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}
__global__ __launch_bounds__(kBlock) void k_dot(long long n, const double2* x, const double2* y, Reduce red,
                                                double* out) {
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    double2 a = x[i], b = y[i];
    s += a.x * b.x + a.y * b.y;
  }
  block_partial<kBlock>(s, red.partials, blockIdx.x);
}

static dim3 flat_grid(long long n) { return dim3((unsigned)((n + 255) / 256)); }

whmc_status axpby_f64(whmc_ctx* c, double* y, double a, const double* x, double b, int nhalf) {
  const long long n = 12LL * c->Vh * nhalf;
  hipLaunchKernelGGL(k_axpby, flat_grid(n), dim3(256), 0, c->stream, n, (double2*)y, a, (const double2*)x, b);
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}
whmc_status copy_f64(whmc_ctx* c, double* y, const double* x, int nhalf) {
  WHMC_HIP(hipMemcpyAsync(y, x, (size_t)c->Vh * 192 * nhalf, hipMemcpyDeviceToDevice, c->stream));
  return WHMC_OK;
}
whmc_status gamma5_f64(whmc_ctx* c, double* y, const double* x, int nhalf) {
  const long long n = (long long)c->Vh * nhalf;
  hipLaunchKernelGGL(k_gamma5, flat_grid(n), dim3(256), 0, c->stream, c->Vh, nhalf, (double2*)y, (const double2*)x);
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}
whmc_status zero_bytes(whmc_ctx* c, void* p, size_t bytes) {
  const long long n = (long long)(bytes / 4);
  if (n > 0) {
    hipLaunchKernelGGL(k_fill, flat_grid(n), dim3(256), 0, c->stream, n, (unsigned int*)p);
    WHMC_HIP(hipGetLastError());
  }
  return WHMC_OK;
}
static int reduce_blocks(whmc_ctx* c, long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  return (int)(b < 1024 ? b : 1024);
}
whmc_status finish_sum(whmc_ctx* c, int nparts, double* dev_out) {
  hipLaunchKernelGGL(k_finish_sum<256>, dim3(1), dim3(256), 0, c->stream, c->red.partials, nparts, dev_out);
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

whmc_status dot_re_f64(whmc_ctx* c, const double* x, const double* y, int nhalf, double* dev_out) {
  const long long n = 12LL * c->Vh * nhalf;
  const int nb = reduce_blocks(c, n);
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kBlock), 0, c->stream, n, (const double2*)x, (const double2*)y, c->red,
                     dev_out);
  WHMC_HIP(hipGetLastError());
  return finish_sum(c, nb, dev_out);
}
whmc_status norm2_f64(whmc_ctx* c, const double* x, int nhalf, double* dev_out) {
  return dot_re_f64(c, x, x, nhalf, dev_out);
}
whmc_status read_scalar(whmc_ctx* c, const double* dev, double* host) {
  WHMC_HIP(hipMemcpyAsync(c->host_pinned, dev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  WHMC_HIP(hipStreamSynchronize(c->stream));
  *host = c->host_pinned[0];
  return WHMC_OK;
}

// ------------------------------------------------------------------ composed operators
// out = a x + K in with K = kappa^2 H_oe H_eo (or K^dag = kappa^2 H_eo^dag H_oe^dag ... applied as
// (H^dag)_oe (H^dag)_eo); even_out receives the even-site intermediate H_eo in (or (H^dag)_eo in).
whmc_status apply_K_f64(whmc_ctx* c, double* out, const double* in, double kappa, int dagger, double* even_out,
                        const double* x, double a) {
  WHMC_TRY(hop(c, WHMC_F64, WHMC_L18, 0, dagger, even_out, in, nullptr, 0.0, 1.0, nullptr));
  if (x) return hop(c, WHMC_F64, WHMC_L18, 1, dagger, out, even_out, x, a, kappa * kappa, nullptr);
  return hop(c, WHMC_F64, WHMC_L18, 1, dagger, out, even_out, nullptr, 0.0, kappa * kappa, nullptr);
}

whmc_status apply_Moo_f64(whmc_ctx* c, double* out, const double* in, double kappa, int dagger, double* tmp_even) {
  WHMC_TRY(hop(c, WHMC_F64, WHMC_L18, 0, dagger, tmp_even, in, nullptr, 0.0, 1.0, nullptr));
  return hop(c, WHMC_F64, WHMC_L18, 1, dagger, out, tmp_even, in, 1.0, -kappa * kappa, nullptr);
}

whmc_status apply_MdagM_f64(whmc_ctx* c, double* out, const double* in, double kappa, double* tmp_even,
                            double* tmp_odd) {
  WHMC_TRY(apply_Moo_f64(c, tmp_odd, in, kappa, 0, tmp_even));
  return apply_Moo_f64(c, out, tmp_odd, kappa, 1, tmp_even);
}

}  // namespace whmc

// ====================================================================== C ABI: context and layouts
using namespace whmc;

extern "C" {

int whmc_abi_version(void) { return WHMC_ABI_VERSION; }
const char* whmc_last_error(void) { return g_last_error.c_str(); }

whmc_status whmc_create(whmc_ctx** out, const int dims[4], int device, void* stream) {
  WHMC_CHECK(out && dims, WHMC_EARG, "whmc_create: null argument");
  *out = nullptr;
  long long V = 1;
  for (int mu = 0; mu < 4; ++mu) {
    WHMC_CHECK(dims[mu] >= 2 && dims[mu] % 2 == 0, WHMC_EARG,
               "whmc_create: every extent must be even and >= 2 (even/odd ordering)");
    V *= dims[mu];
  }
  WHMC_CHECK(V / 2 < (1LL << 31) / 12, WHMC_EARG, "whmc_create: lattice too large for 32-bit component indexing");
  int ndev = 0;
  WHMC_HIP(hipGetDeviceCount(&ndev));
  WHMC_CHECK(device >= 0 && device < ndev, WHMC_EARG, "whmc_create: no such device");
  WHMC_HIP(hipSetDevice(device));
  whmc_ctx* c = new whmc_ctx();
  for (int mu = 0; mu < 4; ++mu) c->dims[mu] = dims[mu], c->g.L[mu] = dims[mu];
  c->V = V;
  c->Vh = (int)(V / 2);
  c->g.Vh = c->Vh;
  c->g.Lxh = dims[3] / 2;
  {
    const long long slice = (long long)dims[1] * dims[2] * dims[3] / 2;
    const bool split = slice % kBlock == 0 && slice / kBlock >= 8;
    c->g.nbs = split ? (int)(slice / kBlock) : 0;
    c->g.xq = split ? (c->g.nbs + 7) / 8 : 0;
    c->g.sched = 0;
    c->hop_chunk = c->g.xq;   // chunk of the time-slab schedule: one XCD's range of a slice
  }
  c->device = device;
  c->stream = (hipStream_t)stream;
  if (hipDeviceGetAttribute(&c->lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) !=
          hipSuccess ||
      hipDeviceGetAttribute(&c->lds_per_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
    c->lds_per_cu = c->lds_per_wg = 0;   // no occupancy cap on this device
  const size_t nlinks = (size_t)8 * c->Vh;
  hipError_t e = hipMalloc(&c->U18, nlinks * 9 * sizeof(double2));
  // partial sums: up to 8 rows per rhs (multi-RHS sub-blocks) of stencil_blocks() slots each
  const int maxb = c->stencil_blocks() * (8 * kMaxRhs + 4) + 1024 * kMaxRhs;
  if (e == hipSuccess) e = hipMalloc(&c->red.partials, (size_t)maxb * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&c->red.counter, 64 * sizeof(unsigned));
  if (e == hipSuccess) e = hipMalloc(&c->red.result, 64 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&c->scal, kMaxRhs * sizeof(CGScalars));
  if (e == hipSuccess) e = hipHostMalloc(&c->scal_host, kMaxRhs * sizeof(CGScalars), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(&c->host_pinned, 64 * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemsetAsync(c->red.counter, 0, 64 * sizeof(unsigned), c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    set_error(std::string("whmc_create: ") + hipGetErrorString(e));
    whmc_destroy(c);
    return WHMC_EHIP;
  }
  // the no-allocation entry point's scratch on this device (device current)
  if (scratch_address(device, &c->noalloc_scratch) != WHMC_OK) {
    whmc_destroy(c);
    return WHMC_EHIP;
  }
  *out = c;
  return WHMC_OK;
}

void whmc_destroy(whmc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(c->U18);
  (void)hipFree(c->U12);
  (void)hipFree(c->U32_18);
  (void)hipFree(c->U32_12);
  (void)hipFree(c->U16_12);
  (void)hipFree(c->U8);
  (void)hipFree(c->U32_8);
  (void)hipFree(c->U16_8);
  (void)hipFree(c->red.partials);
  (void)hipFree(c->red.counter);
  (void)hipFree(c->red.result);
  (void)hipFree(c->scal);
  if (c->scal_host) (void)hipHostFree(c->scal_host);
  if (c->host_pinned) (void)hipHostFree(c->host_pinned);
  for (auto& kv : c->ws) (void)hipFree(kv.second.first);
  delete c;
}

whmc_status whmc_set_stream(whmc_ctx* c, void* stream) {
  WHMC_CHECK(c, WHMC_EARG, "null context");
  WHMC_HIP(hipStreamSynchronize(c->stream));
  c->stream = (hipStream_t)stream;
  return WHMC_OK;
}

whmc_status whmc_field_bytes(const whmc_ctx* c, int kind, int prec, size_t* bytes) {
  WHMC_CHECK(c && bytes, WHMC_EARG, "null argument");
  WHMC_CHECK(prec >= 0 && prec <= 2, WHMC_EARG, "bad precision");
  const size_t hb = prec == WHMC_F64 ? 192 : (prec == WHMC_F32 ? 96 : 52);
  switch (kind) {
    case 0: *bytes = hb * c->Vh; break;
    case 1: *bytes = 2 * hb * c->Vh; break;
    case 2: *bytes = (size_t)c->V * 4 * 8 * sizeof(double); break;
    case 3: *bytes = (size_t)c->V * 4 * 9 * 16; break;
    default: set_error("bad field kind"); return WHMC_EARG;
  }
  return WHMC_OK;
}

whmc_status whmc_load_gauge(whmc_ctx* c, const double* U, double tol) {
  WHMC_CHECK(c && U, WHMC_EARG, "whmc_load_gauge: null argument");
  WHMC_HIP(hipSetDevice(c->device));
  const long long V = c->V;
  hipLaunchKernelGGL(k_pack_gauge, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, c->stream, c->g,
                     (const double2*)U, c->U18, 0);
  WHMC_HIP(hipGetLastError());
  c->gauge_loaded = true;
  gauge_changed(c);
  if (tol > 0) {
    void* w;
    WHMC_TRY(workspace(c, "unitarity", sizeof(unsigned long long), &w));
    WHMC_TRY(zero_bytes(c, w, sizeof(unsigned long long)));
    const int n = 8 * c->Vh;
    hipLaunchKernelGGL(k_unitarity, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, c->U18, c->Vh,
                       (unsigned long long*)w);
    WHMC_HIP(hipGetLastError());
    unsigned long long bits = 0;
    WHMC_HIP(hipMemcpyAsync(c->host_pinned, w, sizeof(bits), hipMemcpyDeviceToHost, c->stream));
    WHMC_HIP(hipStreamSynchronize(c->stream));
    std::memcpy(&bits, c->host_pinned, sizeof(bits));
    double dev;
    std::memcpy(&dev, &bits, sizeof(dev));
    if (!(dev <= tol)) {
      set_error("whmc_load_gauge: link not in SU(3): max deviation " + std::to_string(dev));
      return WHMC_ENOTSU3;
    }
  }
  return WHMC_OK;
}

whmc_status whmc_export_gauge(whmc_ctx* c, double* U) {
  WHMC_CHECK(c && U, WHMC_EARG, "whmc_export_gauge: null argument");
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const long long V = c->V;
  hipLaunchKernelGGL(k_pack_gauge, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, c->stream, c->g,
                     (const double2*)U, c->U18, 1);
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

static whmc_status pack_impl(whmc_ctx* c, double* dst, const double* src, int parity, int nfields, int unpack) {
  WHMC_CHECK(c && dst && src, WHMC_EARG, "pack/unpack spinor: null argument");
  WHMC_CHECK(parity >= -1 && parity <= 1 && nfields >= 1, WHMC_EARG, "pack/unpack spinor: bad parity or nfields");
  WHMC_CHECK(dst != src, WHMC_EARG, "pack/unpack spinor: in-place conversion not supported");
  const long long n = (parity < 0 ? c->V : (long long)c->Vh) * nfields;
  hipLaunchKernelGGL(k_pack_spinor, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->g, (double2*)dst,
                     (const double2*)src, parity, unpack, nfields);
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}
whmc_status whmc_pack_spinor(whmc_ctx* c, double* dst, const double* src, int parity, int nfields) {
  return pack_impl(c, dst, src, parity, nfields, 0);
}
whmc_status whmc_unpack_spinor(whmc_ctx* c, double* dst, const double* src, int parity, int nfields) {
  return pack_impl(c, dst, src, parity, nfields, 1);
}
whmc_status whmc_convert_spinor(whmc_ctx* c, void* dst, int dst_prec, const void* src, int src_prec, int nhalf) {
  WHMC_CHECK(c, WHMC_EARG, "null context");
  return convert_spinor(c, dst, dst_prec, src, src_prec, nhalf);
}

whmc_status whmc_apply_H(whmc_ctx* c, void* out, const void* in, int out_parity, int dagger, int prec, int links) {
  WHMC_CHECK(c && out && in, WHMC_EARG, "whmc_apply_H: null argument");
  WHMC_CHECK(out != in, WHMC_EARG, "whmc_apply_H: in and out must differ");
  WHMC_CHECK(out_parity >= -1 && out_parity <= 1, WHMC_EARG, "whmc_apply_H: out_parity must be -1, 0 or 1");
  WHMC_CHECK(prec >= 0 && prec <= 2, WHMC_EARG, "whmc_apply_H: bad precision");
  WHMC_CHECK(links == WHMC_L8 || links == WHMC_L12 || links == WHMC_L18, WHMC_EARG,
             "whmc_apply_H: links must be 8, 12 or 18");
  const int dag = dagger ? 1 : 0;
  if (out_parity >= 0) return hop(c, prec, links, out_parity, dag, out, in, nullptr, 0.0, 1.0, nullptr, true);
  return hop_full(c, prec, links, dag, out, in);
}

whmc_status whmc_apply_Moo(whmc_ctx* c, double* out, const double* in, double kappa, int dagger) {
  WHMC_CHECK(c && out && in, WHMC_EARG, "whmc_apply_Moo: null argument");
  WHMC_CHECK(out != in, WHMC_EARG, "whmc_apply_Moo: in and out must differ");
  void* tmp;
  WHMC_TRY(workspace(c, "moo_tmp_even", (size_t)c->Vh * 192, &tmp));
  return apply_Moo_f64(c, out, in, kappa, dagger ? 1 : 0, (double*)tmp);
}

whmc_status whmc_apply_MdagM(whmc_ctx* c, double* out, const double* in, const double* kappas, int nrhs, int eo) {
  WHMC_CHECK(c && out && in && kappas && nrhs >= 1, WHMC_EARG, "whmc_apply_MdagM: bad argument");
  WHMC_CHECK(out != in, WHMC_EARG, "whmc_apply_MdagM: in and out must differ");
  WHMC_CHECK(eo == 0 || eo == 1, WHMC_EARG, "whmc_apply_MdagM: eo must be 0 (full lattice) or 1 (even/odd)");
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const size_t hb = (size_t)c->Vh * 192;
  if (!eo) {
    void* tf;
    WHMC_TRY(workspace(c, "mdm_tmp_full", 2 * hb, &tf));
    for (int r = 0; r < nrhs; ++r)
      WHMC_TRY(apply_MdagM_full(c, out + (size_t)r * 48 * c->Vh, in + (size_t)r * 48 * c->Vh, kappas[r], (double*)tf));
    return WHMC_OK;
  }
  void *te, *to;
  WHMC_TRY(workspace(c, "mdm_tmp_even", hb, &te));
  WHMC_TRY(workspace(c, "mdm_tmp_odd", hb, &to));
  for (int r = 0; r < nrhs; ++r)
    WHMC_TRY(apply_MdagM_f64(c, out + (size_t)r * 24 * c->Vh, in + (size_t)r * 24 * c->Vh, kappas[r], (double*)te,
                             (double*)to));
  return WHMC_OK;
}

whmc_status whmc_apply_MdagM_noalloc(whmc_ctx* c, double* out, const double* in, const double* kappas, int nrhs,
                                     int eo) {
  WHMC_CHECK(c && out && in && kappas && nrhs >= 1, WHMC_EARG, "whmc_apply_MdagM_noalloc: bad argument");
  WHMC_CHECK(out != in, WHMC_EARG, "whmc_apply_MdagM_noalloc: in and out must differ");
  WHMC_CHECK(eo == 0 || eo == 1, WHMC_EARG, "whmc_apply_MdagM_noalloc: eo must be 0 (full lattice) or 1 (even/odd)");
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  WHMC_CHECK(c->noalloc_scratch, WHMC_ESTATE, "whmc_apply_MdagM_noalloc: no scratch address for this context");
  // intermediates: even and odd half fields (eo = 1) or one full field (eo = 0), V * 192 bytes either way
  const size_t hb = (size_t)c->Vh * 192;
  WHMC_CHECK(2 * hb <= kNoAllocScratch, WHMC_EARG,
             "whmc_apply_MdagM_noalloc: the lattice needs " + std::to_string(2 * hb) + " bytes of scratch, more than the " +
                 std::to_string(kNoAllocScratch) + " bytes of the static buffer (V <= " +
                 std::to_string(kNoAllocScratch / 192) + " sites)");
  double* t0 = (double*)c->noalloc_scratch;
  double* t1 = (double*)((char*)c->noalloc_scratch + hb);
  for (int r = 0; r < nrhs; ++r) {
    if (eo)
      WHMC_TRY(apply_MdagM_f64(c, out + (size_t)r * 24 * c->Vh, in + (size_t)r * 24 * c->Vh, kappas[r], t0, t1));
    else
      WHMC_TRY(apply_MdagM_full(c, out + (size_t)r * 48 * c->Vh, in + (size_t)r * 48 * c->Vh, kappas[r], t0));
  }
  return WHMC_OK;
}

// Autotuner of the single-RHS stencil schedule: times the FP64 even/odd hop pair t = H_eo x,
// x' = H_oe t (18-real links, the order of the even/odd operator) on zero fields for the slice-range
// schedule and the time-slab schedule with chunks of nbs/16 .. nbs/2 blocks, keeps the fastest.
whmc_status whmc_autotune_hop(whmc_ctx* c, int* schedule, int* chunk, double* us) {
  WHMC_CHECK(c, WHMC_EARG, "whmc_autotune_hop: null context");
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const size_t hb = (size_t)c->Vh * 192;
  void *x, *t;
  WHMC_TRY(workspace(c, "tune_hop_x", hb, &x));
  WHMC_TRY(workspace(c, "tune_hop_t", hb, &t));
  WHMC_TRY(zero_bytes(c, x, hb));
  // candidates: (schedule, chunk, workgroups per CU)
  struct Cand {
    int sched, chunk, cap;
  };
  std::vector<std::pair<int, int>> sc{{0, c->hop_chunk}};
  if (c->g.nbs > 0 && c->g.L[0] % 8 == 0)
    for (int d : {16, 8, 4, 2}) {
      const int q = (c->g.nbs + d - 1) / d;
      bool seen = false;
      for (auto& p : sc) seen |= (p.first == 1 && p.second == q);
      if (!seen) sc.push_back({1, q});
    }
  const int saved_cap = c->hop_wg_per_cu;
  std::vector<Cand> cand;
  for (auto& p : sc)
    for (int cap : {0, 2})
      if (c->set_wg_cap(cap)) cand.push_back({p.first, p.second, cap});
  hipEvent_t e0, e1;
  WHMC_HIP(hipEventCreate(&e0));
  WHMC_HIP(hipEventCreate(&e1));
  const Geom saved = c->g;
  // every candidate is timed in each of kRounds rounds (rounds interleave the candidates, so clock
  // and temperature drifts hit all of them alike) and keeps its best round: the differences between
  // candidates (a few per cent) are below the spread of a single short timing
  constexpr int kRounds = 4, kPairs = 8;
  std::vector<double> best_us(cand.size(), 1e30);
  whmc_status rc = WHMC_OK;
  auto pair = [&]() -> whmc_status {   // the hops of whmc_apply_H (non-temporal stores on large lattices)
    WHMC_TRY(hop(c, WHMC_F64, WHMC_L18, 0, 0, t, x, nullptr, 0.0, 1.0, nullptr, true));
    return hop(c, WHMC_F64, WHMC_L18, 1, 0, x, t, nullptr, 0.0, 1.0, nullptr, true);
  };
  for (int round = 0; round < kRounds && rc == WHMC_OK; ++round)
    for (size_t q = 0; q < cand.size() && rc == WHMC_OK; ++q) {
      c->set_schedule(cand[q].sched, cand[q].chunk);
      c->set_wg_cap(cand[q].cap);
      float ms = 0.f;
      rc = pair();   // warm-up of this candidate
      if (rc == WHMC_OK && hipEventRecord(e0, c->stream) != hipSuccess) rc = WHMC_EHIP;
      for (int rep = 0; rep < kPairs && rc == WHMC_OK; ++rep) rc = pair();
      if (rc == WHMC_OK && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = WHMC_EHIP;
      if (rc == WHMC_OK) best_us[q] = std::min(best_us[q], ms * 1e3 / (2.0 * kPairs));
    }
  size_t qbest = 0;
  for (size_t q = 1; q < cand.size(); ++q)
    if (best_us[q] < best_us[qbest]) qbest = q;
  const Cand pick = cand[qbest];
  const double best = best_us[qbest];
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->g = saved;
  if (rc != WHMC_OK) {
    c->set_wg_cap(saved_cap);
    return rc;
  }
  c->set_schedule(pick.sched, pick.chunk);
  if (pick.sched == 1) c->hop_chunk = pick.chunk;
  c->set_wg_cap(pick.cap);
  if (schedule) *schedule = c->g.sched;
  if (chunk) *chunk = c->hop_chunk;
  if (us) *us = best;
  return WHMC_OK;
}

whmc_status whmc_set_option(whmc_ctx* c, int option, long long value) {
  WHMC_CHECK(c, WHMC_EARG, "whmc_set_option: null context");
  switch (option) {
    case WHMC_OPT_STREAM_THRESHOLD:
      WHMC_CHECK(value >= -1, WHMC_EARG, "whmc_set_option: the stream threshold must be >= -1");
      c->stream_threshold = value;
      return WHMC_OK;
    case WHMC_OPT_HOP_CHUNK:
      WHMC_CHECK(c->g.nbs > 0 && value >= 1 && value <= c->g.nbs, WHMC_EARG,
                 "whmc_set_option: the chunk must be 1 .. blocks per time slice (" + std::to_string(c->g.nbs) + ")");
      c->hop_chunk = (int)value;
      if (c->g.sched == 1) c->set_schedule(1, c->hop_chunk);
      return WHMC_OK;
    case WHMC_OPT_FORCE_KERNEL:
      WHMC_CHECK(value == 0 || value == 1, WHMC_EARG, "whmc_set_option: the force kernel must be 0 or 1");
      c->force_kernel = (int)value;
      return WHMC_OK;
    case WHMC_OPT_FORCE_CHUNK:
      WHMC_CHECK(value >= 1 && value <= 24, WHMC_EARG, "whmc_set_option: pairs per force launch must be 1 .. 24");
      c->force_chunk = (int)value;
      return WHMC_OK;
    case WHMC_OPT_HOP_WG_PER_CU:
      WHMC_CHECK(value == 0 || (value >= 2 && value <= 8 && c->set_wg_cap((int)value)), WHMC_EARG,
                 "whmc_set_option: workgroups per compute unit must be 0 (no cap) or 2 .. 8");
      if (value == 0) c->set_wg_cap(0);
      return WHMC_OK;
    case WHMC_OPT_HOP_SCHEDULE:
      WHMC_CHECK(value == 0 || value == 1, WHMC_EARG, "whmc_set_option: the schedule must be 0 or 1");
      WHMC_CHECK(c->set_schedule((int)value, c->hop_chunk), WHMC_EARG,
                 "whmc_set_option: the time-slab schedule needs L_t divisible by 8 and time slices of whole "
                 "128-site blocks");
      return WHMC_OK;
    default:
      set_error("whmc_set_option: unknown option " + std::to_string(option));
      return WHMC_EARG;
  }
}

whmc_status whmc_get_option(const whmc_ctx* c, int option, long long* value) {
  WHMC_CHECK(c && value, WHMC_EARG, "whmc_get_option: null argument");
  switch (option) {
    case WHMC_OPT_STREAM_THRESHOLD: *value = c->stream_threshold; return WHMC_OK;
    case WHMC_OPT_HOP_SCHEDULE: *value = c->g.sched; return WHMC_OK;
    case WHMC_OPT_HOP_WG_PER_CU: *value = c->hop_wg_per_cu; return WHMC_OK;
    case WHMC_OPT_HOP_CHUNK: *value = c->hop_chunk; return WHMC_OK;
    case WHMC_OPT_FORCE_KERNEL: *value = c->force_kernel; return WHMC_OK;
    case WHMC_OPT_FORCE_CHUNK: *value = c->force_chunk; return WHMC_OK;
    default:
      set_error("whmc_get_option: unknown option " + std::to_string(option));
      return WHMC_EARG;
  }
}

whmc_status whmc_pack_algebra(whmc_ctx* c, double* dst, const double* src) {
  WHMC_CHECK(c && dst && src && dst != src, WHMC_EARG, "whmc_pack_algebra: bad argument");
  return pack_algebra(c, dst, src, 0);
}
whmc_status whmc_unpack_algebra(whmc_ctx* c, double* dst, const double* src) {
  WHMC_CHECK(c && dst && src && dst != src, WHMC_EARG, "whmc_unpack_algebra: bad argument");
  return pack_algebra(c, dst, src, 1);
}

}  // extern "C"
