// Device-side building blocks for the Wilson hot path on gfx950: complex and SU(3) arithmetic,
// the storage formats of spinors and links in every precision, and checkerboard geometry.
//
// Storage (over the V/2 sites of one parity, in 64-site AoSoA blocks -- see aos() -- so that the
// 64 lanes of a wavefront touch 64 consecutive 8/16-byte words of one component):
//   spinor F64 : double2, 12 components      component c = 3*spin + colour, one complex each
//   spinor F32 : float4, 6 components        two complex components per float4
//   spinor F16 : uint4, 3 components, then float [Vh] per-site scales (max |component|); four
//                                             complex (8 halves) per uint4, divided by the scale
//   link  F64-18 : double2 [2][4] x 9 comps  [parity of x][mu] block of U_{x,mu}[row*3+col]
//   link  F64-12 : double2 [2][4] x 6 comps  rows 0 and 1; row 2 = conj(row0 x row1)
//   link  F32-18 : float2  [2][4] x 9 comps
//   link  F32-12 : float4  [2][4] x 3 comps  rows 0,1 as 3 float4 (2 complex each)
//   link  F16-12 : uint2   [2][4] x 3 comps  rows 0,1 as 3 x (4 halves = 2 complex)
//   link  F64-8  : double2 [2][4] x 4 comps  U01, U02, U10, (phase of U00, phase of U20)
//   link  F32-8  : float4  [2][4] x 2 comps  (U01, U02), (U10, phase of U00, phase of U20)
//   link  F16-8  : uint4   [2][4] x 1 comp   8 halves: U01, U02, U10, phases / pi of U00 and U20
// Link entries are bounded by 1 in modulus, so half precision links need no scale.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

#define WHMC_DEV __device__ __forceinline__

namespace whmc {

template <typename R>
struct cplx {
  R re, im;
};

template <typename R> WHMC_DEV cplx<R> mk(R a, R b) { return {a, b}; }
template <typename R> WHMC_DEV cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> WHMC_DEV cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> WHMC_DEV cplx<R> operator-(cplx<R> a) { return {-a.re, -a.im}; }
template <typename R> WHMC_DEV cplx<R> operator*(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> WHMC_DEV cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename R> WHMC_DEV cplx<R> cjmul(cplx<R> a, cplx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R> WHMC_DEV cplx<R> conj(cplx<R> a) { return {a.re, -a.im}; }
template <typename R> WHMC_DEV cplx<R> times_i(cplx<R> a) { return {-a.im, a.re}; }
template <typename R> WHMC_DEV cplx<R> times_mi(cplx<R> a) { return {a.im, -a.re}; }
template <typename R> WHMC_DEV R norm2(cplx<R> a) { return a.re * a.re + a.im * a.im; }

template <typename R>
struct Spinor {
  cplx<R> c[4][3];
};
template <typename R>
struct HalfSpinor {
  cplx<R> c[2][3];
};
template <typename R>
struct SU3 {
  cplx<R> e[3][3];
};

template <typename R> WHMC_DEV void zero(Spinor<R>& s) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) s.c[a][b] = {R(0), R(0)};
}

// y = U x   and   y = U^dag x   on a colour vector
template <typename R> WHMC_DEV void mul(const SU3<R>& U, const cplx<R>* x, cplx<R>* y) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<R> s = cmul(U.e[a][0], x[0]);
    s = s + cmul(U.e[a][1], x[1]);
    s = s + cmul(U.e[a][2], x[2]);
    y[a] = s;
  }
}
template <typename R> WHMC_DEV void mul_dag(const SU3<R>& U, const cplx<R>* x, cplx<R>* y) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<R> s = cjmul(U.e[0][a], x[0]);
    s = s + cjmul(U.e[1][a], x[1]);
    s = s + cjmul(U.e[2][a], x[2]);
    y[a] = s;
  }
}
// third row of an SU(3) matrix from the first two: r2 = conj(r0 x r1)
template <typename R> WHMC_DEV void reconstruct_row2(SU3<R>& U) {
  U.e[2][0] = conj(cmul(U.e[0][1], U.e[1][2]) - cmul(U.e[0][2], U.e[1][1]));
  U.e[2][1] = conj(cmul(U.e[0][2], U.e[1][0]) - cmul(U.e[0][0], U.e[1][2]));
  U.e[2][2] = conj(cmul(U.e[0][0], U.e[1][1]) - cmul(U.e[0][1], U.e[1][0]));
}

// 8 real parameters per link, the form of Clark, Babich, Barros, Brower and Rebbi (Comput. Phys.
// Commun. 181 (2010) 1517): U01, U02, one of U10 / U20 and the phases of U00 and of the other one.
// Unit rows and columns give n = |U01|^2 + |U02|^2 = 1 - |U00|^2 = |U10|^2 + |U20|^2, hence the
// moduli of U00 and of the entry stored by its phase; the other four entries follow from det U = 1,
// which makes every entry the complex conjugate of its cofactor, together with the orthogonality
// of column 0 to columns 1 and 2:
//   U11 = -(conj(U00) U01 U10 + conj(U02) conj(U20)) / n,   U12 = (conj(U01) conj(U20) - conj(U00) U02 U10) / n,
//   U21 = -(conj(U00) U01 U20 - conj(U02) conj(U10)) / n,   U22 = -(conj(U00) U02 U20 + conj(U01) conj(U10)) / n.
// Of U10, U20 the one of smaller modulus is stored in full (FP64 and FP32): the other's modulus,
// sqrt(n - |stored|^2) >= sqrt(n / 2), then suffers no cancellation.  The choice is flagged by
// storing the phase plus 8 (phases lie in [-pi, pi]).  A link with n = 0 (U00 of modulus 1) has no
// such form; the derivation of the format rejects fields with such links.
// Double precision: e^{it} for |t| <= pi + 1e-6 (the stored phases), without the general library
// routine, whose reduction of arbitrary arguments needs many registers.  Cody-Waite reduction
// (W. J. Cody and W. Waite, Software Manual for the Elementary Functions, 1980): t = k pi/2 + r with
// k = rint(2t / pi) in {-2, ..., 2} and pi/2 split into a head (the double nearest to pi/2) and a
// tail, so that t - k * head is exact (Sterbenz) and |r| <= pi/4 (1 + 1e-16).  Then the Taylor series
// of sin r and cos r up to r^17 / 17! and r^18 / 18!, whose first omitted terms are below 2e-19 on
// that range, summed by Horner's rule in r^2; the quadrant k mod 4 permutes and signs the results.
WHMC_DEV void phase(double t, cplx<double>& e) {
  constexpr double two_over_pi = 0.63661977236758134308;
  constexpr double pio2_hi = 1.5707963267948966192;     // the double nearest to pi / 2
  constexpr double pio2_lo = 6.1232339957367658e-17;    // pi / 2 - pio2_hi
  const double k = rint(t * two_over_pi);
  const double r = (t - k * pio2_hi) - k * pio2_lo;
  const double r2 = r * r;
  // sin r = r (1 - r^2/3! + r^4/5! - ... + r^16/17!), cos r = 1 - r^2/2! + ... + r^18/18!
  double sp = 1.0 / 355687428096000.0;                  // 1 / 17!
  sp = fma(sp, r2, -1.0 / 1307674368000.0);             // 1 / 15!
  sp = fma(sp, r2, 1.0 / 6227020800.0);                 // 1 / 13!
  sp = fma(sp, r2, -1.0 / 39916800.0);                  // 1 / 11!
  sp = fma(sp, r2, 1.0 / 362880.0);                     // 1 / 9!
  sp = fma(sp, r2, -1.0 / 5040.0);                      // 1 / 7!
  sp = fma(sp, r2, 1.0 / 120.0);                        // 1 / 5!
  sp = fma(sp, r2, -1.0 / 6.0);                         // 1 / 3!
  const double sn = fma(r * r2, sp, r);
  double cp = 1.0 / 6402373705728000.0;                 // 1 / 18!
  cp = fma(cp, r2, -1.0 / 20922789888000.0);            // 1 / 16!
  cp = fma(cp, r2, 1.0 / 87178291200.0);                // 1 / 14!
  cp = fma(cp, r2, -1.0 / 479001600.0);                 // 1 / 12!
  cp = fma(cp, r2, 1.0 / 3628800.0);                    // 1 / 10!
  cp = fma(cp, r2, -1.0 / 40320.0);                     // 1 / 8!
  cp = fma(cp, r2, 1.0 / 720.0);                        // 1 / 6!
  cp = fma(cp, r2, -1.0 / 24.0);                        // 1 / 4!
  cp = fma(cp, r2, 0.5);                                // 1 / 2!
  const double cs = fma(-r2, cp, 1.0);
  const int q = (int)k & 3;   // two's complement: -1 -> 3, -2 -> 2
  const double s_ = (q & 1) ? cs : sn, c_ = (q & 1) ? sn : cs;
  e.im = (q & 2) ? -s_ : s_;
  e.re = ((q + 1) & 2) ? -c_ : c_;
}
// single precision: the hardware sine / cosine (absolute error about 5e-7 on [-pi, pi], the range
// the stored phases lie in), below the rounding of the FP32 / FP16 formats themselves
WHMC_DEV void phase(float t, cplx<float>& e) { __sincosf(t, &e.im, &e.re); }
WHMC_DEV double rsq(double x) { return sqrt(x); }
WHMC_DEV float rsq(float x) { return sqrtf(x); }

// U.e[0][1], U.e[0][2] set; s = U10 (t_s < 4: phase of U20) or U20 (t_s = phase of U10 + 8)
template <typename R> WHMC_DEV void reconstruct8(SU3<R>& U, cplx<R> s, R t00, R t_s) {
  const cplx<R> a2 = U.e[0][1], a3 = U.e[0][2];
  const R n = norm2(a2) + norm2(a3);
  const bool swapped = t_s > R(4);
  cplx<R> e00, eo;
  phase(t00, e00);
  phase(swapped ? t_s - R(8) : t_s, eo);
  const cplx<R> a1 = rsq(fmax(R(1) - n, R(0))) * e00;
  const cplx<R> o = rsq(fmax(n - norm2(s), R(0))) * eo;
  const cplx<R> b1 = swapped ? o : s, c1 = swapped ? s : o;
  const R inv = R(1) / n;
  const cplx<R> ca1 = conj(a1), ca2 = conj(a2), ca3 = conj(a3), cb1 = conj(b1), cc1 = conj(c1);
  U.e[0][0] = a1;
  U.e[1][0] = b1;
  U.e[2][0] = c1;
  U.e[1][1] = -inv * (cmul(cmul(ca1, a2), b1) + cmul(ca3, cc1));
  U.e[1][2] = inv * (cmul(ca2, cc1) - cmul(cmul(ca1, a3), b1));
  U.e[2][1] = -inv * (cmul(cmul(ca1, a2), c1) - cmul(ca3, cb1));
  U.e[2][2] = -inv * (cmul(cmul(ca1, a3), c1) + cmul(ca2, cb1));
}

// ------------------------------------------------------------------ geometry
// dims L[0..3] = (L_t, L_z, L_y, L_x); direction mu is axis mu.  Checkerboard index
// cb = lex / 2 with lex = ((t L_z + z) L_y + y) L_x + x.
struct Geom {
  int L[4];
  int Vh;
  int Lxh;   // L_x / 2
  int nbs;   // blocks per time slice for site_block (0: a slice is not a whole number of blocks)
  int xq;    // workgroups per XCD per time slice, ceil(nbs / 8); 0: plain eighths of the lattice
  // single-RHS stencil schedule (site_block): 0 = slice ranges (site_block_xq); 1 = time slabs:
  // XCD k owns the tx = L_t / 8 slices [k tx, (k + 1) tx) and sweeps them in chunks of tq blocks of
  // a slice, all tx slices of a chunk before the next chunk (site_block_slab); nch = ceil(nbs / tq)
  int sched, tx, tq, nch;
};

struct Coords {
  int t, z, y, x, row, xh;
};

WHMC_DEV Coords coords_of(const Geom& g, int i, int par) {
  Coords c;
  c.row = i / g.Lxh;
  c.xh = i - c.row * g.Lxh;
  int tz = c.row / g.L[2];
  c.y = c.row - tz * g.L[2];
  c.t = tz / g.L[1];
  c.z = tz - c.t * g.L[1];
  c.x = 2 * c.xh + ((par + c.t + c.z + c.y) & 1);
  return c;
}

// checkerboard index of the neighbour x + dir*mu_hat (dir = +1 / -1); also returns whether the
// hop crosses the time boundary (fermion sign -1).
template <int MU, int DIR>
WHMC_DEV int neighbour(const Geom& g, const Coords& c, bool& wrap_t) {
  wrap_t = false;
  if (MU == 3) {
    int x = c.x + DIR;
    x = (x == g.L[3]) ? 0 : (x < 0 ? g.L[3] - 1 : x);
    return c.row * g.Lxh + (x >> 1);
  } else if (MU == 2) {
    int y = c.y + DIR;
    int d = DIR;
    if (y == g.L[2]) d = 1 - g.L[2];
    if (y < 0) d = g.L[2] - 1;
    return (c.row + d) * g.Lxh + c.xh;
  } else if (MU == 1) {
    int z = c.z + DIR;
    int d = DIR;
    if (z == g.L[1]) d = 1 - g.L[1];
    if (z < 0) d = g.L[1] - 1;
    return (c.row + d * g.L[2]) * g.Lxh + c.xh;
  } else {
    int t = c.t + DIR;
    int d = DIR;
    if (t == g.L[0]) { d = 1 - g.L[0]; wrap_t = true; }
    if (t < 0) { d = g.L[0] - 1; wrap_t = true; }
    return (c.row + d * g.L[2] * g.L[1]) * g.Lxh + c.xh;
  }
}

// ------------------------------------------------------------------ cache-policy helpers
// NT = non-temporal: data streamed once (links of a large lattice, outputs that are not read back
// soon) is marked so that it does not evict reusable neighbour spinors from L2 / Infinity Cache.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));

template <bool NT> WHMC_DEV double2 ldg(const double2* p) {
  if (NT) { d2v v = __builtin_nontemporal_load((const d2v*)p); return make_double2(v.x, v.y); }
  return *p;
}
template <bool NT> WHMC_DEV float4 ldg(const float4* p) {
  if (NT) { f4v v = __builtin_nontemporal_load((const f4v*)p); return make_float4(v.x, v.y, v.z, v.w); }
  return *p;
}
template <bool NT> WHMC_DEV float2 ldg(const float2* p) {
  if (NT) { f2v v = __builtin_nontemporal_load((const f2v*)p); return make_float2(v.x, v.y); }
  return *p;
}
template <bool NT> WHMC_DEV uint2 ldg(const uint2* p) {
  if (NT) { u2v v = __builtin_nontemporal_load((const u2v*)p); return make_uint2(v.x, v.y); }
  return *p;
}
template <bool NT> WHMC_DEV void stg(double2* p, double2 v) {
  if (NT) __builtin_nontemporal_store(d2v{v.x, v.y}, (d2v*)p);
  else *p = v;
}
template <bool NT> WHMC_DEV void stg(float4* p, float4 v) {
  if (NT) __builtin_nontemporal_store(f4v{v.x, v.y, v.z, v.w}, (f4v*)p);
  else *p = v;
}
template <bool NT> WHMC_DEV void stg(uint4* p, uint4 v) {
  if (NT) __builtin_nontemporal_store(u4v{v.x, v.y, v.z, v.w}, (u4v*)p);
  else *p = v;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.  Renumber them so
// that XCD k works on the k-th contiguous eighth of the sites: neighbours in y, z (and x) then
// sit in the same L2.  Bijective on [0, nb) for any nb.
WHMC_DEV int xcd_remap(int B, int nb) {
  const int k = B & 7, m = B >> 3, q = nb >> 3, r = nb & 7;
  return k * q + (k < r ? k : r) + m;
}

// Workgroup -> block of sites for the stencil kernels.  A time slice is a contiguous range of cb
// indices.  When a slice holds a whole number g.nbs >= 8 of blocks, it is cut into 8 ranges of
// floor or ceil(g.nbs / 8) blocks, XCD k takes range k of every slice and sweeps t upwards: an
// input spinor is then read by its t-1 and t+1 neighbours a few ranges apart, while both are in the
// same L2, instead of a whole slice of the lattice apart.  The grid then has nb = 8 * g.xq * L_t
// workgroups, g.xq = ceil(g.nbs / 8); a workgroup beyond its XCD's range gets the block index
// L_t * g.nbs, whose sites all lie past the last site.  Otherwise (g.xq = 0, nb = ceil(Vh / block))
// XCD k takes the k-th contiguous eighth of the blocks.
WHMC_DEV int site_block_xq(const Geom& g, int B, int nb) {
  if (g.xq == 0) return xcd_remap(B, nb);
  const int k = B & 7, m = B >> 3;
  const int t = m / g.xq, j = m - t * g.xq;
  const int lo = k * g.nbs / 8, hi = (k + 1) * g.nbs / 8;
  if (lo + j >= hi) return g.L[0] * g.nbs;
  return t * g.nbs + lo + j;
}

// Time-slab schedule: XCD k owns the tx consecutive time slices starting at k tx and works through
// them chunk by chunk, a chunk being tq consecutive blocks of a slice (a few z planes): the tx
// slices of chunk 0, then of chunk 1, ...  A spinor is then read by its t +- 1 and z +- 1 neighbours
// while it is in the same L2 (z neighbours across a chunk edge one chunk later), and only the two
// slices at the slab's ends are also read by another XCD.  The grid has 8 tx nch tq workgroups;
// one whose chunk runs past the slice's nbs blocks gets the block index L_t nbs (all sites past the
// last one).
WHMC_DEV int site_block_slab(const Geom& g, int B) {
  const int k = B & 7, m = B >> 3;
  const int per = g.tx * g.tq;
  const int ch = m / per, r = m - ch * per;
  const int t = r / g.tq, j = r - t * g.tq;
  const int blk = ch * g.tq + j;
  if (blk >= g.nbs) return g.L[0] * g.nbs;
  return (k * g.tx + t) * g.nbs + blk;
}

// workgroup -> block of sites for the single-RHS stencil, solver and BiCGstab kernels
WHMC_DEV int site_block(const Geom& g, int B, int nb) {
  return g.sched == 1 ? site_block_slab(g, B) : site_block_xq(g, B, nb);
}

// G groups (e.g. of right-hand sides) per block of sites in one 1D grid of nb = G * (site grid)
// workgroups: the G groups of a block run back to back on the same XCD.  grp receives the group;
// slot numbers the workgroups of one group without repeats in [0, nb / G).
WHMC_DEV int site_block_grp(const Geom& g, int B, int nb, int G, int& grp, int& slot) {
  if (g.xq == 0) {
    const int b = xcd_remap(B, nb);
    slot = b / G;
    grp = b - slot * G;
    return slot;
  }
  const int k = B & 7, m = B >> 3;
  const int per_t = g.xq * G;
  const int t = m / per_t, r = m - t * per_t;
  const int j = r / G;
  grp = r - j * G;
  slot = (t * g.xq + j) * 8 + k;
  const int lo = k * g.nbs / 8, hi = (k + 1) * g.nbs / 8;
  if (lo + j >= hi) return g.L[0] * g.nbs;
  return t * g.nbs + lo + j;
}

// Both parities in one grid of 2 nb workgroups: the XCD's m-th workgroup does parity m & 1 of its
// (m >> 1)-th block, so each XCD applies both parities to the same region.
WHMC_DEV int site_block_pair(const Geom& g, int B, int nb, int& par) {
  const int k = B & 7, m = B >> 3;
  if (g.xq == 0) {
    const int b = xcd_remap(B, 2 * nb);
    par = b & 1;
    return b >> 1;
  }
  par = m & 1;
  return site_block_xq(g, ((m >> 1) << 3) | k, nb);
}

// ------------------------------------------------------------------ AoSoA addressing
// Per-site fields with K components over n sites are stored in blocks of 64 sites (one
// wavefront): component k of site i lives at (i/64)*64*K + k*w + i%64, with w = 64 for full blocks
// and w = n%64 for the last, partial block.  A wavefront's load of one component is a single
// contiguous 1 KiB (FP64) run, the fields of a block share DRAM pages, and a field occupies
// exactly K*n elements for any n.
WHMC_DEV size_t aos(int k, int i, int K, int n) {
  const int blk = i >> 6;
  const int w = blk < (n >> 6) ? 64 : (n & 63);
  return (size_t)blk * 64 * K + (size_t)k * w + (i & 63);
}

// ------------------------------------------------------------------ spinor storage
struct SpinorF64 {
  using Real = double;
  double2* p;
  int stride;
  WHMC_DEV void load(int i, Spinor<double>& s) const {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      double2 v = p[aos(k, i, 12, stride)];
      s.c[k / 3][k % 3] = {v.x, v.y};
    }
  }
  template <bool NT = false>
  WHMC_DEV void store(int i, const Spinor<double>& s) const {
#pragma unroll
    for (int k = 0; k < 12; ++k)
      stg<NT>(p + aos(k, i, 12, stride), make_double2(s.c[k / 3][k % 3].re, s.c[k / 3][k % 3].im));
  }
};

struct SpinorF32 {
  using Real = float;
  float4* p;
  int stride;
  WHMC_DEV void load(int i, Spinor<float>& s) const {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float4 v = p[aos(k, i, 6, stride)];
      s.c[(2 * k) / 3][(2 * k) % 3] = {v.x, v.y};
      s.c[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v.z, v.w};
    }
  }
  template <bool NT = false>
  WHMC_DEV void store(int i, const Spinor<float>& s) const {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      cplx<float> a = s.c[(2 * k) / 3][(2 * k) % 3], b = s.c[(2 * k + 1) / 3][(2 * k + 1) % 3];
      stg<NT>(p + aos(k, i, 6, stride), make_float4(a.re, a.im, b.re, b.im));
    }
  }
};

WHMC_DEV float h2f(unsigned short h) { return __half2float(__ushort_as_half(h)); }
WHMC_DEV unsigned short f2h(float f) { return __half_as_ushort(__float2half_rn(f)); }

struct SpinorF16 {
  using Real = float;
  uint4* p;
  float* scale;
  int stride;
  WHMC_DEV void load(int i, Spinor<float>& s) const {
    float sc = scale[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint4 v = p[aos(k, i, 3, stride)];
      unsigned int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int comp = 4 * k + j;
        s.c[comp / 3][comp % 3] = {sc * h2f((unsigned short)(w[j] & 0xffffu)), sc * h2f((unsigned short)(w[j] >> 16))};
      }
    }
  }
  template <bool NT = false>
  WHMC_DEV void store(int i, const Spinor<float>& s) const {
    float m = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) m = fmaxf(m, fmaxf(fabsf(s.c[a][b].re), fabsf(s.c[a][b].im)));
    float inv = m > 0.f ? 1.0f / m : 0.f;
    scale[i] = m;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      unsigned int w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int comp = 4 * k + j;
        w[j] = (unsigned int)f2h(inv * s.c[comp / 3][comp % 3].re) |
               ((unsigned int)f2h(inv * s.c[comp / 3][comp % 3].im) << 16);
      }
      stg<NT>(p + aos(k, i, 3, stride), make_uint4(w[0], w[1], w[2], w[3]));
    }
  }
};

// ------------------------------------------------------------------ link storage
// every link type: load(par, mu, i) -> U_{x,mu} for the site x of parity `par`, cb index i.
template <bool NT = false>
struct LinkF64_18T {
  using Real = double;
  const double2* p;
  int Vh;
  WHMC_DEV void load(int par, int mu, int i, SU3<double>& U) const {
    const double2* q = p + (size_t)(par * 4 + mu) * 9 * Vh;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      double2 v = ldg<NT>(q + aos(k, i, 9, Vh));
      U.e[k / 3][k % 3] = {v.x, v.y};
    }
  }
};

template <bool NT = false>
struct LinkF64_12T {
  using Real = double;
  const double2* p;
  int Vh;
  WHMC_DEV void load(int par, int mu, int i, SU3<double>& U) const {
    const double2* q = p + (size_t)(par * 4 + mu) * 6 * Vh;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double2 v = ldg<NT>(q + aos(k, i, 6, Vh));
      U.e[k / 3][k % 3] = {v.x, v.y};
    }
    reconstruct_row2(U);
  }
};

template <bool NT = false>
struct LinkF32_12T {
  using Real = float;
  const float4* p;
  int Vh;
  WHMC_DEV void load(int par, int mu, int i, SU3<float>& U) const {
    const float4* q = p + (size_t)(par * 4 + mu) * 3 * Vh;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float4 v = ldg<NT>(q + aos(k, i, 3, Vh));
      U.e[(2 * k) / 3][(2 * k) % 3] = {v.x, v.y};
      U.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v.z, v.w};
    }
    reconstruct_row2(U);
  }
};

template <bool NT = false>
struct LinkF32_18T {
  using Real = float;
  const float2* p;
  int Vh;
  WHMC_DEV void load(int par, int mu, int i, SU3<float>& U) const {
    const float2* q = p + (size_t)(par * 4 + mu) * 9 * Vh;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float2 v = ldg<NT>(q + aos(k, i, 9, Vh));
      U.e[k / 3][k % 3] = {v.x, v.y};
    }
  }
};

template <bool NT = false>
struct LinkF16_12T {
  using Real = float;
  const uint2* p;
  int Vh;
  WHMC_DEV void load(int par, int mu, int i, SU3<float>& U) const {
    const uint2* q = p + (size_t)(par * 4 + mu) * 3 * Vh;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint2 v = ldg<NT>(q + aos(k, i, 3, Vh));
      U.e[(2 * k) / 3][(2 * k) % 3] = {h2f((unsigned short)(v.x & 0xffffu)), h2f((unsigned short)(v.x >> 16))};
      U.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = {h2f((unsigned short)(v.y & 0xffffu)), h2f((unsigned short)(v.y >> 16))};
    }
    reconstruct_row2(U);
  }
};

template <bool NT = false>
struct LinkF64_8T {
  using Real = double;
  const double2* p;
  int Vh;
  WHMC_DEV void load(int par, int mu, int i, SU3<double>& U) const {
    const double2* q = p + (size_t)(par * 4 + mu) * 4 * Vh;
    const double2 v0 = ldg<NT>(q + aos(0, i, 4, Vh)), v1 = ldg<NT>(q + aos(1, i, 4, Vh));
    const double2 v2 = ldg<NT>(q + aos(2, i, 4, Vh)), v3 = ldg<NT>(q + aos(3, i, 4, Vh));
    U.e[0][1] = {v0.x, v0.y};
    U.e[0][2] = {v1.x, v1.y};
    reconstruct8(U, cplx<double>{v2.x, v2.y}, v3.x, v3.y);
  }
};

template <bool NT = false>
struct LinkF32_8T {
  using Real = float;
  const float4* p;
  int Vh;
  WHMC_DEV void load(int par, int mu, int i, SU3<float>& U) const {
    const float4* q = p + (size_t)(par * 4 + mu) * 2 * Vh;
    const float4 v0 = ldg<NT>(q + aos(0, i, 2, Vh)), v1 = ldg<NT>(q + aos(1, i, 2, Vh));
    U.e[0][1] = {v0.x, v0.y};
    U.e[0][2] = {v0.z, v0.w};
    reconstruct8(U, cplx<float>{v1.x, v1.y}, v1.z, v1.w);
  }
};

// FP16: always U10 in full and the phase of U20 (halves of the phases / pi)
template <bool NT = false>
struct LinkF16_8T {
  using Real = float;
  const uint4* p;
  int Vh;
  WHMC_DEV void load(int par, int mu, int i, SU3<float>& U) const {
    const uint4* q = p + (size_t)(par * 4 + mu) * Vh + aos(0, i, 1, Vh);
    u4v w;
    if (NT) w = __builtin_nontemporal_load((const u4v*)q);
    else { const uint4 v = *q; w = u4v{v.x, v.y, v.z, v.w}; }
    U.e[0][1] = {h2f((unsigned short)(w.x & 0xffffu)), h2f((unsigned short)(w.x >> 16))};
    U.e[0][2] = {h2f((unsigned short)(w.y & 0xffffu)), h2f((unsigned short)(w.y >> 16))};
    const cplx<float> b1 = {h2f((unsigned short)(w.z & 0xffffu)), h2f((unsigned short)(w.z >> 16))};
    const float pi = 3.14159265358979f;
    reconstruct8(U, b1, pi * h2f((unsigned short)(w.w & 0xffffu)), pi * h2f((unsigned short)(w.w >> 16)));
  }
};

// 8-real accessors (their reconstruction makes the hop arithmetic-heavy: not occupancy-capped)
template <class L> struct is_8real : std::false_type {};
template <bool NT> struct is_8real<LinkF64_8T<NT>> : std::true_type {};
template <bool NT> struct is_8real<LinkF32_8T<NT>> : std::true_type {};
template <bool NT> struct is_8real<LinkF16_8T<NT>> : std::true_type {};

using LinkF64_18 = LinkF64_18T<false>;
using LinkF64_12 = LinkF64_12T<false>;
using LinkF32_18 = LinkF32_18T<false>;
using LinkF32_12 = LinkF32_12T<false>;
using LinkF16_12 = LinkF16_12T<false>;

// ------------------------------------------------------------------ reductions
// wavefront (64 lanes) then workgroup sum; result valid in thread 0.
template <int BLOCK>
WHMC_DEV double block_sum(double v, double* lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) s += lds[w];
  }
  return s;
}

struct Reduce {
  double* partials;    // per-block partial sums
  unsigned* counter;   // unused by the two-pass scheme (kept for the ABI-internal layout)
  double* result;      // final sums
};

// Two-pass deterministic reductions.  Pass 1: each block reduces its values and writes one
// partial per value with a plain store -- no fence or atomic, which on gfx950 would force an
// L2 write-back per block (the 8 XCD L2s are not coherent within a kernel).  Pass 2 (a separate,
// tiny kernel, so the kernel boundary makes the partials visible) adds the partials of each value
// in a fixed order.  Every thread of the pass-1 grid must call block_partial.
template <int BLOCK>
WHMC_DEV void block_partial(double v, double* partials, int slot) {
  __shared__ double lds[BLOCK / 64];
  __syncthreads();
  const double s = block_sum<BLOCK>(v, lds);
  if (threadIdx.x == 0) partials[slot] = s;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_finish_sum(const double* partials, int n, double* out);

// pass 2 helper: sum of p[0..n) by one block of BLOCK threads in a fixed order; valid in thread 0
template <int BLOCK>
WHMC_DEV double sum_partials(const double* p, int n) {
  __shared__ double lds[BLOCK / 64];
  double t = 0.0;
  for (int k = threadIdx.x; k < n; k += BLOCK) t += p[k];
  __syncthreads();
  return block_sum<BLOCK>(t, lds);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_finish_sum(const double* partials, int n, double* out) {
  const double t = sum_partials<BLOCK>(partials, n);
  if (threadIdx.x == 0) *out = t;
}

}  // namespace whmc
