/*
 * whmc.h -- C ABI of the MI355X (gfx950) hot path of two-flavour Wilson-fermion HMC with
 * hopping-parameter-expansion filtering, after M. Hasenbusch, arXiv:1805.03560.
 *
 * Conventions (the paper leaves them open):
 *   - lattice dims are (L_t, L_z, L_y, L_x); direction mu is axis mu (mu = 0 is time).
 *     lex = ((t L_z + z) L_y + y) L_x + x, parity = (t+z+y+x) mod 2, cb = lex / 2.
 *     All extents must be even and >= 2 (even/odd ordering, Sec. 2.2).
 *   - gauge field periodic; fermion hops across the time boundary carry -1 (Sec. 4).
 *   - chiral Euclidean gamma basis: gamma_0 = [[0,1],[1,0]], gamma_k = [[0,-i s_k],[i s_k,0]]
 *     (s_k Pauli matrices, k = 1,2,3 acting along axes 1,2,3), gamma_5 = g0 g1 g2 g3.
 *   - H has no factor 1/2:  M = 1 - kappa H,  M_oo = 1 - kappa^2 H_oe H_eo on the odd sites.
 *   - momenta and forces are antihermitian traceless 3x3 matrices stored as 8 real coordinates on
 *     T_a = i lambda_a / 2 (Gell-Mann lambda_a), so (Pi,Pi) = -2 sum Tr Pi^2 = sum pi_a^2.
 *
 * Memory.  Every field pointer is DEVICE memory owned by the caller (e.g. a torch tensor on the
 * context's GPU); the library never frees it.  Device layouts ("whmc layout"): per-site fields of
 * K components over the Vh sites of one parity are stored in blocks of 64 sites -- component k of
 * site cb at element (cb/64)*64*K + k*w + cb%64, w = 64 for full blocks and w = Vh%64 for the last
 * block -- so a field is exactly K*Vh elements:
 *   half spinor F64   double2, K = 12         complex component 3*spin+colour
 *   half spinor F32   float4,  K = 6          complex components (2k, 2k+1) in float4 k
 *   half spinor F16   uint4,   K = 3, then float [Vh] per-site scales (4 complex as halves per
 *                                             uint4, divided by the site's scale)
 *   full spinor       two half spinors, even parity first
 *   nrhs spinors      nrhs consecutive fields
 *   algebra field     double [2][4][8][Vh]    [parity][mu][a][cb]  (momenta, forces; plain SoA)
 * Canonical layouts (for import/export only):
 *   gauge    complex128 [V][4][3][3]          U_{x,mu}[row][col], x in lex order
 *   spinor   complex128 [V][4][3] (full) or [Vh][4][3] (one parity, cb order)
 *   algebra  float64 [V][4][8]
 *
 * Streams.  All work is enqueued on the context's HIP stream and is asynchronous unless the
 * function returns a host scalar (solver statistics, actions, trajectory results), in which case
 * it synchronises that stream before returning.
 *
 * Errors.  Every function returns a whmc_status; on failure whmc_last_error() holds a message
 * for the calling thread.  Nothing aborts or throws across the ABI.  Unless noted, functions are
 * not re-entrant on one context (one context = one stream of work).
 */
#ifndef WHMC_H
#define WHMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WHMC_ABI_VERSION 2

typedef enum whmc_status {
  WHMC_OK = 0,
  WHMC_EARG = 1,     /* bad argument: null pointer, odd extent, unknown enum, nrhs < 1, ... */
  WHMC_EHIP = 2,     /* a HIP runtime call failed (message names it) */
  WHMC_ENOCONV = 3,  /* solver hit maxiter; statistics are still filled in */
  WHMC_EUNSUP = 4,   /* valid but unsupported combination (e.g. filter order k > 2) */
  WHMC_ENOTSU3 = 5,  /* gauge field not unitary / det != 1 within the given tolerance */
  WHMC_ESTATE = 6,   /* call out of order (e.g. no gauge field loaded yet) */
  WHMC_ENONFINITE = 7 /* a NaN or infinity in an input or in a solver's scalars (e.g. a NaN in phi) */
} whmc_status;

typedef enum whmc_prec { WHMC_F64 = 0, WHMC_F32 = 1, WHMC_F16 = 2 } whmc_prec;
/* link storage: 18 reals (all entries), 12 (rows 0 and 1; row 2 = conj(row 0 x row 1)) or 8 (U01, U02,
 * one of U10 / U20 and two phases; the 8-parameter form of Clark et al., Comput. Phys. Commun. 181
 * (2010) 1517).  The 8-real form needs |U01|^2 + |U02|^2 > 0 on every link (> 1e-20 in FP64 and
 * FP32, > 1e-6 in FP16); a field with a link that violates it gives WHMC_EUNSUP when the format is
 * first used (e.g. unit links). */
typedef enum whmc_links { WHMC_L8 = 8, WHMC_L12 = 12, WHMC_L18 = 18 } whmc_links;
typedef enum whmc_integrator { WHMC_LEAPFROG = 0, WHMC_OMELYAN = 1 } whmc_integrator;

typedef struct whmc_ctx whmc_ctx;

/* ------------------------------------------------------------------ context */

int whmc_abi_version(void);
const char* whmc_last_error(void);

/* Create a context for a lattice of extents dims = {L_t, L_z, L_y, L_x} on HIP device `device`,
 * enqueueing on `stream` (a hipStream_t; NULL = the default stream).  Allocates the gauge
 * storage (~ V * 4 * 144 B in FP64 plus compressed copies on first use) and small scratch.
 * EARG for odd or < 2 extents or V/2 >= 2^31. */
whmc_status whmc_create(whmc_ctx** ctx, const int dims[4], int device, void* stream);
void whmc_destroy(whmc_ctx* ctx);
whmc_status whmc_set_stream(whmc_ctx* ctx, void* stream);

/* Context options (values are 64-bit integers):
 *   WHMC_OPT_STREAM_THRESHOLD  link arrays larger than this many bytes are read with non-temporal
 *                              (streaming) loads in every stencil, solver and force kernel, so that
 *                              they do not evict neighbour spinors from the caches; -1 = never,
 *                              0 = always.  Default 128 MiB (streaming pays once a link array no
 *                              longer fits the caches; smaller lattices run faster without it).
 * EARG for an unknown option or a value below -1. */
#define WHMC_OPT_STREAM_THRESHOLD 1
/*   WHMC_OPT_HOP_SCHEDULE      order of the workgroups of the single-RHS stencil, solver and
 *                              BiCGstab kernels: 0 = each XCD takes one eighth of every time slice
 *                              and sweeps t (default); 1 = each XCD takes L_t / 8 consecutive time
 *                              slices and works through them in chunks of WHMC_OPT_HOP_CHUNK blocks
 *                              of 128 sites of a slice (needs L_t divisible by 8 and time slices of
 *                              whole blocks, else EARG).  Results do not depend on it.
 *   WHMC_OPT_HOP_CHUNK         chunk of schedule 1, 1 .. blocks per time slice.
 *   WHMC_OPT_FORCE_KERNEL      pseudo-fermion force contraction: 0 = one thread per link, the eight
 *                              (parity, mu) links of 64 sites in one workgroup stepping through the
 *                              pairs together (default; lattices of more than 2^32 / 192 sites per
 *                              parity use 1), 1 = one thread per site and its four links.
 *   WHMC_OPT_FORCE_CHUNK       (X, Y) pairs summed per launch of that contraction, 1 .. 24 (default
 *                              24); later launches accumulate.  Results agree to rounding.
 *   WHMC_OPT_HOP_WG_PER_CU     occupancy cap of those kernels that work on FP64 spinors with 18- or
 *                              12-real links: 0 = none (default), 2 .. 8 = at most that many
 *                              128-thread workgroups per compute unit (each reserves LDS it does not
 *                              use).  Fewer sites in flight keep their neighbour spinors in the L2
 *                              of their XCD.  FP32 / FP16 kernels and 8-real links are never capped.
 *                              EARG if the device's LDS limits do not allow the value.  Results do
 *                              not depend on it. */
#define WHMC_OPT_HOP_SCHEDULE 2
#define WHMC_OPT_HOP_CHUNK 3
#define WHMC_OPT_FORCE_KERNEL 4
#define WHMC_OPT_FORCE_CHUNK 5
#define WHMC_OPT_HOP_WG_PER_CU 6
whmc_status whmc_set_option(whmc_ctx* ctx, int option, long long value);
whmc_status whmc_get_option(const whmc_ctx* ctx, int option, long long* value);

/* Autotuner of the single-RHS stencil schedule: times the FP64 even/odd hop pair (H_eo then H_oe,
 * 18-real links) for schedule 0 and for schedule 1 with chunks of 1/16 .. 1/2 of a time slice, each
 * without and with a cap of 2 workgroups per compute unit (each candidate's best of four interleaved
 * rounds of eight pairs), and keeps the fastest in the context
 * (WHMC_OPT_HOP_SCHEDULE / WHMC_OPT_HOP_CHUNK / WHMC_OPT_HOP_WG_PER_CU, read back with
 * whmc_get_option).  Outputs may be NULL; us receives the time per hop in microseconds.  Uses context
 * scratch of two half fields.  On an error the schedule and cap are left as they were. */
whmc_status whmc_autotune_hop(whmc_ctx* ctx, int* schedule, int* chunk, double* us);

/* Bytes of one field of the given kind in the whmc layout:
 * kind 0 = half spinor, 1 = full spinor, 2 = algebra field (prec ignored), 3 = canonical gauge. */
whmc_status whmc_field_bytes(const whmc_ctx* ctx, int kind, int prec, size_t* bytes);

/* ------------------------------------------------------------------ gauge field (Sec. 1)
 * Copy a canonical complex128 gauge field (device pointer) into the context.  The library keeps
 * an FP64 18-real master copy and derives 12-real / FP32 / FP16 copies when an operator asks for
 * them.  If unitarity_tol > 0 every link is checked: max |U U^dag - 1| and |det U - 1| must not
 * exceed it, else ENOTSU3 (the field is still loaded; 12-real formats assume det = 1). */
whmc_status whmc_load_gauge(whmc_ctx* ctx, const double* U, double unitarity_tol);
whmc_status whmc_export_gauge(whmc_ctx* ctx, double* U);

/* ------------------------------------------------------------------ layout conversion
 * parity 0 / 1: one half field (canonical [Vh][4][3]); parity -1: full field (canonical [V][4][3]
 * <-> two halves, even first).  nfields consecutive fields are converted. */
whmc_status whmc_pack_spinor(whmc_ctx* ctx, double* dst, const double* src, int parity, int nfields);
whmc_status whmc_unpack_spinor(whmc_ctx* ctx, double* dst, const double* src, int parity, int nfields);
/* Convert nhalf half-spinor fields between precisions (both in whmc layout). */
whmc_status whmc_convert_spinor(whmc_ctx* ctx, void* dst, int dst_prec, const void* src, int src_prec, int nhalf);
/* canonical float64 [V][4][8] <-> whmc algebra layout */
whmc_status whmc_pack_algebra(whmc_ctx* ctx, double* dst, const double* src);
whmc_status whmc_unpack_algebra(whmc_ctx* ctx, double* dst, const double* src);

/* ------------------------------------------------------------------ hopping matrix (Sec. 1, 2.2)
 * out_parity p in {0, 1}: out (half field of parity p) = H_{p,1-p} in (half field of parity 1-p),
 * i.e. H_eo for p = 0 and H_oe for p = 1; dagger = 1 applies the same block of H^dag.
 * out_parity = -1: out (full) = H in (full), computed as both blocks.
 * prec selects the spinor format of in/out, links the link format (F64 and F32 support L18, L12
 * and L8; F16 supports L12 and L8).  in and out must not overlap. */
whmc_status whmc_apply_H(whmc_ctx* ctx, void* out, const void* in, int out_parity, int dagger, int prec, int links);

/* Multi right-hand-side form of the even/odd hop: out_r = H_{p,1-p} in_r for r < nrhs (nrhs
 * consecutive half fields in and out, 1 <= nrhs <= 16).  Blocking: each thread applies the links
 * of its site to rhs_block right-hand sides held in registers (one link load and decode serves
 * them all), and rhs_lanes lanes of a wavefront hold the same site for further right-hand sides,
 * sharing each link load instruction.  The right-hand sides thus form groups of
 * rhs_block * rhs_lanes; rhs_order chooses the order of the workgroups:
 *   0 (block-major): the groups of a site block run back to back on one XCD, so the links are
 *     reused from its L2 (each link read from memory once per call);
 *   1 (group-major): each group sweeps the whole lattice before the next, so the neighbour
 *     spinors of the group stay in L2 (the links are read once per group).
 * Allowed: FP64 (18-, 12- or 8-real links) rhs_block = 1 with rhs_lanes = 1, 2 or 4, or rhs_block = 2
 * with rhs_lanes = 1 or 2; FP32 / FP16 (12- or 8-real links) rhs_block = 1, 2 or 4 with
 * rhs_lanes = 1 or 2; other formats WHMC_EUNSUP.  rhs_block = rhs_lanes = 0
 * takes the autotuned blocking and order (rhs_order ignored); one of them 0 reads as 1; anything
 * else is WHMC_EARG. */
whmc_status whmc_apply_H_multi(whmc_ctx* ctx, void* out, const void* in, int out_parity, int dagger, int prec,
                               int links, int nrhs, int rhs_block, int rhs_lanes, int rhs_order);

/* Autotuner: time the multi-RHS hop for every allowed blocking and order not wider than needed
 * for nrhs at this lattice size, precision and link format, remember the fastest in the context
 * and return it (rhs_order may be NULL; us, if not NULL, receives its time per launch in
 * microseconds).  Later calls with the same key return the stored choice without timing. */
whmc_status whmc_autotune(whmc_ctx* ctx, int prec, int links, int nrhs, int* rhs_block, int* rhs_lanes,
                          int* rhs_order, double* us);

/* out = M_oo in = in - kappa^2 H_oe H_eo in (dagger = 0) or M_oo^dag in (dagger = 1), FP64,
 * odd-site half fields (Sec. 2.2).  Uses context scratch for the even-site intermediate. */
whmc_status whmc_apply_Moo(whmc_ctx* ctx, double* out, const double* in, double kappa, int dagger);

/* Full-lattice fermion matrix of Sec. 1, M = 1 - kappa H (dagger = 1: M^dag = gamma_5 M gamma_5),
 * on full spinors (even half then odd half, whmc layout, FP64, 18-real links).  in and out must
 * not overlap. */
whmc_status whmc_apply_M(whmc_ctx* ctx, double* out, const double* in, double kappa, int dagger);

/* out_r = A(kappa_r) in_r for r < nrhs, FP64, with
 *   eo = 1: A = M_oo^dag M_oo on odd-site half fields (even/odd form, Sec. 2.2),
 *   eo = 0: A = M^dag M on full spinors, M = 1 - kappa H (Sec. 1).
 * The nrhs fields are consecutive (half or full fields).  in and out must not overlap.
 * Uses context scratch for the intermediates (allocated on first use). */
whmc_status whmc_apply_MdagM(whmc_ctx* ctx, double* out, const double* in, const double* kappas, int nrhs, int eo);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): whmc_apply_MdagM without any allocation.  The
 * intermediates live in a static device buffer of WHMC_NOALLOC_SCRATCH_BYTES that the library holds
 * on every GPU it runs on until the process ends (its address is looked up in whmc_create), so the
 * lattice must satisfy V * 192 <= WHMC_NOALLOC_SCRATCH_BYTES (V <= 174762 sites, e.g. 16^3 x 32),
 * else WHMC_EARG.  All calls on one GPU share that buffer: calls that overlap in time on one GPU
 * (several streams or contexts) race and give wrong results.  The buffer keeps the last call's
 * contents; nothing in it needs to start at zero.  Arguments and results as for whmc_apply_MdagM. */
#define WHMC_NOALLOC_SCRATCH_BYTES (32u << 20)
whmc_status whmc_apply_MdagM_noalloc(whmc_ctx* ctx, double* out, const double* in, const double* kappas, int nrhs,
                                     int eo);

/* ------------------------------------------------------------------ solver (Sec. 1, 4)
 * Solve M_oo(kappa_r)^dag M_oo(kappa_r) x_r = b_r (odd-site half fields, FP64 whmc layout) by CG
 * from x_r = 0, until the true FP64 residual |b - A x| / |b| <= tol for every r.
 *   prec = WHMC_F64: plain FP64 CG (links = WHMC_L12 rebuilds the third link row in FP64).
 *   prec = WHMC_F32 / WHMC_F16: mixed precision; the Krylov bulk runs with spinors in that
 *     format and `links`-real links of the same precision, FP64 reliable updates recompute
 *     r = b - A x whenever the iterated residual drops below delta times its maximum since the
 *     last update; dot products accumulate in FP64.
 *   nrhs > 1: all right-hand sides advance together through the multi-RHS kernels (mixed
 *     precision with 18-real links, which they lack, solves them one after the other), blocked as
 *     in whmc_apply_H_multi (rhs_block = rhs_lanes = 0: autotuned); a converged rhs is frozen
 *     (masked) while the others continue; the FP64 true residuals of reliable updates and of
 *     the final check are computed for all right-hand sides concerned in one multi-RHS pass.
 * stats (may be NULL) receives nrhs entries.  Returns ENOCONV if any rhs misses tol. */
typedef struct whmc_cg_params {
  double tol;         /* target true relative residual, e.g. 1e-10 */
  int maxiter;        /* per solve (counting sloppy iterations in mixed mode) */
  int prec;           /* whmc_prec of the Krylov bulk */
  int links;          /* whmc_links of the bulk operator */
  double delta;       /* reliable-update trigger (mixed only), e.g. 0.1 */
  int check_every;    /* iterations enqueued between host convergence checks (>= 1) */
  int rhs_block;      /* multi-RHS register block (right-hand sides per thread), 0 = autotuned */
  int rhs_lanes;      /* multi-RHS lanes per site sharing link loads, 0 = autotuned */
  int rhs_order;      /* multi-RHS workgroup order (see whmc_apply_H_multi); ignored when autotuned */
} whmc_cg_params;

typedef struct whmc_cg_stats {
  int iters;             /* iterations (sloppy iterations in mixed mode) */
  int reliable_updates;  /* FP64 residual recomputations (mixed mode) */
  int converged;         /* 1 if the true residual reached tol */
  double true_residual;  /* final |b - A x| / |b|, computed in FP64 */
  double seconds;        /* wall time of the whole solve (all rhs) */
} whmc_cg_stats;

whmc_status whmc_cg_solve(whmc_ctx* ctx, double* x, const double* b, const double* kappas, int nrhs,
                          const whmc_cg_params* params, whmc_cg_stats* stats);

/* Solve M^dag M x = b on the full lattice (M = 1 - kappa H, Sec. 1; full spinors, whmc layout) by
 * FP64 CG from x = 0 until the true residual |b - A x| / |b| <= params->tol.  params->prec must be
 * WHMC_F64 (else WHMC_EUNSUP); params->links selects 18- or 12-real links; maxiter and check_every
 * as for whmc_cg_solve (one iteration applies H four times, two launches of both parities).
 * stats (may be NULL) receives one entry.  ENOCONV if tol is not reached, ENONFINITE if b or an
 * iterate is not finite. */
whmc_status whmc_cg_solve_full(whmc_ctx* ctx, double* x, const double* b, double kappa, const whmc_cg_params* params,
                               whmc_cg_stats* stats);

/* Solve M_oo(kappa) x = b (dagger = 0) or M_oo(kappa)^dag x = b (dagger = 1) for one odd-site half
 * field (FP64 whmc layout) by BiCGstab, the Krylov solver the paper uses (Sec. 4), from x = 0 until
 * the true FP64 residual |b - A x| / |b| <= params->tol.  params->prec must be WHMC_F64 (else
 * WHMC_EUNSUP); params->links selects 18- or 12-real links for the iteration (the true residual
 * always uses 18-real links); maxiter and check_every as for whmc_cg_solve; one iteration applies
 * A twice.  A breakdown restarts from the true residual (at most 4 passes).  stats (may be NULL)
 * receives one entry.  Returns WHMC_ENOCONV if tol is not reached. */
whmc_status whmc_bicgstab_solve(whmc_ctx* ctx, double* x, const double* b, double kappa, int dagger,
                                const whmc_cg_params* params, whmc_cg_stats* stats);

/* ------------------------------------------------------------------ filter, actions, forces
 * Hopping-parameter-expansion filter (Sec. 2, 2.2): with K = kappa^2 H_oe H_eo,
 *   M~ = M_oo exp(sum_{j<=k} K^j / j),  M~^{-1} = sum_n b_n K^n + alpha M_oo^{-1}.
 * k = 0 is the plain action S_PF = |M_oo^{-1} phi|^2, k = 1 kappa^2-, k = 2 kappa^4-filtering.
 * n_t truncates the force, n_max the action and the heat bath.  The gauge action becomes
 * S_G at beta + 96 kappa^4 for k = 2 (Sec. 2; exact when no lattice extent is 2 or 4). */
typedef struct whmc_filter {
  int k;
  int n_t;
  int n_max;
} whmc_filter;

/* coefficient tables: b[0..n], c[0..n] (c_n = Taylor coefficients of exp(+sum_{j<=k} x^j/j),
 * used by the heat bath phi = M~ eta) and alpha; computed on the host in extended precision. */
whmc_status whmc_filter_coefficients(int k, int n, double* b, double* c, double* alpha);

/* phi = M~ eta = M_oo sum_{n<=n_max} c_n K^n eta  (eq. initPseudo for M~), odd-site FP64. */
whmc_status whmc_heatbath_phi(whmc_ctx* ctx, double* phi, const double* eta, const whmc_filter* f, double kappa);

/* S_G (with the filter's beta shift) and S~_PF = |M~^{-1} phi|^2 at n_max; either output may be
 * NULL to skip it.  solver may be NULL (FP64 CG to 1e-12). */
whmc_status whmc_action(whmc_ctx* ctx, double* S_G, double* S_PF, const double* phi, const whmc_filter* f,
                        double kappa, double beta, const whmc_cg_params* solver);

/* plaquette <P> = sum_p Re Tr U_p / (3 N_p)  (Sec. 4.1), FP64, deterministic. */
whmc_status whmc_plaquette(whmc_ctx* ctx, double* plaq);

/* Forces in the whmc algebra layout, defined by (omega, F) = delta_omega S with
 * delta U = omega U (Sec. 1).  flags: bit 0 pseudo-fermion force of S~_PF truncated at n_t
 * (Sec. 2, Horner scheme), bit 1 gauge force of S_G at beta (+ the filter's shift),
 * bit 2 accumulate into F instead of overwriting.  solver may be NULL (FP64 CG to 1e-12). */
#define WHMC_FORCE_PF 1
#define WHMC_FORCE_GAUGE 2
#define WHMC_FORCE_ACCUMULATE 4
whmc_status whmc_force(whmc_ctx* ctx, double* F, const double* phi, const whmc_filter* f, double kappa,
                       double beta, const whmc_cg_params* solver, int flags);

/* Full-lattice pseudo-fermion action and force without even/odd preconditioning (Sec. 1):
 * S_PF = |M^{-1} phi|^2 for a full spinor phi, force from delta S = -X^dag delta M Y + h.c. with
 * X = (M M^dag)^{-1} phi = gamma_5 (M^dag M)^{-1} gamma_5 phi (one full-lattice CG) and Y = M^dag X.
 * whmc_force_full flags as for whmc_force (WHMC_FORCE_GAUGE adds the gauge force at beta, no shift).
 * solver may be NULL (FP64 CG to 1e-12). */
whmc_status whmc_action_full(whmc_ctx* ctx, double* S_PF, const double* phi, double kappa,
                             const whmc_cg_params* solver);
whmc_status whmc_force_full(whmc_ctx* ctx, double* F, const double* phi, double kappa, double beta,
                            const whmc_cg_params* solver, int flags);

/* Molecular-dynamics primitives (Sec. 1, with the step conventions of this library):
 * T step  U_{x,mu} <- exp(eps Pi_{x,mu}) U_{x,mu}  (exact SU(3) exponential, FP64 master copy;
 *         lower-precision copies are re-derived on next use), and
 * P step  Pi <- Pi - eps F  (algebra layout). */
whmc_status whmc_update_links(whmc_ctx* ctx, const double* pi, double eps);
whmc_status whmc_update_momenta(whmc_ctx* ctx, double* pi, const double* F, double eps);

/* Chain rule through the exponential chart U(omega) = exp(omega) U0: given the force F at U(omega)
 * (algebra layout), out = sum_k (-ad_omega)^k F / (k+1)!, the gradient of S(exp(omega) U0) with
 * respect to the coordinates of omega (equal to F at omega = 0).  out must not alias the inputs. */
whmc_status whmc_dexp_transpose(whmc_ctx* ctx, double* out, const double* omega, const double* F);

/* ------------------------------------------------------------------ HMC (Sec. 1, 4.1)
 * One trajectory: phi = M~ eta, H0, molecular dynamics with Sexton-Weingarten levels (gauge on
 * level 0 with m0 steps per coarse step, pseudo-fermion on level 1 with m steps over tau),
 * H1, accept if u < exp(-dH).  The random inputs are passed in: pi0 (algebra layout, pi_a ~ N(0,1)),
 * eta (odd-site FP64 spinor with density exp(-|eta|^2)), u uniform in [0,1).  On acceptance the
 * context's gauge field becomes the new one, otherwise it is restored.  Steps: P(e): Pi -= e F,
 * T(e): U = exp(e Pi) U; Omelyan with lambda, or leapfrog.  Consecutive P steps of one level that
 * evaluate the force on the same field are merged. */
typedef struct whmc_hmc_params {
  double beta;
  double kappa;
  whmc_filter filter;
  int integrator;   /* whmc_integrator */
  double lambda;    /* Omelyan parameter, 1/6 in the paper */
  int m;            /* coarse steps per trajectory */
  int m0;           /* gauge steps per coarse (half) step */
  double tau;       /* trajectory length */
  whmc_cg_params md_solver;      /* solves inside the force */
  whmc_cg_params action_solver;  /* solves for H0 / H1 */
} whmc_hmc_params;

typedef struct whmc_traj_result {
  double dH, H0, H1;
  int accepted;
  double plaquette;       /* of the field kept after the accept/reject step */
  long long cg_iters;     /* total M_oo^dag M_oo solver iterations in the trajectory */
  int n_solves;
  double seconds;
  long long poly_iters;   /* CG iterations on p_j^dag p_j in the rooted heat bath (0 otherwise) */
} whmc_traj_result;

whmc_status whmc_hmc_trajectory(whmc_ctx* ctx, const whmc_hmc_params* p, const double* pi0, const double* eta,
                                double u, whmc_traj_result* res);

/* Molecular dynamics only: integrates the context's gauge field and pi (in place, algebra layout)
 * over tau with phi fixed (for reversibility and dH-scaling studies). */
whmc_status whmc_md_integrate(whmc_ctx* ctx, const whmc_hmc_params* p, double* pi, const double* phi);

/* Hamiltonian H = (1/2)(Pi,Pi) + S~_G + S~_PF for the context's gauge field. */
whmc_status whmc_hamiltonian(whmc_ctx* ctx, const whmc_hmc_params* p, const double* pi, const double* phi,
                             double* H);

/* ------------------------------------------------------------------ rooted polynomials (Sec. 2.1)
 * Starting from M_1 = M~ of the kappa^(2k) filter (M_oo for k = 0) and with x = K, the chain
 *   p_j(x) = W_j^{-1} = Taylor polynomial of degree n_j of M_j(x)^{-1/N},   M_{j+1} = p_j(x)^N M_j,
 * j = 1 .. jmax (one root order N for all j, as in the paper's runs), leaves the remainder
 *   M_{jmax+1}^{-1} = sum_n b_n K^n + alpha M_oo^{-1}                      (eq. restM).
 * Since det M~ = prod_j det(W_j)^N det M_{jmax+1}, two flavours are represented by jmax*N + 1
 * pseudo-fermion fields with the terms
 *   S_j = sum_{i=1..N} |p_j(K) phi_{j,i}|^2   (j = 1 .. jmax),
 *   S_r = |(sum_{n<=n_max} b_n K^n + alpha M_oo^{-1}) phi_r|^2   (term jmax + 1),
 * plus the gauge action at beta (+ 96 kappa^4 for k = 2).  n_t truncates the remainder series in
 * the force, n_max in the action and the heat bath.  jmax = 0 is the kappa^(2k) filter itself.
 * Fields: phi and eta hold the jmax*N + 1 odd-site FP64 fields (whmc layout) back to back in the
 * order phi_{1,1} .. phi_{1,N}, phi_{2,1}, ..., phi_r.  Scratch grows with max(n_j, n_t) + 1 fields
 * of each of four kinds (the Horner vectors of the force). */
#define WHMC_MAX_POLY 4
#define WHMC_ROOTED_MAX_N 1000
typedef struct whmc_rooted {
  int N;                   /* root order, 1 .. 64 */
  int jmax;                /* number of polynomials, 0 .. WHMC_MAX_POLY */
  int n[WHMC_MAX_POLY];    /* degrees n_1 .. n_jmax, each 1 .. WHMC_ROOTED_MAX_N */
  int k;                   /* filter order of M_1: 0, 1 or 2 */
  int n_t;                 /* remainder truncation in the force, 0 .. WHMC_ROOTED_MAX_N */
  int n_max;               /* remainder (and M~ eta) truncation in action and heat bath, same range */
} whmc_rooted;

/* Coefficient tables on the host, in extended precision: p receives p_1[0..n_1], p_2[0..n_2], ...
 * back to back (sum_j (n_j + 1) doubles), b receives b[0..nb] (nb <= WHMC_ROOTED_MAX_N), alpha the
 * alpha of eq. (restM).  Any output may be NULL.  Needs no GPU. */
whmc_status whmc_rooted_coefficients(const whmc_rooted* r, double* p, double* b, int nb, double* alpha);

/* Heat bath (eq. initPseudo for each term): phi_{j,i} = p_j(K)^{-1} eta_{j,i} by CG on
 * p_j^dag p_j to solver->tol (relative residual; FP64; solver->maxiter bounds each solve),
 * phi_r = prod_j p_j(K)^N M~ eta_r with M~ eta truncated at n_max.  solver may be NULL (1e-12).
 * iters (may be NULL) receives the total CG iterations.  WHMC_ENOCONV if a solve hits maxiter. */
whmc_status whmc_rooted_heatbath(whmc_ctx* ctx, double* phi, const double* eta, const whmc_rooted* r, double kappa,
                                 const whmc_cg_params* solver, long long* iters);

/* S[0 .. jmax]: S_1 .. S_jmax and S_r (at n_max).  solver (may be NULL: FP64 CG to 1e-12) inverts
 * M_oo^dag M_oo for the alpha term. */
whmc_status whmc_rooted_action(whmc_ctx* ctx, double* S, const double* phi, const whmc_rooted* r, double kappa,
                               const whmc_cg_params* solver);

/* Force of one term in the algebra layout (the Horner scheme of Sec. 2 with the term's
 * coefficients; the polynomial terms need no solve): term 1 .. jmax is S_j summed over its N
 * fields, term jmax + 1 is S_r with the series truncated at n_t, term 0 is all of them.
 * flags: WHMC_FORCE_ACCUMULATE adds to F instead of overwriting it. */
whmc_status whmc_rooted_force(whmc_ctx* ctx, double* F, const double* phi, const whmc_rooted* r, int term,
                              double kappa, const whmc_cg_params* solver, int flags);

/* Multi-level trajectory with the rooted action (Sec. 2.1, 4.2): the gauge action on level 0 and
 * term j on level j, the remainder on level jmax + 1.  One (half, for Omelyan) step of level l
 * holds msub[l-1] steps of level l - 1; the remainder takes m steps over tau.  In the paper's
 * notation (jmax = 2) msub = {m_0, m_1, m_2}.  Otherwise as whmc_hmc_trajectory; eta holds the
 * jmax*N + 1 Gaussian sources, heatbath_solver drives the polynomial heat baths. */
typedef struct whmc_rooted_hmc_params {
  double beta;
  double kappa;
  whmc_rooted rooted;
  int integrator;                 /* whmc_integrator */
  double lambda;                  /* Omelyan parameter */
  int m;                          /* remainder steps per trajectory */
  int msub[WHMC_MAX_POLY + 1];    /* msub[l-1]: level l-1 steps per step of level l, l = 1 .. jmax+1 */
  double tau;
  whmc_cg_params md_solver;
  whmc_cg_params action_solver;
  whmc_cg_params heatbath_solver;
} whmc_rooted_hmc_params;

whmc_status whmc_rooted_trajectory(whmc_ctx* ctx, const whmc_rooted_hmc_params* p, const double* pi0,
                                   const double* eta, double u, whmc_traj_result* res);

/* Molecular dynamics only, with the jmax*N + 1 fields phi fixed (pi integrated in place). */
whmc_status whmc_rooted_md_integrate(whmc_ctx* ctx, const whmc_rooted_hmc_params* p, double* pi, const double* phi);

/* H = (1/2)(Pi,Pi) + S_G + sum_j S_j + S_r for the context's gauge field. */
whmc_status whmc_rooted_hamiltonian(whmc_ctx* ctx, const whmc_rooted_hmc_params* p, const double* pi,
                                    const double* phi, double* H);

/* ------------------------------------------------------------------ mass preconditioning (Sec. 1, 5)
 * The fermion determinant split into factors with a pseudo-fermion each (Sec. 1), combined with the
 * kappa^(2k) filter as the conclusion proposes: with heavier hopping parameters
 * 0 < kappa_1 < ... < kappa_n < kappa_{n+1} = kappa every factor carries the filter and one gauge
 * term remains, that of kappa (gauge action at beta + 96 kappa^4 for k = 2):
 *   det M_oo(kappa) = det M~(kappa_1) prod_{i=1..n} det M~(kappa_{i+1}) / det M~(kappa_i) * (gauge term).
 * Term 1 is S_1 = |M~(kappa_1)^{-1} phi_1|^2; term i + 1 the ratio
 *   S_{i+1} = |M~(kappa_{i+1})^{-1} M~(kappa_i) phi_{i+1}|^2 = |(sum_n b_n K^n + alpha M_oo^{-1}) phi_{i+1}|^2
 * at kappa_{i+1}, with b_n, alpha of g(x)/(1 - x), g = (1 - rho x) exp(sum_{j<=k} (rho^j - 1) x^j / j),
 * rho = kappa_i^2 / kappa_{i+1}^2 (all factors are functions of H_oe H_eo, so they commute); the
 * series is truncated at n_max in the action and at n_t in the force.  Without the filter (k = 0)
 * the ratio is rho + (1 - rho) M_oo(kappa_{i+1})^{-1}.  n = 0 is the filter alone at kappa.
 * phi and eta hold n + 1 odd-site FP64 fields back to back, term 1 first. */
#define WHMC_MAX_MASSPRE 4
typedef struct whmc_masspre {
  int n;                              /* heavier hopping parameters, 0 .. WHMC_MAX_MASSPRE */
  double kappas[WHMC_MAX_MASSPRE];    /* 0 < kappa_1 < ... < kappa_n < kappa */
  whmc_filter filter;                 /* the filter of every factor (k <= 2) */
} whmc_masspre;

/* Coefficient table of one ratio on the host, in extended precision: b[0..n] (n <= WHMC_ROOTED_MAX_N)
 * and alpha of M~(kappa_{i+1})^{-1} M~(kappa_i) = sum_n b_n K^n + alpha M_oo^{-1} for
 * rho = kappa_i^2 / kappa_{i+1}^2 in (0, 1) and filter order k in 0..2.  Needs no GPU. */
whmc_status whmc_masspre_coefficients(double rho, int k, int n, double* b, double* alpha);

/* phi_1 = M~(kappa_1) eta_1, phi_{i+1} = M~(kappa_i)^{-1} M~(kappa_{i+1}) eta_{i+1} (series at n_max,
 * one solve at kappa_i each).  solver may be NULL (FP64 CG to 1e-12). */
whmc_status whmc_masspre_heatbath(whmc_ctx* ctx, double* phi, const double* eta, const whmc_masspre* mp,
                                  double kappa, const whmc_cg_params* solver);

/* S[0 .. n]: the heavy filtered term, then the ratios. */
whmc_status whmc_masspre_action(whmc_ctx* ctx, double* S, const double* phi, const whmc_masspre* mp, double kappa,
                                const whmc_cg_params* solver);

/* Force of term 1 .. n + 1 (0: all), algebra layout; flags: WHMC_FORCE_ACCUMULATE. */
whmc_status whmc_masspre_force(whmc_ctx* ctx, double* F, const double* phi, const whmc_masspre* mp, int term,
                               double kappa, const whmc_cg_params* solver, int flags);

/* Multi-level trajectory: gauge action on level 0, term t on level t (the heavy filtered field on
 * level 1, the lightest ratio outermost with m steps); msub[l-1] steps of level l - 1 per (half)
 * step of level l.  Otherwise as whmc_hmc_trajectory; eta holds the n + 1 Gaussian sources. */
typedef struct whmc_masspre_hmc_params {
  double beta;
  double kappa;
  whmc_masspre mp;
  int integrator;
  double lambda;
  int m;
  int msub[WHMC_MAX_MASSPRE + 1];
  double tau;
  whmc_cg_params md_solver;
  whmc_cg_params action_solver;
} whmc_masspre_hmc_params;

whmc_status whmc_masspre_trajectory(whmc_ctx* ctx, const whmc_masspre_hmc_params* p, const double* pi0,
                                    const double* eta, double u, whmc_traj_result* res);
whmc_status whmc_masspre_md_integrate(whmc_ctx* ctx, const whmc_masspre_hmc_params* p, double* pi,
                                      const double* phi);
whmc_status whmc_masspre_hamiltonian(whmc_ctx* ctx, const whmc_masspre_hmc_params* p, const double* pi,
                                     const double* phi, double* H);

#ifdef __cplusplus
}
#endif
#endif
