// Host-side internals shared by the translation units of libwhmc: the context, error reporting,
// scratch management and the launchers each .hip file exports to the others.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <map>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/whmc.h"
#include "device.h"
#include "occupancy.h"

namespace whmc {

void set_error(const std::string& msg);

#define WHMC_HIP(call)                                                                         \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      ::whmc::set_error(std::string(#call) + " failed: " + hipGetErrorString(e_) + " at " +    \
                        __FILE__ + ":" + std::to_string(__LINE__));                            \
      return WHMC_EHIP;                                                                        \
    }                                                                                          \
  } while (0)

#define WHMC_CHECK(cond, code, msg) \
  do {                              \
    if (!(cond)) {                  \
      ::whmc::set_error(msg);       \
      return code;                  \
    }                               \
  } while (0)

#define WHMC_TRY(expr)              \
  do {                              \
    whmc_status s_ = (expr);        \
    if (s_ != WHMC_OK) return s_;   \
  } while (0)

constexpr int kBlock = 128;   // threads per workgroup of the stencil and reduction kernels

// roctx range over a host scope (solver iterations, MD steps, trajectories), seen by rocprofv3
// --marker-trace; a no-op call when no tool is attached
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// per-solve scalar state that lives on the device so that iterations can be enqueued without a
// host round trip; `done` / `pause` make the remaining queued kernels exit at once.
struct CGScalars {
  double rr;        // |r|^2 of the current residual
  double pAp;       // (p, A p)
  double alpha, beta;
  double rr_old;    // |r|^2 before the last update (reliable-update restart of p)
  double stop_rr;   // convergence threshold on |r|^2
  double rmax2;     // mixed precision: max |r|^2 since the last reliable update
  double delta2;    // mixed precision: reliable update when |r|^2 < delta2 * rmax2
  int done;         // converged (or broken down)
  int pause;        // mixed precision: reliable update requested
  int iter;         // iterations completed
  int active;       // multi-RHS: 1 while the rhs still iterates
};

constexpr int kMaxRhs = 16;

}  // namespace whmc

struct whmc_ctx {
  int dims[4];
  long long V;
  int Vh;
  whmc::Geom g;
  int device;
  hipStream_t stream;
  // gauge field copies
  double2* U18 = nullptr;          // master FP64 18-real
  double2* U12 = nullptr;          // FP64 12-real
  float2* U32_18 = nullptr;
  float4* U32_12 = nullptr;
  uint2* U16_12 = nullptr;
  double2* U8 = nullptr;           // FP64 8-real
  float4* U32_8 = nullptr;
  uint4* U16_8 = nullptr;
  bool gauge_loaded = false;
  bool derived_valid[7] = {};      // U12, U32_18, U32_12, U16_12, U8, U32_8, U16_8
  // scratch
  std::map<std::string, std::pair<void*, size_t>> ws;
  std::map<std::string, std::pair<int, double>> tuned;   // autotuned multi-RHS blockings (16 nb + lanes, us)
  whmc::Reduce red{};
  void* noalloc_scratch = nullptr;   // device address of the static scratch of whmc_apply_MdagM_noalloc
  whmc::CGScalars* scal = nullptr;   // kMaxRhs entries
  whmc::CGScalars* scal_host = nullptr;  // pinned mirror
  double* host_pinned = nullptr;     // small pinned buffer for scalar read-back
  // cache policy: stream (non-temporal) link loads when the link array of a format is larger
  // than stream_threshold bytes; -1 = never, 0 = always.  Default 128 MiB; callers change it with
  // whmc_set_option(WHMC_OPT_STREAM_THRESHOLD).
  long long stream_threshold = 128LL << 20;
  int hop_chunk = 0;   // tq of the time-slab schedule (WHMC_OPT_HOP_CHUNK)
  int force_kernel = 0;   // pair-force kernel: 0 link-parallel, 1 site-parallel (WHMC_OPT_FORCE_KERNEL)
  int force_chunk = 24;   // (X, Y) pairs per launch of the pair-force kernel (WHMC_OPT_FORCE_CHUNK)
  // occupancy cap of the single-RHS stencil kernels (WHMC_OPT_HOP_WG_PER_CU): each workgroup
  // reserves stencil_lds bytes of LDS it does not use, so that at most hop_wg_per_cu workgroups fit
  // on a compute unit (0 = no cap, stencil_lds = 0).  Fewer sites in flight per XCD keep the
  // neighbour spinors of the sites in flight inside that XCD's L2.
  int hop_wg_per_cu = 0;
  unsigned stencil_lds = 0;
  int lds_per_cu = 0, lds_per_wg = 0;   // device limits, read at creation
  bool stream_links(int prec, int links) const {
    if (stream_threshold < 0) return false;
    const long long per = links == 8 ? (prec == 0 ? 64 : prec == 1 ? 32 : 16)
                                     : prec == 0 ? (links == 18 ? 144 : 96) : (prec == 1 ? (links == 18 ? 72 : 48) : 24);
    return (long long)8 * Vh * per > stream_threshold;
  }
  int num_blocks() const { return (Vh + whmc::kBlock - 1) / whmc::kBlock; }
  // grid of the kernels on the slice-range schedule (site_block_xq, site_block_grp,
  // site_block_pair): may exceed num_blocks() by padding workgroups
  int stencil_blocks() const { return g.xq ? 8 * g.xq * g.L[0] : num_blocks(); }
  // grid of the single-RHS stencil kernels (site_block), for the schedule in g.sched
  int site_blocks() const { return g.sched == 1 ? 8 * g.tx * g.nch * g.tq : stencil_blocks(); }
  // at most k workgroups per compute unit for the single-RHS stencil kernels (k = 0: no cap; else
  // 2 <= k <= 8, reserving whmc::lds_reservation bytes; false, unchanged, if the device cannot do it)
  bool set_wg_cap(int k) {
    if (k == 0) {
      hop_wg_per_cu = 0;
      stencil_lds = 0;
      return true;
    }
    const unsigned b = whmc::lds_reservation(lds_per_cu, lds_per_wg, k);
    if (b == 0) return false;
    hop_wg_per_cu = k;
    stencil_lds = b;
    return true;
  }
  // time-slab schedule with chunks of tq blocks, if the lattice allows it (else false, unchanged)
  bool set_schedule(int sched, int tq) {
    if (sched == 0) { g.sched = 0; return true; }
    if (sched != 1 || g.nbs == 0 || g.L[0] % 8 != 0 || tq < 1 || tq > g.nbs) return false;
    g.sched = 1;
    g.tx = g.L[0] / 8;
    g.tq = tq;
    g.nch = (g.nbs + tq - 1) / tq;
    return true;
  }
};

namespace whmc {

// scratch buffer owned by the context, grown on demand, freed in whmc_destroy
whmc_status workspace(whmc_ctx* c, const std::string& name, size_t bytes, void** out);

// ---- gauge copies (core.hip)
whmc_status ensure_links(whmc_ctx* c, int prec, int links);
whmc_status gauge_changed(whmc_ctx* c);   // invalidate derived copies after the master changed

// ---- hopping matrix launchers (core.hip).  All operate on half fields in whmc layout.
// out = a * x + b * H_{par,1-par}^{(dag)} in   (x may be null: then out = b * H in)
// if norm_out != null the FP64 sum |out|^2 is written there (device pointer).
whmc_status hop(whmc_ctx* c, int prec, int links, int par, int dag, void* out, const void* in, const void* x,
                double a, double b, double* norm_out, bool nt_store = false);

// ---- FP64 BLAS on half fields (core.hip); n = number of half fields
whmc_status axpby_f64(whmc_ctx* c, double* y, double a, const double* x, double b, int nhalf);  // y = a x + b y
whmc_status copy_f64(whmc_ctx* c, double* y, const double* x, int nhalf);
whmc_status gamma5_f64(whmc_ctx* c, double* y, const double* x, int nhalf);
whmc_status norm2_f64(whmc_ctx* c, const double* x, int nhalf, double* dev_out);      // async, device result
whmc_status dot_re_f64(whmc_ctx* c, const double* x, const double* y, int nhalf, double* dev_out);
whmc_status read_scalar(whmc_ctx* c, const double* dev, double* host);                // synchronises
whmc_status finish_sum(whmc_ctx* c, int nparts, double* dev_out);   // pass 2 over red.partials[0..nparts)
whmc_status convert_spinor(whmc_ctx* c, void* dst, int dst_prec, const void* src, int src_prec, int nhalf);
whmc_status zero_bytes(whmc_ctx* c, void* p, size_t bytes);   // fill kernel (graph-safe)

// ---- operators composed from hops (core.hip)
whmc_status apply_Moo_f64(whmc_ctx* c, double* out, const double* in, double kappa, int dagger, double* tmp_even);
whmc_status apply_MdagM_f64(whmc_ctx* c, double* out, const double* in, double kappa, double* tmp_even,
                            double* tmp_odd);
whmc_status apply_K_f64(whmc_ctx* c, double* out, const double* in, double kappa, int dagger, double* even_out,
                        const double* x, double a);   // out = a x + K^(dag) in; even_out = H_eo^(dag) in
// full lattice (full spinors = even half, odd half): out = M in or M^dag in, M = 1 - kappa H (full.hip)
whmc_status apply_M_full(whmc_ctx* c, double* out, const double* in, double kappa, int dagger);
whmc_status apply_MdagM_full(whmc_ctx* c, double* out, const double* in, double kappa, double* tmp_full);

// ---- solvers (cg.hip)
whmc_status cg_solve(whmc_ctx* c, double* x, const double* b, const double* kappas, int nrhs,
                     const whmc_cg_params* p, whmc_cg_stats* st);

// ---- gauge and force kernels (gauge.hip)
whmc_status plaquette_sum(whmc_ctx* c, double* host_out);
whmc_status gauge_force(whmc_ctx* c, double* F, double beta_eff, double scale, int accumulate);
whmc_status pf_force_pairs(whmc_ctx* c, double* F, const double* const* X_e, const double* const* X_o,
                           const double* const* Y_e, const double* const* Y_o, int npairs, double kappa_eff,
                           int accumulate);
whmc_status mom_update(whmc_ctx* c, double* pi, const double* F, double eps);   // pi -= eps F
whmc_status link_update(whmc_ctx* c, const double* pi, double eps);              // U = exp(eps pi) U
whmc_status algebra_norm2(whmc_ctx* c, const double* pi, double* host_out);
whmc_status pack_algebra(whmc_ctx* c, double* dst, const double* src, int unpack);

// ---- actions, forces and molecular dynamics (hmc.hip)
// named odd-site FP64 scratch fields of the context
struct Fields {
  whmc_ctx* c;
  size_t hb;
  whmc_status get(const char* name, int idx, double** p) {
    void* v;
    WHMC_TRY(workspace(c, std::string(name) + std::to_string(idx), hb, &v));
    *p = (double*)v;
    return WHMC_OK;
  }
};
struct SolveLog {   // M_oo^dag M_oo solver statistics of one action / force / trajectory
  long long iters = 0;
  int n = 0;
};
struct MDLevel {    // one Sexton-Weingarten level: pi += scale F_l, and its substep count
  std::function<whmc_status(double scale)> force;
  int nsub = 0;
};
// filter tables: b_0..b_n and alpha of M~^{-1}, c_0..c_n of exp(+sum_{j<=k} x^j/j)
void coefficients(int k, int n, std::vector<double>& b, std::vector<double>& c, double& alpha);
double delta_beta(double kappa, int k);
whmc_cg_params default_solver();
whmc_status solve(whmc_ctx* c, double* x, const double* rhs, double kappa, const whmc_cg_params* p, SolveLog* log);
whmc_status poly_K(whmc_ctx* c, double* out, const double* v, const std::vector<double>& coef, double kappa,
                   double* tmp_e, double* tmp_o, int dagger);
whmc_status series_inverse(whmc_ctx* c, double* out, const double* phi, std::vector<double> b, double alpha,
                           double kappa, const whmc_cg_params* sp, SolveLog* log);
whmc_status series_force(whmc_ctx* c, double* out, const double* phi, const std::vector<double>& b, double alpha,
                         double kappa, const whmc_cg_params* sp, double scale, int accumulate, SolveLog* log);
whmc_status heatbath(whmc_ctx* c, double* phi, const double* eta, const whmc_filter* f, double kappa);
whmc_status check_filter(const whmc_filter* f);
whmc_status pf_action(whmc_ctx* c, const double* phi, const whmc_filter* f, double kappa, const whmc_cg_params* sp,
                      double* S, SolveLog* log);
whmc_status pf_force(whmc_ctx* c, double* out, const double* phi, const whmc_filter* f, double kappa,
                     const whmc_cg_params* sp, double scale, int accumulate, SolveLog* log);
whmc_status md_levels(whmc_ctx* c, double* pi, const std::vector<MDLevel>& lv, int integrator, double lambda,
                      double tau, int m);

// A pseudo-fermion action of several terms (term t on MD level t, the gauge action on level 0),
// with the trajectory that the rooted and the mass-preconditioned actions share.
struct TermAction {
  int nfields = 1;          // odd-site FP64 fields in phi and eta
  int nterms = 1;           // pseudo-fermion terms
  double beta_eff = 0.0;    // gauge coupling including the filter's shift
  // phi from the Gaussian sources eta; M_oo^dag M_oo solves go to log, other Krylov iterations
  // (the polynomial heat bath of the rooted action) to aux_iters
  std::function<whmc_status(double* phi, const double* eta, long long* aux_iters, SolveLog* log)> heatbath;
  std::function<whmc_status(double* S, const double* phi, SolveLog* log)> action;   // S[0 .. nterms)
  // F (or pi) += scale * force of term t (1 .. nterms); overwrite unless accumulate
  std::function<whmc_status(double* F, const double* phi, int t, double scale, int accumulate, SolveLog* log)> force;
};
struct TermMD {
  int integrator;
  double lambda, tau;
  int m;            // steps of the outermost term per trajectory
  const int* msub;  // msub[l-1]: level l-1 steps per step of level l
};
whmc_status term_hamiltonian(whmc_ctx* c, const TermAction& A, const double* pi, const double* phi, double* H,
                             SolveLog* log);
whmc_status term_md(whmc_ctx* c, const TermAction& A, const TermMD& md, double* pi, const double* phi, SolveLog* log);
whmc_status term_trajectory(whmc_ctx* c, const TermAction& A, const TermMD& md, const double* pi0, const double* eta,
                            double u, whmc_traj_result* res);

}  // namespace whmc
