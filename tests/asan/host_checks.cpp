// Host-side checks of libwhmc under AddressSanitizer and UndefinedBehaviorSanitizer: the coefficient
// generators over their whole input ranges, and the argument checks of every entry point, which
// must reject null contexts and invalid arguments with a status before touching a GPU.  Built from
// host-only objects of the library (no device code, no GPU needed); every failure exits non-zero.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "whmc.h"
#include "../../paper_1805_03560_amd/csrc/occupancy.h"

static int g_checks = 0;

#define EXPECT(cond)                                                          \
  do {                                                                        \
    ++g_checks;                                                               \
    if (!(cond)) {                                                            \
      std::fprintf(stderr, "host check failed at line %d: %s\n", __LINE__, #cond); \
      std::exit(1);                                                           \
    }                                                                         \
  } while (0)

static bool finite_all(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

static void filter_coefficients() {
  for (int k = 0; k <= 3; ++k)
    for (int n : {0, 1, 7, 15, 19, 29, 200, 1000}) {
      std::vector<double> b(n + 1), c(n + 1);
      double alpha = 0.0;
      EXPECT(whmc_filter_coefficients(k, n, b.data(), c.data(), &alpha) == WHMC_OK);
      EXPECT(finite_all(b) && finite_all(c) && alpha > 0.0 && alpha <= 1.0);
      EXPECT(whmc_filter_coefficients(k, n, nullptr, nullptr, nullptr) == WHMC_OK);
    }
  double b[4], c[4], a;
  EXPECT(whmc_filter_coefficients(-1, 3, b, c, &a) == WHMC_EARG);
  EXPECT(whmc_filter_coefficients(65, 3, b, c, &a) == WHMC_EARG);
  EXPECT(whmc_filter_coefficients(1, -1, b, c, &a) == WHMC_EARG);
  EXPECT(whmc_filter_coefficients(1, 1001, b, c, &a) == WHMC_EARG);
}

static whmc_rooted rooted(int N, std::vector<int> ns, int k, int nt, int nmax) {
  whmc_rooted r{};
  r.N = N;
  r.jmax = (int)ns.size();
  for (size_t j = 0; j < ns.size() && j < WHMC_MAX_POLY; ++j) r.n[j] = ns[j];
  r.k = k;
  r.n_t = nt;
  r.n_max = nmax;
  return r;
}

static void rooted_coefficients() {
  const std::vector<std::vector<int>> degrees = {{}, {8}, {8, 32}, {16, 42}, {3, 7, 15, 31}, {1000}};
  for (int N : {1, 2, 4, 8, 64})
    for (int k = 0; k <= 2; ++k)
      for (const auto& ns : degrees) {
        whmc_rooted r = rooted(N, ns, k, 160, 400);
        int np = 0;
        for (int n : ns) np += n + 1;
        std::vector<double> p(np > 0 ? np : 1), b(401);
        double alpha = 0.0;
        EXPECT(whmc_rooted_coefficients(&r, p.data(), b.data(), 400, &alpha) == WHMC_OK);
        EXPECT(finite_all(p) && finite_all(b) && std::isfinite(alpha));
      }
  std::vector<double> p(64), b(64);
  double alpha;
  whmc_rooted bad = rooted(0, {8}, 0, 10, 10);
  EXPECT(whmc_rooted_coefficients(&bad, p.data(), b.data(), 10, &alpha) == WHMC_EARG);
  bad = rooted(65, {8}, 0, 10, 10);
  EXPECT(whmc_rooted_coefficients(&bad, p.data(), b.data(), 10, &alpha) == WHMC_EARG);
  bad = rooted(2, {0}, 0, 10, 10);
  EXPECT(whmc_rooted_coefficients(&bad, p.data(), b.data(), 10, &alpha) == WHMC_EARG);
  bad = rooted(2, {1001}, 0, 10, 10);
  EXPECT(whmc_rooted_coefficients(&bad, p.data(), b.data(), 10, &alpha) == WHMC_EARG);
  bad = rooted(2, {8}, 3, 10, 10);
  EXPECT(whmc_rooted_coefficients(&bad, p.data(), b.data(), 10, &alpha) != WHMC_OK);
  bad = rooted(2, {8}, 0, 10, 10);
  bad.jmax = WHMC_MAX_POLY + 1;
  EXPECT(whmc_rooted_coefficients(&bad, p.data(), b.data(), 10, &alpha) == WHMC_EARG);
  EXPECT(whmc_rooted_coefficients(nullptr, p.data(), b.data(), 10, &alpha) == WHMC_EARG);
  whmc_rooted ok = rooted(2, {8}, 0, 10, 10);
  EXPECT(whmc_rooted_coefficients(&ok, p.data(), b.data(), WHMC_ROOTED_MAX_N + 1, &alpha) == WHMC_EARG);
}

static void masspre_coefficients() {
  for (double rho : {1e-6, 0.1, 0.5, 0.81, 0.99, 0.999999})
    for (int k = 0; k <= 2; ++k)
      for (int n : {0, 1, 15, 29, 400, 1000}) {
        std::vector<double> b(n + 1);
        double alpha = 0.0;
        EXPECT(whmc_masspre_coefficients(rho, k, n, b.data(), &alpha) == WHMC_OK);
        EXPECT(finite_all(b) && std::isfinite(alpha));
      }
  double b[8], alpha;
  for (double rho : {0.0, 1.0, -0.5, 2.0, (double)NAN}) EXPECT(whmc_masspre_coefficients(rho, 1, 5, b, &alpha) == WHMC_EARG);
  EXPECT(whmc_masspre_coefficients(0.5, 3, 5, b, &alpha) != WHMC_OK);
  EXPECT(whmc_masspre_coefficients(0.5, 1, -1, b, &alpha) == WHMC_EARG);
  EXPECT(whmc_masspre_coefficients(0.5, 1, 1001, b, &alpha) == WHMC_EARG);
}

// every entry point taking a context rejects a null one with WHMC_EARG and a message
static void null_context() {
  whmc_ctx* c = nullptr;
  double buf[64] = {0};
  double* d = buf;
  double kap[2] = {0.15, 0.15};
  int ib = 0, il = 0, io = 0;
  double us = 0;
  long long v = 0;
  size_t sz = 0;
  whmc_cg_params prm{1e-10, 100, WHMC_F64, WHMC_L18, 0.1, 8, 0, 0, 0};
  whmc_cg_stats st{};
  whmc_filter f{2, 15, 29};
  whmc_hmc_params hp{};
  hp.filter = f;
  hp.md_solver = hp.action_solver = prm;
  whmc_traj_result tr{};
  whmc_rooted r = rooted(2, {8}, 0, 10, 10);
  whmc_rooted_hmc_params rp{};
  rp.rooted = r;
  whmc_masspre mp{};
  mp.filter = f;
  whmc_masspre_hmc_params mpp{};
  mpp.mp = mp;
  long long it = 0;
  const whmc_status E = WHMC_EARG;
  EXPECT(whmc_set_stream(c, nullptr) == E);
  EXPECT(whmc_set_option(c, WHMC_OPT_STREAM_THRESHOLD, 0) == E);
  EXPECT(whmc_get_option(c, WHMC_OPT_STREAM_THRESHOLD, &v) == E);
  EXPECT(whmc_autotune_hop(c, &ib, &il, &us) == E);
  EXPECT(whmc_field_bytes(c, 0, 0, &sz) == E);
  EXPECT(whmc_load_gauge(c, d, 1e-12) == E);
  EXPECT(whmc_export_gauge(c, d) == E);
  EXPECT(whmc_pack_spinor(c, d, d + 1, 0, 1) == E);
  EXPECT(whmc_unpack_spinor(c, d, d + 1, 0, 1) == E);
  EXPECT(whmc_convert_spinor(c, d, 0, d + 1, 1, 1) == E);
  EXPECT(whmc_pack_algebra(c, d, d + 1) == E);
  EXPECT(whmc_unpack_algebra(c, d, d + 1) == E);
  EXPECT(whmc_apply_H(c, d, d + 1, 0, 0, WHMC_F64, WHMC_L18) == E);
  EXPECT(whmc_apply_H_multi(c, d, d + 1, 0, 0, WHMC_F64, WHMC_L18, 2, 0, 0, 0) == E);
  EXPECT(whmc_autotune(c, WHMC_F64, WHMC_L18, 2, &ib, &il, &io, &us) == E);
  EXPECT(whmc_apply_Moo(c, d, d + 1, 0.15, 0) == E);
  EXPECT(whmc_apply_M(c, d, d + 1, 0.15, 0) == E);
  EXPECT(whmc_apply_MdagM(c, d, d + 1, kap, 1, 1) == E);
  EXPECT(whmc_apply_MdagM_noalloc(c, d, d + 1, kap, 1, 1) == E);
  EXPECT(whmc_cg_solve(c, d, d + 1, kap, 1, &prm, &st) == E);
  EXPECT(whmc_cg_solve_full(c, d, d + 1, 0.15, &prm, &st) == E);
  EXPECT(whmc_bicgstab_solve(c, d, d + 1, 0.15, 0, &prm, &st) == E);
  EXPECT(whmc_heatbath_phi(c, d, d + 1, &f, 0.15) == E);
  EXPECT(whmc_action(c, d, d + 1, d + 2, &f, 0.15, 5.6, &prm) == E);
  EXPECT(whmc_action_full(c, d, d + 1, 0.15, &prm) == E);
  EXPECT(whmc_plaquette(c, d) == E);
  EXPECT(whmc_force(c, d, d + 1, &f, 0.15, 5.6, &prm, WHMC_FORCE_PF) == E);
  EXPECT(whmc_force_full(c, d, d + 1, 0.15, 5.6, &prm, WHMC_FORCE_PF) == E);
  EXPECT(whmc_update_links(c, d, 0.1) == E);
  EXPECT(whmc_update_momenta(c, d, d + 1, 0.1) == E);
  EXPECT(whmc_dexp_transpose(c, d, d + 1, d + 2) == E);
  EXPECT(whmc_hmc_trajectory(c, &hp, d, d + 1, 0.5, &tr) == E);
  EXPECT(whmc_md_integrate(c, &hp, d, d + 1) == E);
  EXPECT(whmc_hamiltonian(c, &hp, d, d + 1, d + 2) == E);
  EXPECT(whmc_rooted_heatbath(c, d, d + 1, &r, 0.15, &prm, &it) == E);
  EXPECT(whmc_rooted_action(c, d, d + 1, &r, 0.15, &prm) == E);
  EXPECT(whmc_rooted_force(c, d, d + 1, &r, 0, 0.15, &prm, 0) == E);
  EXPECT(whmc_rooted_trajectory(c, &rp, d, d + 1, 0.5, &tr) == E);
  EXPECT(whmc_rooted_md_integrate(c, &rp, d, d + 1) == E);
  EXPECT(whmc_rooted_hamiltonian(c, &rp, d, d + 1, d + 2) == E);
  EXPECT(whmc_masspre_heatbath(c, d, d + 1, &mp, 0.15, &prm) == E);
  EXPECT(whmc_masspre_action(c, d, d + 1, &mp, 0.15, &prm) == E);
  EXPECT(whmc_masspre_force(c, d, d + 1, &mp, 0, 0.15, &prm, 0) == E);
  EXPECT(whmc_masspre_trajectory(c, &mpp, d, d + 1, 0.5, &tr) == E);
  EXPECT(whmc_masspre_md_integrate(c, &mpp, d, d + 1) == E);
  EXPECT(whmc_masspre_hamiltonian(c, &mpp, d, d + 1, d + 2) == E);
  whmc_destroy(nullptr);
  EXPECT(whmc_last_error() != nullptr);
}

static void create_arguments() {
  whmc_ctx* c = nullptr;
  const int odd[4] = {4, 4, 4, 5}, zero[4] = {4, 0, 4, 4}, huge[4] = {1024, 1024, 1024, 1024};
  EXPECT(whmc_create(nullptr, odd, 0, nullptr) == WHMC_EARG);
  EXPECT(whmc_create(&c, nullptr, 0, nullptr) == WHMC_EARG);
  EXPECT(whmc_create(&c, odd, 0, nullptr) == WHMC_EARG && c == nullptr);
  EXPECT(whmc_create(&c, zero, 0, nullptr) == WHMC_EARG && c == nullptr);
  EXPECT(whmc_create(&c, huge, 0, nullptr) == WHMC_EARG && c == nullptr);
  EXPECT(whmc_abi_version() == WHMC_ABI_VERSION);
}

// the LDS reservation of the occupancy cap: k workgroups fit, k + 1 do not, for every k and any
// plausible LDS size; impossible requests give 0
static void lds_reservation() {
  int possible = 0;
  for (long long cu = 32768; cu <= 262144; cu += 1024)
    for (int k = 2; k <= 8; ++k) {
      const unsigned b = whmc::lds_reservation(cu, cu, k);
      if (b == 0) continue;
      ++possible;
      EXPECT(b % 2048 == 0);
      EXPECT(((long long)b + 2048) * k <= cu);   // k fit even with each allocation rounded up by 2 KiB
      EXPECT((long long)b * (k + 1) > cu);       // k + 1 never fit
    }
  EXPECT(possible > 1000);
  for (int k : {2, 3, 4, 5, 6, 8}) EXPECT(whmc::lds_reservation(163840, 163840, k) > 0);   // gfx950: 160 KiB per CU
  EXPECT(whmc::lds_reservation(163840, 65536, 2) == 55296);
  EXPECT(whmc::lds_reservation(163840, 65536, 1) == 0);
  EXPECT(whmc::lds_reservation(163840, 65536, 9) == 0);
  EXPECT(whmc::lds_reservation(0, 65536, 2) == 0);
  EXPECT(whmc::lds_reservation(163840, 16384, 2) == 0);   // more than one workgroup may allocate
}

int main() {
  filter_coefficients();
  rooted_coefficients();
  masspre_coefficients();
  null_context();
  create_arguments();
  lds_reservation();
  std::printf("host checks passed: %d\n", g_checks);
  return 0;
}
