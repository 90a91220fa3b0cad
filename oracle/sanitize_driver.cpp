// Test infrastructure: a host program that runs every exported oracle entry
// point on tiny grids, built with AddressSanitizer and UndefinedBehavior-
// Sanitizer by the CPU tests (out-of-bounds accesses, use after free, integer
// overflow, misaligned or null accesses abort the run).  It checks nothing
// numerically; the numerical pins live in the Python tests.
#include "msc_oracle.cpp"

#include <cstdio>
#include <random>
#include <vector>

namespace {

std::mt19937_64 rng(12345);

std::vector<double> noise(size_t n, double scale) {
  std::normal_distribution<double> g(0.0, scale);
  std::vector<double> v(n);
  for (auto& x : v) x = g(rng);
  return v;
}

int Qof(int d) { return d == 2 ? 9 : 19; }

// populations near a resting equilibrium: feq(1e-3 noise) plus small noise
std::vector<double> pops(int d, const int* n) {
  int64_t NS = (int64_t)n[0] * n[1] * (d == 3 ? n[2] : 1);
  auto p0 = noise(NS, 1e-6);
  auto u0 = noise((size_t)d * NS, 1e-3);
  std::vector<double> f((size_t)Qof(d) * NS);
  orc_init_populations(d, n, p0.data(), u0.data(), f.data());
  for (auto& x : f) x += 1e-5 * std::normal_distribution<double>(0.0, 1.0)(rng);
  return f;
}

int fail(const char* what, int rc) {
  std::fprintf(stderr, "%s returned %d\n", what, rc);
  return 1;
}

int run_lattice(int d, const int* n) {
  const int Q = Qof(d);
  const int64_t NS = (int64_t)n[0] * n[1] * (d == 3 ? n[2] : 1);
  const size_t FQ = (size_t)Q * NS, FM = (size_t)(d + 1) * NS;
  const double a = 3.0 / 128.0;
  auto f = pops(d, n);
  auto h = noise(FM, 1e-5);
  std::vector<double> fT(FQ), Pr(FM), dm(FM), fn(FQ);
  double R = 0;
  int rc;
  if ((rc = orc_sweep(d, n, f.data(), h.data(), a, 1.0, 1.0, fT.data(), Pr.data(), &R))) return fail("sweep", rc);
  if ((rc = orc_sweep(d, n, f.data(), h.data(), a, 1 / 0.8, 1 / 1.3, fT.data(), Pr.data(), &R)))
    return fail("sweep off-design", rc);
  if ((rc = orc_corrected_iteration(d, n, f.data(), h.data(), a, 1.0, 1.0, 1.0 / 6.0, fn.data(), fT.data(),
                                    Pr.data(), dm.data(), &R)))
    return fail("corrected_iteration", rc);
  if ((rc = orc_full_symbol_iteration(d, n, f.data(), h.data(), a, 1.0, 1.0, 0.0, fn.data(), fT.data(), &R)))
    return fail("full_symbol_iteration", rc);
  std::vector<double> lam = noise(FQ, 1.0), lout(FQ), lh(FM);
  if ((rc = orc_sweep_adjoint(d, n, f.data(), h.data(), a, 1.0, 1.0, lam.data(), lout.data(), lh.data())))
    return fail("sweep_adjoint", rc);
  std::vector<double> y = noise(FM, 1.0), yo(FM);
  if ((rc = orc_shadow_adjoint(d, n, y.data(), a, 1.0 / 6.0, yo.data()))) return fail("shadow_adjoint", rc);
  std::vector<int32_t> nbr(FQ), sidx(n[0] + n[1] + (d == 3 ? n[2] : 0));
  std::vector<uint8_t> mask(NS);
  if ((rc = orc_tables(d, n, nbr.data(), sidx.data(), mask.data()))) return fail("tables", rc);
  std::vector<double> re = noise(NS, 1.0), im = noise(NS, 1.0);
  if ((rc = orc_fft(d, n, re.data(), im.data(), 0)) || (rc = orc_fft(d, n, re.data(), im.data(), 1)))
    return fail("fft", rc);
  std::vector<double> fe = f;
  if ((rc = orc_explicit(d, n, 1.0, 1.0, fe.data(), 5))) return fail("explicit", rc);

  // marches: shadow (paper trial rule and the linear cap), Picard, full symbol
  auto p0 = noise(NS, 1e-7);
  auto u0 = noise((size_t)d * NS, 1e-4);
  std::vector<double> state(3 * FQ + 2 * FM);
  if ((rc = orc_initial_state(d, n, p0.data(), u0.data(), state.data()))) return fail("initial_state", rc);
  orc_params P{};
  P.d = d;
  for (int i = 0; i < 3; ++i) P.n[i] = (i < d) ? n[i] : 1;
  P.tau_plus = P.tau_minus = 1.0;
  P.dt = 24.0;
  P.eps = 1e-10;
  P.kmax = 300;
  P.nmin = 2;
  const int S = 4;
  std::vector<orc_step_stats> st(S);
  std::vector<double> Rh((size_t)S * P.kmax);
  std::vector<double> fo(FQ), mo(FM);
  int done = 0;
  const int correctors[3] = {1, 0, 2};
  for (int ci = 0; ci < 3; ++ci) {
    P.corrector = correctors[ci];
    for (int ex : {0, 2}) {
      P.extrap_states = ex;
      if ((rc = orc_march(&P, p0.data(), u0.data(), S, nullptr, st.data(), Rh.data(), fo.data(), mo.data(), &done)))
        return fail("march", rc);
    }
  }
  // march state and its adjoint at the recorded counts
  P.corrector = 1;
  P.extrap_states = 0;
  std::vector<double> s1 = state;
  int64_t bc = 0;
  if ((rc = orc_march_state(&P, s1.data(), &bc, S, nullptr, st.data(), nullptr, &done))) return fail("march_state", rc);
  std::vector<int> K(S);
  for (int i = 0; i < S; ++i) K[i] = st[i].iters;
  std::vector<double> lam_s = noise(state.size(), 1.0);
  if ((rc = orc_march_adjoint(&P, state.data(), 0, S, K.data(), lam_s.data()))) return fail("march_adjoint", rc);
  std::vector<double> lp(NS), lu((size_t)d * NS);
  if ((rc = orc_initial_state_adjoint(d, n, p0.data(), u0.data(), lam_s.data(), lp.data(), lu.data())))
    return fail("initial_state_adjoint", rc);
  return 0;
}

int run_cavity() {
  const int n[2] = {8, 6};
  const int64_t NS = 48;
  const size_t FQ = 9 * NS, FM = 3 * NS;
  const double a = 3.0 / 64.0;
  auto f = pops(2, n);
  auto h = noise(FM, 1e-5);
  std::vector<double> fT(FQ);
  double R = 0;
  int rc;
  if ((rc = orc_sweep_cavity(n, f.data(), h.data(), a, 1.0, 1.0, 1e-3, fT.data(), &R))) return fail("sweep_cavity", rc);
  auto mref = noise(FM, 1e-4), sref = noise(FM, 1e-6);
  std::vector<double> Jc((size_t)NS * 81);
  if ((rc = orc_cavity_local_jacobians(NS, a, mref.data(), sref.data(), Jc.data())))
    return fail("cavity_local_jacobians", rc);
  return 0;
}

}  // namespace

int main() {
  const int g2[3] = {8, 4, 1}, g2b[3] = {4, 8, 1}, g3[3] = {4, 8, 4};
  if (run_lattice(2, g2) || run_lattice(2, g2b) || run_lattice(3, g3) || run_cavity()) return 1;
  std::printf("sanitized oracle run: ok\n");
  return 0;
}
