// Solver<L, T>: device buffers and kernel sequencing for one lattice and
// storage type.  Included by one translation unit per instantiation.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <string>
#include <type_traits>
#include <vector>

#include <hip/hip_ext.h>

#include "msc_aa.h"
#include "msc_adjoint.h"
#include "msc_sweep_launch.h"
#include "msc_fullsym.h"
#include "msc_walls.h"
#include "msc_solver.h"

namespace msc {

#define MSC_HIPCK(x)                                                                 \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) throw DeviceError{e_, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

struct OomError {};

inline int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Buffers of one run of the correction transforms in one precision.
template <class CX, class TX>
struct XformBufs {
  const TX* in;
  TX* out;
  cpx<CX>* spec1;
  cpx<CX>* spec2;
  const cpx<CX>* tw[3];
};

// ----------------------------------------------------------------- solver --
template <class L, class T>
class Solver : public SolverBase {
 public:
  using CT = typename CompT<T>::type;
  using TM = CT;
  static constexpr int Q = L::Q, D = L::D;
  static constexpr bool DV = PopDev<T>::value;  // FP16 deviation storage

  Solver(const msc_params& p, const Geometry& g, hipStream_t s) : P(p), G(g), st(s) {
    wp = 1.0 / P.tau_plus;
    wm = 1.0 / P.tau_minus;
    nu = (P.tau_plus - 0.5) / 3.0;  // Eq. (trt): nu = cs^2 (tau+ - 1/2)
  }
  ~Solver() override { release(); }

  Tuning& tuning() override { return tune; }

  void krylov_stats(int64_t* solves, int64_t* iters, int64_t* refreshes, double* worst) const override {
    if (solves) *solves = kr_solves;
    if (iters) *iters = kr_iters;
    if (refreshes) *refreshes = kr_refresh;
    if (worst) *worst = kr_worst;
  }

  msc_status reconfigure() override {
    return guard([&]() {
      sync();
      choose_sweep();
      ensure_partials(sweep_grid_max());
      if (spec && corrector_supported()) set_fft_attrs();
      if (gexec) (void)hipGraphExecDestroy(gexec);
      if (graph) (void)hipGraphDestroy(graph);
      gexec = nullptr;
      graph = nullptr;
      return MSC_OK;
    });
  }

  // ----------------------------------------------------------------- init --
  msc_status init(const double* phat0, const double* u0, bool on_device) override {
    return guard([&]() -> msc_status {
      if (P.corrector == MSC_CORRECTOR_SHADOW && !corrector_supported()) {
        last_error = "the shadow corrector is not available for this lattice/grid size";
        return MSC_ERR_UNSUPPORTED;
      }
      if (wallkin() && !wall_supported()) {
        last_error = "the wall-kinetic corrector needs the D2Q9 cavity, FP64 storage, tau+ = tau- = 1 and "
                     "extents up to 256";
        return MSC_ERR_UNSUPPORTED;
      }
      if (fullsym() && !fs_supported()) {
        last_error = "the full-symbol corrector needs D2Q9 with FP64 or FP32 storage and its transforms "
                     "in LDS (N_x, N_y <= 512 FP32 / 256 FP64 per line pass)";
        return MSC_ERR_UNSUPPORTED;
      }
      allocate();
      // Algorithm 2: the initial wall operator is assembled at rest with the
      // BDF2 coefficient
      wk_aA = 1.5 / P.dt;
      wk_rest = true;
      const int64_t NS = G.NS;
      double* pd = nullptr;
      double* ud = nullptr;
      if (on_device) {
        pd = const_cast<double*>(phat0);
        ud = const_cast<double*>(u0);
      } else {
        double* stg = staging();
        MSC_HIPCK(hipMemcpyAsync(stg, phat0, sizeof(double) * NS, hipMemcpyHostToDevice, st));
        MSC_HIPCK(hipMemcpyAsync(stg + NS, u0, sizeof(double) * D * NS, hipMemcpyHostToDevice, st));
        pd = stg;
        ud = stg + NS;
      }
      // control block: slots 0,1,2 hold f^n, f^{n-1}, f^{n-2}; 3,4 work.
      std::memset(ctl_h, 0, sizeof(DevCtl));
      ctl_h->phase = make_phase(-1, 0, PH_ACCEPTED);
      for (int r = 0; r < 2; ++r) {
        Roles& ro = ctl_h->roles[r];
        for (int i = 0; i < 3; ++i) ro.slot_hist[i] = i;
        ro.slot_w[0] = 3;
        ro.slot_w[1] = 4;
        for (int i = 0; i < 3; ++i) ro.slot_m[i] = i;
      }
      n_next = 0;
      MSC_HIPCK(hipMemcpyAsync(ctl, ctl_h, sizeof(DevCtl), hipMemcpyHostToDevice, st));
      if (DV) sig = choose_sigma(0.0, std::max(absmax(pd, NS), absmax(ud, (int64_t)D * NS)));
      hipLaunchKernelGGL((k_init_feq<L, T>), dim3(ew_grid()), dim3(256), 0, st, pd, ud, fb.p[0], NS);
      MSC_HIPCK(hipGetLastError());
      reset_history_from_current();
      sync();
      n_next = 0;
      return MSC_OK;
    });
  }

  // ------------------------------------------------------- BDF dual time --
  msc_status bdf2_step(int32_t nsteps, msc_step_stats* out) override {
    if (wallkin()) return bdf2_step_walls(nsteps, out);
    return guard([&]() -> msc_status {
      if (nsteps <= 0) return MSC_OK;
      ensure_stats(nsteps);
      const int stat_base = n_next;
      const int n_end = n_next + nsteps;
      // schedule replay for these steps
      const bool use_sched = sched_pos < (int64_t)sched_h.size();
      if (use_sched) {
        std::vector<int32_t> K(nsteps, 0);
        for (int i = 0; i < nsteps; ++i) {
          const int64_t j = sched_pos + i;
          K[i] = (j < (int64_t)sched_h.size()) ? sched_h[j] : P.k_max;
        }
        ensure_sched(nsteps);
        MSC_HIPCK(hipMemcpyAsync(sched_d, K.data(), sizeof(int32_t) * nsteps, hipMemcpyHostToDevice, st));
        sched_host_view = K;
      }
      int n_dev = n_next, ell_dev = 1;
      int64_t bdf_dev = bdf_count;
      int batch = 1;
      msc_status rc = MSC_OK;
      if (recording) pull_ctl();
      while (n_dev < n_end) {
        // while recording, one step per synchronisation so that the state at
        // each step's start can be checkpointed
        const int B = recording ? 1 : std::min(batch, n_end - n_dev);
        if (recording && ell_dev == 1) take_checkpoint(n_dev, bdf_dev);
        for (int i = 0; i < B; ++i) {
          const int n = n_dev + i;
          const int64_t bc = bdf_dev + i;
          const int q = (bc == 0) ? 1 : 2;
          const int max_order = (P.extrap_states == 0) ? 2 : P.extrap_states - 1;
          const int order = (int)std::min<int64_t>(bc, max_order);
          const double a = (q == 1) ? 1.0 / P.dt : 3.0 / (2.0 * P.dt);
          const int ell0 = (i == 0) ? ell_dev : 1;
          int want;
          if (use_sched)
            want = sched_host_view[n - stat_base];
          else
            want = std::max(P.n_min, last_iters + tune.spec_extra);
          int ell1 = (ell0 == 1) ? want : ell0 - 1 + std::max(8, want);
          ell1 = std::min(std::max(ell1, ell0), P.k_max);
          // resuming a step: the previous batch ended it at sweep ell0 - 1
          // without the correction's later passes
          if (ell0 > 1) enqueue_correction_tail(n, ell0 - 1, a);
          // within one call, each step's acceptance leaves m^{n+1} to the next
          // step's setup sweep (which reads the same populations anyway); the
          // call's last step reconstructs it so that the state is complete
          // when the call returns, and recording keeps every step complete for
          // its checkpoint
          const bool recon = !recording && n > stat_base;
          const double a_prev = (bc - 1 == 0) ? 1.0 / P.dt : 3.0 / (2.0 * P.dt);
          const bool defer = !recording && n < n_end - 1;
          for (int ell = ell0; ell <= ell1; ++ell)
            enqueue_iteration(n, ell, q, order, a, use_sched, stat_base, ell == ell1, recon, a_prev, defer);
        }
        MSC_HIPCK(hipMemcpyAsync(ctl_h, ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, st));
        sync();
        const uint64_t ph = ctl_h->phase;
        const int pn = phase_n(ph), pell = phase_ell(ph);
        const uint32_t ps = phase_state(ph);
        if (ps == PH_FAILED) {
          if (recording && !records.empty() && records.back().K == 0) drop_last_record();
          bdf_dev += (pn - n_dev);
          rc = (ctl_h->fail_code == 5) ? MSC_ERR_NONCONVERGED : MSC_ERR_NONFINITE;
          last_error = std::string(rc == MSC_ERR_NONCONVERGED ? "nonconvergent" : "non-finite residual") +
                       " at physical step " + std::to_string(pn) + ", inner iteration " + std::to_string(pell);
          // the march stays at the last accepted step
          ctl_h->phase = make_phase(pn - 1, 0, PH_ACCEPTED);
          ctl_h->fail_code = 0;
          MSC_HIPCK(hipMemcpyAsync(ctl, ctl_h, sizeof(DevCtl), hipMemcpyHostToDevice, st));
          copy_stats(out, stat_base, pn - stat_base + 1);
          n_next = pn;
          bdf_count = bdf_dev;
          sched_pos += (pn - stat_base);
          sync();
          return rc;
        }
        if (ps == PH_ACCEPTED) {
          if (recording && !records.empty() && records.back().K == 0) records.back().K = pell;
          bdf_dev += (pn - n_dev + 1);
          n_dev = pn + 1;
          ell_dev = 1;
          last_iters = pell;
          batch = std::min(batch * 2, std::max(1, tune.batch_steps));
        } else {
          // still iterating step pn after pell sweeps
          bdf_dev += (pn - n_dev);
          n_dev = pn;
          ell_dev = pell + 1;
          last_iters = std::max(last_iters, pell + 1);
          batch = 1;
        }
      }
      copy_stats(out, stat_base, nsteps);
      n_next = n_end;
      bdf_count = bdf_dev;
      if (use_sched) sched_pos += nsteps;
      return rc;
    });
  }

  // -------------------------------------------------------- explicit march --
  msc_status explicit_step(int64_t nsteps) override {
    return guard([&]() -> msc_status {
      pull_ctl();
      T* A = fb.p[cur_roles().slot_hist[0]];
      T* B = fb.p[cur_roles().slot_w[0]];
      SweepArgs<T, TM> S = sweep_args(0.0);
      const int64_t chunk = 64;
      int64_t done = 0;
      const bool aa = aa_ok();
      // AA march: pairs of steps in place on A; an odd count ends with one
      // two-buffer sweep
      const int64_t paired = aa ? (nsteps & ~(int64_t)1) : 0;
      if (tune.use_graph && (aa ? paired : nsteps) >= chunk && !timing) {
        hipGraphExec_t ge = explicit_graph(A, B, (int)chunk, aa);
        for (; done + chunk <= (aa ? paired : nsteps); done += chunk) MSC_HIPCK(hipGraphLaunch(ge, st));
      }
      for (; done < paired; done += 2) {
        launch_aa(A, false);
        launch_aa(A, true);
      }
      const bool swapped = aa ? (nsteps & 1) : false;
      for (; done < nsteps; ++done) {
        const int64_t i = aa ? 0 : done;
        S.src = (i & 1) ? B : A;
        S.dst = (i & 1) ? A : B;
        launch_sweep_timed(SW_EXPLICIT, S, 1);
      }
      if (aa ? swapped : (nsteps & 1)) std::swap(cur_roles().slot_hist[0], cur_roles().slot_w[0]);
      MSC_HIPCK(hipMemcpyAsync(ctl, ctl_h, sizeof(DevCtl), hipMemcpyHostToDevice, st));
      reset_history_from_current();
      // non-finite check on the final state
      const double ss = pop_sumsq(fb.p[cur_roles().slot_hist[0]]);
      if (!std::isfinite(ss)) {
        last_error = "non-finite population after the explicit march";
        return MSC_ERR_NONFINITE;
      }
      return MSC_OK;
    });
  }

  // The in-place (AA) explicit march: periodic boundaries and full-population
  // storage (FP64, FP32); the cavity and FP16-deviation storage keep the
  // two-buffer sweep.
  bool aa_ok() const { return tune.explicit_aa && !walls() && !PopDev<T>::value && G.NS < ((int64_t)1 << 31); }

  // one AA kernel (odd = false: the even kernel) on the population array f
  void launch_aa(T* f, bool odd) {
    if constexpr (!PopDev<T>::value) {
      AaArgs<T> A{};
      A.f = f;
      A.N0 = G.N0;
      A.N1 = G.N1;
      A.N2 = G.N2;
      A.lg1 = ilog2(G.N1);
      A.lg2 = ilog2(G.N2);
      A.NS = (int)G.NS;
      A.wp = 1.0 / P.tau_plus;
      A.wm = 1.0 / P.tau_minus;
      EvPair ep{};
      if (timing) {
        ep = timed_pair(1, 2.0 * Q * (double)G.NS * sizeof(T));
        A.did_run = run_flags + ep.flag;
        MSC_HIPCK(hipEventRecord(ep.a, st));
      }
      const int grid = (int)((G.NS + 255) / 256);
      if (odd)
        hipLaunchKernelGGL((k_aa_odd<L, T>), dim3(grid), dim3(256), 0, st, A);
      else
        hipLaunchKernelGGL((k_aa_even<L, T>), dim3(grid), dim3(256), 0, st, A);
      MSC_HIPCK(hipGetLastError());
      if (timing) {
        MSC_HIPCK(hipEventRecord(ep.b, st));
        ev_live.push_back(ep);
        if ((int)ev_live.size() >= kFlagCap) collect_timing();
      }
    }
  }

  // -------------------------------------------------------------- outputs --
  msc_status moments(double* phat, double* u, bool on_device) override {
    return guard([&]() {
      pull_ctl();
      const double* m = mb[cur_roles().slot_m[0]];
      const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
      if (phat) MSC_HIPCK(hipMemcpyAsync(phat, m, sizeof(double) * G.NS, kind, st));
      if (u) MSC_HIPCK(hipMemcpyAsync(u, m + G.NS, sizeof(double) * D * G.NS, kind, st));
      sync();
      return MSC_OK;
    });
  }

  msc_status export_tables(int32_t* nbr, int32_t* sidx, uint8_t* mask) override {
    return guard([&]() {
      const int64_t NS = G.NS;
      const int nsum = G.n[0] + G.n[1] + (D == 3 ? G.n[2] : 0);
      int32_t* dn = (int32_t*)dalloc(sizeof(int32_t) * Q * NS);
      uint8_t* dmk = (uint8_t*)dalloc(NS);
      int32_t* ds = (int32_t*)dalloc(sizeof(int32_t) * nsum);
      hipLaunchKernelGGL((k_tables<L>), dim3(ew_grid()), dim3(256), 0, st, G.N0, G.N1, G.N2, dn, dmk, ds);
      MSC_HIPCK(hipGetLastError());
      if (nbr) MSC_HIPCK(hipMemcpyAsync(nbr, dn, sizeof(int32_t) * Q * NS, hipMemcpyDeviceToHost, st));
      if (mask) MSC_HIPCK(hipMemcpyAsync(mask, dmk, NS, hipMemcpyDeviceToHost, st));
      if (sidx) MSC_HIPCK(hipMemcpyAsync(sidx, ds, sizeof(int32_t) * nsum, hipMemcpyDeviceToHost, st));
      sync();
      dfree(dn);
      dfree(dmk);
      dfree(ds);
      return MSC_OK;
    });
  }

  msc_status get_populations(double* f) override {
    return guard([&]() {
      pull_ctl();
      download_pop(fb.p[cur_roles().slot_hist[0]], f);
      return MSC_OK;
    });
  }

  msc_status set_populations(const double* f) override {
    return guard([&]() {
      pull_ctl();
      if (DV) sig = sigma_for({f});
      upload_pop(f, fb.p[cur_roles().slot_hist[0]]);
      reset_history_from_current();
      sync();
      return MSC_OK;
    });
  }

  // ------------------------------------------------------------ diagnostics --
  msc_status sweep(const double* f, const double* h_in, double a, double* fT, double* Pr_out,
                   double* R) override {
    return guard([&]() {
      pull_ctl();
      T* A = fb.p[cur_roles().slot_w[0]];
      T* B = fb.p[cur_roles().slot_w[1]];
      const float sig_state = sig;  // the work buffers may take another scale
      if (DV) sig = sigma_for({f});
      upload_pop(f, A);
      upload_h(h_in);
      SweepArgs<T, TM> S = sweep_args(a);
      S.src = A;
      S.dst = B;
      launch_sweep_timed(SW_DTS, S, 0);
      const double Rv = reduce_partials(S);
      if (R) *R = Rv;
      if (fT) download_pop(B, fT);
      if (Pr_out) download_tm(Pr, Pr_out, (int64_t)(D + 1) * G.NS);
      sync();
      sig = sig_state;
      return MSC_OK;
    });
  }

  msc_status correct(const double* f, const double* h_in, double a, double* fnext, double* dm_out,
                     double* R) override {
    if (fullsym()) return correct_fullsym(f, h_in, a, fnext, dm_out, R);
    if (wallkin()) return correct_walls(f, h_in, a, fnext, dm_out, R);
    return guard([&]() -> msc_status {
      if (!corrector_supported()) {
        last_error = "the shadow corrector is not available for this lattice/grid";
        return MSC_ERR_UNSUPPORTED;
      }
      pull_ctl();
      T* A = fb.p[cur_roles().slot_w[0]];
      T* B = fb.p[cur_roles().slot_w[1]];
      const float sig_state = sig;
      if (DV) sig = sigma_for({f});
      upload_pop(f, A);
      upload_h(h_in);
      SweepArgs<T, TM> S = sweep_args(a);
      S.src = A;
      S.dst = B;
      launch_sweep_timed(SW_DTS, S, 0);
      const double Rv = reduce_partials(S);
      if (R) *R = Rv;
      enqueue_correction(nullptr, 0, 0, a, nullptr);
      // f_next = f_T + E dm: the same lift the next sweep applies on load,
      // here through an explicit no-op-collision pass is not available, so
      // apply it element-wise.
      hipLaunchKernelGGL((k_lift<L, T, TM>), dim3(ew_grid()), dim3(256), 0, st, B, dm, A, G.NS, sig, 1.0f / sig);
      MSC_HIPCK(hipGetLastError());
      if (fnext) download_pop(A, fnext);
      if (dm_out) download_tm(dm, dm_out, (int64_t)(D + 1) * G.NS);
      sync();
      sig = sig_state;
      return MSC_OK;
    });
  }

  // One full-symbol corrected iteration from host arrays: f_T = T(f), the
  // correction of Eq. (full-symbol), f_next = f + df; dm_out (no macroscopic
  // correction field here) is zeroed.
  msc_status correct_fullsym(const double* f, const double* h_in, double a, double* fnext, double* dm_out,
                             double* R) {
    return guard([&]() -> msc_status {
      pull_ctl();
      T* A = fb.p[cur_roles().slot_w[0]];
      T* B = fb.p[cur_roles().slot_w[1]];
      upload_pop(f, A);
      upload_h(h_in);
      SweepArgs<T, TM> S = sweep_args(a);
      S.src = A;
      S.dst = B;
      S.rout = rfs;
      launch_sweep_timed(SW_DTS, S, 0);
      const double Rv = reduce_partials(S);
      if (R) *R = Rv;
      enqueue_fullsym(nullptr, 0, 0, a, nullptr, nullptr, true, true, B);
      if (fnext) download_pop(B, fnext);
      sync();
      if (dm_out) std::memset(dm_out, 0, sizeof(double) * (D + 1) * G.NS);
      return MSC_OK;
    });
  }

  // ------------------------------------------- wall-bounded correction --
  void wall_allocate() {
    const int64_t n = (int64_t)Q * G.NS;
    wk_m = P.wall_restart > 0 ? P.wall_restart : 50;
    wk_V = keep((double*)dalloc(sizeof(double) * (wk_m + 1) * n));
    wk_R = keep((double*)dalloc(sizeof(double) * n));
    wk_Y = keep((double*)dalloc(sizeof(double) * n));
    wk_Z = keep((double*)dalloc(sizeof(double) * n));
    wk_D = keep((double*)dalloc(sizeof(double) * n));
    wk_W = keep((double*)dalloc(sizeof(double) * n));
    wk_vc = keep((double*)dalloc(sizeof(double) * n));
    wk_mu = keep((double*)dalloc(sizeof(double) * 3 * G.NS));
    wk_mref = keep((double*)dalloc(sizeof(double) * 3 * G.NS));
    wk_sref = keep((double*)dalloc(sizeof(double) * 3 * G.NS));
    wk_part = keep((double*)dalloc(sizeof(double) * kDotBlocks * (wk_m + 2)));
    wk_coef = keep((double*)dalloc(sizeof(double) * (wk_m + 2)));
    const size_t small = (size_t)wk_m * wk_m + 2 * wk_m + (wk_m + 1) + (wk_m + 2) + 1 + wk_m;
    wk_small = keep((double*)dalloc(sizeof(double) * small));
    MSC_HIPCK(hipHostMalloc((void**)&wk_part_h, sizeof(double) * kDotBlocks * (wk_m + 2), hipHostMallocDefault));
    MSC_HIPCK(hipHostMalloc((void**)&wk_coef_h, sizeof(double) * (wk_m + 2), hipHostMallocDefault));
    MSC_HIPCK(hipHostMalloc((void**)&wk_small_h, sizeof(double) * small, hipHostMallocDefault));
  }

  int vec_grid() const {
    const int64_t n = (int64_t)Q * G.NS;
    return (int)std::min<int64_t>((n + 255) / 256, 2048);
  }

  // <V_i, w> for i < nv, summed on the host in block order
  void wall_dots(const double* V, int nv, const double* w, double* out) {
    const int64_t n = (int64_t)Q * G.NS;
    hipLaunchKernelGGL(k_dots<double>, dim3(kDotBlocks), dim3(256), 0, st, V, n, nv, w, n, wk_part, 0);
    MSC_HIPCK(hipGetLastError());
    MSC_HIPCK(hipMemcpyAsync(wk_part_h, wk_part, sizeof(double) * kDotBlocks * nv, hipMemcpyDeviceToHost, st));
    sync();
    for (int i = 0; i < nv; ++i) {
      double acc = 0.0;
      for (int b = 0; b < kDotBlocks; ++b) acc += wk_part_h[(int64_t)i * kDotBlocks + b];
      out[i] = acc;
    }
  }

  void upload_coef(const double* c, int nv) {
    for (int i = 0; i < nv; ++i) wk_coef_h[i] = c[i];
    MSC_HIPCK(hipMemcpyAsync(wk_coef, wk_coef_h, sizeof(double) * nv, hipMemcpyHostToDevice, st));
  }

  void lincomb(double* out, const double* x, double alpha, const double* y, double beta) {
    hipLaunchKernelGGL(k_lincomb<0>, dim3(vec_grid()), dim3(256), 0, st, out, x, alpha, y, beta,
                       (int64_t)Q * G.NS);
    MSC_HIPCK(hipGetLastError());
  }

  // w = (I - L) z with the current operator (Eq. wall-global-jacobian)
  void wall_apply(const double* z, double* w) {
    const int g = ew_grid();
    hipLaunchKernelGGL(k_wall_mu<0>, dim3(g), dim3(256), 0, st, z, wk_mu, G.NS, 1.0 / (1.0 + 0.5 * wk_aA));
    MSC_HIPCK(hipGetLastError());
    hipLaunchKernelGGL(k_wall_apply<0>, dim3(g), dim3(256), 0, st, z, (const double*)wk_mu,
                       wk_rest ? (const double*)nullptr : (const double*)wk_mref,
                       wk_rest ? (const double*)nullptr : (const double*)wk_sref, wk_aA, G.N0, G.N2, w);
    MSC_HIPCK(hipGetLastError());
  }

  // out = M^{-1} in: the periodic full-symbol inverse at rest (omega = 1, a_A)
  void wall_precondition(const double* in, double* out) {
    if constexpr (std::is_same<T, double>::value && std::is_same<TM, double>::value)
      enqueue_fullsym(nullptr, 0, 0, wk_aA, nullptr, nullptr, true, true, (T*)out, (const TM*)in, 1);
  }

  // Restarted GMRES(m), right-preconditioned, classical Gram-Schmidt (with
  // one re-orthogonalisation when krylov_tol < 1e-8; a single projection
  // otherwise, which halves the passes over the basis): delta ~ (I - L)^{-1}
  // rhs to the relative residual krylov_tol.  The basis is stored in FP32 when
  // krylov_tol >= 1e-5 (half the bytes of the passes over it; its rounding,
  // ~1e-7 relative, stays far below such tolerances), else in FP64; the new
  // vector, the coefficients and every sum are FP64.  The orthogonalisation
  // coefficients, the Hessenberg columns and the Givens rotations stay on the
  // device (k_gs_first, k_gs_second); the host reads the residual estimate
  // every kCheck iterations and the small triangular system once per cycle.
  // Returns the iteration count; rel receives the final true relative
  // residual.
  static constexpr int kCheck = 4;
  int wall_gmres(const double* rhs, double* delta, double& rel) {
    const double tol = P.krylov_tol > 0.0 ? P.krylov_tol : 1e-12;
    return tol >= 1e-5 ? wall_gmres_t<float>(rhs, delta, rel) : wall_gmres_t<double>(rhs, delta, rel);
  }

  template <class VT>
  int wall_gmres_t(const double* rhs, double* delta, double& rel) {
    const int64_t n = (int64_t)Q * G.NS;
    const int m = wk_m;
    const double tol = P.krylov_tol > 0.0 ? P.krylov_tol : 1e-12;
    const int max_restarts = 40;
    VT* V = reinterpret_cast<VT*>(wk_V);
    double b2 = 0.0;
    wall_dots(rhs, 1, rhs, &b2);
    const double beta0 = std::sqrt(b2);
    lincomb(delta, rhs, 0.0, nullptr, 0.0);
    rel = 0.0;
    if (!(beta0 > 0.0)) return 0;
    if (!std::isfinite(beta0)) {
      rel = beta0;
      return 0;
    }
    // device scratch of the cycle: Hd (m x m, row stride m), cs, sn, g,
    // hcol, scale, resid
    double* Hd = wk_small;
    double* cs = Hd + (size_t)m * m;
    double* sn = cs + m;
    double* g = sn + m;
    double* hcol = g + (m + 1);
    double* scale = hcol + (m + 2);
    double* resid = scale + 1;
    lincomb(wk_R, rhs, 1.0, nullptr, 0.0);
    double beta = beta0;
    int iters = 0;
    std::vector<double> y(m);
    const bool reorth = tol < 1e-8;
    if (!reorth) MSC_HIPCK(hipMemsetAsync(hcol, 0, sizeof(double) * (m + 2), st));
    for (int rs = 0; rs < max_restarts; ++rs) {
      hipLaunchKernelGGL(k_scale_to<VT>, dim3(vec_grid()), dim3(256), 0, st, V, wk_vc, (const double*)wk_R,
                         1.0 / beta, n);
      MSC_HIPCK(hipGetLastError());
      for (int i = 0; i <= m; ++i) wk_small_h[i] = (i == 0) ? beta : 0.0;
      MSC_HIPCK(hipMemcpyAsync(g, wk_small_h, sizeof(double) * (m + 1), hipMemcpyHostToDevice, st));
      int jend = 0;
      bool done = false;
      for (int j = 0; j < m; ++j) {
        VT* vj1 = V + (int64_t)(j + 1) * n;
        // w = (I - L) M^{-1} v_j, from the FP64 copy of v_j
        wall_precondition(wk_vc, wk_Z);
        wall_apply(wk_Z, wk_W);
        if (reorth) {
          hipLaunchKernelGGL(k_dots<VT>, dim3(kDotBlocks), dim3(256), 0, st, (const VT*)V, n, j + 1,
                             (const double*)wk_W, n, wk_part, 0);
          hipLaunchKernelGGL(k_gs_first<0>, dim3(1), dim3(1024), 0, st, (const double*)wk_part, j + 1, wk_coef,
                             hcol);
          hipLaunchKernelGGL(k_axpy_multi<VT>, dim3(vec_grid()), dim3(256), 0, st, wk_W, (const VT*)V, n, j + 1,
                             (const double*)wk_coef, n);
        }
        hipLaunchKernelGGL(k_dots<VT>, dim3(kDotBlocks), dim3(256), 0, st, (const VT*)V, n, j + 1,
                           (const double*)wk_W, n, wk_part, 1);
        hipLaunchKernelGGL(k_gs_second<0>, dim3(1), dim3(1024), 0, st, (const double*)wk_part, j, m,
                           wk_coef, (const double*)hcol, Hd, cs, sn, g, scale, resid);
        hipLaunchKernelGGL(k_axpy_scale<VT>, dim3(vec_grid()), dim3(256), 0, st, vj1, wk_vc, (const double*)wk_W,
                           (const VT*)V, n, j + 1, (const double*)wk_coef, (const double*)scale, n);
        MSC_HIPCK(hipGetLastError());
        ++iters;
        jend = j + 1;
        if ((j + 1) % kCheck == 0 || j == m - 1) {
          MSC_HIPCK(hipMemcpyAsync(wk_small_h, resid + j, sizeof(double), hipMemcpyDeviceToHost, st));
          sync();
          const double res = wk_small_h[0];
          if (res <= tol * beta0 || !std::isfinite(res)) {
            done = true;
            break;
          }
        }
      }
      // y = R^{-1} g (upper triangular, jend x jend), delta += M^{-1} V y;
      // the columns after the first converged or broken-down one are unused
      const size_t hsz = (size_t)m * m + 2 * m + (m + 1) + (m + 2) + 1 + m;
      MSC_HIPCK(hipMemcpyAsync(wk_small_h, Hd, sizeof(double) * hsz, hipMemcpyDeviceToHost, st));
      sync();
      const double* Hh = wk_small_h;
      const double* gh = wk_small_h + (size_t)m * m + 2 * m;
      const double* rh = gh + (m + 1) + (m + 2) + 1;
      for (int i = 0; i < jend; ++i) {
        if (!(std::fabs(Hh[(size_t)i * m + i]) > 0.0)) {
          jend = i;
          break;
        }
        if (rh[i] <= tol * beta0) {
          jend = i + 1;
          break;
        }
      }
      for (int i = jend - 1; i >= 0; --i) {
        double acc = gh[i];
        for (int k = i + 1; k < jend; ++k) acc -= Hh[(size_t)i * m + k] * y[k];
        y[i] = acc / Hh[(size_t)i * m + i];
      }
      upload_coef(y.data(), jend);
      hipLaunchKernelGGL(k_combine<VT>, dim3(vec_grid()), dim3(256), 0, st, wk_Y, (const VT*)V, n, jend,
                         (const double*)wk_coef, n);
      MSC_HIPCK(hipGetLastError());
      wall_precondition(wk_Y, wk_Z);
      lincomb(delta, delta, 1.0, wk_Z, 1.0);
      // true residual
      wall_apply(delta, wk_Y);
      lincomb(wk_R, rhs, 1.0, wk_Y, -1.0);
      double r2 = 0.0;
      wall_dots(wk_R, 1, wk_R, &r2);
      beta = std::sqrt(r2);
      rel = beta / beta0;
      if (done || rel <= tol || !(beta > 0.0)) break;
    }
    kr_solves += 1;
    kr_iters += iters;
    kr_worst = std::max(kr_worst, rel);
    return iters;
  }

  // f_T <- f_T + (delta - r) = f + delta, f the sweep's input
  void wall_update(double* fT, const double* delta, const double* r) {
    lincomb(wk_Y, delta, 1.0, r, -1.0);
    lincomb(fT, fT, 1.0, wk_Y, 1.0);
  }

  // Algorithm 2 driven from the host: each inner iteration is the sweep (with
  // the wall rows) and the device-side acceptance decision, then, when the
  // step goes on, the residual guard (adaptive branch) and the correction.
  msc_status bdf2_step_walls(int32_t nsteps, msc_step_stats* out) {
    return guard([&]() -> msc_status {
      if constexpr (std::is_same<T, double>::value) {
        if (nsteps <= 0) return MSC_OK;
        ensure_stats(nsteps);
        const int stat_base = n_next;
        const bool use_sched = sched_pos < (int64_t)sched_h.size();
        if (use_sched) {
          std::vector<int32_t> K(nsteps, 0);
          for (int i = 0; i < nsteps; ++i) {
            const int64_t j = sched_pos + i;
            K[i] = (j < (int64_t)sched_h.size()) ? sched_h[j] : P.k_max;
          }
          ensure_sched(nsteps);
          MSC_HIPCK(hipMemcpyAsync(sched_d, K.data(), sizeof(int32_t) * nsteps, hipMemcpyHostToDevice, st));
        }
        wall_refreshes.assign(nsteps, 0);
        const int64_t NS = G.NS;
        double Rdev = 0.0;
        for (int i = 0; i < nsteps; ++i) {
          const int n = n_next;
          const int64_t bc = bdf_count;
          const int q = (bc == 0) ? 1 : 2;
          const int max_order = (P.extrap_states == 0) ? 2 : P.extrap_states - 1;
          const int order = (int)std::min<int64_t>(bc, max_order);
          const double a = (q == 1) ? 1.0 / P.dt : 3.0 / (2.0 * P.dt);
          int n_grow = 0, n_ref = 0;
          double Rref = 0.0, Rprev = 0.0;
          for (int ell = 1; ell <= P.k_max; ++ell) {
            enqueue_iteration(n, ell, q, order, a, use_sched, stat_base, true);
            MSC_HIPCK(hipMemcpyAsync(ctl_h, ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, st));
            MSC_HIPCK(hipMemcpyAsync(&Rdev, Rhist + (ell - 1), sizeof(double), hipMemcpyDeviceToHost, st));
            sync();
            const uint32_t ps = phase_state(ctl_h->phase);
            if (ps == PH_ACCEPTED) {
              bdf_count += 1;
              n_next = n + 1;
              last_iters = ell;
              break;
            }
            if (ps == PH_FAILED) {
              const msc_status rc = (ctl_h->fail_code == 5) ? MSC_ERR_NONCONVERGED : MSC_ERR_NONFINITE;
              last_error = std::string(rc == MSC_ERR_NONCONVERGED ? "nonconvergent" : "non-finite residual") +
                           " at physical step " + std::to_string(n) + ", inner iteration " + std::to_string(ell);
              ctl_h->phase = make_phase(n - 1, 0, PH_ACCEPTED);
              ctl_h->fail_code = 0;
              MSC_HIPCK(hipMemcpyAsync(ctl, ctl_h, sizeof(DevCtl), hipMemcpyHostToDevice, st));
              copy_stats(out, stat_base, n - stat_base + 1);
              if (use_sched) sched_pos += (n - stat_base);
              sync();
              return rc;
            }
            // Algorithm 2: residual guard of the adaptive operator
            const double R = Rdev;
            if (ell == 1) Rref = R;
            n_grow = (ell > 1 && R > Rprev) ? n_grow + 1 : 0;
            Rprev = R;
            T* fT = fb.p[ctl_h->roles[n & 1].slot_w[ell & 1]];
            if (P.wall_operator == MSC_WALL_ADAPTIVE && n_ref < 3 &&
                (n_grow >= 2 || R > 10.0 * Rref || (P.wall_forced > 0 && ell % P.wall_forced == 0))) {
              hipLaunchKernelGGL(k_wall_reference<0>, dim3(ew_grid()), dim3(256), 0, st, (const double*)fT,
                                 (const double*)rfs, (const double*)h, a, NS, wk_mref, wk_sref);
              MSC_HIPCK(hipGetLastError());
              wk_aA = a;
              wk_rest = false;
              ++n_ref;
              ++kr_refresh;
              wall_refreshes[i] = n_ref;
              n_grow = 0;
              Rref = R;
            }
            double rel = 0.0;
            wall_gmres(rfs, wk_D, rel);
            wall_update(fT, wk_D, rfs);
          }
        }
        copy_stats(out, stat_base, nsteps);
        if (use_sched) sched_pos += nsteps;
        return MSC_OK;
      } else {
        (void)nsteps, (void)out;
        return MSC_ERR_UNSUPPORTED;
      }
    });
  }

  // One wall-corrected iteration from host arrays with the current operator.
  msc_status correct_walls(const double* f, const double* h_in, double a, double* fnext, double* dm_out,
                           double* R) {
    return guard([&]() -> msc_status {
      if constexpr (std::is_same<T, double>::value) {
        pull_ctl();
        T* A = fb.p[cur_roles().slot_w[0]];
        T* B = fb.p[cur_roles().slot_w[1]];
        upload_pop(f, A);
        upload_h(h_in);
        SweepArgs<T, TM> S = sweep_args(a);
        S.src = A;
        S.dst = B;
        S.rout = rfs;
        launch_sweep_timed(SW_DTS, S, 0);
        const double Rv = reduce_partials(S);
        if (R) *R = Rv;
        double rel = 0.0;
        wall_gmres(rfs, wk_D, rel);
        wall_update(B, wk_D, rfs);
        if (fnext) download_pop(B, fnext);
        sync();
        if (dm_out) std::memset(dm_out, 0, sizeof(double) * (D + 1) * G.NS);
        return MSC_OK;
      } else {
        (void)f, (void)h_in, (void)a, (void)fnext, (void)dm_out, (void)R;
        return MSC_ERR_UNSUPPORTED;
      }
    });
  }

  msc_status set_schedule(const int32_t* K, int32_t nsteps) override {
    sched_h.clear();
    sched_pos = 0;
    if (K && nsteps > 0) {
      for (int i = 0; i < nsteps; ++i) {
        if (K[i] < 1) {
          last_error = "schedule entries must be >= 1";
          sched_h.clear();
          return MSC_ERR_INVALID_ARG;
        }
        sched_h.push_back(std::min(K[i], P.k_max));
      }
    }
    return MSC_OK;
  }

  int64_t state_size() const override {
    return 3 * (int64_t)Q * G.NS + 2 * (int64_t)(D + 1) * G.NS;
  }

  msc_status get_state(double* state, int64_t* bc) override {
    return guard([&]() {
      pull_ctl();
      const int64_t FQ = (int64_t)Q * G.NS, FM = (int64_t)(D + 1) * G.NS;
      for (int i = 0; i < 3; ++i) download_pop(fb.p[cur_roles().slot_hist[i]], state + i * FQ);
      MSC_HIPCK(hipMemcpyAsync(state + 3 * FQ, mb[cur_roles().slot_m[0]], sizeof(double) * FM,
                               hipMemcpyDeviceToHost, st));
      MSC_HIPCK(hipMemcpyAsync(state + 3 * FQ + FM, mb[cur_roles().slot_m[1]], sizeof(double) * FM,
                               hipMemcpyDeviceToHost, st));
      sync();
      if (bc) *bc = bdf_count;
      return MSC_OK;
    });
  }

  msc_status set_state(const double* state, int64_t bc) override {
    return guard([&]() {
      pull_ctl();
      const int64_t FQ = (int64_t)Q * G.NS, FM = (int64_t)(D + 1) * G.NS;
      if (DV) sig = sigma_for({state, state + FQ, state + 2 * FQ});
      for (int i = 0; i < 3; ++i) upload_pop(state + i * FQ, fb.p[cur_roles().slot_hist[i]]);
      MSC_HIPCK(hipMemcpyAsync(mb[cur_roles().slot_m[0]], state + 3 * FQ, sizeof(double) * FM,
                               hipMemcpyHostToDevice, st));
      MSC_HIPCK(hipMemcpyAsync(mb[cur_roles().slot_m[1]], state + 3 * FQ + FM, sizeof(double) * FM,
                               hipMemcpyHostToDevice, st));
      sync();
      bdf_count = bc;
      return MSC_OK;
    });
  }

  // ------------------------------------------------------------- adjoint --
  msc_status set_recording(int enable) override {
    return guard([&]() {
      sync();
      clear_records();
      recording = enable != 0;
      if (!recording) free_adjoint_buffers();
      return MSC_OK;
    });
  }

  int32_t recorded_steps() const override { return (int32_t)records.size(); }

  msc_status bdf2_adjoint(int32_t nsteps, double* lam, bool on_device) override {
    return guard([&]() -> msc_status {
      if (nsteps < 1 || nsteps > (int32_t)records.size()) {
        last_error = "nsteps must be between 1 and the number of recorded steps (" +
                     std::to_string(records.size()) + ")";
        return MSC_ERR_INVALID_ARG;
      }
      if (P.corrector == MSC_CORRECTOR_SHADOW && !fft_fits(sizeof(cpx<double>))) {
        last_error = "the FP64 transforms of the adjoint correction do not fit this grid size";
        return MSC_ERR_UNSUPPORTED;
      }
      if (fullsym() || wallkin() || walls()) {
        last_error = "the adjoint covers the periodic Picard and shadow marches only";
        return MSC_ERR_UNSUPPORTED;
      }
      int kmax = 1;
      for (int r = 0; r < nsteps; ++r) kmax = std::max(kmax, records[records.size() - 1 - r].K);
      ensure_adjoint_buffers(kmax);
      const int64_t SZ = state_size();
      double* cur = adj_lam[0];
      double* nxt = adj_lam[1];
      MSC_HIPCK(hipMemcpyAsync(cur, lam, sizeof(double) * SZ,
                               on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
      for (int r = 0; r < nsteps; ++r) {
        backward_step(records[records.size() - 1 - r], cur, nxt);
        std::swap(cur, nxt);
      }
      MSC_HIPCK(hipMemcpyAsync(lam, cur, sizeof(double) * SZ,
                               on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
      sync();
      for (int r = 0; r < nsteps; ++r) drop_last_record();
      return MSC_OK;
    });
  }

  msc_status init_adjoint(const double* phat0, const double* u0, const double* lam, double* lam_phat0,
                          double* lam_u0, bool on_device) override {
    return guard([&]() -> msc_status {
      const int64_t NS = G.NS, SZ = state_size();
      const double *pd = phat0, *ud = u0, *ld = lam;
      double *lp = lam_phat0, *lu = lam_u0;
      double* tmp = nullptr;
      if (!on_device) {
        tmp = (double*)dalloc(sizeof(double) * (SZ + 2 * (D + 1) * NS));
        double* t = tmp;
        MSC_HIPCK(hipMemcpyAsync(t, phat0, sizeof(double) * NS, hipMemcpyHostToDevice, st));
        MSC_HIPCK(hipMemcpyAsync(t + NS, u0, sizeof(double) * D * NS, hipMemcpyHostToDevice, st));
        MSC_HIPCK(hipMemcpyAsync(t + (D + 1) * NS, lam, sizeof(double) * SZ, hipMemcpyHostToDevice, st));
        pd = t;
        ud = t + NS;
        ld = t + (D + 1) * NS;
        lp = t + (D + 1) * NS + SZ;
        lu = lp + NS;
      }
      hipLaunchKernelGGL((k_adj_init<L>), dim3(ew_grid()), dim3(256), 0, st, NS, pd, ud, ld, lp, lu);
      MSC_HIPCK(hipGetLastError());
      if (!on_device) {
        MSC_HIPCK(hipMemcpyAsync(lam_phat0, lp, sizeof(double) * NS, hipMemcpyDeviceToHost, st));
        MSC_HIPCK(hipMemcpyAsync(lam_u0, lu, sizeof(double) * D * NS, hipMemcpyDeviceToHost, st));
      }
      sync();
      if (tmp) dfree(tmp);
      return MSC_OK;
    });
  }

  msc_status set_kernel_timing(int enable) override {
    return guard([&]() {
      sync();
      collect_timing();
      timing = enable != 0;
      for (int k = 0; k < 2; ++k) {
        t_sum[k] = 0.0;
        t_count[k] = 0;
        t_bytes[k] = 0.0;
      }
      return MSC_OK;
    });
  }

  msc_status kernel_time(int kind, double* seconds, int64_t* launches, double* bytes) override {
    return guard([&]() -> msc_status {
      if (kind < 0 || kind > 1) return MSC_ERR_INVALID_ARG;
      sync();
      collect_timing();
      if (seconds) *seconds = t_sum[kind];
      if (launches) *launches = t_count[kind];
      if (bytes) *bytes = t_count[kind] ? t_bytes[kind] / (double)t_count[kind] : sweep_bytes(kind == 1 ? SW_EXPLICIT : SW_DTS_LIFT);
      return MSC_OK;
    });
  }

 private:
  msc_params P;
  Geometry G;
  hipStream_t st;
  Tuning tune;
  double wp, wm, nu;

  FBufs<T> fb{};
  double* mb[3] = {nullptr, nullptr, nullptr};
  double* h = nullptr;
  // history term of odd physical steps (even steps use h): a setup sweep that
  // forms m^n from the previous step's h writes its own step's h meanwhile
  double* h_alt = nullptr;
  TM* Pr = nullptr;
  TM* dm = nullptr;
  cpx<CT>* spec = nullptr;
  cpx<CT>* spec2 = nullptr;
  cpx<CT>* spec_alt = nullptr;  // 2D: second band spectrum (inverse rows in the sweep)
  TM* rfs = nullptr;           // full symbol / wall corrector: residual of every field (Q x NS)
  // wall-bounded kinetic corrector (Algorithm 2): Krylov basis and work
  // vectors (FP64, Q x NS each), the reference field of the current operator
  // and the assembly coefficient a_A, dot-product partials and coefficients
  double* wk_V = nullptr;
  double* wk_R = nullptr;
  double* wk_Y = nullptr;
  double* wk_Z = nullptr;
  double* wk_D = nullptr;
  double* wk_W = nullptr;   // the new Krylov vector before its orthogonalisation
  double* wk_vc = nullptr;  // FP64 copy of the newest basis vector (preconditioner input)
  double* wk_mu = nullptr;
  double* wk_mref = nullptr;
  double* wk_sref = nullptr;
  double* wk_part = nullptr;
  double* wk_part_h = nullptr;
  double* wk_coef = nullptr;
  double* wk_coef_h = nullptr;
  double* wk_small = nullptr;    // GMRES cycle bookkeeping on the device
  double* wk_small_h = nullptr;  // its pinned host mirror
  int wk_m = 50;
  double wk_aA = 0.0;
  bool wk_rest = true;
  int64_t kr_solves = 0, kr_iters = 0, kr_refresh = 0;
  double kr_worst = 0.0;
  std::vector<int32_t> wall_refreshes;
  cpx<CT>* spec_fs = nullptr;  // full symbol: half spectrum (Q x N_x x (N_y/2 + 1))
  double* partials = nullptr;
  double* partials_h = nullptr;
  double* presum = nullptr;                   // folded partials for large sweep grids
  static constexpr int kFusedParts = 4096;    // decision kernels sum at most this many partials
  int nparts_cap = 0;
  DevCtl* ctl = nullptr;
  DevCtl* ctl_h = nullptr;
  double* Rhist = nullptr;
  StepStat* stats_d = nullptr;
  StepStat* stats_h = nullptr;
  int stats_cap = 0;
  int32_t* sched_d = nullptr;
  int sched_cap = 0;
  std::vector<int32_t> sched_h, sched_host_view;
  int64_t sched_pos = 0;
  cpx<CT>* tw[3] = {nullptr, nullptr, nullptr};
  double* stage = nullptr;
  std::vector<void*> allocs;

  int n_next = 0;
  int64_t bdf_count = 0;
  int last_iters = 4;
  float sig = 1.0f;  // scale of FP16 deviation storage (unused otherwise)

  // explicit-march graph cache
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  // key of the captured explicit-march graph: the sweep arguments it holds by
  // value (buffers, chunk length and the deviation-storage scale)
  const T* g_a = nullptr;
  const T* g_b = nullptr;
  int g_chunk = 0;
  float g_sig = 0.0f;
  bool g_aa = false;

  // kernel timing
  bool timing = false;
  struct EvPair {
    hipEvent_t a, b;
    int kind;
    int flag;
    double bytes;
  };
  int* run_flags = nullptr;  // device, one per timed launch since the last collection
  int32_t* run_flags_h = nullptr;
  static constexpr int kFlagCap = 4096;
  double t_bytes[2] = {0, 0};
  std::vector<EvPair> ev_live;
  std::vector<hipEvent_t> ev_free;
  double t_sum[2] = {0, 0};
  int64_t t_count[2] = {0, 0};

  // adjoint records and buffers
  struct Record {
    void* mem;   // f^n, f^{n-1}, f^{n-2} (storage format), then m^n, m^{n-1} (FP64)
    int64_t bc;  // BDF steps accepted before this step
    int K;       // inner sweeps at acceptance; 0 while the step is in flight
    float sig;   // deviation-storage scale of the checkpointed populations
  };
  bool recording = false;
  std::vector<Record> records;
  std::vector<void*> adj_allocs;
  double* adj_lam[2] = {nullptr, nullptr};  // state-layout adjoints (in, out)
  double* adj_LT = nullptr;
  double* adj_LF = nullptr;
  double* adj_carry = nullptr;
  double* adj_lh = nullptr;
  double* adj_h = nullptr;
  double* adj_fT = nullptr;
  double* adj_it = nullptr;  // FP64 inner iterates f^(1..K) of the step being reversed
  int adj_it_cap = 0;
  // FP64 transform buffers: P r of a recomputed sweep, or y = E^T Lambda, in
  // adj_y; dm, or z = Sh^T y, out in adj_z
  double* adj_y = nullptr;
  double* adj_z = nullptr;
  XformBufs<double, double> adj_x{};

  // ------------------------------------------------------------- helpers --
  template <class F>
  msc_status guard(F&& fn) {
    if (broken) return MSC_ERR_STATE;
    try {
      return fn();
    } catch (const DeviceError& e) {
      broken = true;
      last_error = e.what;
      return MSC_ERR_DEVICE;
    } catch (const OomError&) {
      last_error = "device allocation failed";
      return MSC_ERR_OUT_OF_MEMORY;
    }
  }

  void sync() { MSC_HIPCK(hipStreamSynchronize(st)); }

  void* dalloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 1;
    if (P.alloc_fn) {
      p = P.alloc_fn(bytes, P.alloc_user);
      if (!p) throw OomError{};
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e == hipErrorOutOfMemory) throw OomError{};
      if (e != hipSuccess) throw DeviceError{e, std::string("hipMalloc: ") + hipGetErrorString(e)};
    }
    return p;
  }
  void dfree(void* p) {
    if (!p) return;
    if (P.alloc_fn) {
      if (P.free_fn) P.free_fn(p, P.alloc_user);
    } else {
      (void)hipFree(p);
    }
  }
  template <class X>
  X* keep(X* p) {
    allocs.push_back((void*)p);
    return p;
  }

  int ew_grid() const {
    const int64_t b = (G.NS + 255) / 256;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 4096);
  }

  bool corrector_supported() const { return fft_fits(); }

  bool fullsym() const { return P.corrector == MSC_CORRECTOR_FULL_SYMBOL; }
  // Shadow corrector with FP64 or FP32 populations, 3D or 2D with the row
  // transforms as passes of their own: the lift sweep enqueued as the last of
  // its step leaves P r out (the step is predicted to accept there);
  // k_recompute_pr forms it if the step goes on
  bool skip_pr_ok() const {
    return tune.skip_pr != 0 && P.corrector == MSC_CORRECTOR_SHADOW && !PopDev<T>::value &&
           (D == 3 || !fuse_rows);
  }
  bool wallkin() const { return P.corrector == MSC_CORRECTOR_WALL_KINETIC; }
  bool walls() const { return P.boundary == MSC_BOUNDARY_CAVITY; }
  bool wall_supported() const {
    return D == 2 && std::is_same<T, double>::value && walls() && P.tau_plus == 1.0 && P.tau_minus == 1.0 &&
           fs_supported();
  }
  // the full-symbol passes at their minimum block shape: one row of
  // (Q+1)/2 packed lines, one column of Q lines, each with its LDS ping-pong
  bool fs_supported(size_t c = sizeof(cpx<CT>)) const {
    if (D != 2 || DV) return false;
    return (size_t)2 * ((Q + 1) / 2) * G.N2 * c <= 131072 && (size_t)2 * Q * G.N0 * c <= 131072;
  }

  // LDS of the transform passes at their minimum block shape
  bool fft_fits(size_t c = sizeof(cpx<CT>)) const {
    if (D == 2) return (size_t)4 * G.N2 * c <= 131072 && (size_t)6 * G.N0 * c <= 131072;
    const int Nmax = std::max(G.n[0], std::max(G.n[1], G.n[2]));
    return (size_t)4 * G.n[2] * c <= 131072 && (size_t)8 * Nmax * c <= 131072;
  }

  void allocate() {
    const int64_t NS = G.NS;
    const size_t fbytes = pop_bytes();
    for (int i = 0; i < 5; ++i) fb.p[i] = keep((T*)dalloc(fbytes));
    for (int i = 0; i < 3; ++i) mb[i] = keep((double*)dalloc(sizeof(double) * (D + 1) * NS));
    h = keep((double*)dalloc(sizeof(double) * (D + 1) * NS));
    h_alt = keep((double*)dalloc(sizeof(double) * (D + 1) * NS));
    Pr = keep((TM*)dalloc(sizeof(TM) * (D + 1) * NS));
    dm = keep((TM*)dalloc(sizeof(TM) * (D + 1) * NS));
    MSC_HIPCK(hipMemsetAsync(h, 0, sizeof(double) * (D + 1) * NS, st));
    MSC_HIPCK(hipMemsetAsync(h_alt, 0, sizeof(double) * (D + 1) * NS, st));
    MSC_HIPCK(hipMemsetAsync(dm, 0, sizeof(TM) * (D + 1) * NS, st));
    ctl = keep((DevCtl*)dalloc(sizeof(DevCtl)));
    MSC_HIPCK(hipHostMalloc((void**)&ctl_h, sizeof(DevCtl), hipHostMallocDefault));
    Rhist = keep((double*)dalloc(sizeof(double) * std::max(P.k_max, 1)));
    presum = keep((double*)dalloc(sizeof(double)));
    choose_sweep();
    ensure_partials(sweep_grid_max());
    if (corrector_supported()) {
      if (D == 2) {
        const int NB = G.N2 / 4 + 1;
        spec = keep((cpx<CT>*)dalloc(sizeof(cpx<CT>) * 3 * (int64_t)G.N0 * NB));
        spec_alt = keep((cpx<CT>*)dalloc(sizeof(cpx<CT>) * 3 * (int64_t)G.N0 * NB));
        tw[0] = make_twiddles(G.N0);
        tw[2] = make_twiddles(G.N2);
      } else {
        const int NBz = G.n[2] / 4 + 1, NBy = 2 * (G.n[1] / 4) + 1;
        spec = keep((cpx<CT>*)dalloc(sizeof(cpx<CT>) * 4 * (int64_t)G.n[0] * G.n[1] * NBz));
        spec2 = keep((cpx<CT>*)dalloc(sizeof(cpx<CT>) * 4 * (int64_t)G.n[0] * NBy * NBz));
        for (int a = 0; a < 3; ++a) tw[a] = make_twiddles(G.n[a]);
      }
      set_fft_attrs();
    }
    if (wallkin() && wall_supported()) wall_allocate();
    if ((fullsym() || wallkin()) && fs_supported()) {
      rfs = keep((TM*)dalloc(sizeof(TM) * (int64_t)Q * NS));
      spec_fs = keep((cpx<CT>*)dalloc(sizeof(cpx<CT>) * (int64_t)Q * G.N0 * (G.N2 / 2 + 1)));
      if (!tw[0]) tw[0] = make_twiddles(G.N0);
      if (!tw[2]) tw[2] = make_twiddles(G.N2);
      set_fs_attrs();
    }
  }

  void release() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    for (auto& e : ev_live) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    for (auto& e : ev_free) (void)hipEventDestroy(e);
    ev_live.clear();
    ev_free.clear();
    if (st) (void)hipStreamSynchronize(st);
    for (auto& r : records) dfree(r.mem);
    records.clear();
    for (void* p : adj_allocs) dfree(p);
    adj_allocs.clear();
    for (void* p : allocs) dfree(p);
    allocs.clear();
    if (ctl_h) (void)hipHostFree(ctl_h);
    if (stats_h) (void)hipHostFree(stats_h);
    if (partials_h) (void)hipHostFree(partials_h);
    if (run_flags_h) (void)hipHostFree(run_flags_h);
    run_flags_h = nullptr;
    if (wk_part_h) (void)hipHostFree(wk_part_h);
    if (wk_coef_h) (void)hipHostFree(wk_coef_h);
    if (wk_small_h) (void)hipHostFree(wk_small_h);
    wk_part_h = nullptr;
    wk_coef_h = nullptr;
    wk_small_h = nullptr;
    ctl_h = nullptr;
    stats_h = nullptr;
    partials_h = nullptr;
  }

  template <class CX = CT>
  cpx<CX>* make_twiddles(int N, std::vector<void*>* owner = nullptr) {
    std::vector<cpx<CX>> t(N);
    const double two_pi = 6.283185307179586476925286766559;
    for (int i = 0; i < N; ++i) {
      const double ang = -two_pi * (double)i / (double)N;
      t[i] = {(CX)std::cos(ang), (CX)std::sin(ang)};
    }
    cpx<CX>* d = (cpx<CX>*)dalloc(sizeof(cpx<CX>) * N);
    (owner ? owner : &allocs)->push_back((void*)d);
    MSC_HIPCK(hipMemcpyAsync(d, t.data(), sizeof(cpx<CX>) * N, hipMemcpyHostToDevice, st));
    sync();  // t goes out of scope
    return d;
  }

  double* staging() {
    if (!stage) stage = keep((double*)dalloc(sizeof(double) * std::max<int64_t>(Q, 2 * (D + 1)) * G.NS));
    return stage;
  }

  void ensure_partials(int n) {
    if (n <= nparts_cap) return;
    partials = keep((double*)dalloc(sizeof(double) * n));
    if (partials_h) (void)hipHostFree(partials_h);
    MSC_HIPCK(hipHostMalloc((void**)&partials_h, sizeof(double) * n, hipHostMallocDefault));
    nparts_cap = n;
  }

  void ensure_stats(int n) {
    if (n <= stats_cap) return;
    stats_d = keep((StepStat*)dalloc(sizeof(StepStat) * n));
    if (stats_h) (void)hipHostFree(stats_h);
    MSC_HIPCK(hipHostMalloc((void**)&stats_h, sizeof(StepStat) * n, hipHostMallocDefault));
    stats_cap = n;
  }

  void ensure_sched(int n) {
    if (n <= sched_cap) return;
    sched_d = keep((int32_t*)dalloc(sizeof(int32_t) * n));
    sched_cap = n;
  }

  void copy_stats(msc_step_stats* out, int base, int count) {
    (void)base;
    if (!out || count <= 0) return;
    MSC_HIPCK(hipMemcpyAsync(stats_h, stats_d, sizeof(StepStat) * count, hipMemcpyDeviceToHost, st));
    sync();
    for (int i = 0; i < count; ++i) {
      out[i].q = stats_h[i].q;
      out[i].iters = stats_h[i].iters;
      out[i].R_first = stats_h[i].R_first;
      out[i].R_final = stats_h[i].R_final;
      out[i].rho_obs = stats_h[i].rho_obs;
      out[i].converged = stats_h[i].converged;
      out[i].refreshes = (i < (int)wall_refreshes.size()) ? wall_refreshes[i] : 0;
    }
  }

  // Buffer roles of the next step to run (host copy; pull_ctl first).
  Roles& cur_roles() { return ctl_h->roles[n_next & 1]; }

  void pull_ctl() {
    MSC_HIPCK(hipMemcpyAsync(ctl_h, ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, st));
    sync();
  }

  // m^n = P f^n, m^{n-1} = m^n, f^{n-1} = f^{n-2} = f^n, BDF history reset
  // (next step BDF1, whose trial uses f^n alone).
  void reset_history_from_current() {
    for (int i = 1; i < 3; ++i)
      MSC_HIPCK(hipMemcpyAsync(fb.p[cur_roles().slot_hist[i]], fb.p[cur_roles().slot_hist[0]], pop_bytes(),
                               hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL((k_moments<L, T>), dim3(ew_grid()), dim3(256), 0, st, fb.p[cur_roles().slot_hist[0]],
                       mb[cur_roles().slot_m[0]], G.NS);
    MSC_HIPCK(hipGetLastError());
    MSC_HIPCK(hipMemcpyAsync(mb[cur_roles().slot_m[1]], mb[cur_roles().slot_m[0]], sizeof(double) * (D + 1) * G.NS,
                             hipMemcpyDeviceToDevice, st));
    bdf_count = 0;
  }

  // bytes of one population buffer: Q N_sites values, plus the FP32 moments
  // of deviation storage
  size_t pop_bytes() const {
    return sizeof(T) * (size_t)Q * G.NS + (DV ? sizeof(float) * (size_t)(D + 1) * G.NS : 0);
  }

  void upload_pop(const double* f, T* dst) {
    double* stg = staging();
    const int64_t n = (int64_t)Q * G.NS;
    MSC_HIPCK(hipMemcpyAsync(stg, f, sizeof(double) * n, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL((k_pop_from_f64<L, T>), dim3(ew_grid()), dim3(256), 0, st, (const double*)stg, dst, G.NS,
                       1.0f / sig);
    MSC_HIPCK(hipGetLastError());
  }
  void download_pop(const T* src, double* f) {
    double* stg = staging();
    const int64_t n = (int64_t)Q * G.NS;
    hipLaunchKernelGGL((k_pop_to_f64<L, T>), dim3(ew_grid()), dim3(256), 0, st, src, stg, G.NS, sig);
    MSC_HIPCK(hipGetLastError());
    MSC_HIPCK(hipMemcpyAsync(f, stg, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    sync();
  }
  void download_tm(const TM* src, double* out, int64_t n) {
    double* stg = staging();
    hipLaunchKernelGGL((k_convert<TM, double>), dim3(ew_grid()), dim3(256), 0, st, src, stg, n);
    MSC_HIPCK(hipGetLastError());
    MSC_HIPCK(hipMemcpyAsync(out, stg, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    sync();
  }
  void upload_h(const double* h_in) {
    const int64_t n = (int64_t)(D + 1) * G.NS;
    if (h_in)
      MSC_HIPCK(hipMemcpyAsync(h, h_in, sizeof(double) * n, hipMemcpyHostToDevice, st));
    else
      MSC_HIPCK(hipMemsetAsync(h, 0, sizeof(double) * n, st));
  }

  // Scale of deviation storage: a power of two with |g| <= 2^12 for the
  // given populations (max deviation from equilibrium) and <= 2^10 times the
  // deviation over the largest moment (headroom for the march: a post-stream
  // deviation is a difference of neighbouring equilibria, a few times the
  // largest moment at most); FP16 overflows at 65504.
  static float choose_sigma(double maxdev, double maxm) {
    const double want = std::max(std::max(maxdev * 0x1p-12, maxm * 0x1p-10), 0x1p-100);
    return (float)std::exp2(std::ceil(std::log2(want)));
  }

  // Scale for populations uploaded from host FP64 arrays.
  float sigma_for(std::initializer_list<const double*> fs) {
    double md = 0.0, mm = 0.0;
    double* stg = staging();
    const int grid = 512;
    ensure_partials(2 * grid);
    for (const double* f : fs) {
      MSC_HIPCK(hipMemcpyAsync(stg, f, sizeof(double) * Q * G.NS, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL((k_pop_maxdev<L>), dim3(grid), dim3(256), 0, st, (const double*)stg, G.NS, partials);
      MSC_HIPCK(hipGetLastError());
      MSC_HIPCK(hipMemcpyAsync(partials_h, partials, sizeof(double) * 2 * grid, hipMemcpyDeviceToHost, st));
      sync();
      for (int i = 0; i < grid; ++i) {
        md = std::max(md, partials_h[2 * i]);
        mm = std::max(mm, partials_h[2 * i + 1]);
      }
    }
    return choose_sigma(md, mm);
  }

  double absmax(const double* v, int64_t n) {
    const int grid = 512;
    ensure_partials(grid);
    hipLaunchKernelGGL(k_absmax<0>, dim3(grid), dim3(256), 0, st, v, n, partials);
    MSC_HIPCK(hipGetLastError());
    MSC_HIPCK(hipMemcpyAsync(partials_h, partials, sizeof(double) * grid, hipMemcpyDeviceToHost, st));
    sync();
    double m = 0.0;
    for (int i = 0; i < grid; ++i) m = std::max(m, partials_h[i]);
    return m;
  }

  double pop_sumsq(const T* p) {
    double s = sumsq(p, (int64_t)Q * G.NS);
    if (DV) s += sumsq(dev_moments(p, Q, G.NS), (int64_t)(D + 1) * G.NS);
    return s;
  }

  template <class X>
  double sumsq(const X* v, int64_t n) {
    const int grid = 1024;
    ensure_partials(grid);
    hipLaunchKernelGGL((k_sumsq<X>), dim3(grid), dim3(256), 0, st, v, n, partials);
    MSC_HIPCK(hipGetLastError());
    MSC_HIPCK(hipMemcpyAsync(partials_h, partials, sizeof(double) * grid, hipMemcpyDeviceToHost, st));
    sync();
    double s = 0.0;
    for (int i = 0; i < grid; ++i) s += partials_h[i];
    return s;
  }

  double reduce_partials(const SweepArgs<T, TM>& S) {
    const int nb = sweep_grid();
    MSC_HIPCK(hipMemcpyAsync(partials_h, S.partials, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    sync();
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += partials_h[i];
    return std::sqrt(s / ((double)Q * (double)G.NS));
  }

  // ------------------------------------------------------ adjoint pieces --
  size_t record_bytes() const { return 3 * pop_bytes() + 2 * sizeof(double) * (size_t)(D + 1) * G.NS; }

  // Enqueue a copy of the state at the start of step n (ctl_h must be current).
  void take_checkpoint(int n, int64_t bc) {
    const Roles& ro = ctl_h->roles[n & 1];
    Record r{};
    r.mem = dalloc(record_bytes());
    r.bc = bc;
    r.K = 0;
    r.sig = sig;
    records.push_back(r);
    const size_t fq = pop_bytes(), fm = sizeof(double) * (size_t)(D + 1) * G.NS;
    char* b = (char*)r.mem;
    for (int i = 0; i < 3; ++i)
      MSC_HIPCK(hipMemcpyAsync(b + i * fq, fb.p[ro.slot_hist[i]], fq, hipMemcpyDeviceToDevice, st));
    for (int i = 0; i < 2; ++i)
      MSC_HIPCK(hipMemcpyAsync(b + 3 * fq + i * fm, mb[ro.slot_m[i]], fm, hipMemcpyDeviceToDevice, st));
  }

  void drop_last_record() {
    sync();
    dfree(records.back().mem);
    records.pop_back();
  }

  void clear_records() {
    for (auto& r : records) dfree(r.mem);
    records.clear();
  }

  void free_adjoint_buffers() {
    for (void* p : adj_allocs) dfree(p);
    adj_allocs.clear();
    adj_lam[0] = adj_lam[1] = nullptr;
    adj_LT = adj_LF = adj_carry = adj_lh = adj_h = nullptr;
    adj_fT = adj_it = nullptr;
    adj_it_cap = 0;
    adj_y = adj_z = nullptr;
    adj_x = XformBufs<double, double>{};
  }

  void ensure_adjoint_buffers(int K) {
    const int64_t NS = G.NS, FQ = (int64_t)Q * NS, FM = (int64_t)(D + 1) * NS;
    auto get = [&](size_t bytes) {
      void* p = dalloc(bytes);
      adj_allocs.push_back(p);
      return p;
    };
    if (!adj_LT) {
      for (int i = 0; i < 2; ++i) adj_lam[i] = (double*)get(sizeof(double) * state_size());
      adj_LT = (double*)get(sizeof(double) * FQ);
      adj_LF = (double*)get(sizeof(double) * FQ);
      adj_carry = (double*)get(sizeof(double) * FQ);
      adj_lh = (double*)get(sizeof(double) * FM);
      adj_h = (double*)get(sizeof(double) * FM);
      adj_fT = (double*)get(sizeof(double) * FQ);
      adj_y = (double*)get(sizeof(double) * FM);
      adj_z = (double*)get(sizeof(double) * FM);
      if (P.corrector == MSC_CORRECTOR_SHADOW) {
        adj_x.in = adj_y;
        adj_x.out = adj_z;
        if constexpr (std::is_same<CT, double>::value) {
          adj_x.spec1 = spec;
          adj_x.spec2 = spec2;
          for (int i = 0; i < 3; ++i) adj_x.tw[i] = tw[i];
        } else {
          using C2 = cpx<double>;
          if (D == 2) {
            adj_x.spec1 = (C2*)get(sizeof(C2) * 3 * (size_t)G.N0 * (G.N2 / 4 + 1));
            adj_x.tw[0] = make_twiddles<double>(G.N0, &adj_allocs);
            adj_x.tw[2] = make_twiddles<double>(G.N2, &adj_allocs);
          } else {
            const int NBz = G.n[2] / 4 + 1, NBy = 2 * (G.n[1] / 4) + 1;
            adj_x.spec1 = (C2*)get(sizeof(C2) * 4 * (size_t)G.n[0] * G.n[1] * NBz);
            adj_x.spec2 = (C2*)get(sizeof(C2) * 4 * (size_t)G.n[0] * NBy * NBz);
            for (int a = 0; a < 3; ++a) adj_x.tw[a] = make_twiddles<double>(G.n[a], &adj_allocs);
          }
          set_fft_attrs<double, double>();
        }
      }
    }
    if (K > adj_it_cap) {
      adj_it = (double*)get(sizeof(double) * FQ * (size_t)K);
      adj_it_cap = K;
    }
  }

  // FP64 dual-time sweep of src into dst (diagnostic mode, no control
  // block) for the recompute of the adjoint: P r into adj_y.
  void sweep64(const double* src, double* dst, double a) {
    SweepArgs<double, double> S{};
    S.N0 = G.N0;
    S.N1 = G.N1;
    S.N2 = G.N2;
    S.L = strip_L;
    const TileCfg tm = tile_of(SW_DTS);
    S.ntile1 = G.N1 / tm.T1;
    S.ntile2 = G.N2 / tm.T2;
    S.nstrip = G.N0 / strip_L;
    S.NS = G.NS;
    S.ctl = nullptr;
    S.src = src;
    S.dst = dst;
    S.h = adj_h;
    S.dm = adj_z;
    S.Pr = adj_y;
    S.partials = partials;
    S.a = a;
    S.inv1pa2 = 1.0 / (1.0 + a / 2.0);
    S.wp = wp;
    S.wm = wm;
    if (D == 2)
      launch_sweep_d2<double, double>(tile_id, SW_DTS, S, sweep_grid(), st);
    else if (wide_mode(SW_DTS))
      launch_sweep_dual_wide<double, double>(SW_DTS, S, sweep_grid(), st);
    else
      launch_sweep_d3<double, double>(tile_id, SW_DTS, S, sweep_grid(), st);
    MSC_HIPCK(hipGetLastError());
  }

  // Reverse one recorded step: recompute its inner iterates from the
  // checkpoint, then run the transposed stages from the last sweep to the
  // first and through the history combination.  lin is the adjoint of the
  // state after the step, lout receives the adjoint of the state before it.
  void backward_step(const Record& R, const double* lin, double* lout) {
    const int64_t NS = G.NS, FQ = (int64_t)Q * NS, FM = (int64_t)(D + 1) * NS;
    const bool shadow = (P.corrector == MSC_CORRECTOR_SHADOW);
    const size_t pb = pop_bytes();
    const T* f0 = (const T*)R.mem;
    const T* f1 = (const T*)((const char*)R.mem + pb);
    const T* f2 = (const T*)((const char*)R.mem + 2 * pb);
    const double* m0 = (const double*)((const char*)R.mem + 3 * pb);
    const double* m1 = m0 + FM;
    const int q = (R.bc == 0) ? 1 : 2;
    const int max_order = (P.extrap_states == 0) ? 2 : P.extrap_states - 1;
    const int order = (int)std::min<int64_t>(R.bc, max_order);
    const double a = (q == 1) ? 1.0 / P.dt : 3.0 / (2.0 * P.dt);
    const int K = R.K;
    auto it = [&](int ell) { return adj_it + (size_t)(ell - 1) * FQ; };
    const int eg = ew_grid();

    // forward recompute of f^(1..K) in FP64
    hipLaunchKernelGGL((k_extrap_h<L, T>), dim3(eg), dim3(256), 0, st, NS, order, q, P.dt, f0, f1, f2, m0, m1,
                       R.sig, it(1), adj_h);
    MSC_HIPCK(hipGetLastError());
    for (int ell = 1; ell < K; ++ell) {
      sweep64(it(ell), shadow ? adj_fT : it(ell + 1), a);
      if (shadow) {
        enqueue_transform<double, double>(nullptr, 0, 0, a, nullptr, false, adj_x);
        hipLaunchKernelGGL((k_lift<L, double, double>), dim3(eg), dim3(256), 0, st, (const double*)adj_fT,
                           (const double*)adj_z, it(ell + 1), NS, 1.0f, 1.0f);
        MSC_HIPCK(hipGetLastError());
      }
    }

    // backward through the inner iterations
    const double* lf0 = lin;
    const double* lf1 = lin + FQ;
    const double* lf2 = lin + 2 * FQ;
    const double* lm0 = lin + 3 * FQ;
    const double* lm1 = lin + 3 * FQ + FM;
    double* LT = adj_LT;
    double* LF = adj_LF;
    hipLaunchKernelGGL((k_adj_seed<L>), dim3(eg), dim3(256), 0, st, NS, lf0, lm0, a, LT, adj_lh);
    MSC_HIPCK(hipGetLastError());
    const AdjGeom ag{G.N0, G.N1, G.N2, NS};
    const double* carry = nullptr;
    for (int ell = K; ell >= 1; --ell) {
      hipLaunchKernelGGL((k_adj_sweep<L, double>), dim3(eg), dim3(256), 0, st, ag, (const double*)it(ell),
                         (const double*)adj_h, (const double*)LT, carry, LF, adj_lh, a, wp, wm);
      MSC_HIPCK(hipGetLastError());
      if (ell == 1) break;
      if (shadow) {
        hipLaunchKernelGGL((k_adj_Et<L, double>), dim3(eg), dim3(256), 0, st, NS, (const double*)LF, adj_y);
        MSC_HIPCK(hipGetLastError());
        enqueue_transform<double, double>(nullptr, 0, 0, a, nullptr, true, adj_x);
        hipLaunchKernelGGL((k_adj_lift<L, double>), dim3(eg), dim3(256), 0, st, NS, (const double*)adj_z,
                           (const double*)LF, LT, adj_carry);
        MSC_HIPCK(hipGetLastError());
        carry = adj_carry;
      } else {
        std::swap(LT, LF);
        carry = nullptr;
      }
    }
    // LF holds the adjoint of the trial f^(1)
    AdjSetupArgs A{};
    A.NS = NS;
    A.Q = Q;
    A.D1 = D + 1;
    A.order = order;
    A.q = q;
    A.dt = P.dt;
    A.lf1n = lf1;
    A.lf2n = lf2;
    A.lm1n = lm1;
    A.Lam1 = LF;
    A.lam_h = adj_lh;
    A.of0 = lout;
    A.of1 = lout + FQ;
    A.of2 = lout + 2 * FQ;
    A.om0 = lout + 3 * FQ;
    A.om1 = lout + 3 * FQ + FM;
    hipLaunchKernelGGL(k_adj_setup<0>, dim3(eg), dim3(256), 0, st, A);
    MSC_HIPCK(hipGetLastError());
  }

  // ------------------------------------------------------ sweep config --
  int tile_id = 0, strip_L = 1;
  bool wide_dual = false;  // dual-time sweeps after the first of a step on kWideDualTile3
  int strip_setup = 1;     // planes per strip of the first sweep of a step
  int strip_explicit = 1;  // planes per strip of the tiled explicit sweep
  TileCfg tile{};
  // 2D with the shadow corrector and tiles spanning whole rows: the sweep
  // also does the forward row transform of P r
  bool fuse_rows = false;
  // ... and the inverse row transform before the lift (one-plane strips): the
  // correction's spectrum then alternates between spec and spec_alt
  bool fuse_inv = false;

  void choose_sweep() {
    const int n = TileSet<L>::count;
    int best = -1;
    if (tune.sweep_tile_index > 0 && tune.sweep_tile_index <= n) {
      const TileCfg t = TileSet<L>::get(tune.sweep_tile_index - 1);
      if (t.T1 <= G.N1 && t.T2 <= G.N2) best = tune.sweep_tile_index - 1;
    }
    if (best < 0 && tune.sweep_tile > 0) {
      for (int i = 0; i < n; ++i) {
        const TileCfg t = TileSet<L>::get(i);
        if (t.T1 * t.T2 == tune.sweep_tile && t.T1 <= G.N1 && t.T2 <= G.N2) best = i;
      }
    }
    if (best < 0) best = auto_sweep_tile<L>(G.N1, G.N2);
    tile_id = best;
    tile = TileSet<L>::get(best);
    wide_dual = D == 3 && tune.wide_dual && tile.T1 == 2 && tile.T2 == 128 && G.N2 == 128 && G.N1 >= 4;
    strip_L = wide_dual ? sweep_strip_for<L, T>(kWideDualTile3, G.N0, G.N1, G.N2, tune.sweep_strip, STRIP_DUAL_WIDE)
                        : sweep_strip_for<L, T>(tile, G.N0, G.N1, G.N2, tune.sweep_strip, STRIP_DUAL);
    strip_setup = sweep_strip_for<L, T>(tile, G.N0, G.N1, G.N2, tune.sweep_strip, STRIP_SETUP);
    strip_explicit = sweep_strip_for<L, T>(tile, G.N0, G.N1, G.N2, tune.sweep_strip, STRIP_EXPLICIT);
    fuse_rows = D == 2 && P.corrector == MSC_CORRECTOR_SHADOW && tile.T1 == 1 && tile.T2 == G.N2 &&
                tile.NT == tile.T2 && corrector_supported() && tune.fuse_rows != 0;
    fuse_inv = fuse_rows && strip_L == 1 && tune.fuse_rows >= 2;
  }

  int strip_of(int mode) const {
    return (mode == SW_DTS_SETUP) ? strip_setup : (mode == SW_EXPLICIT ? strip_explicit : strip_L);
  }
  bool wide_mode(int mode) const { return wide_dual && (mode == SW_DTS || mode == SW_DTS_LIFT); }
  TileCfg tile_of(int mode) const { return wide_mode(mode) ? kWideDualTile3 : tile; }
  int sweep_grid(int mode = SW_DTS) const {
    const TileCfg t = tile_of(mode);
    return (int)((int64_t)(G.N1 / t.T1) * (G.N2 / t.T2) * (G.N0 / strip_of(mode)));
  }
  int sweep_grid_max() const {
    return std::max({sweep_grid(), sweep_grid(SW_DTS_SETUP), sweep_grid(SW_EXPLICIT)});
  }

  SweepArgs<T, TM> sweep_args(double a) {
    SweepArgs<T, TM> S{};
    S.N0 = G.N0;
    S.N1 = G.N1;
    S.N2 = G.N2;
    S.L = strip_L;
    S.ntile1 = G.N1 / tile.T1;
    S.ntile2 = G.N2 / tile.T2;
    S.nstrip = G.N0 / strip_L;
    S.NS = G.NS;
    S.ctl = nullptr;
    S.fb = fb;
    S.h = h;
    S.dm = dm;
    S.Pr = Pr;
    S.partials = partials;
    S.a = a;
    S.inv1pa2 = 1.0 / (1.0 + a / 2.0);
    S.wp = wp;
    S.wm = wm;
    S.sig = sig;
    S.isig = 1.0f / sig;
    S.walls = walls() ? 1 : 0;
    S.ulid = P.u_lid;
    return S;
  }

  // algorithmic bytes per sweep launch (one read and one write of the
  // populations, plus h, dm in, P r out for the dual-time sweep)
  // algorithmic HBM bytes of one sweep launch: populations read once per
  // history state used and written once; h read (or, in setup mode, m^n and
  // m^{n-1} read and h written); the lift input and P r output
  double sweep_bytes(int mode, int order = 0, int q = 1) const {
    const double NS = (double)G.NS;
    const double fb1 = (double)pop_bytes(), mb1 = (double)(D + 1) * NS;
    if (mode == SW_EXPLICIT) return 2.0 * fb1;
    double b = 2.0 * fb1 + mb1 * sizeof(TM);  // f in, f_T out, P r out
    if (fullsym()) b += (double)(Q - D - 1) * NS * sizeof(TM);  // r of every field instead of P r
    if (fuse_rows && (lift_mode(mode) || mode == SW_DTS_SETUP))  // row spectrum out instead of P r
      b += (double)(D + 1) * G.N0 * (G.N2 / 4 + 1) * sizeof(cpx<TM>) - mb1 * sizeof(TM);
    if (mode == SW_DTS_SETUP)
      b += order * fb1 + mb1 * sizeof(double) * (q == 2 ? 3.0 : 2.0);
    else
      b += mb1 * sizeof(double);
    if (mode == SW_DTS_LIFT) b += mb1 * sizeof(TM);
    if (mode == SW_DTS_LIFT_ROWS)  // the band spectrum rows in instead of dm
      b += (double)(D + 1) * G.N0 * (G.N2 / 4 + 1) * sizeof(cpx<TM>);
    return b;
  }

  hipEvent_t get_event() {
    if (!ev_free.empty()) {
      hipEvent_t e = ev_free.back();
      ev_free.pop_back();
      return e;
    }
    hipEvent_t e;
    MSC_HIPCK(hipEventCreate(&e));
    return e;
  }

  void collect_timing() {
    if (ev_live.empty()) return;
    MSC_HIPCK(hipMemcpyAsync(run_flags_h, run_flags, sizeof(int) * ev_live.size(), hipMemcpyDeviceToHost, st));
    sync();
    for (auto& e : ev_live) {
      if (run_flags_h[e.flag]) {
        float ms = 0.f;
        MSC_HIPCK(hipEventElapsedTime(&ms, e.a, e.b));
        t_sum[e.kind] += 1e-3 * ms;
        t_count[e.kind] += 1;
        t_bytes[e.kind] += e.bytes;
      }
      ev_free.push_back(e.a);
      ev_free.push_back(e.b);
    }
    ev_live.clear();
    MSC_HIPCK(hipMemsetAsync(run_flags, 0, sizeof(int) * kFlagCap, st));
    sync();
  }

  // events and run flag of one timed launch (kind 0: dual-time sweep, 1:
  // explicit march)
  EvPair timed_pair(int kind, double bytes) {
    if (!run_flags) {
      run_flags = keep((int*)dalloc(sizeof(int) * kFlagCap));
      MSC_HIPCK(hipHostMalloc((void**)&run_flags_h, sizeof(int) * kFlagCap, hipHostMallocDefault));
      MSC_HIPCK(hipMemsetAsync(run_flags, 0, sizeof(int) * kFlagCap, st));
    }
    EvPair ep{};
    ep.a = get_event();
    ep.b = get_event();
    ep.kind = kind;
    ep.flag = (int)ev_live.size();
    ep.bytes = bytes;
    return ep;
  }

  void launch_sweep_timed(int mode, SweepArgs<T, TM> S, int kind) {
    EvPair ep{};
    (void)kind;
    if (timing) {
      ep = timed_pair((mode == SW_EXPLICIT) ? 1 : 0,
                      sweep_bytes(mode, S.order, S.q) - (S.skip_pr ? (double)(D + 1) * G.NS * sizeof(TM) : 0.0) +
                          ((mode == SW_DTS_SETUP && S.recon) ? (double)(D + 1) * G.NS * 8.0 : 0.0));
      S.did_run = run_flags + ep.flag;
    }
    S.L = strip_of(mode);
    S.nstrip = G.N0 / S.L;
    const TileCfg tm = tile_of(mode);
    S.ntile1 = G.N1 / tm.T1;
    S.ntile2 = G.N2 / tm.T2;
    if (D == 2)
      launch_sweep_d2<T, TM>(tile_id, mode, S, sweep_grid(mode), st, timing ? ep.a : nullptr, timing ? ep.b : nullptr);
    else if (wide_mode(mode))
      launch_sweep_dual_wide<T, TM>(mode, S, sweep_grid(mode), st, timing ? ep.a : nullptr, timing ? ep.b : nullptr);
    else
      launch_sweep_d3<T, TM>(tile_id, mode, S, sweep_grid(mode), st, timing ? ep.a : nullptr, timing ? ep.b : nullptr);
    MSC_HIPCK(hipGetLastError());
    if (timing) {
      ev_live.push_back(ep);
      if ((int)ev_live.size() >= kFlagCap) collect_timing();
    }
  }

  hipGraphExec_t explicit_graph(T* A, T* B, int chunk, bool aa) {
    if (gexec && g_a == A && g_b == B && g_chunk == chunk && g_sig == sig && g_aa == aa) return gexec;
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    sync();
    MSC_HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    SweepArgs<T, TM> S = sweep_args(0.0);
    S.L = strip_explicit;
    S.nstrip = G.N0 / strip_explicit;
    for (int i = 0; i < chunk; ++i) {
      if (aa) {
        launch_aa(A, (i & 1) != 0);
        continue;
      }
      S.src = (i & 1) ? B : A;
      S.dst = (i & 1) ? A : B;
      if (D == 2)
        launch_sweep_d2<T, TM>(tile_id, SW_EXPLICIT, S, sweep_grid(SW_EXPLICIT), st);
      else
        launch_sweep_d3<T, TM>(tile_id, SW_EXPLICIT, S, sweep_grid(SW_EXPLICIT), st);
    }
    MSC_HIPCK(hipStreamEndCapture(st, &graph));
    MSC_HIPCK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    g_a = A;
    g_b = B;
    g_chunk = chunk;
    g_sig = sig;
    g_aa = aa;
    return gexec;
  }

  // --------------------------------------------------- Algorithm 1 pieces --
  // One inner iteration of Algorithm 1 for (step n, sweep ell), guarded on the
  // device: the sweep (the first one of a step also forms h_q and the
  // extrapolated trial), the one-block acceptance test, then either the
  // reconstruction of m^{n+1} (accepted) or the shadow correction.
  // last: the final iteration enqueued for this step; its correction passes
  // after the first are left out (they run only if the step goes on, and then
  // enqueue_correction_tail supplies them before the next sweep).
  // recon: this step's setup sweep forms m^n (the previous step, coefficient
  // a_prev, left it); defer: this step's acceptance leaves m^{n+1} to the
  // next step's setup sweep.
  void enqueue_iteration(int n, int ell, int q, int order, double a, bool use_sched, int stat_base,
                         bool last = false, bool recon = false, double a_prev = 0.0, bool defer = false) {
    SweepArgs<T, TM> S = sweep_args(a);
    S.ctl = ctl;
    S.h = h_of(n);
    S.recon = (ell == 1 && recon) ? 1 : 0;
    S.h_prev = h_of(n - 1);
    S.a_prev = a_prev;
    S.inv1pa2_prev = 1.0 / (1.0 + a_prev / 2.0);
    S.inv_dt = 1.0 / P.dt;
    S.inv_2dt = 1.0 / (2.0 * P.dt);
    S.n = n;
    S.ell = ell;
    for (int i = 0; i < 3; ++i) S.mb[i] = mb[i];
    S.q = q;
    S.order = order;
    S.dt = P.dt;
    FinishArgs F{};
    F.ctl = ctl;
    F.n = n;
    F.ell = ell;
    F.inv_count = 1.0 / ((double)Q * (double)G.NS);
    F.eps = P.eps;
    F.nmin = P.n_min;
    F.kmax = P.k_max;
    F.q = q;
    F.mcap = (D == 2) ? 10 : 8;
    F.sched = use_sched ? sched_d : nullptr;
    F.Rhist = Rhist;
    F.stats = stats_d;
    F.stat_base = stat_base;
    F.partials = partials;
    int mode;
    if (ell == 1)
      mode = SW_DTS_SETUP;
    else if (P.corrector == MSC_CORRECTOR_SHADOW)
      mode = fuse_inv ? SW_DTS_LIFT_ROWS : SW_DTS_LIFT;
    else
      mode = SW_DTS;
    F.nparts = sweep_grid(mode);
    if (fullsym() || wallkin()) S.rout = rfs;
    const bool skip_pr = skip_pr_ok() && last && mode == SW_DTS_LIFT;
    S.skip_pr = skip_pr ? 1 : 0;
    if (fuse_rows) {
      S.fuse_rows = 1;
      S.lgr = ilog2(G.N2);
      S.NBr = G.N2 / 4 + 1;
      S.spec = spec_of(ell);
      S.twr = tw[2];
      if (mode == SW_DTS_LIFT_ROWS) S.spec_in = spec_of(ell - 1);
    }
    launch_sweep_timed(mode, S, 0);
    if (F.nparts > kFusedParts) {
      // many sweep blocks: fold the partials once instead of in every block
      hipLaunchKernelGGL(k_presum<0>, dim3(1), dim3(256), 0, st, (const double*)partials, F.nparts, presum);
      MSC_HIPCK(hipGetLastError());
      F.partials = presum;
      F.nparts = 1;
    }

    AcceptArgs<L, T> Ac = accept_args(n, ell, a);
    Ac.defer = defer ? 1 : 0;
    if (P.corrector == MSC_CORRECTOR_SHADOW) {
      XformBufs<CT, TM> B{Pr, dm, spec_of(ell), spec2, {tw[0], tw[1], tw[2]}};
      enqueue_transform<CT, TM>(ctl, n, ell, a, &Ac, false, B, &F, true, !last && !fuse_inv, fuse_rows, skip_pr);
    } else if (fullsym()) {
      enqueue_fullsym(ctl, n, ell, a, &Ac, &F, true, !last, nullptr);
    } else {
      hipLaunchKernelGGL((k_accept<L, T>), dim3(ew_grid()), dim3(256), 0, st, Ac, F);
      MSC_HIPCK(hipGetLastError());
    }
  }

  // The correction passes after the first for (step n, sweep ell), guarded on
  // the device (they run only if that sweep was not accepted).
  void enqueue_correction_tail(int n, int ell, double a) {
    if (fullsym()) {
      enqueue_fullsym(ctl, n, ell, a, nullptr, nullptr, false, true, nullptr);
      return;
    }
    if (P.corrector != MSC_CORRECTOR_SHADOW) return;
    if (fuse_inv) return;  // the next sweep inverts the rows itself
    XformBufs<CT, TM> B{Pr, dm, spec_of(ell), spec2, {tw[0], tw[1], tw[2]}};
    if constexpr (!PopDev<T>::value) {
      // the tail follows the last sweep enqueued for the step; a lift sweep
      // there left P r out: form it, then every pass, the first one guarded
      // rather than deciding (the decision was taken)
      if (skip_pr_ok() && ell >= 2) {
        PrArgs<T, TM> R{ctl, n, ell, fb, dm, Pr, G.NS};
        hipLaunchKernelGGL((k_recompute_pr<L, T, TM>), dim3(ew_grid()), dim3(256), 0, st, R);
        MSC_HIPCK(hipGetLastError());
        enqueue_transform<CT, TM>(ctl, n, ell, a, nullptr, false, B, nullptr, true, true, false);
        return;
      }
    }
    AcceptArgs<L, T> Ac = accept_args(n, ell, a);
    enqueue_transform<CT, TM>(ctl, n, ell, a, &Ac, false, B, nullptr, false, true, fuse_rows);
  }

  // band spectrum of the correction after sweep ell (alternating buffers
  // when the sweep inverts the previous correction's rows while writing its
  // own forward rows)
  cpx<CT>* spec_of(int ell) const { return (fuse_inv && (ell & 1)) ? spec_alt : spec; }

  // history term of physical step n (see h_alt); the wall corrector keeps one
  double* h_of(int n) const { return (!wallkin() && (n & 1)) ? h_alt : h; }

  AcceptArgs<L, T> accept_args(int n, int ell, double a) {
    AcceptArgs<L, T> Ac{};
    Ac.ctl = ctl;
    Ac.n = n;
    Ac.ell = ell;
    Ac.fb = fb;
    for (int i = 0; i < 3; ++i) Ac.mb[i] = mb[i];
    Ac.h = h_of(n);
    Ac.NS = G.NS;
    Ac.a = a;
    Ac.inv1pa2 = 1.0 / (1.0 + a / 2.0);
    return Ac;
  }

  // FFT launch shapes
  // rows per block of the row passes: LDS-limited, and small enough that the
  // grid has >= 1024 blocks (four per CU) when the grid is large enough: these
  // passes are latency-bound, and one row per block instead of four cuts the
  // corrected march by 18% at N = 512 FP32, one instead of two by 4% at N = 1024
  int fft_rows_per_block(size_t c = sizeof(cpx<CT>)) const {
    int R = (int)std::max<size_t>(1, (size_t)65536 / (4 * G.N2 * c));
    int p = 1;
    while (p * 2 <= R) p *= 2;
    while (p > 1 && G.N0 / p < 1024) p >>= 1;
    return std::min(p, G.N0);
  }
  // columns per block of the column pass: LDS-limited, and as few as give
  // >= 256 blocks (one per CU: at N = 512 one column per block instead of
  // two cuts the corrected march by 7%, at N = 1024 FP32 by 5%)
  int fft_cols_per_block(size_t c = sizeof(cpx<CT>)) const {
    int J = (int)std::max<size_t>(1, (size_t)98304 / (6 * G.N0 * c));
    J = std::min(J, 16);
    const int NB = G.N2 / 4 + 1;
    while (J > 1 && (NB + J - 1) / J < 256) J >>= 1;
    return std::max(J, 1);
  }

  // 3D launch shapes: pencils per block of the z passes, j_z columns per
  // block of the y and x passes
  int fft3_pencils_per_block(size_t c = sizeof(cpx<CT>)) const {
    int R = (int)std::max<size_t>(1, (size_t)65536 / (4 * G.n[2] * c));
    int p = 1;
    while (p * 2 <= R) p *= 2;
    if (tune.fft3_pencils > 0) {
      int q = 1;
      while (q * 2 <= tune.fft3_pencils) q *= 2;
      return std::min(p, q);
    }
    // at most four pencils per block: more, smaller blocks hide the latency
    // of the LDS passes better (measured at N = 128: 7% per step over 16)
    p = std::min(p, 4);
    while (p > 1 && ((int64_t)G.n[0] * G.n[1]) / p < 256) p >>= 1;
    return p;
  }
  int fft3_cols_per_block(size_t c = sizeof(cpx<CT>)) const {
    const int Nmax = std::max(G.n[0], G.n[1]);
    int J = (int)std::max<size_t>(1, (size_t)98304 / (8 * Nmax * c));
    J = std::min(J, 8);
    if (tune.fft3_cols > 0)
      J = std::min(J, tune.fft3_cols);
    else
      J = std::min(J, 2);  // as for the pencils: smaller blocks, more of them per CU
                           // (N = 128 march: FP64 0.835 -> 0.807 ms per step, FP32
                           // 0.558 -> 0.546 against four columns)
    return std::max(J, 1);
  }

  // Blocks of a kernel that the device holds at once (occupancy per CU times
  // the CU count) for a block size and dynamic LDS size, cached: the grid of
  // the grid-resident passes (any grid size gives the same results).
  struct Resident {
    const void* k;
    int threads;
    size_t lds;
    int blocks;
  };
  std::vector<Resident> resident_cache;
  int resident_blocks(const void* k, int threads, size_t lds) {
    for (const auto& e : resident_cache)
      if (e.k == k && e.threads == threads && e.lds == lds) return e.blocks;
    int dev = 0, cus = 0, per_cu = 0;
    MSC_HIPCK(hipGetDevice(&dev));
    MSC_HIPCK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MSC_HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, lds));
    const int n = std::max(1, per_cu) * std::max(1, cus);
    resident_cache.push_back({k, threads, lds, n});
    return n;
  }

  template <class CX = CT, class TX = TM>
  void set_fft_attrs() {
    const size_t c = sizeof(cpx<CX>);
    if constexpr (D == 2) {
      const int rows_b = (int)(4 * fft_rows_per_block(c) * G.N2 * c);
      const int cols_b = (int)(6 * fft_cols_per_block(c) * G.N0 * c);
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fft2_rows_fwd<L, T, CX, TX>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, rows_b));
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fft2_rows_inv<CX, TX>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, rows_b));
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fft2_cols_solve<L, T, CX, TX>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, cols_b));
    } else {
      const int zb = (int)(4 * fft3_pencils_per_block(c) * G.n[2] * c);
      const int Nmax = std::max(G.n[0], G.n[1]);
      const int cb = (int)(8 * fft3_cols_per_block(c) * Nmax * c);
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fft3_z_fwd<L, T, CX, TX>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, zb));
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fft3_z_inv<CX, TX>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, zb));
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fft3_y_fwd<CX, TX>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, cb));
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fft3_y_inv<CX, TX>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, cb));
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fft3_x_solve<CX, TX>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, cb));
      resident_blocks((const void*)k_fft3_z_fwd<L, T, CX, TX>, 256, zb);
    }
  }


  // Full-symbol launch shapes: rows per block of the row passes (LDS-limited,
  // >= 512 blocks where the grid allows), j_y columns per block of the
  // column pass (>= 256 blocks where possible).  At N <= 512 every pass is
  // latency-bound, so these keep one row / one column per block there.
  int fs_rows_per_block() const {
    const size_t c = sizeof(cpx<CT>);
    int R = (int)std::max<size_t>(1, (size_t)65536 / (2 * ((Q + 1) / 2) * G.N2 * c));
    int p = 1;
    while (p * 2 <= R) p *= 2;
    while (p > 1 && G.N0 / p < 512) p >>= 1;
    return std::min(p, G.N0);
  }
  int fs_cols_per_block() const {
    const size_t c = sizeof(cpx<CT>);
    int J = (int)std::max<size_t>(1, (size_t)98304 / (2 * Q * G.N0 * c));
    J = std::min(J, 8);
    const int NH = G.N2 / 2 + 1;
    while (J > 1 && (NH + J - 1) / J < 256) J >>= 1;
    return std::max(J, 1);
  }
  size_t fs_rows_lds() const { return (size_t)2 * ((Q + 1) / 2) * fs_rows_per_block() * G.N2 * sizeof(cpx<CT>); }
  size_t fs_cols_lds() const { return (size_t)2 * Q * fs_cols_per_block() * G.N0 * sizeof(cpx<CT>); }
  // split column pass: lines per block of the x transforms
  int fs_lines_per_block() const { return std::max(1, std::min(8, 2048 / G.N0)); }
  size_t fs_lines_lds() const { return (size_t)2 * fs_lines_per_block() * G.N0 * sizeof(cpx<CT>); }

  void set_fs_attrs() {
    if constexpr (D == 2 && !DV) {
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fs_rows_fwd<L, T, CT, TM>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)fs_rows_lds()));
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fs_rows_inv<L, T, CT, TM>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)fs_rows_lds()));
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fs_cols_fft<L, T, CT, TM>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)fs_lines_lds()));
      MSC_HIPCK(hipFuncSetAttribute((const void*)k_fs_cols_solve<L, T, CT, TM>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)fs_cols_lds()));
    }
  }

  // The full-symbol correction of Eq. (full-symbol) for (step n, sweep ell),
  // guarded on the device like the shadow passes.  head: the rows pass (with
  // Ac and Fin, it decides acceptance first); tail: the column pass and the
  // inverse rows pass, which leave f_{l+1} in the sweep's output buffer (out
  // when c is null).
  void enqueue_fullsym(const DevCtl* c, int n, int ell, double a, const AcceptArgs<L, T>* Ac,
                       const FinishArgs* Fin, bool head, bool tail, T* out, const TM* rin = nullptr,
                       int plain = 0) {
    if constexpr (D == 2 && !DV) {
      FsArgs<T, CT, TM> F{};
      F.g = CorrGuard{c, n, ell};
      F.do_accept = (Ac && Fin) ? 1 : 0;
      F.Nx = G.N0;
      F.Ny = G.N2;
      F.lgx = ilog2(G.N0);
      F.lgy = ilog2(G.N2);
      F.NH = G.N2 / 2 + 1;
      F.rows_per_block = fs_rows_per_block();
      F.cols_per_block = fs_cols_per_block();
      F.r = rin ? rin : rfs;
      F.plain = plain;
      F.spec = spec_fs;
      F.twx = tw[0];
      F.twy = tw[2];
      F.a = a;
      F.wp = wp;
      F.wm = wm;
      F.inv_ns = 1.0 / (double)G.NS;
      F.fb = fb;
      F.out = out;
      const int rgrid = G.N0 / F.rows_per_block;
      if (head) {
        AcceptArgs<L, T> none{};
        const FinishArgs nofin{};
        hipLaunchKernelGGL((k_fs_rows_fwd<L, T, CT, TM>), dim3(rgrid), dim3(256), fs_rows_lds(), st, F,
                           Ac ? *Ac : none, Fin ? *Fin : nofin);
        MSC_HIPCK(hipGetLastError());
      }
      if (tail) {
        const int cgrid = pad8((F.NH + F.cols_per_block - 1) / F.cols_per_block);  // XCD-aware order
        // split column pass where it is faster (measured: N_x = 512, 12% per
        // iteration; at N_x <= 256 the extra launches cost more than the
        // parallelism gains)
        const bool split = (tune.fs_split == 1) || (tune.fs_split == 0 && G.N0 >= 512);
        if (split) {
          FsArgs<T, CT, TM> Fl = F;
          Fl.cols_per_block = fs_lines_per_block();
          const int lgrid = pad8((Q * F.NH + Fl.cols_per_block - 1) / Fl.cols_per_block);
          const int64_t nk = (int64_t)G.N0 * F.NH;
          const int sgrid = (int)std::min<int64_t>((nk + 63) / 64, 4096);
          hipLaunchKernelGGL((k_fs_cols_fft<L, T, CT, TM>), dim3(lgrid), dim3(256), fs_lines_lds(), st, Fl, -1);
          hipLaunchKernelGGL((k_fs_solve_k<L, T, CT, TM>), dim3(sgrid), dim3(64), 0, st, F);
          hipLaunchKernelGGL((k_fs_cols_fft<L, T, CT, TM>), dim3(lgrid), dim3(256), fs_lines_lds(), st, Fl, +1);
        } else {
          hipLaunchKernelGGL((k_fs_cols_solve<L, T, CT, TM>), dim3(cgrid), dim3(256), fs_cols_lds(), st, F);
        }
        MSC_HIPCK(hipGetLastError());
        hipLaunchKernelGGL((k_fs_rows_inv<L, T, CT, TM>), dim3(rgrid), dim3(256), fs_rows_lds(), st, F);
        MSC_HIPCK(hipGetLastError());
      }
    } else {
      (void)c, (void)n, (void)ell, (void)a, (void)Ac, (void)Fin, (void)head, (void)tail, (void)out, (void)rin,
          (void)plain;
    }
  }

  // The shadow correction of Eq. (shadow-update) for (step n, sweep ell):
  // transforms of P r, per-wavevector Schur solve, inverse transforms into dm
  // (the lift is fused into the next sweep).  With Ac the first pass instead
  // reconstructs m^{n+1} when the step was accepted at this sweep.
  void enqueue_correction(const DevCtl* c, int n, int ell, double a, const AcceptArgs<L, T>* Ac) {
    XformBufs<CT, TM> B{Pr, dm, spec, spec2, {tw[0], tw[1], tw[2]}};
    enqueue_transform<CT, TM>(c, n, ell, a, Ac, false, B);
  }

  template <class CX, class TX>
  void enqueue_transform(const DevCtl* c, int n, int ell, double a, const AcceptArgs<L, T>* Ac, bool adjoint,
                         const XformBufs<CX, TX>& B, const FinishArgs* Fin = nullptr, bool head = true,
                         bool tail = true, bool rows_in_sweep = false, bool decide_only = false) {
    AcceptArgs<L, T> none{};
    const FinishArgs nofin{};
    const size_t cb = sizeof(cpx<CX>);
    if constexpr (D == 2) {
      Fft2Args<CX, TX> F{};
      F.g = CorrGuard{c, n, ell};
      F.do_accept = Ac ? 1 : 0;
      F.decide_only = (Ac && decide_only) ? 1 : 0;
      F.adjoint = adjoint ? 1 : 0;
      F.Nx = G.N0;
      F.Ny = G.N2;
      F.lgx = ilog2(G.N0);
      F.lgy = ilog2(G.N2);
      F.NBy = G.N2 / 4 + 1;
      F.rows_per_block = fft_rows_per_block(cb);
      F.cols_per_block = fft_cols_per_block(cb);
      F.Pr = B.in;
      F.spec = B.spec1;
      F.dm = B.out;
      F.twx = B.tw[0];
      F.twy = B.tw[2];
      F.a = a;
      F.nu = nu;
      F.inv_ns = 1.0 / (double)G.NS;
      const size_t rows_b = 4 * (size_t)F.rows_per_block * G.N2 * cb;
      const size_t cols_b = 6 * (size_t)F.cols_per_block * G.N0 * cb;
      const int grows = G.N0 / F.rows_per_block;
      // column blocks rounded up to a multiple of 8 (the XCD-aware order)
      const int gcols = pad8((F.NBy + F.cols_per_block - 1) / F.cols_per_block);
      if (rows_in_sweep) {
        // the sweep wrote the row spectrum; the column pass decides
        F.do_accept = 0;
        F.decide = 1;
        if (head) {
          // enough blocks for the reconstruction of an accepted step; blocks
          // beyond the column count stop after the decision otherwise
          const int gdec = std::max<int>(gcols, (int)std::min<int64_t>((G.NS + 255) / 256, 4096));
          hipLaunchKernelGGL((k_fft2_cols_solve<L, T, CX, TX>), dim3(gdec), dim3(256), cols_b, st, F,
                             Ac ? *Ac : none, Fin ? *Fin : nofin);
          MSC_HIPCK(hipGetLastError());
        }
        if (tail) {
          hipLaunchKernelGGL((k_fft2_rows_inv<CX, TX>), dim3(grows), dim3(256), rows_b, st, F);
          MSC_HIPCK(hipGetLastError());
        }
        return;
      }
      if (head) {
        hipLaunchKernelGGL((k_fft2_rows_fwd<L, T, CX, TX>), dim3(grows), dim3(256), rows_b, st, F,
                           Ac ? *Ac : none, Fin ? *Fin : nofin);
        MSC_HIPCK(hipGetLastError());
      }
      if (tail) {
        // 512 threads: two waves per SIMD on the one block per CU that the
        // column count allows (N = 1024 FP64 march 0.361 -> 0.347 ms per step,
        // N = 512 and 2048 FP32 4-5%; 1024 threads no better)
        hipLaunchKernelGGL((k_fft2_cols_solve<L, T, CX, TX>), dim3(gcols), dim3(512), cols_b, st, F, none, nofin);
        MSC_HIPCK(hipGetLastError());
        hipLaunchKernelGGL((k_fft2_rows_inv<CX, TX>), dim3(grows), dim3(256), rows_b, st, F);
        MSC_HIPCK(hipGetLastError());
      }
    } else {
      Fft3Args<CX, TX> F{};
      F.g = CorrGuard{c, n, ell};
      F.do_accept = Ac ? 1 : 0;
      F.decide_only = (Ac && decide_only) ? 1 : 0;
      F.adjoint = adjoint ? 1 : 0;
      F.Nx = G.n[0];
      F.Ny = G.n[1];
      F.Nz = G.n[2];
      F.lgx = ilog2(F.Nx);
      F.lgy = ilog2(F.Ny);
      F.lgz = ilog2(F.Nz);
      F.NBz = F.Nz / 4 + 1;
      F.NBy = 2 * (F.Ny / 4) + 1;
      F.pencils_per_block = fft3_pencils_per_block(cb);
      F.cols_per_block = fft3_cols_per_block(cb);
      F.Pr = B.in;
      F.dm = B.out;
      F.spec1 = B.spec1;
      F.spec2 = B.spec2;
      F.twx = B.tw[0];
      F.twy = B.tw[1];
      F.twz = B.tw[2];
      F.a = a;
      F.nu = nu;
      F.inv_ns = 1.0 / (double)G.NS;
      const int R = F.pencils_per_block, JB = F.cols_per_block;
      const size_t zb = 4 * (size_t)R * F.Nz * cb;
      const size_t yb = 8 * (size_t)JB * F.Ny * cb;
      const size_t xb = 8 * (size_t)JB * F.Nx * cb;
      const int ng = (F.NBz + JB - 1) / JB;
      // z passes: pencil groups of R; the forward pass (which takes the
      // acceptance decision) at most one block per resident slot, each
      // looping over groups (measured at N = 128 FP64: full launches 46.5 ->
      // 42.9 us, decision-only ones 8.1 -> 4.9 us; the same loop made the
      // inverse pass slower, 34.5 -> 38.3 us, so it keeps one group per block)
      const int gz = (int)(((int64_t)F.Nx * F.Ny) / R);
      const int gzf = std::min(gz, resident_blocks((const void*)k_fft3_z_fwd<L, T, CX, TX>, 256, zb));
      if (head) {
        hipLaunchKernelGGL((k_fft3_z_fwd<L, T, CX, TX>), dim3(gzf), dim3(256), zb, st, F, Ac ? *Ac : none,
                           Fin ? *Fin : nofin);
        MSC_HIPCK(hipGetLastError());
      }
      if (!tail) return;
      hipLaunchKernelGGL((k_fft3_y_fwd<CX, TX>), dim3(pad8(F.Nx * ng)), dim3(256), yb, st, F);
      MSC_HIPCK(hipGetLastError());
      hipLaunchKernelGGL((k_fft3_x_solve<CX, TX>), dim3(pad8(F.NBy * ng)), dim3(256), xb, st, F);
      MSC_HIPCK(hipGetLastError());
      hipLaunchKernelGGL((k_fft3_y_inv<CX, TX>), dim3(pad8(F.Nx * ng)), dim3(256), yb, st, F);
      MSC_HIPCK(hipGetLastError());
      hipLaunchKernelGGL((k_fft3_z_inv<CX, TX>), dim3(gz), dim3(256), zb, st, F);
      MSC_HIPCK(hipGetLastError());
    }
  }
};

}  // namespace msc
