// Fused population sweep T_{q,h}(f) (paper Eq. sweep) with the raw residual
// r = T(f) - f (Eq. residual), the conserved residual moments P r and the
// FP64 sum of r^2, on a periodic lattice.  One kernel serves the dual-time
// sweep of Algorithm 1 (with or without the equilibrium lift of the previous
// correction, Eq. lift / shadow-update, fused into the load) and the explicit
// source-free march (a = 0, h = 0), so both use the same collision and
// streaming code (Sec. 4.1).
//
// Work decomposition.  A block owns a tile of T1 x T2 sites of the (p1, p2)
// plane and a strip of L consecutive planes along x.  It walks the strip plane
// by plane (plus one plane on each side): for each source plane it loads the
// populations, reconstructs m and s, collides (Eq. collision), and pushes the
// post-collision values (Eq. sweep, push streaming) of the directions that
// leave the thread's own (p1, p2) position into LDS ring buffers indexed by
// the destination; directions that stay on the thread's position (rest and
// +-x) stay in registers.  After one barrier the plane behind is complete and
// each thread finalises its own sites: f_T, r, P r, sum r^2.  Source sites on
// a one-site ring around the tile (only along axes the tile does not span)
// are collided as well so that every destination in the tile is served.  HBM
// traffic is one read and one write of every population per sweep plus the
// moment fields; halo re-reads hit L2.
#pragma once

#include <type_traits>

#include "msc_common.h"
#include "msc_ldsfft.h"

namespace msc {

// Sweep modes: the source-free explicit map; the dual-time sweep on a given
// trial; the same with the previous correction's lift fused into the load;
// and the first sweep of a physical step, which also forms the BDF history
// term h_q (Eq. bdf2) and the extrapolated trial (Sec. 3.1) while loading.
enum { SW_EXPLICIT = 0, SW_DTS = 1, SW_DTS_LIFT = 2, SW_DTS_SETUP = 3, SW_DTS_LIFT_ROWS = 4, SW_DTS_SETUP1 = 5 };
// SW_DTS_LIFT_ROWS: the lift mode with the correction's inverse row transform
// done by the sweep itself (2D, tiles spanning whole rows, one-plane strips):
// each block inverts the band spectrum rows of its source planes in LDS
// instead of reading dm.
__host__ __device__ constexpr bool lift_mode(int m) { return m == SW_DTS_LIFT || m == SW_DTS_LIFT_ROWS; }
// SW_DTS_SETUP1: the first sweep of a step with a trial extrapolated from at
// most two states (order <= 1), which holds no f^{n-2} registers
__host__ __device__ constexpr bool setup_mode(int m) { return m == SW_DTS_SETUP || m == SW_DTS_SETUP1; }
// first sweep whose halo loads are issued a plane ahead (see k_sweep)
template <class L, class T, int MODE>
__host__ __device__ constexpr bool setup_halo_prefetch() {
  return MODE == SW_DTS_SETUP1 && L::D == 3 && sizeof(T) != 4;
}
// sweep whose owned loads for the next plane are issued after the halo (see k_sweep)
template <class L, class T, int MODE>
__host__ __device__ constexpr bool late_owned_prefetch() {
  return L::D == 3 && (((MODE == SW_DTS || MODE == SW_DTS_LIFT) && sizeof(T) == 8) ||
                       (MODE == SW_DTS_SETUP1 && sizeof(T) == 4));
}
// halo ring sites of a T1 x T2 tile (one ring along each axis the tile does
// not span)
__host__ __device__ inline int tile_halo_sites(int T1, int T2, int N1, int N2) {
  const int h1 = (T1 < N1) ? 1 : 0, h2 = (T2 < N2) ? 1 : 0;
  return 2 * h1 * (T2 + 2 * h2) + 2 * h2 * T1;
}

template <class T>
struct CompT;
template <>
struct CompT<double> {
  using type = double;
};
template <>
struct CompT<float> {
  using type = float;
};
template <>
struct CompT<_Float16> {
  using type = float;
};

// Acceptance test of Algorithm 1.  It runs at the start of the kernel that
// follows the sweep (the first transform pass, or the reconstruction kernel
// without the shadow corrector): every block sums the sweep's per-block
// partials of r^2 in the same fixed order, so every block reaches the same
// decision without waiting for another; block 0 alone records it.
struct FinishArgs {
  DevCtl* ctl;
  int n, ell;
  double inv_count;  // 1/(Q N_sites)
  double eps;
  int nmin, kmax, q, mcap;
  const int32_t* sched;  // accept count of step n at sched[n - stat_base], or null
  double* Rhist;         // residual history of the current step
  StepStat* stats;       // stats[n - stat_base]
  int stat_base;
  const double* partials;  // the sweep's per-block sums of r^2
  int nparts;
};

enum { DEC_SKIP = -1, DEC_RUNNING = 0, DEC_ACCEPTED = 1, DEC_FAILED = 2 };

// Raw residual RMS (Eq. residual) and the acceptance decision: accept when
// ell >= n_min and the residual is finite and below eps (or at the scheduled
// count in replay mode); a non-finite residual fails the step (Sec. 4.1);
// reaching K_max fails it as nonconvergent.
__device__ inline int accept_decision(const FinishArgs& A, double R, int* fail_out) {
  const int ell = A.ell;
  const bool fin = isfinite(R);
  const bool pass = A.sched ? (ell == A.sched[A.n - A.stat_base]) : (ell >= A.nmin && fin && R < A.eps);
  int fail = 0;
  if (!pass) {
    if (!fin)
      fail = 6;  // MSC_ERR_NONFINITE
    else if (ell >= A.kmax)
      fail = 5;  // MSC_ERR_NONCONVERGED
  }
  *fail_out = fail;
  return pass ? DEC_ACCEPTED : (fail ? DEC_FAILED : DEC_RUNNING);
}

// Block 0's record of the decision: residual history, statistics (Eq.
// rho-observed), on acceptance the rotated roles of step n + 1 (Sec. 3.1,
// last paragraph: the histories shift; the moment slot that becomes m^{n+1}
// is the spare, filled by the reconstruction of the same kernel), and the
// phase word.
__device__ inline void finish_commit(const FinishArgs& A, double R, int dec, int fail) {
  const int ell = A.ell;
  A.Rhist[ell - 1] = R;
  DevCtl* c = A.ctl;
  if (dec != DEC_RUNNING) {
    StepStat& st = A.stats[A.n - A.stat_base];
    st.q = A.q;
    st.iters = ell;
    st.R_first = A.Rhist[0];
    st.R_final = R;
    double rho = __builtin_nan("");
    if (ell >= 3) {
      // tail geometric mean over m_rho = min(mcap, ell-1)
      const int mr = (A.mcap < ell - 1) ? A.mcap : ell - 1;
      double sl = 0.0;
      for (int j = ell - mr + 1; j <= ell; ++j) sl += log(A.Rhist[j - 1] / A.Rhist[j - 2]);
      rho = exp(sl / mr);
    }
    st.rho_obs = rho;
    st.converged = (dec == DEC_ACCEPTED) ? 1 : 0;
    st.fail = fail;
  }
  if (dec == DEC_ACCEPTED) {
    const Roles& o = c->roles[A.n & 1];
    Roles& r = c->roles[(A.n + 1) & 1];
    r.slot_hist[0] = o.slot_w[ell & 1];
    r.slot_hist[1] = o.slot_hist[0];
    r.slot_hist[2] = o.slot_hist[1];
    r.slot_w[ell & 1] = o.slot_hist[2];
    r.slot_w[(ell + 1) & 1] = o.slot_w[(ell + 1) & 1];
    r.slot_m[0] = o.slot_m[2];  // becomes m^{n+1}
    r.slot_m[1] = o.slot_m[0];
    r.slot_m[2] = o.slot_m[1];
    c->phase = make_phase(A.n, ell, PH_ACCEPTED);
  } else if (dec == DEC_FAILED) {
    c->fail_code = fail;
    c->phase = make_phase(A.n, ell, PH_FAILED);
  } else {
    c->phase = make_phase(A.n, ell, PH_RUNNING);
  }
}

// Block-uniform decision for (step n, sweep ell), or DEC_SKIP when the march
// is not right after that sweep.  The phase word is either still the one the
// sweep saw or already block 0's record of this very decision.  Uses red[] (one entry per wavefront).
__device__ inline int finish_block(const FinishArgs& A, double* red) {
  __shared__ int sh_mine;
  if (threadIdx.x == 0) {
    const uint64_t ph = A.ctl->phase;
    const bool after = phase_n(ph) == A.n && phase_ell(ph) == A.ell && phase_state(ph) != 0;
    sh_mine = (phase_ready(ph, A.n, A.ell) || after) ? 1 : 0;
  }
  __syncthreads();
  if (!sh_mine) return DEC_SKIP;
  // fixed-order fold: strided per thread, then within each wavefront by
  // shuffles, then across the (blockDim / 64) wavefronts in order
  double acc = 0.0;
  for (int i = threadIdx.x; i < A.nparts; i += blockDim.x) acc += A.partials[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  double tot = 0.0;
  for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) tot += red[wv];
  const double R = sqrt(tot * A.inv_count);
  int fail = 0;
  const int dec = accept_decision(A, R, &fail);
  if (blockIdx.x == 0 && threadIdx.x == 0) finish_commit(A, R, dec, fail);
  return dec;
}

template <class T, class TM>
struct SweepArgs {
  int N0, N1, N2;  // extents along x, p1, p2
  int L;           // planes per strip
  int ntile1, ntile2, nstrip;
  int64_t NS;
  // Algorithm 1 mode when ctl != nullptr: buffers come from the control slots
  const DevCtl* ctl;
  int n, ell;
  FBufs<T> fb;
  const T* src;  // used when ctl == nullptr
  T* dst;
  double* h;        // (d+1) x NS FP64 history term h_q: read, or written in setup mode
  const TM* dm;     // (d+1) x NS, previous shadow correction
  TM* Pr;           // (d+1) x NS, residual moments out
  TM* rout;         // Q x NS, the raw residual of every field out instead of
                    // P r (full-symbol correction), or null
  double* partials; // one FP64 partial sum of r^2 per block
  double a, inv1pa2;  // a_q and 1/(1 + a_q/2)
  double wp, wm;      // omega+, omega-
  float sig, isig;    // FP16 deviation storage: scale sigma and 1/sigma
  int* did_run;       // optional: set to 1 when the launch passed its guard
  // setup mode: moment buffers (roles from control slots), BDF order,
  // extrapolation order, physical step
  double* mb[3];
  int q, order;
  double dt;
  // setup mode, recon = 1: the previous step's acceptance left m^n to this
  // sweep, which forms it from f^n with that step's history term h_prev and
  // coefficient a_prev (Eq. macro-reconstruct) and writes it for the owned
  // sites; h (this step's) is then a different buffer from h_prev
  int recon;
  const double* h_prev;
  double a_prev;
  // reciprocals formed once on the host: 1/(1 + a_prev/2), 1/dt, 1/(2 dt)
  double inv1pa2_prev, inv_dt, inv_2dt;
  // fused forward row transform (2D, tiles spanning whole rows, Algorithm 1
  // with the shadow corrector): the band spectrum of P r goes to spec
  // ([field][x][j <= N_y/4], as the first transform pass writes it) instead
  // of P r to Pr
  int fuse_rows, lgr, NBr;
  cpx<TM>* spec;
  const cpx<TM>* twr;
  // SW_DTS_LIFT_ROWS: the solved band spectrum of the previous correction
  // ([field][x][j <= N_y/4]), inverted along y by the sweep to give dm
  const cpx<TM>* spec_in;
  // D2Q9 lid-driven cavity: wall rows after streaming (every mode)
  int walls;
  double ulid;
  // lift mode: leave P r out (the sweep predicted to end its step; if the
  // step goes on, k_recompute_pr forms it from this sweep's input and output)
  int skip_pr;
};

// ---- compile-time direction classification -----------------------------
template <class L>
__host__ __device__ constexpr bool is_local(int k) {
  return L::c1(k) == 0 && L::c2(k) == 0;
}
// group of a non-local direction by its x component: 0 -> +x, 1 -> 0, 2 -> -x
template <class L>
__host__ __device__ constexpr int xgroup(int k) {
  return L::cx(k) > 0 ? 0 : (L::cx(k) == 0 ? 1 : 2);
}
template <class L>
__host__ __device__ constexpr int group_count(int g) {
  int n = 0;
  for (int k = 0; k < L::Q; ++k)
    if (!is_local<L>(k) && xgroup<L>(k) == g) ++n;
  return n;
}
template <class L>
__host__ __device__ constexpr int group_index(int k) {
  int n = 0;
  for (int j = 0; j < k; ++j)
    if (!is_local<L>(j) && xgroup<L>(j) == xgroup<L>(k)) ++n;
  return n;
}
template <class L>
__host__ __device__ constexpr int local_dir(int cxv) {
  for (int k = 0; k < L::Q; ++k)
    if (is_local<L>(k) && L::cx(k) == cxv) return k;
  return -1;
}

// ring depth per group: a value pushed towards plane x+1 is read two plane
// steps later, towards x one step later, towards x-1 in the same step; with
// one barrier per step the rings need 4, 3 and 2 slots, with a second
// barrier after the finalisation 3, 2 and 1 (a third less LDS).
__host__ __device__ constexpr int ring_depth(int g, bool two_bar) {
  return two_bar ? (g == 0 ? 3 : (g == 1 ? 2 : 1)) : (g == 0 ? 4 : (g == 1 ? 3 : 2));
}

// Two barriers per plane step where the LDS of the one-barrier rings would
// hold the block count per CU down: D3Q19 with FP64 populations (96 KB per
// 256-thread block, one block per CU; 64 KB with two barriers, two blocks per
// CU for the explicit and lift sweeps: N = 128 explicit sweep 184 -> 166 us,
// corrected march 1% faster).
template <class L, class T>
__host__ __device__ constexpr bool sweep_two_barriers() {
  return L::D == 3 && sizeof(T) == 8;
}

__device__ inline int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Source pointers of one launch, resolved once per block.
template <class T>
struct SrcPtrs {
  const T* s0;  // trial populations (f^n in setup mode)
  const T* s1;  // f^{n-1} (setup mode)
  const T* s2;  // f^{n-2} (setup mode)
  const double* mc;  // m^n (setup mode), or the previous h with recon
  const double* mp;  // m^{n-1} (setup mode)
  double* mw;        // m^n written (setup mode with recon)
};

// Raw loads of one site, issued one plane ahead of their use so that the
// memory latency overlaps the previous plane's collision.
template <class L, class T, class TM, int MODE>
struct RawSite {
  static constexpr int Q = L::Q, D1 = L::D + 1;
  static constexpr bool DV = PopDev<T>::value;
  T f0[Q];
  T f1[setup_mode(MODE) ? Q : 1];
  T f2[MODE == SW_DTS_SETUP ? Q : 1];
  float M0[DV ? D1 : 1];  // stored moments of each deviation buffer
  float M1[DV && setup_mode(MODE) ? D1 : 1];
  float M2[DV && MODE == SW_DTS_SETUP ? D1 : 1];
  TM dmv[lift_mode(MODE) ? D1 : 1];
  double hv[MODE == SW_EXPLICIT ? 1 : D1];  // h, or m^n in setup mode
  double mpv[setup_mode(MODE) ? D1 : 1];
};

template <class L, class T, class TM, int MODE>
__device__ __forceinline__ void load_raw(const SweepArgs<T, TM>& A, const SrcPtrs<T>& P, int64_t site,
                                         RawSite<L, T, TM, MODE>& r) {
  constexpr int Q = L::Q, D = L::D;
  constexpr bool DV = PopDev<T>::value;
  const int64_t NS = A.NS;
#pragma unroll
  for (int k = 0; k < Q; ++k) r.f0[k] = P.s0[k * NS + site];
  if constexpr (DV) {
#pragma unroll
    for (int b = 0; b <= D; ++b) r.M0[b] = dev_moments(P.s0, Q, NS)[b * NS + site];
  }
  if constexpr (setup_mode(MODE)) {
    if (A.order >= 1) {
#pragma unroll
      for (int k = 0; k < Q; ++k) r.f1[k] = P.s1[k * NS + site];
      if constexpr (DV) {
#pragma unroll
        for (int b = 0; b <= D; ++b) r.M1[b] = dev_moments(P.s1, Q, NS)[b * NS + site];
      }
    }
    if constexpr (MODE == SW_DTS_SETUP) {
      if (A.order >= 2) {
#pragma unroll
        for (int k = 0; k < Q; ++k) r.f2[k] = P.s2[k * NS + site];
        if constexpr (DV) {
#pragma unroll
          for (int b = 0; b <= D; ++b) r.M2[b] = dev_moments(P.s2, Q, NS)[b * NS + site];
        }
      }
    }
#pragma unroll
    for (int b = 0; b <= D; ++b) r.hv[b] = P.mc[b * NS + site];
    if (A.q == 2) {
#pragma unroll
      for (int b = 0; b <= D; ++b) r.mpv[b] = P.mp[b * NS + site];
    }
  } else if (MODE != SW_EXPLICIT) {
#pragma unroll
    for (int b = 0; b <= D; ++b) r.hv[b] = A.h[b * NS + site];
  }
  if (MODE == SW_DTS_LIFT) {
#pragma unroll
    for (int b = 0; b <= D; ++b) r.dmv[b] = A.dm[b * NS + site];
  }
  // SW_DTS_LIFT_ROWS: dmv is filled by the caller from the inverted rows
}

// From the raw loads: the trial populations (extrapolated in setup mode, with
// the lift of Eq. lift added in lift mode), then reconstruct (Eq.
// macro-reconstruct), form the source (Eq. source-moments) and collide (Eq.
// collision with Eq. feq and Eq. source-distribution).  hout receives h_q
// (setup mode).
template <class L, class T, class TM, int MODE>
__device__ __forceinline__ void collide_raw(const SweepArgs<T, TM>& A, const RawSite<L, T, TM, MODE>& r,
                                            typename CompT<T>::type* f, typename CompT<T>::type* C,
                                            double* hout, double* Mtrial = nullptr, double* mnout = nullptr) {
  // Multiply-adds are fused only within one expression, as written here, not
  // by the optimiser across statements: every kernel that inlines the
  // collision (the tiled sweep, the in-place march) then rounds it the same
  // way and their results agree bit for bit.
#pragma clang fp contract(on)
  using CT = typename CompT<T>::type;
  constexpr int Q = L::Q, D = L::D;
  constexpr bool DV = PopDev<T>::value;
  double h[4] = {0, 0, 0, 0};
  if constexpr (setup_mode(MODE)) {
    // m^n: loaded, or with recon formed here from f^n and the previous step's
    // history term (Eq. macro-reconstruct, the reconstruction the previous
    // step's acceptance left to this sweep)
    double mn[4];
    if (A.recon) {
      double Mn[4] = {0, 0, 0, 0};
      if constexpr (DV) {
#pragma unroll
        for (int b = 0; b <= D; ++b) Mn[b] = (double)r.M0[b];
      } else {
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          const double fk = (double)r.f0[k];
          Mn[0] += fk;
#pragma unroll
          for (int b = 0; b < D; ++b) {
            if (ca<L>(k, b) > 0)
              Mn[1 + b] += fk;
            else if (ca<L>(k, b) < 0)
              Mn[1 + b] -= fk;
          }
        }
      }
#pragma unroll
      for (int b = 0; b <= D; ++b) mn[b] = (Mn[b] + 0.5 * r.hv[b]) * A.inv1pa2_prev;
      if (mnout) {
#pragma unroll
        for (int b = 0; b <= D; ++b) mnout[b] = mn[b];
      }
    } else {
#pragma unroll
      for (int b = 0; b <= D; ++b) mn[b] = r.hv[b];
    }
    // Eq. (bdf2) in FP64, and the extrapolated initial trial (Sec. 3.1)
#pragma unroll
    for (int b = 0; b <= D; ++b)
      h[b] = (A.q == 1) ? mn[b] * A.inv_dt : (4.0 * mn[b] - r.mpv[b]) * A.inv_2dt;
    if constexpr (DV) {
      CT g1[Q], g2[MODE == SW_DTS_SETUP ? Q : 1];
      dev_rebuild<L>(r.f0, r.M0, A.sig, f);
      if (A.order >= 1) dev_rebuild<L>(r.f1, r.M1, A.sig, g1);
      if constexpr (MODE == SW_DTS_SETUP) {
        if (A.order >= 2) dev_rebuild<L>(r.f2, r.M2, A.sig, g2);
      }
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (A.order == 1) {
          f[k] = (CT)2 * f[k] - g1[k];
        } else if constexpr (MODE == SW_DTS_SETUP) {
          if (A.order >= 2) f[k] = (CT)3 * f[k] - (CT)3 * g1[k] + g2[k];
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (A.order == 0) {
          f[k] = (CT)r.f0[k];
        } else if (A.order == 1) {
          f[k] = (CT)2 * (CT)r.f0[k] - (CT)r.f1[k];
        } else if constexpr (MODE == SW_DTS_SETUP) {
          f[k] = (CT)3 * (CT)r.f0[k] - (CT)3 * (CT)r.f1[k] + (CT)r.f2[k];
        }
      }
    }
#pragma unroll
    for (int b = 0; b <= D; ++b) hout[b] = h[b];
  } else {
    if constexpr (DV) {
      dev_rebuild<L>(r.f0, r.M0, A.sig, f);
    } else {
#pragma unroll
      for (int k = 0; k < Q; ++k) f[k] = (CT)r.f0[k];
    }
    if (MODE != SW_EXPLICIT) {
#pragma unroll
      for (int b = 0; b <= D; ++b) h[b] = r.hv[b];
    }
  }
  if (lift_mode(MODE)) {
    const CT d0 = (CT)r.dmv[0];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      CT cu = 0;
#pragma unroll
      for (int b = 0; b < D; ++b) cu += (CT)ca<L>(k, b) * (CT)r.dmv[1 + b];
      f[k] += (CT)L::w(k) * (d0 + (CT)3 * cu);
    }
  }
  // Collision arithmetic type: FP64 temporaries in every mode and storage
  // type; the populations, the trial and the residual stay in the storage's
  // compute type.  In the dual-time modes the inner fixed point amplifies the
  // rounding of the collision's conserved moments by about dt (the slow
  // hydrodynamic modes of I - J have eigenvalues near a_q): FP32 arithmetic
  // there would put an error of ~eps32 dt sqrt(S) on the velocity.  In the
  // explicit map the FP32 weights (1/9, 1/36 and 1/18, 1/36 are not binary
  // fractions) make the equilibrium's mass and momentum differ from the
  // moments it is built from by a fixed relative ~1e-8 of one sign, so each
  // step scales them by 1 + O(1e-8) and the drift grows linearly with the
  // step count (a 2% velocity error after the 6.3e5 steps of 0.1 N^2/nu at
  // N = 1024).
  using KT = double;
  KT M[4] = {0, 0, 0, 0};
  if constexpr (DV) {
    // deviation storage keeps P f itself: combine the stored FP32 moments
    // (P of the rebuild is exactly M; P of the lift E dm is dm)
#pragma unroll
    for (int b = 0; b <= D; ++b) {
      if constexpr (MODE == SW_DTS_SETUP)
        M[b] = (A.order == 0) ? (KT)r.M0[b]
                              : (A.order == 1 ? (KT)2 * (KT)r.M0[b] - (KT)r.M1[b]
                                              : (KT)3 * (KT)r.M0[b] - (KT)3 * (KT)r.M1[b] + (KT)r.M2[b]);
      else if constexpr (MODE == SW_DTS_SETUP1)
        M[b] = (A.order == 0) ? (KT)r.M0[b] : (KT)2 * (KT)r.M0[b] - (KT)r.M1[b];
      else
        M[b] = (KT)r.M0[b];
      if constexpr (lift_mode(MODE)) M[b] += (KT)r.dmv[b];
    }
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      M[0] += (KT)f[k];
#pragma unroll
      for (int b = 0; b < D; ++b)
        if (ca<L>(k, b) != 0) M[1 + b] += (KT)ca<L>(k, b) * (KT)f[k];
    }
  }
  if constexpr (DV) {
    if (Mtrial) {
#pragma unroll
      for (int b = 0; b <= D; ++b) Mtrial[b] = (double)M[b];
    }
  }
  KT m[4], s[4];
  if (MODE == SW_EXPLICIT) {
#pragma unroll
    for (int b = 0; b <= D; ++b) {
      m[b] = M[b];
      s[b] = 0;
    }
  } else {
    // BDF history combination in FP64: s = h - a m is a small difference of
    // two O(m/dt) terms.
#pragma unroll
    for (int b = 0; b <= D; ++b) {
      const double mb = ((double)M[b] + 0.5 * h[b]) * A.inv1pa2;
      m[b] = (KT)mb;
      s[b] = (KT)(h[b] - A.a * mb);
    }
  }
  // Equilibrium (Eq. feq) and source distribution (Eq. source-distribution)
  // split into the parts even and odd under k -> opposite(k), which is what
  // the TRT update (Eq. collision) takes: with cu = c_k.u and cs = c_k.s_u,
  //   feq+ = w (p - 1.5 u.u + 4.5 cu^2),   feq- = 3 w cu,
  //   Phi+ = w (s_0 - 3 u.s_u + 9 cu cs),  Phi- = 3 w cs,
  // so each pair of opposite directions is collided from two dot products.
  KT uu = 0, us = 0;
#pragma unroll
  for (int b = 1; b <= D; ++b) {
    uu += m[b] * m[b];
    us += m[b] * s[b];
  }
  const KT Be = m[0] - (KT)1.5 * uu;
  const KT Ae = s[0] - (KT)3 * us;
  const KT wp = (KT)A.wp, wm = (KT)A.wm;
  const KT hp = (KT)1 - (KT)0.5 * wp, hm = (KT)1 - (KT)0.5 * wm;
  const KT gp = (KT)1 - wp, gm = (KT)1 - wm;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const int kb = L::opp(k);
    if (kb < k) continue;
    const KT wk = (KT)L::w(k);
    const KT fk = (KT)f[k];
    if (kb == k) {
      // rest direction: only even parts
      KT ck = gp * fk + wp * (wk * Be);
      if (MODE != SW_EXPLICIT) ck += hp * (wk * Ae);
      C[k] = (CT)ck;
      continue;
    }
    KT cu = 0, cs = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
      if (ca<L>(k, b) > 0) {
        cu += m[1 + b];
        if (MODE != SW_EXPLICIT) cs += s[1 + b];
      } else if (ca<L>(k, b) < 0) {
        cu -= m[1 + b];
        if (MODE != SW_EXPLICIT) cs -= s[1 + b];
      }
    }
    const KT fkb = (KT)f[kb];
    const KT fp = (KT)0.5 * (fk + fkb), fm = (KT)0.5 * (fk - fkb);
    const KT ep = wk * (Be + (KT)4.5 * cu * cu), em = (KT)3 * wk * cu;
    KT ev = gp * fp + wp * ep;
    KT od = gm * fm + wm * em;
    if (MODE != SW_EXPLICIT) {
      ev += hp * (wk * (Ae + (KT)9 * cu * cs));
      od += hm * ((KT)3 * wk * cs);
    }
    C[k] = (CT)(ev + od);
    C[kb] = (CT)(ev - od);
  }
}

// Minimum waves per SIMD of a sweep instantiation: the D2Q9 FP64 first sweep
// of a step (three history states in flight) needs 266 registers and would
// run one wave per SIMD; bounded to two it spills 40 bytes per lane and is
// 9-12% faster per step at N = 512 and 1024 (3% slower at N = 256, where one
// block per CU runs anyway).
// The D2Q9 FP32 dual-time and lift sweeps need 129-131 registers, one or
// three above the 128 that allow four waves per SIMD; bounded to four.
// The D3Q19 FP32 first sweep (order-1 trial, owned loads issued late) fits
// two waves with 12 bytes of spills per lane: N = 128 march 0.474 -> 0.441 ms
// per step against one wave with the halo prefetch.
template <class L, class T, int MODE, int T1>
__host__ __device__ constexpr int sweep_min_waves() {
  return (L::D == 2 && sizeof(T) == 8 && setup_mode(MODE))                              ? 2
         : (L::D == 2 && sizeof(T) == 4 && (MODE == SW_DTS || MODE == SW_DTS_LIFT)) ? 4
         : (sweep_two_barriers<L, T>() && !setup_mode(MODE) && T1 > 1)                 ? 2
         : (L::D == 3 && sizeof(T) == 4 && MODE == SW_DTS_SETUP1 && T1 > 1)           ? 2
                                                                                       : 1;
}

template <class L, class T, class TM, int NT, int T1, int T2, int MODE>
__global__ __launch_bounds__(NT, (sweep_min_waves<L, T, MODE, T1>())) void k_sweep(SweepArgs<T, TM> A) {
  using CT = typename CompT<T>::type;
  constexpr int Q = L::Q, D = L::D;
  constexpr int NI = T1 * T2;
  static_assert(NI % NT == 0, "tile must be a multiple of the block");
  constexpr int SPT = NI / NT;
  constexpr int NGP = group_count<L>(0), NG0 = group_count<L>(1), NGM = group_count<L>(2);
  constexpr int KPX = local_dir<L>(1), KMX = local_dir<L>(-1);
  static_assert(KPX > 0 && KMX > 0 && local_dir<L>(0) == 0, "lattice layout");

  // post-collision values travel through LDS in the storage type, or FP32
  // for deviation storage (they are full populations there)
  using LT = typename std::conditional<PopDev<T>::value, float, T>::type;
  constexpr bool ROWFFT = (T1 == 1 && MODE != SW_EXPLICIT && NT == T2);
  constexpr bool ROWINV = (MODE == SW_DTS_LIFT_ROWS);
  static_assert(!ROWINV || (ROWFFT && L::D == 2), "inverse rows need 2D tiles spanning whole rows");
  __shared__ cpx<CT> fbuf[ROWFFT ? 4 * T2 : 1];
  // inverted dm rows of the three source planes of a one-plane strip: line
  // 2p packs (dm_0 + i dm_1) of plane p, line 2p+1 holds dm_2; ping-pong
  __shared__ cpx<CT> ibuf[ROWINV ? 12 * T2 : 1];
  constexpr bool TWOBAR = sweep_two_barriers<L, T>();
  constexpr int DP = ring_depth(0, TWOBAR), DZ = ring_depth(1, TWOBAR), DM = ring_depth(2, TWOBAR);
  __shared__ LT ldsP[DP][NGP][NI];
  __shared__ LT ldsZ[DZ][NG0][NI];
  __shared__ LT ldsM[DM][NGM][NI];
  __shared__ double red[NT];

  SrcPtrs<T> P{A.src, nullptr, nullptr, nullptr, nullptr, nullptr};
  T* __restrict__ dst = A.dst;
  if (A.ctl) {
    const uint64_t ph = A.ctl->phase;
    if (!phase_ready(ph, A.n, A.ell)) return;  // uniform for the grid
    const Roles& ro = A.ctl->roles[A.n & 1];
    if (setup_mode(MODE)) {
      P.s0 = A.fb.p[ro.slot_hist[0]];
      P.s1 = A.fb.p[ro.slot_hist[1]];
      P.s2 = A.fb.p[ro.slot_hist[2]];
      P.mc = A.recon ? A.h_prev : A.mb[ro.slot_m[0]];
      P.mp = A.mb[ro.slot_m[1]];
      P.mw = A.mb[ro.slot_m[0]];
    } else {
      P.s0 = A.fb.p[ro.slot_w[(A.ell - 1) & 1]];
    }
    dst = A.fb.p[ro.slot_w[A.ell & 1]];
  }
  if (A.did_run && blockIdx.x == 0 && threadIdx.x == 0) *A.did_run = 1;

  // XCD-aware tile order: blocks b, b+8, b+16, ... run on one XCD, so give
  // them consecutive (spatially adjacent) tiles and let halos hit that L2.
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int lb = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int t2 = lb % A.ntile2;
  const int rr = lb / A.ntile2;
  const int t1 = rr % A.ntile1;
  const int strip = rr / A.ntile1;
  const int b1 = t1 * T1, b2 = t2 * T2, x0 = strip * A.L;
  const int N0 = A.N0, N1 = A.N1, N2 = A.N2;
  const int64_t NS = A.NS;
  const int h1 = (T1 < N1) ? 1 : 0, h2 = (T2 < N2) ? 1 : 0;
  const int S2 = T2 + 2 * h2;
  const int nhalo = 2 * h1 * S2 + 2 * h2 * T1;
  const int tid = threadIdx.x;

  CT fprev[SPT][Q], fcur[SPT][Q];
  // The D3Q19 first sweep with the halo prefetch (one wave per SIMD) keeps
  // the destination plane's trial values, which every thread holds for a
  // whole plane step, in LDS instead of registers (each thread reads and
  // writes only its own entries): FP64 446 -> 370 registers, fewer moves
  // through the accumulation registers; N = 128 FP64 march 0.703 -> 0.689 ms
  // per step
  constexpr bool FPLDS = setup_halo_prefetch<L, T, MODE>() && SPT == 1;
  __shared__ CT fpl[FPLDS ? Q * NT : 1];
  // deviation storage: the trial's moments at the owned sites, for P r
  constexpr int NMT = (PopDev<T>::value && MODE != SW_EXPLICIT) ? D + 1 : 1;
  double mprev[SPT][NMT], mcur[SPT][NMT];
  CT c0prev[SPT], cpx1[SPT], cpx2[SPT], cmxc[SPT], c0c[SPT], cpxc[SPT];
  RawSite<L, T, TM, MODE> raw[SPT];
  double r2 = 0.0;

  // tile-relative coordinates of halo ring site t (rows along p1 first, then
  // columns along p2)
  auto halo_at = [&](int t, int& i1, int& i2) {
    if (t < 2 * h1 * S2) {
      i1 = (t < S2) ? -1 : T1;
      i2 = (t % S2) - h2;
    } else {
      const int u = t - 2 * h1 * S2;
      i2 = (u < T1) ? -1 : T2;
      i1 = u % T1;
    }
  };
  // prefetch the owned sites of the first source plane
  {
    const int xs0 = wrapi(x0 - 1, N0);
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      const int s = tid + j * NT;
      const int i1 = s / T2, i2 = s - (s / T2) * T2;
      load_raw<L, T, TM, MODE>(A, P, ((int64_t)xs0 * N1 + (b1 + i1)) * N2 + (b2 + i2), raw[j]);
    }
  }
  // The D3Q19 first sweep with FP64 and FP16-deviation storage runs one wave
  // per SIMD (history states and the FP64 collision in flight), so nothing
  // would hide the latency of its halo loads: they are issued one plane ahead
  // like the owned ones.  The launcher takes this instantiation only when
  // every thread has at most one halo site (setup_halo_prefetch).  With FP32
  // storage the first sweep fits two waves per SIMD instead, with the owned
  // loads issued late (below).
  constexpr bool HPF = setup_halo_prefetch<L, T, MODE>();
  // D3Q19 FP64 sweeps after the first of a step: the owned sites' loads for
  // the next plane are issued after this plane's halo sites, so that a block
  // fetches its halo rows soon after the neighbouring blocks fetched the same
  // rows as owned ones (more of them still in L2): N = 128 march 0.760 ->
  // 0.745 ms per step (FP32 sweeps after the first gain nothing).  The FP32
  // first sweep issues them late too: no loads in flight during the
  // collision, which brings it to 256 registers and two waves per SIMD
  constexpr bool LATE = late_owned_prefetch<L, T, MODE>();
  const bool hown = HPF && tid < nhalo;
  int hi1 = 0, hi2 = 0;
  RawSite<L, T, TM, MODE> hraw;
  if constexpr (HPF) {
    if (hown) {
      halo_at(tid, hi1, hi2);
      const int xs0 = wrapi(x0 - 1, N0);
      load_raw<L, T, TM, MODE>(A, P, ((int64_t)xs0 * N1 + wrapi(b1 + hi1, N1)) * N2 + wrapi(b2 + hi2, N2), hraw);
    }
  }
  // SW_DTS_LIFT_ROWS: inverse transform along y of the band spectrum rows of
  // the source planes x0-1, x0, x0+1 (Eq. fft-convention, the 1/N_Omega is in
  // the spectrum): the conjugate-symmetric extension of each field's half
  // band, fields 0 and 1 packed in one complex line, field 2 in a second;
  // the same arithmetic as the separate inverse row pass
  const cpx<CT>* dmr = nullptr;
  if constexpr (ROWINV) {
    const int NB = A.NBr;
    const int64_t FS = (int64_t)N0 * NB;
    for (int i = tid; i < 3 * T2; i += NT) {
      const int p = i / T2, jj = i - p * T2;
      const int64_t o = (int64_t)wrapi(x0 - 1 + p, N0) * NB;
      cpx<CT> a0 = {0, 0}, a1 = {0, 0}, a2 = {0, 0};
      if (jj < NB) {
        a0 = A.spec_in[o + jj];
        a1 = A.spec_in[FS + o + jj];
        a2 = A.spec_in[2 * FS + o + jj];
        if (jj == 0) {
          a0.y = 0;
          a1.y = 0;
          a2.y = 0;
        }
      } else if (T2 - jj < NB) {
        const int jm = T2 - jj;
        a0 = A.spec_in[o + jm];
        a1 = A.spec_in[FS + o + jm];
        a2 = A.spec_in[2 * FS + o + jm];
        a0.y = -a0.y;
        a1.y = -a1.y;
        a2.y = -a2.y;
      }
      ibuf[(2 * p) * T2 + jj] = {a0.x - a1.y, a0.y + a1.x};
      ibuf[(2 * p + 1) * T2 + jj] = a2;
    }
    __syncthreads();
    dmr = lds_fft<CT>(ibuf, ibuf + 6 * T2, A.lgr, 6, +1, A.twr);
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      const int i2 = tid + j * NT;
      raw[j].dmv[0] = (TM)dmr[i2].x;
      raw[j].dmv[1] = (TM)dmr[i2].y;
      raw[j].dmv[2] = (TM)dmr[T2 + i2].x;
    }
  }

  for (int it = 0; it < A.L + 2; ++it) {
    const int xs = wrapi(x0 - 1 + it, N0);
    const bool wP = it <= A.L - 1;             // dest plane it+1 is finalised later
    const bool wZ = it >= 1 && it <= A.L;      // dest plane it
    const bool wM = it >= 2;                   // dest plane it-1
    // slots keyed by the destination plane's index modulo the ring depth
    const int sP = (it + 1) % DP, sZ = it % DZ, sM = (it + DM - 1) % DM;

    // ---- owned interior sources --------------------------------------------
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      const int s = tid + j * NT;
      const int i1 = s / T2, i2 = s - (s / T2) * T2;
      // next plane's loads: issued before this plane's collision (a full
      // plane step to land), or with the halo prefetch after it (the
      // registers of this plane's loads are free again; half a plane step)
      RawSite<L, T, TM, MODE> cur;
      auto load_next = [&](RawSite<L, T, TM, MODE>& dstr) {
        if (it + 1 < A.L + 2) {
          const int xn = wrapi(x0 + it, N0);
          load_raw<L, T, TM, MODE>(A, P, ((int64_t)xn * N1 + (b1 + i1)) * N2 + (b2 + i2), dstr);
          if constexpr (ROWINV) {
            const cpx<CT>* row = dmr + 2 * (it + 1) * T2;
            dstr.dmv[0] = (TM)row[i2].x;
            dstr.dmv[1] = (TM)row[i2].y;
            dstr.dmv[2] = (TM)row[T2 + i2].x;
          }
        }
      };
      CT C[Q];
      double hs[4], mns[4];
      if constexpr (HPF && sizeof(T) == 8) {
        // FP64: the next plane's owned loads before this plane's collision, a
        // full plane step to land (the registers allow a second set since the
        // destination plane's trial moved to LDS: 418 registers; N = 128
        // march 0.686 -> 0.680 ms per step)
        cur = raw[j];
        load_next(raw[j]);
        __builtin_amdgcn_sched_barrier(0);
        collide_raw<L, T, TM, MODE>(A, cur, fcur[j], C, hs, mcur[j], mns);
      } else if constexpr (HPF) {
        collide_raw<L, T, TM, MODE>(A, raw[j], fcur[j], C, hs, mcur[j], mns);
        // keep the next plane's loads below the collision that frees their
        // registers (the scheduler would otherwise hoist them)
        __builtin_amdgcn_sched_barrier(0);
        load_next(raw[j]);
      } else if constexpr (LATE) {
        collide_raw<L, T, TM, MODE>(A, raw[j], fcur[j], C, hs, mcur[j], mns);
      } else {
        cur = raw[j];
        load_next(raw[j]);
        collide_raw<L, T, TM, MODE>(A, cur, fcur[j], C, hs, mcur[j], mns);
      }
      if (setup_mode(MODE) && it >= 1 && it <= A.L) {
        const int64_t site = ((int64_t)xs * N1 + (b1 + i1)) * N2 + (b2 + i2);
#pragma unroll
        for (int bb = 0; bb <= D; ++bb) A.h[bb * NS + site] = hs[bb];
        if (A.recon) {
#pragma unroll
          for (int bb = 0; bb <= D; ++bb) P.mw[bb * NS + site] = mns[bb];
        }
      }
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (is_local<L>(k)) continue;
        int j1 = i1 + L::c1(k), j2 = i2 + L::c2(k);
        bool ok = true;
        if (h1) ok = ok && (j1 >= 0 && j1 < T1); else j1 = (j1 + T1) % T1;
        if (h2) ok = ok && (j2 >= 0 && j2 < T2); else j2 = (j2 + T2) % T2;
        if (!ok) continue;
        const int di = j1 * T2 + j2;
        const int g = xgroup<L>(k), gi = group_index<L>(k);
        if (g == 0) {
          if (wP) ldsP[sP][gi][di] = (LT)C[k];
        } else if (g == 1) {
          if (wZ) ldsZ[sZ][gi][di] = (LT)C[k];
        } else {
          if (wM) ldsM[sM][gi][di] = (LT)C[k];
        }
      }
      c0c[j] = C[0];
      cpxc[j] = C[KPX];
      cmxc[j] = C[KMX];
    }
    // ---- halo ring sources (only along axes the tile does not span) -------
    auto push_halo = [&](int i1, int i2, const CT* C) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (is_local<L>(k)) continue;
        int j1 = i1 + L::c1(k), j2 = i2 + L::c2(k);
        bool ok = true;
        if (h1) ok = ok && (j1 >= 0 && j1 < T1); else j1 = (j1 + T1) % T1;
        if (h2) ok = ok && (j2 >= 0 && j2 < T2); else j2 = (j2 + T2) % T2;
        if (!ok) continue;
        const int di = j1 * T2 + j2;
        const int g = xgroup<L>(k), gi = group_index<L>(k);
        if (g == 0) {
          if (wP) ldsP[sP][gi][di] = (LT)C[k];
        } else if (g == 1) {
          if (wZ) ldsZ[sZ][gi][di] = (LT)C[k];
        } else {
          if (wM) ldsM[sM][gi][di] = (LT)C[k];
        }
      }
    };
    if constexpr (HPF) {
      if (hown) {
        CT f[Q], C[Q];
        double hs[4];
        collide_raw<L, T, TM, MODE>(A, hraw, f, C, hs);
        __builtin_amdgcn_sched_barrier(0);
        if (it + 1 < A.L + 2) {
          const int xn = wrapi(x0 + it, N0);
          load_raw<L, T, TM, MODE>(A, P, ((int64_t)xn * N1 + wrapi(b1 + hi1, N1)) * N2 + wrapi(b2 + hi2, N2), hraw);
        }
        push_halo(hi1, hi2, C);
      }
    } else {
      for (int t = tid; t < nhalo; t += NT) {
        int i1, i2;
        halo_at(t, i1, i2);
        const int p1 = wrapi(b1 + i1, N1), p2 = wrapi(b2 + i2, N2);
        RawSite<L, T, TM, MODE> hr;
        load_raw<L, T, TM, MODE>(A, P, ((int64_t)xs * N1 + p1) * N2 + p2, hr);
        CT f[Q], C[Q];
        double hs[4];
        collide_raw<L, T, TM, MODE>(A, hr, f, C, hs);
        push_halo(i1, i2, C);
      }
    }
    if constexpr (LATE) {
      if (it + 1 < A.L + 2) {
        const int xn = wrapi(x0 + it, N0);
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
          const int s = tid + j * NT;
          const int i1 = s / T2, i2 = s - (s / T2) * T2;
          __builtin_amdgcn_sched_barrier(0);
          load_raw<L, T, TM, MODE>(A, P, ((int64_t)xn * N1 + (b1 + i1)) * N2 + (b2 + i2), raw[j]);
        }
      }
    }
    __syncthreads();

    // ---- finalise destination plane it-1 ----------------------------------
    if (it >= 2) {
      const int id = it - 1;
      const int xd = wrapi(x0 + id - 1, N0);
      const int rP = id % DP, rZ = id % DZ, rM = id % DM;
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        const int s = tid + j * NT;
        const int i1 = s / T2, i2 = s - (s / T2) * T2;
        const int64_t site = ((int64_t)xd * N1 + (b1 + i1)) * N2 + (b2 + i2);
        CT pr[4] = {0, 0, 0, 0};
        CT vv[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          if (k == 0) {
            vv[k] = c0prev[j];
          } else if (k == KPX) {
            vv[k] = cpx2[j];
          } else if (k == KMX) {
            vv[k] = cmxc[j];
          } else {
            const int g = xgroup<L>(k), gi = group_index<L>(k);
            vv[k] = (g == 0) ? (CT)ldsP[rP][gi][s] : ((g == 1) ? (CT)ldsZ[rZ][gi][s] : (CT)ldsM[rM][gi][s]);
          }
        }
        if constexpr (L::D == 2) {
          if (A.walls) cavity_rows<CT>(vv, xd, b2 + i2, N0, N2, (CT)A.ulid);
        }
        float Mq[PopDev<T>::value ? D + 1 : 1];
        if constexpr (PopDev<T>::value) {
          // store (g, M); the residual is then taken against the stored
          // output, so that the iterate of the stored iteration is what it
          // measures (and its fixed point has r = 0)
          T gq[Q];
          dev_split<L, typename std::conditional<MODE == SW_EXPLICIT, float, double>::type>(vv, A.isig, gq, Mq);
#pragma unroll
          for (int k = 0; k < Q; ++k) __builtin_nontemporal_store(gq[k], &dst[k * NS + site]);
          float* dM = dev_moments(dst, Q, NS);
#pragma unroll
          for (int bb = 0; bb <= D; ++bb) __builtin_nontemporal_store(Mq[bb], &dM[bb * NS + site]);
          if (MODE != SW_EXPLICIT) dev_rebuild<L>(gq, Mq, A.sig, vv);
        }
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          const CT v = vv[k];
          if constexpr (!PopDev<T>::value) __builtin_nontemporal_store((T)v, &dst[k * NS + site]);
          if (MODE != SW_EXPLICIT) {
            const CT r = v - (FPLDS ? fpl[k * NT + tid] : fprev[j][k]);
            if (A.rout) __builtin_nontemporal_store((TM)r, &A.rout[k * NS + site]);
            pr[0] += r;
#pragma unroll
            for (int bb = 0; bb < D; ++bb)
              if (ca<L>(k, bb) != 0) pr[1 + bb] += (CT)ca<L>(k, bb) * r;
            r2 += (double)r * (double)r;
          }
        }
        if constexpr (PopDev<T>::value && MODE != SW_EXPLICIT) {
          // P r exactly: the stored output moments minus the trial's.  The
          // rebuilt populations each carry FP32 rounding of about eps32 |f|,
          // so their differences would put a floor of that size under P r,
          // which the shadow solve amplifies by up to dt at small k.
#pragma unroll
          for (int bb = 0; bb <= D; ++bb) pr[bb] = (CT)((double)Mq[bb] - mprev[j][bb]);
        }
        if (MODE != SW_EXPLICIT) {
          if (ROWFFT && A.fuse_rows) {
            // the row of P r (fields 0 and 1 packed in one complex line, field 2 in a second)
            fbuf[i2] = {pr[0], pr[1]};
            fbuf[T2 + i2] = {pr[2], (CT)0};
          } else if (!A.rout && !A.skip_pr) {
#pragma unroll
            for (int bb = 0; bb <= D; ++bb) __builtin_nontemporal_store((TM)pr[bb], &A.Pr[bb * NS + site]);
          }
        }
      }
      if constexpr (ROWFFT) {
        if (A.fuse_rows) {
          // forward transform along y of this plane's P r, band j <= N_y/4
          // kept (Eq. fft-convention, shadow-mask); unpack the packed pair
          __syncthreads();
          const cpx<CT>* out = lds_fft<CT>(fbuf, fbuf + 2 * T2, A.lgr, 2, -1, A.twr);
          const int NB = A.NBr;
          const int64_t FS = (int64_t)N0 * NB;
          for (int j = tid; j < NB; j += NT) {
            const cpx<CT> z = out[j];
            const cpx<CT> zc = out[(T2 - j) & (T2 - 1)];
            const int64_t o = (int64_t)xd * NB + j;
            A.spec[o] = {(CT)0.5 * (z.x + zc.x), (CT)0.5 * (z.y - zc.y)};
            A.spec[FS + o] = {(CT)0.5 * (z.y + zc.y), (CT)0.5 * (zc.x - z.x)};
            A.spec[2 * FS + o] = out[T2 + j];
          }
          __syncthreads();  // fbuf is refilled by the next plane
        }
      }
    }
    if constexpr (TWOBAR) __syncthreads();  // the rings' slots are refilled next step
    // ---- roll registers ------------------------------------------------------
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if constexpr (FPLDS)
          fpl[k * NT + tid] = fcur[j][k];
        else
          fprev[j][k] = fcur[j][k];
      }
#pragma unroll
      for (int b = 0; b < NMT; ++b) mprev[j][b] = mcur[j][b];
      c0prev[j] = c0c[j];
      cpx2[j] = cpx1[j];
      cpx1[j] = cpxc[j];
    }
  }

  if (MODE != SW_EXPLICIT) {
    // FP64 block reduction of sum r^2 (wave shuffles, then LDS across waves;
    // blocks narrower than a wavefront sum serially).
    double acc = 0.0;
    if (NT >= 64) {
      double v = r2;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if ((tid & 63) == 0) red[tid >> 6] = v;
      __syncthreads();
      if (tid == 0)
        for (int wv = 0; wv < NT / 64; ++wv) acc += red[wv];
    } else {
      red[tid] = r2;
      __syncthreads();
      if (tid == 0)
        for (int i = 0; i < NT; ++i) acc += red[i];
    }
    if (tid == 0) A.partials[blockIdx.x] = acc;
  }
}

// Large sweep grids: one block first folds the partials into partials_out[0]
// (fixed order), so that the decision kernel's blocks each read one value.
template <int UNUSED = 0>
__global__ __launch_bounds__(256) void k_presum(const double* __restrict__ partials, int nparts,
                                                double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) acc += partials[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace msc
