// Element-wise and control kernels around the sweep: BDF setup and trial
// extrapolation, the device-side acceptance test of Algorithm 1, the
// accepted-state reconstruction, initialisation, conversions and the index
// tables.
#pragma once

#include "msc_sweep.h"

namespace msc {

// ---------------------------------------------------------------- setup --
// Eq. (bdf2): h_1 = m^n/dt, h_2 = (4 m^n - m^{n-1})/(2 dt) in FP64, and the
// initial trial of the inner solve by population-history extrapolation
// (Sec. 3.1): f^n, then 2 f^n - f^{n-1}, then 3 f^n - 3 f^{n-1} + f^{n-2}.
template <class T>
struct SetupArgs {
  const DevCtl* ctl;
  int n;
  FBufs<T> fb;
  double* mb[3];
  double* h;
  int64_t NS;
  int D1;      // d + 1
  int Q;
  int q;       // BDF order of this step
  int order;   // extrapolation order 0, 1, 2
  double dt;
};

template <class T>
__global__ void k_setup(SetupArgs<T> A) {
  using CT = typename CompT<T>::type;
  const uint64_t ph = A.ctl->phase;
  if (!phase_ready(ph, A.n, 1)) return;
  const T* f0 = A.fb.p[A.ctl->slot_hist[0]];
  const T* f1 = A.fb.p[A.ctl->slot_hist[1]];
  const T* f2 = A.fb.p[A.ctl->slot_hist[2]];
  T* tr = A.fb.p[A.ctl->slot_w[0]];
  const double* mc = A.mb[A.ctl->slot_m[0]];
  const double* mp = A.mb[A.ctl->slot_m[1]];
  const int64_t NS = A.NS;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
    for (int b = 0; b < A.D1; ++b) {
      const double m0 = mc[b * NS + s];
      A.h[b * NS + s] = (A.q == 1) ? m0 / A.dt : (4.0 * m0 - mp[b * NS + s]) / (2.0 * A.dt);
    }
    for (int k = 0; k < A.Q; ++k) {
      const int64_t i = (int64_t)k * NS + s;
      CT v;
      if (A.order == 0)
        v = (CT)f0[i];
      else if (A.order == 1)
        v = (CT)2 * (CT)f0[i] - (CT)f1[i];
      else
        v = (CT)3 * (CT)f0[i] - (CT)3 * (CT)f1[i] + (CT)f2[i];
      tr[i] = (T)v;
    }
  }
}

// ---------------------------------------------------------- acceptance --
// One block: FP64 sum of the sweep's block partials in a fixed order, the
// raw-residual RMS (Eq. residual), and the acceptance test of Algorithm 1:
// accept when ell >= n_min and the residual is finite and below eps (or at
// the scheduled count in replay mode); a non-finite residual fails the step
// (Sec. 4.1); reaching K_max fails it as nonconvergent.  On acceptance the
// population and moment history slots rotate (Sec. 3.1, last paragraph).
struct FinishArgs {
  DevCtl* ctl;
  int n, ell;
  const double* partials;
  int nparts;
  double inv_count;  // 1/(Q N_sites)
  double eps;
  int nmin, kmax, q, mcap;
  const int32_t* sched;  // accept count of step n at sched[n - stat_base], or null
  double* Rhist;         // residual history of the current step
  StepStat* stats;       // stats[n - stat_base]
  int stat_base;
};

template <int UNUSED = 0>
__global__ __launch_bounds__(256) void k_finish(FinishArgs A) {
  __shared__ double red[256];
  const uint64_t ph = A.ctl->phase;
  if (!phase_ready(ph, A.n, A.ell)) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < A.nparts; i += 256) acc += A.partials[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double R = sqrt(red[0] * A.inv_count);
  const int ell = A.ell;
  A.Rhist[ell - 1] = R;
  const bool fin = isfinite(R);
  const bool pass = A.sched ? (ell == A.sched[A.n - A.stat_base]) : (ell >= A.nmin && fin && R < A.eps);
  DevCtl* c = A.ctl;
  int fail = 0;
  if (!pass) {
    if (!fin)
      fail = 6;  // MSC_ERR_NONFINITE
    else if (ell >= A.kmax)
      fail = 5;  // MSC_ERR_NONCONVERGED
  }
  if (pass || fail) {
    StepStat& st = A.stats[A.n - A.stat_base];
    st.q = A.q;
    st.iters = ell;
    st.R_first = A.Rhist[0];
    st.R_final = R;
    double rho = __builtin_nan("");
    if (ell >= 3) {
      const int mr = (A.mcap < ell - 1) ? A.mcap : ell - 1;
      double sl = 0.0;
      for (int j = ell - mr + 1; j <= ell; ++j) sl += log(A.Rhist[j - 1] / A.Rhist[j - 2]);
      rho = exp(sl / mr);
    }
    st.rho_obs = rho;
    st.converged = pass ? 1 : 0;
    st.fail = fail;
  }
  if (pass) {
    const int accb = c->slot_w[ell & 1];
    const int old2 = c->slot_hist[2];
    c->slot_hist[2] = c->slot_hist[1];
    c->slot_hist[1] = c->slot_hist[0];
    c->slot_hist[0] = accb;
    c->slot_w[ell & 1] = old2;
    const int mc = c->slot_m[0], mp = c->slot_m[1], ms = c->slot_m[2];
    c->slot_m[0] = ms;  // filled with m^{n+1} by k_accept
    c->slot_m[1] = mc;
    c->slot_m[2] = mp;
    c->phase = make_phase(A.n, ell, PH_ACCEPTED);
  } else if (fail) {
    c->fail_code = fail;
    c->phase = make_phase(A.n, ell, PH_FAILED);
  } else {
    c->phase = make_phase(A.n, ell, PH_RUNNING);
  }
}

// m^{n+1} = R_{q,h}(f_T) with the step's unchanged history (Alg. 1 accept,
// Eq. macro-reconstruct), from the accepted populations (now f^n slot).
template <class L, class T>
struct AcceptArgs {
  const DevCtl* ctl;
  int n, ell;
  FBufs<T> fb;
  double* mb[3];
  const double* h;
  int64_t NS;
  double a;
};

template <class L, class T>
__global__ void k_accept(AcceptArgs<L, T> A) {
  const uint64_t ph = A.ctl->phase;
  if (!phase_accepted(ph, A.n, A.ell)) return;
  const T* f = A.fb.p[A.ctl->slot_hist[0]];
  double* m = A.mb[A.ctl->slot_m[0]];
  const int64_t NS = A.NS;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
    double M[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      const double v = (double)f[(int64_t)k * NS + s];
      M[0] += v;
#pragma unroll
      for (int b = 0; b < L::D; ++b)
        if (ca<L>(k, b) != 0) M[1 + b] += (double)ca<L>(k, b) * v;
    }
#pragma unroll
    for (int b = 0; b <= L::D; ++b) m[b * NS + s] = (M[b] + A.h[b * NS + s] / 2.0) / (1.0 + A.a / 2.0);
  }
}

// ------------------------------------------------------ initialisation --
// f = feq(p, u) (Eq. feq) from FP64 fields; the initial state of Sec. 4.1.
template <class L, class T>
__global__ void k_init_feq(const double* __restrict__ p, const double* __restrict__ u, T* __restrict__ f,
                           int64_t NS) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
    double m[4] = {p[s], 0, 0, 0};
    double uu = 0;
#pragma unroll
    for (int b = 0; b < L::D; ++b) {
      m[1 + b] = u[b * NS + s];
      uu += m[1 + b] * m[1 + b];
    }
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      double cu = 0;
#pragma unroll
      for (int b = 0; b < L::D; ++b)
        if (ca<L>(k, b) != 0) cu += (double)ca<L>(k, b) * m[1 + b];
      const double cs2 = 1.0 / 3.0;
      f[(int64_t)k * NS + s] =
          (T)(L::w(k) * (m[0] + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2)));
    }
  }
}

// P f in FP64 (Eq. moments), written to m.
template <class L, class T>
__global__ void k_moments(const T* __restrict__ f, double* __restrict__ m, int64_t NS) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
    double M[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      const double v = (double)f[(int64_t)k * NS + s];
      M[0] += v;
#pragma unroll
      for (int b = 0; b < L::D; ++b)
        if (ca<L>(k, b) != 0) M[1 + b] += (double)ca<L>(k, b) * v;
    }
#pragma unroll
    for (int b = 0; b <= L::D; ++b) m[b * NS + s] = M[b];
  }
}

// out = fT + E dm (Eq. lift, Eq. shadow-update) with the same arithmetic the
// sweep applies when it fuses the lift into its load.
template <class L, class T, class TM>
__global__ void k_lift(const T* __restrict__ fT, const TM* __restrict__ dm, T* __restrict__ out,
                       int64_t NS) {
  using CT = typename CompT<T>::type;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
    const CT d0 = (CT)dm[s];
    CT du[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < L::D; ++b) du[b] = (CT)dm[(1 + b) * NS + s];
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      CT cu = 0;
#pragma unroll
      for (int b = 0; b < L::D; ++b) cu += (CT)ca<L>(k, b) * du[b];
      out[(int64_t)k * NS + s] = (T)((CT)fT[(int64_t)k * NS + s] + (CT)L::w(k) * (d0 + (CT)3 * cu));
    }
  }
}

template <class A, class B>
__global__ void k_convert(const A* __restrict__ in, B* __restrict__ out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = (B)in[i];
}

// Per-block partial sums of v^2 (a non-finite entry makes the sum non-finite).
template <class T>
__global__ __launch_bounds__(256) void k_sumsq(const T* __restrict__ v, int64_t n, double* partials) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double x = (double)v[i];
    acc += x * x;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// ------------------------------------------------------------- tables --
// Signed wavenumber index of Eq. (wavenumbers) and the integer mask test of
// Eq. (shadow-mask); the transform kernels use these same functions.
__host__ __device__ inline int signed_index(int j, int N) { return (j <= N / 2) ? j : j - N; }
__host__ __device__ inline bool in_band(int sj, int N) { return 4 * (sj < 0 ? -sj : sj) <= N; }

// Push targets with the sweep's own index arithmetic: the destination of
// direction k from site (x, p1, p2) is (x + cx, p1 + c1, p2 + c2) wrapped.
template <class L>
__global__ void k_tables(int N0, int N1, int N2, int32_t* nbr, uint8_t* mask, int32_t* sidx) {
  const int64_t NS = (int64_t)N0 * N1 * N2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
    const int p2 = (int)(s % N2);
    const int p1 = (int)((s / N2) % N1);
    const int x = (int)(s / ((int64_t)N1 * N2));
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      const int xd = wrapi(x + L::cx(k), N0);
      const int d1 = wrapi(p1 + L::c1(k), N1);
      const int d2 = wrapi(p2 + L::c2(k), N2);
      nbr[(int64_t)k * NS + s] = (int32_t)(((int64_t)xd * N1 + d1) * N2 + d2);
    }
    bool keep = in_band(signed_index(x, N0), N0) && in_band(signed_index(p2, N2), N2);
    if (L::D == 3) keep = keep && in_band(signed_index(p1, N1), N1);
    mask[s] = keep ? 1 : 0;
  }
  if (blockIdx.x == 0) {
    const int Ns[3] = {N0, (L::D == 3) ? N1 : N2, N2};
    int off = 0;
    for (int ax = 0; ax < L::D; ++ax) {
      for (int j = threadIdx.x; j < Ns[ax]; j += blockDim.x) sidx[off + j] = signed_index(j, Ns[ax]);
      off += Ns[ax];
    }
  }
}

}  // namespace msc
