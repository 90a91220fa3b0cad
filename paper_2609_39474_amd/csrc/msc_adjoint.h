// Discrete adjoint of the dual-time march: the transpose of the unrolled
// computation of each physical step at its recorded inner count.  The step's
// inner iterates are recomputed from its checkpoint (kept in the storage
// precision) in FP64, and the adjoint runs in FP64, whatever the storage
// precision: the corrected iteration's transpose cancels terms amplified by
// the shadow solve (up to 1/a_q at low wavenumbers), so it is linearised at
// FP64 iterates.
//
// Stages (transposes of the forward stages):
//   sweep: push streaming transposes to a pull, mu_k(x) = lamT_k(x + c_k);
//     the TRT collision with source, Eq. (collision), transposes sitewise
//     through the even/odd projections, the derivatives of Eq. (feq) and Eq.
//     (source-distribution) in m and s, s = h - a m and
//     m = (P f + h/2)/(1 + a/2) (Eq. macro-reconstruct);
//   correction: f' = f_T + E Sh P (f_T - f) with Sh the shadow multiplier;
//     its transpose uses E^T, Sh^T = F^{-1}[chi H^{-H} F[.]] (same transform
//     kernels, conjugate-transposed Schur solve) and P^T;
//   acceptance m^{n+1} = (P f_T + h/2)/(1 + a/2), the rotation of the
//   histories, the BDF history term h_q (Eq. bdf2) and the trial
//   extrapolation.
#pragma once

#include "msc_fft.h"

namespace msc {

struct AdjGeom {
  int N0, N1, N2;
  int64_t NS;
};

__device__ __forceinline__ int64_t adj_neighbor(const AdjGeom& g, int64_t s, int cx, int c1, int c2) {
  const int p2 = (int)(s % g.N2);
  const int p1 = (int)((s / g.N2) % g.N1);
  const int x = (int)(s / ((int64_t)g.N1 * g.N2));
  return ((int64_t)wrapi(x + cx, g.N0) * g.N1 + wrapi(p1 + c1, g.N1)) * g.N2 + wrapi(p2 + c2, g.N2);
}

// LF = carry + (dT/df)^T LT at the forward trial f; lam_h += (dT/dh)^T LT.
template <class L, class T>
__global__ __launch_bounds__(256) void k_adj_sweep(AdjGeom g, const T* __restrict__ f, const double* __restrict__ h,
                                                   const double* __restrict__ LT, const double* __restrict__ carry,
                                                   double* __restrict__ LF, double* __restrict__ lam_h, double a,
                                                   double wp, double wm) {
  constexpr int Q = L::Q, D = L::D;
  const double cs2 = 1.0 / 3.0;
  const double inv1pa2 = 1.0 / (1.0 + a / 2.0);  // as the forward sweep forms m
  const int64_t NS = g.NS;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < NS; x += stride) {
    double fs[Q], mu[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      fs[k] = (double)f[(int64_t)k * NS + x];
      mu[k] = LT[(int64_t)k * NS + adj_neighbor(g, x, L::cx(k), L::c1(k), L::c2(k))];
    }
    double M[4] = {0, 0, 0, 0}, m[4], s[4], hh[4];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      M[0] += fs[k];
#pragma unroll
      for (int b = 0; b < D; ++b) M[1 + b] += (double)ca<L>(k, b) * fs[k];
    }
#pragma unroll
    for (int b = 0; b <= D; ++b) {
      hh[b] = h[b * NS + x];
      m[b] = (M[b] + 0.5 * hh[b]) * inv1pa2;
      s[b] = hh[b] - a * m[b];
    }
    double lf[Q], gk[Q], pk[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int kb = L::opp(k);
      const double np = 0.5 * (mu[k] + mu[kb]), nm = 0.5 * (mu[k] - mu[kb]);
      lf[k] = mu[k] - wp * np - wm * nm;
      gk[k] = wp * np + wm * nm;
      pk[k] = (1.0 - wp / 2.0) * np + (1.0 - wm / 2.0) * nm;
    }
    double lm[4] = {0, 0, 0, 0}, ls[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      double cu = 0.0, cs = 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        cu += (double)ca<L>(k, b) * m[1 + b];
        cs += (double)ca<L>(k, b) * s[1 + b];
      }
      const double wk = L::w(k);
      lm[0] += wk * gk[k];
      ls[0] += wk * pk[k];
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const double c = (double)ca<L>(k, b);
        lm[1 + b] += wk * (c / cs2 + cu * c / (cs2 * cs2) - m[1 + b] / cs2) * gk[k];
        lm[1 + b] += wk * (-s[1 + b] / cs2 + c * cs / (cs2 * cs2)) * pk[k];
        ls[1 + b] += wk * ((c - m[1 + b]) / cs2 + cu * c / (cs2 * cs2)) * pk[k];
      }
    }
    double lmt[4];
#pragma unroll
    for (int b = 0; b <= D; ++b) {
      lmt[b] = lm[b] - a * ls[b];
      lam_h[b * NS + x] += ls[b] + lmt[b] * 0.5 / (1.0 + a / 2.0);
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      double v = lmt[0];
#pragma unroll
      for (int b = 0; b < D; ++b) v += (double)ca<L>(k, b) * lmt[1 + b];
      LF[(int64_t)k * NS + x] = (carry ? carry[(int64_t)k * NS + x] : 0.0) + lf[k] + v / (1.0 + a / 2.0);
    }
  }
}

// y = E^T Lambda, written in the transform input type.
template <class L, class TM>
__global__ void k_adj_Et(int64_t NS, const double* __restrict__ Lam, TM* __restrict__ y) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < NS; x += stride) {
    double acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      const double v = Lam[(int64_t)k * NS + x];
      acc[0] += L::w(k) * v;
#pragma unroll
      for (int b = 0; b < L::D; ++b) acc[1 + b] += 3.0 * L::w(k) * (double)ca<L>(k, b) * v;
    }
#pragma unroll
    for (int b = 0; b <= L::D; ++b) y[b * NS + x] = (TM)acc[b];
  }
}

// v = P^T z; LT = Lambda + v; carry = -v.
template <class L, class TM>
__global__ void k_adj_lift(int64_t NS, const TM* __restrict__ z, const double* __restrict__ Lam,
                           double* __restrict__ LT, double* __restrict__ carry) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < NS; x += stride) {
    double zz[4];
#pragma unroll
    for (int b = 0; b <= L::D; ++b) zz[b] = (double)z[b * NS + x];
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      double v = zz[0];
#pragma unroll
      for (int b = 0; b < L::D; ++b) v += (double)ca<L>(k, b) * zz[1 + b];
      LT[(int64_t)k * NS + x] = Lam[(int64_t)k * NS + x] + v;
      carry[(int64_t)k * NS + x] = -v;
    }
  }
}

// Seed of one step's backward pass from the adjoint of the new state:
// LT = lam_f0' + P^T lam_m0' / (1 + a/2); lam_h = lam_m0' (1/2)/(1 + a/2).
template <class L>
__global__ void k_adj_seed(int64_t NS, const double* __restrict__ lf0, const double* __restrict__ lm0, double a,
                           double* __restrict__ LT, double* __restrict__ lam_h) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < NS; x += stride) {
    double lm[4];
#pragma unroll
    for (int b = 0; b <= L::D; ++b) {
      lm[b] = lm0[b * NS + x];
      lam_h[b * NS + x] = lm[b] * 0.5 / (1.0 + a / 2.0);
    }
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      double v = lm[0];
#pragma unroll
      for (int b = 0; b < L::D; ++b) v += (double)ca<L>(k, b) * lm[1 + b];
      LT[(int64_t)k * NS + x] = lf0[(int64_t)k * NS + x] + v / (1.0 + a / 2.0);
    }
  }
}

// Adjoint of the rotation, trial extrapolation and h_q: from the adjoint of
// the new state (lf1', lf2', lm1') and of the trial (Lam1) and h (lam_h),
// the adjoint of the old state (f^n, f^{n-1}, f^{n-2}, m^n, m^{n-1}).
struct AdjSetupArgs {
  int64_t NS;
  int Q, D1, order, q;
  double dt;
  const double* lf1n;  // adjoint of f^{n-1}' (= old f^n)
  const double* lf2n;  // adjoint of f^{n-2}' (= old f^{n-1})
  const double* lm1n;  // adjoint of m^{n-1}' (= old m^n)
  const double* Lam1;  // adjoint of the trial f^(1)
  const double* lam_h;
  double* of0;
  double* of1;
  double* of2;
  double* om0;
  double* om1;
};

template <int UNUSED = 0>
__global__ void k_adj_setup(AdjSetupArgs A) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t NQ = (int64_t)A.Q * A.NS, NM = (int64_t)A.D1 * A.NS;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NQ; i += stride) {
    const double l = A.Lam1[i];
    double a0 = A.lf1n[i], a1 = A.lf2n[i], a2 = 0.0;
    if (A.order == 0) {
      a0 += l;
    } else if (A.order == 1) {
      a0 += 2.0 * l;
      a1 -= l;
    } else {
      a0 += 3.0 * l;
      a1 -= 3.0 * l;
      a2 += l;
    }
    A.of0[i] = a0;
    A.of1[i] = a1;
    A.of2[i] = a2;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NM; i += stride) {
    const double lh = A.lam_h[i];
    if (A.q == 1) {
      A.om0[i] = A.lm1n[i] + lh / A.dt;
      A.om1[i] = 0.0;
    } else {
      A.om0[i] = A.lm1n[i] + 4.0 * lh / (2.0 * A.dt);
      A.om1[i] = -lh / (2.0 * A.dt);
    }
  }
}

// Forward recompute helpers: the trial by extrapolation and h_q (Eq. bdf2),
// from checkpointed populations of type T into FP64 iterates.
template <class L, class T>
__global__ void k_extrap_h(int64_t NS, int order, int q, double dt, const T* __restrict__ f0,
                           const T* __restrict__ f1, const T* __restrict__ f2, const double* __restrict__ mc,
                           const double* __restrict__ mp, float sig, double* __restrict__ trial,
                           double* __restrict__ h) {
  using CT = typename CompT<T>::type;
  constexpr int Q = L::Q, D1 = L::D + 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const double inv_dt = 1.0 / dt, inv_2dt = 1.0 / (2.0 * dt);
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
    for (int b = 0; b < D1; ++b)
      h[b * NS + s] = (q == 1) ? mc[b * NS + s] * inv_dt : (4.0 * mc[b * NS + s] - mp[b * NS + s]) * inv_2dt;
    CT a0[Q], a1[Q], a2[Q];
    site_load<L, T>(f0, NS, s, sig, a0);
    if (order >= 1) site_load<L, T>(f1, NS, s, sig, a1);
    if (order >= 2) site_load<L, T>(f2, NS, s, sig, a2);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      double v;
      if (order == 0)
        v = (double)a0[k];
      else if (order == 1)
        v = 2.0 * (double)a0[k] - (double)a1[k];
      else
        v = 3.0 * (double)a0[k] - 3.0 * (double)a1[k] + (double)a2[k];
      trial[(int64_t)k * NS + s] = v;
    }
  }
}

// Adjoint of the initial map: state (f0, f0, f0, P f0, P f0), f0 = feq(p0, u0).
template <class L>
__global__ void k_adj_init(int64_t NS, const double* __restrict__ p0, const double* __restrict__ u0,
                           const double* __restrict__ lam, double* __restrict__ lp, double* __restrict__ lu) {
  constexpr int Q = L::Q, D = L::D;
  const double cs2 = 1.0 / 3.0;
  const int64_t FQ = (int64_t)Q * NS, FM = (int64_t)(D + 1) * NS;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < NS; x += stride) {
    double m[4] = {p0[x], 0, 0, 0};
#pragma unroll
    for (int b = 0; b < D; ++b) m[1 + b] = u0[b * NS + x];
    double acc_p = 0.0, acc_u[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      double lk = lam[k * NS + x] + lam[FQ + k * NS + x] + lam[2 * FQ + k * NS + x];
      lk += lam[3 * FQ + x] + lam[3 * FQ + FM + x];
      double cu = 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        lk += (double)ca<L>(k, b) * (lam[3 * FQ + (1 + b) * NS + x] + lam[3 * FQ + FM + (1 + b) * NS + x]);
        cu += (double)ca<L>(k, b) * m[1 + b];
      }
      acc_p += L::w(k) * lk;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const double c = (double)ca<L>(k, b);
        acc_u[b] += L::w(k) * (c / cs2 + cu * c / (cs2 * cs2) - m[1 + b] / cs2) * lk;
      }
    }
    lp[x] = acc_p;
#pragma unroll
    for (int b = 0; b < D; ++b) lu[b * NS + x] = acc_u[b];
  }
}

}  // namespace msc
