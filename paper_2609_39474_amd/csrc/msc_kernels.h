// Element-wise kernels around the sweep: the accepted-state reconstruction,
// initialisation, conversions and the index tables.
#pragma once

#include "msc_sweep.h"

namespace msc {

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
__device__ inline void accept_sites(const AcceptArgs<L, T>& A, int64_t s0, int64_t s1, int64_t stride) {
  const T* f = A.fb.p[A.ctl->slot_hist[0]];
  double* m = A.mb[A.ctl->slot_m[0]];
  const int64_t NS = A.NS;
  for (int64_t s = s0; s < s1; s += stride) {
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

template <class L, class T>
__global__ void k_accept(AcceptArgs<L, T> A) {
  if (!phase_accepted(A.ctl->phase, A.n, A.ell)) return;
  accept_sites<L, T>(A, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, A.NS, (int64_t)gridDim.x * blockDim.x);
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
