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
  double inv1pa2;  // 1/(1 + a/2), formed once on the host (the setup sweep's
                   // reconstruction uses the same value, so both agree bit for bit)
  // 1: the reconstruction of m^{n+1} is left to the next step's setup sweep,
  // which forms it from the same populations (the next step is enqueued by
  // the same call)
  int defer;
};

// P f in FP64 at one site (for deviation storage the stored moments, which
// the rebuild preserves exactly).
template <class L, class T>
__device__ inline void site_moments(const T* f, int64_t NS, int64_t s, double* M) {
  if constexpr (PopDev<T>::value) {
    const float* Ms = dev_moments(f, L::Q, NS);
#pragma unroll
    for (int b = 0; b <= L::D; ++b) M[b] = (double)Ms[b * NS + s];
  } else {
#pragma unroll
    for (int b = 0; b <= L::D; ++b) M[b] = 0.0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      const double v = (double)f[(int64_t)k * NS + s];
      M[0] += v;
#pragma unroll
      for (int b = 0; b < L::D; ++b)
        if (ca<L>(k, b) != 0) M[1 + b] += (double)ca<L>(k, b) * v;
    }
  }
}

// All Q populations of one site in the compute type.
template <class L, class T>
__device__ inline void site_load(const T* f, int64_t NS, int64_t s, float sig, typename CompT<T>::type* v) {
  if constexpr (PopDev<T>::value) {
    _Float16 g[L::Q];
    float M[L::D + 1];
#pragma unroll
    for (int k = 0; k < L::Q; ++k) g[k] = f[(int64_t)k * NS + s];
    const float* Ms = dev_moments(f, L::Q, NS);
#pragma unroll
    for (int b = 0; b <= L::D; ++b) M[b] = Ms[b * NS + s];
    dev_rebuild<L>(g, M, sig, v);
  } else {
#pragma unroll
    for (int k = 0; k < L::Q; ++k) v[k] = (typename CompT<T>::type)f[(int64_t)k * NS + s];
  }
}

template <class L, class T>
__device__ inline void site_store(T* f, int64_t NS, int64_t s, float isig, const typename CompT<T>::type* v) {
  if constexpr (PopDev<T>::value) {
    _Float16 g[L::Q];
    float M[L::D + 1];
    dev_split<L, double>(v, isig, g, M);
#pragma unroll
    for (int k = 0; k < L::Q; ++k) f[(int64_t)k * NS + s] = g[k];
    float* Ms = dev_moments(f, L::Q, NS);
#pragma unroll
    for (int b = 0; b <= L::D; ++b) Ms[b * NS + s] = M[b];
  } else {
#pragma unroll
    for (int k = 0; k < L::Q; ++k) f[(int64_t)k * NS + s] = (T)v[k];
  }
}

// The accepted populations are step n's working buffer of sweep ell; m^{n+1}
// goes to step n's spare moment slot (the roles of step n + 1 name them f^n
// and m^n).
template <class L, class T>
__device__ inline void accept_sites(const AcceptArgs<L, T>& A, int64_t s0, int64_t s1, int64_t stride) {
  if (A.defer) return;
  const Roles& ro = A.ctl->roles[A.n & 1];
  const T* f = A.fb.p[ro.slot_w[A.ell & 1]];
  double* m = A.mb[ro.slot_m[2]];
  const int64_t NS = A.NS;
  for (int64_t s = s0; s < s1; s += stride) {
    double M[4];
    site_moments<L, T>(f, NS, s, M);
#pragma unroll
    for (int b = 0; b <= L::D; ++b) m[b * NS + s] = (M[b] + 0.5 * A.h[b * NS + s]) * A.inv1pa2;
  }
}

// Without the shadow corrector: the acceptance decision and, if accepted,
// the reconstruction.
template <class L, class T>
__global__ __launch_bounds__(256) void k_accept(AcceptArgs<L, T> A, FinishArgs F) {
  __shared__ double red[256];
  if (finish_block(F, red) != DEC_ACCEPTED) return;
  accept_sites<L, T>(A, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, A.NS, (int64_t)gridDim.x * blockDim.x);
}

// P r of a lift sweep that left it out (the sweep enqueued as the last of its
// step, which then went on): from the sweep's input (the previous f_T), the
// correction it lifted and its output, by the sweep's own arithmetic (the
// trial f_in + E dm of Eq. lift, r = f_T - trial, P r summed over k in order),
// so the values equal those the sweep would have stored.
template <class T, class TM>
struct PrArgs {
  const DevCtl* ctl;
  int n, ell;
  FBufs<T> fb;
  const TM* dm;
  TM* Pr;
  int64_t NS;
};

template <class L, class CT, class TM>
__device__ __forceinline__ void lifted_trial(const CT* fin, const TM* dmv, CT* f) {
#pragma clang fp contract(on)
  const CT d0 = (CT)dmv[0];
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    CT cu = 0;
#pragma unroll
    for (int b = 0; b < L::D; ++b) cu += (CT)ca<L>(k, b) * (CT)dmv[1 + b];
    f[k] = fin[k];
    f[k] += (CT)L::w(k) * (d0 + (CT)3 * cu);
  }
}

template <class L, class T, class TM>
__global__ __launch_bounds__(256) void k_recompute_pr(PrArgs<T, TM> A) {
  static_assert(!PopDev<T>::value, "deviation storage forms P r from its stored moments");
  using CT = typename CompT<T>::type;
  constexpr int Q = L::Q, D = L::D;
  if (!phase_correct(A.ctl->phase, A.n, A.ell)) return;  // uniform for the grid
  const Roles& ro = A.ctl->roles[A.n & 1];
  const T* fin = A.fb.p[ro.slot_w[(A.ell - 1) & 1]];
  const T* fout = A.fb.p[ro.slot_w[A.ell & 1]];
  const int64_t NS = A.NS;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += (int64_t)gridDim.x * blockDim.x) {
    CT f0[Q], f[Q];
    TM dmv[D + 1];
#pragma unroll
    for (int k = 0; k < Q; ++k) f0[k] = (CT)fin[(int64_t)k * NS + s];
#pragma unroll
    for (int b = 0; b <= D; ++b) dmv[b] = A.dm[b * NS + s];
    lifted_trial<L, CT, TM>(f0, dmv, f);
    CT pr[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const CT r = (CT)fout[(int64_t)k * NS + s] - f[k];
      pr[0] += r;
#pragma unroll
      for (int bb = 0; bb < D; ++bb)
        if (ca<L>(k, bb) != 0) pr[1 + bb] += (CT)ca<L>(k, bb) * r;
    }
#pragma unroll
    for (int bb = 0; bb <= D; ++bb) A.Pr[bb * NS + s] = (TM)pr[bb];
  }
}

// ------------------------------------------------------ initialisation --
// f = feq(p, u) (Eq. feq) from FP64 fields; the initial state of Sec. 4.1.
// Deviation storage: g = 0 and M = (p, u) (P feq(p, u) = (p, u)).
template <class L, class T>
__global__ void k_init_feq(const double* __restrict__ p, const double* __restrict__ u, T* __restrict__ f,
                           int64_t NS) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if constexpr (PopDev<T>::value) {
    float* M = dev_moments(f, L::Q, NS);
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
#pragma unroll
      for (int k = 0; k < L::Q; ++k) f[(int64_t)k * NS + s] = (_Float16)0.f;
      M[s] = (float)p[s];
#pragma unroll
      for (int b = 0; b < L::D; ++b) M[(1 + b) * NS + s] = (float)u[b * NS + s];
    }
    return;
  }
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
    double M[4];
    site_moments<L, T>(f, NS, s, M);
#pragma unroll
    for (int b = 0; b <= L::D; ++b) m[b * NS + s] = M[b];
  }
}

// out = fT + E dm (Eq. lift, Eq. shadow-update) with the same arithmetic the
// sweep applies when it fuses the lift into its load.
template <class L, class T, class TM>
__global__ void k_lift(const T* __restrict__ fT, const TM* __restrict__ dm, T* __restrict__ out, int64_t NS,
                       float sig, float isig) {
  using CT = typename CompT<T>::type;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
    const CT d0 = (CT)dm[s];
    CT du[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < L::D; ++b) du[b] = (CT)dm[(1 + b) * NS + s];
    CT v[L::Q];
    site_load<L, T>(fT, NS, s, sig, v);
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      CT cu = 0;
#pragma unroll
      for (int b = 0; b < L::D; ++b) cu += (CT)ca<L>(k, b) * du[b];
      v[k] = v[k] + (CT)L::w(k) * (d0 + (CT)3 * cu);
    }
    site_store<L, T>(out, NS, s, isig, v);
  }
}

// Populations between the storage type and FP64 (canonical layout).
template <class L, class T>
__global__ void k_pop_to_f64(const T* __restrict__ in, double* __restrict__ out, int64_t NS, float sig) {
  using CT = typename CompT<T>::type;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
    CT v[L::Q];
    site_load<L, T>(in, NS, s, sig, v);
#pragma unroll
    for (int k = 0; k < L::Q; ++k) out[(int64_t)k * NS + s] = (double)v[k];
  }
}

template <class L, class T>
__global__ void k_pop_from_f64(const double* __restrict__ in, T* __restrict__ out, int64_t NS, float isig) {
  using CT = typename CompT<T>::type;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
    CT v[L::Q];
#pragma unroll
    for (int k = 0; k < L::Q; ++k) v[k] = (CT)in[(int64_t)k * NS + s];
    site_store<L, T>(out, NS, s, isig, v);
  }
}

// Per-block maxima of |f_k - feq_k(P f)| and of |P f| over FP64 populations:
// partials[2 b] and partials[2 b + 1] (the scale choice of deviation storage).
template <class L>
__global__ __launch_bounds__(256) void k_pop_maxdev(const double* __restrict__ f, int64_t NS,
                                                    double* __restrict__ partials) {
  __shared__ double r0[256], r1[256];
  double md = 0.0, mm = 0.0;
  const double cs2 = 1.0 / 3.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += stride) {
    double M[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      const double v = f[(int64_t)k * NS + s];
      M[0] += v;
#pragma unroll
      for (int b = 0; b < L::D; ++b) M[1 + b] += (double)ca<L>(k, b) * v;
    }
    double uu = 0.0;
#pragma unroll
    for (int b = 0; b <= L::D; ++b) mm = fmax(mm, fabs(M[b]));
#pragma unroll
    for (int b = 0; b < L::D; ++b) uu += M[1 + b] * M[1 + b];
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      double cu = 0.0;
#pragma unroll
      for (int b = 0; b < L::D; ++b) cu += (double)ca<L>(k, b) * M[1 + b];
      const double fe = L::w(k) * (M[0] + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
      md = fmax(md, fabs(f[(int64_t)k * NS + s] - fe));
    }
  }
  r0[threadIdx.x] = md;
  r1[threadIdx.x] = mm;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r0[threadIdx.x] = fmax(r0[threadIdx.x], r0[threadIdx.x + w]);
      r1[threadIdx.x] = fmax(r1[threadIdx.x], r1[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = r0[0];
    partials[2 * blockIdx.x + 1] = r1[0];
  }
}

template <class A, class B>
__global__ void k_convert(const A* __restrict__ in, B* __restrict__ out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = (B)in[i];
}

// Per-block maxima of |v|.
template <int UNUSED = 0>
__global__ __launch_bounds__(256) void k_absmax(const double* __restrict__ v, int64_t n, double* partials) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) acc = fmax(acc, fabs(v[i]));
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
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
