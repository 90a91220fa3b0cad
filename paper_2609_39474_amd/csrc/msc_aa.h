// In-place explicit march (the source-free map of Sec. 4.1, Eq. sweep with
// a = 0, h = 0) by the AA access pattern: two kernels that alternate on one
// population array and together advance two lattice steps.
//
//   even: every site collides its own populations (Eq. collision) and stores
//         the post-collision value of direction k in its own slot of the
//         opposite direction;
//   odd:  every site gathers direction k from the opposite slot of its
//         upstream neighbour x - c_k (the streaming of the even step),
//         collides, and stores direction k in slot k of its downstream
//         neighbour x + c_k (the streaming of the odd step).
//
// The odd step writes exactly the locations it reads, and no other site
// touches them, so one array holds the march: after an odd step it is the
// canonical population field again.  Each population is read and written
// once per step without a halo or a block-level exchange.  The collision is
// the sweep kernel's own code, so the march is bit-identical to the
// two-buffer sweep.
#pragma once

#include "msc_sweep.h"

namespace msc {

template <class T>
struct AaArgs {
  T* f;                 // Q x NS populations, updated in place
  int N0, N1, N2;       // extents in the sweep frame (x, p1, p2), powers of two
  int lg1, lg2;         // log2 N1, log2 N2
  int NS;               // sites (< 2^31)
  double wp, wm;        // omega+, omega-
  int* did_run;         // optional: set when the launch ran (kernel timing)
};

// site of this thread, with the XCD-aware block order of the sweep: the
// blocks b, b + 8, ... that one XCD runs take one contiguous range of sites
__device__ __forceinline__ int aa_site() {
  return xcd_item(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}

template <class L, class T>
__device__ __forceinline__ void aa_collide(const AaArgs<T>& A, const RawSite<L, T, typename CompT<T>::type, SW_EXPLICIT>& r,
                                           typename CompT<T>::type* C) {
  using CT = typename CompT<T>::type;
  SweepArgs<T, CT> S{};
  S.wp = A.wp;
  S.wm = A.wm;
  CT f[L::Q];
  double hs[4];
  collide_raw<L, T, CT, SW_EXPLICIT>(S, r, f, C, hs);
}

template <class L, class T>
__global__ __launch_bounds__(256) void k_aa_even(AaArgs<T> A) {
  using CT = typename CompT<T>::type;
  constexpr int Q = L::Q;
  const int s = aa_site();
  if (A.did_run && s == 0) *A.did_run = 1;
  if (s >= A.NS) return;
  const int64_t NS = A.NS;
  RawSite<L, T, CT, SW_EXPLICIT> r;
#pragma unroll
  for (int k = 0; k < Q; ++k) r.f0[k] = A.f[k * NS + s];
  CT C[Q];
  aa_collide<L, T>(A, r, C);
#pragma unroll
  for (int k = 0; k < Q; ++k) A.f[L::opp(k) * NS + s] = (T)C[k];
}

// index of the site (x + dx, p1 + d1, p2 + d2), periodic
__device__ __forceinline__ int aa_shift(int x, int i1, int i2, int dx, int d1, int d2, const int N0, const int N1,
                                        const int N2, int lg1, int lg2) {
  return ((((x + dx) & (N0 - 1)) << lg1 | ((i1 + d1) & (N1 - 1))) << lg2) | ((i2 + d2) & (N2 - 1));
}

template <class L, class T>
__global__ __launch_bounds__(256) void k_aa_odd(AaArgs<T> A) {
  using CT = typename CompT<T>::type;
  constexpr int Q = L::Q;
  const int s = aa_site();
  if (A.did_run && s == 0) *A.did_run = 1;
  if (s >= A.NS) return;
  const int64_t NS = A.NS;
  const int N0 = A.N0, N1 = A.N1, N2 = A.N2, lg1 = A.lg1, lg2 = A.lg2;
  const int i2 = s & (N2 - 1);
  const int i1 = (s >> lg2) & (N1 - 1);
  const int x = s >> (lg1 + lg2);
  RawSite<L, T, CT, SW_EXPLICIT> r;
#pragma unroll
  for (int k = 0; k < Q; ++k)
    r.f0[k] = A.f[L::opp(k) * NS + aa_shift(x, i1, i2, -L::cx(k), -L::c1(k), -L::c2(k), N0, N1, N2, lg1, lg2)];
  CT C[Q];
  aa_collide<L, T>(A, r, C);
#pragma unroll
  for (int k = 0; k < Q; ++k)
    A.f[k * NS + aa_shift(x, i1, i2, L::cx(k), L::c1(k), L::c2(k), N0, N1, N2, lg1, lg2)] = (T)C[k];
}

}  // namespace msc
