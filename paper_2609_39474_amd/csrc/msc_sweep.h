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

#include "msc_common.h"

namespace msc {

enum { SW_EXPLICIT = 0, SW_DTS = 1, SW_DTS_LIFT = 2 };

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
  const double* h;  // (d+1) x NS, FP64 BDF history term h_q
  const TM* dm;     // (d+1) x NS, previous shadow correction
  TM* Pr;           // (d+1) x NS, residual moments out
  double* partials; // one FP64 partial sum of r^2 per block
  double a, inv1pa2;  // a_q and 1/(1 + a_q/2)
  double wp, wm;      // omega+, omega-
  int* did_run;       // optional: set to 1 when the launch passed its guard
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
// one barrier per step the rings need 4, 3 and 2 slots.
__host__ __device__ constexpr int ring_depth(int g) { return g == 0 ? 4 : (g == 1 ? 3 : 2); }

__device__ inline int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Load the trial populations of one site (with the fused lift), reconstruct
// (Eq. macro-reconstruct), form the source (Eq. source-moments) and collide
// (Eq. collision with Eq. feq and Eq. source-distribution).
template <class L, class T, class TM, int MODE>
__device__ __forceinline__ void load_collide(const SweepArgs<T, TM>& A, const T* __restrict__ src,
                                             int64_t site, typename CompT<T>::type* f,
                                             typename CompT<T>::type* C) {
  using CT = typename CompT<T>::type;
  constexpr int Q = L::Q, D = L::D;
  const int64_t NS = A.NS;
#pragma unroll
  for (int k = 0; k < Q; ++k) f[k] = (CT)src[k * NS + site];
  if (MODE == SW_DTS_LIFT) {
    CT d0 = (CT)A.dm[site];
    CT du[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < D; ++b) du[b] = (CT)A.dm[(1 + b) * NS + site];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      CT cu = 0;
#pragma unroll
      for (int b = 0; b < D; ++b) cu += (CT)ca<L>(k, b) * du[b];
      f[k] += (CT)L::w(k) * (d0 + (CT)3 * cu);
    }
  }
  CT M[4] = {0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    M[0] += f[k];
#pragma unroll
    for (int b = 0; b < D; ++b)
      if (ca<L>(k, b) != 0) M[1 + b] += (CT)ca<L>(k, b) * f[k];
  }
  CT m[4], s[4];
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
      double hb = A.h[b * NS + site];
      double mb = ((double)M[b] + 0.5 * hb) * A.inv1pa2;
      m[b] = (CT)mb;
      s[b] = (CT)(hb - A.a * mb);
    }
  }
  const CT uu = m[1] * m[1] + m[2] * m[2] + (D == 3 ? m[3] * m[3] : (CT)0);
  CT feq[Q], phi[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    CT cu = 0;
#pragma unroll
    for (int b = 0; b < D; ++b)
      if (ca<L>(k, b) != 0) cu += (CT)ca<L>(k, b) * m[1 + b];
    const CT wk = (CT)L::w(k);
    feq[k] = wk * (m[0] + (CT)3 * cu + (CT)4.5 * cu * cu - (CT)1.5 * uu);
    if (MODE == SW_EXPLICIT) {
      phi[k] = 0;
    } else {
      CT ps = s[0];
#pragma unroll
      for (int b = 0; b < D; ++b)
        ps += ((CT)3 * ((CT)ca<L>(k, b) - m[1 + b]) + (CT)9 * cu * (CT)ca<L>(k, b)) * s[1 + b];
      phi[k] = wk * ps;
    }
  }
  const CT wp = (CT)A.wp, wm = (CT)A.wm;
  const CT hp = (CT)1 - (CT)0.5 * wp, hm = (CT)1 - (CT)0.5 * wm;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const int kb = L::opp(k);
    const CT fp = (CT)0.5 * (f[k] + f[kb]), fm = (CT)0.5 * (f[k] - f[kb]);
    const CT ep = (CT)0.5 * (feq[k] + feq[kb]), em = (CT)0.5 * (feq[k] - feq[kb]);
    C[k] = f[k] - wp * (fp - ep) - wm * (fm - em);
    if (MODE != SW_EXPLICIT) {
      const CT pp = (CT)0.5 * (phi[k] + phi[kb]), pm = (CT)0.5 * (phi[k] - phi[kb]);
      C[k] += hp * pp + hm * pm;
    }
  }
}

template <class L, class T, class TM, int NT, int T1, int T2, int MODE>
__global__ __launch_bounds__(NT) void k_sweep(SweepArgs<T, TM> A) {
  using CT = typename CompT<T>::type;
  constexpr int Q = L::Q, D = L::D;
  constexpr int NI = T1 * T2;
  static_assert(NI % NT == 0, "tile must be a multiple of the block");
  constexpr int SPT = NI / NT;
  constexpr int NGP = group_count<L>(0), NG0 = group_count<L>(1), NGM = group_count<L>(2);
  constexpr int KPX = local_dir<L>(1), KMX = local_dir<L>(-1);
  static_assert(KPX > 0 && KMX > 0 && local_dir<L>(0) == 0, "lattice layout");

  __shared__ T ldsP[4][NGP][NI];
  __shared__ T ldsZ[3][NG0][NI];
  __shared__ T ldsM[2][NGM][NI];
  __shared__ double red[NT / 64 + 1];

  const T* __restrict__ src = A.src;
  T* __restrict__ dst = A.dst;
  if (A.ctl) {
    const uint64_t ph = A.ctl->phase;
    if (!phase_ready(ph, A.n, A.ell)) return;  // uniform for the grid
    src = A.fb.p[A.ctl->slot_w[(A.ell - 1) & 1]];
    dst = A.fb.p[A.ctl->slot_w[A.ell & 1]];
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
  CT c0prev[SPT], cpx1[SPT], cpx2[SPT], cmxc[SPT], c0c[SPT], cpxc[SPT];
  double r2 = 0.0;

  for (int it = 0; it < A.L + 2; ++it) {
    const int xs = wrapi(x0 - 1 + it, N0);
    const bool wP = it <= A.L - 1;             // dest plane it+1 is finalised later
    const bool wZ = it >= 1 && it <= A.L;      // dest plane it
    const bool wM = it >= 2;                   // dest plane it-1
    const int sP = (it + 1) & 3, sZ = it % 3, sM = (it + 1) & 1;

    // ---- owned interior sources ------------------------------------------
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      const int s = tid + j * NT;
      const int i1 = s / T2, i2 = s - (s / T2) * T2;
      const int64_t site = ((int64_t)xs * N1 + (b1 + i1)) * N2 + (b2 + i2);
      CT C[Q];
      load_collide<L, T, TM, MODE>(A, src, site, fcur[j], C);
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
          if (wP) ldsP[sP][gi][di] = (T)C[k];
        } else if (g == 1) {
          if (wZ) ldsZ[sZ][gi][di] = (T)C[k];
        } else {
          if (wM) ldsM[sM][gi][di] = (T)C[k];
        }
      }
      c0c[j] = C[0];
      cpxc[j] = C[KPX];
      cmxc[j] = C[KMX];
    }
    // ---- halo ring sources (only along axes the tile does not span) -------
    for (int t = tid; t < nhalo; t += NT) {
      int i1, i2;
      if (t < 2 * h1 * S2) {
        i1 = (t < S2) ? -1 : T1;
        i2 = (t % S2) - h2;
      } else {
        const int u = t - 2 * h1 * S2;
        i2 = (u < T1) ? -1 : T2;
        i1 = u % T1;
      }
      const int p1 = wrapi(b1 + i1, N1), p2 = wrapi(b2 + i2, N2);
      const int64_t site = ((int64_t)xs * N1 + p1) * N2 + p2;
      CT f[Q], C[Q];
      load_collide<L, T, TM, MODE>(A, src, site, f, C);
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
          if (wP) ldsP[sP][gi][di] = (T)C[k];
        } else if (g == 1) {
          if (wZ) ldsZ[sZ][gi][di] = (T)C[k];
        } else {
          if (wM) ldsM[sM][gi][di] = (T)C[k];
        }
      }
    }
    __syncthreads();

    // ---- finalise destination plane it-1 ----------------------------------
    if (it >= 2) {
      const int id = it - 1;
      const int xd = wrapi(x0 + id - 1, N0);
      const int rP = id & 3, rZ = id % 3, rM = id & 1;
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        const int s = tid + j * NT;
        const int i1 = s / T2, i2 = s - (s / T2) * T2;
        const int64_t site = ((int64_t)xd * N1 + (b1 + i1)) * N2 + (b2 + i2);
        CT pr[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          CT v;
          if (k == 0) {
            v = c0prev[j];
          } else if (k == KPX) {
            v = cpx2[j];
          } else if (k == KMX) {
            v = cmxc[j];
          } else {
            const int g = xgroup<L>(k), gi = group_index<L>(k);
            v = (g == 0) ? (CT)ldsP[rP][gi][s] : ((g == 1) ? (CT)ldsZ[rZ][gi][s] : (CT)ldsM[rM][gi][s]);
          }
          dst[k * NS + site] = (T)v;
          if (MODE != SW_EXPLICIT) {
            const CT r = v - fprev[j][k];
            pr[0] += r;
#pragma unroll
            for (int bb = 0; bb < D; ++bb)
              if (ca<L>(k, bb) != 0) pr[1 + bb] += (CT)ca<L>(k, bb) * r;
            r2 += (double)r * (double)r;
          }
        }
        if (MODE != SW_EXPLICIT) {
#pragma unroll
          for (int bb = 0; bb <= D; ++bb) A.Pr[bb * NS + site] = (TM)pr[bb];
        }
      }
    }
    // ---- roll registers ------------------------------------------------------
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
#pragma unroll
      for (int k = 0; k < Q; ++k) fprev[j][k] = fcur[j][k];
      c0prev[j] = c0c[j];
      cpx2[j] = cpx1[j];
      cpx1[j] = cpxc[j];
    }
  }

  if (MODE != SW_EXPLICIT) {
    // FP64 block reduction of sum r^2: wave shuffles, then LDS across waves.
    if (NT >= 64) {
      double v = r2;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if ((tid & 63) == 0) red[tid >> 6] = v;
      __syncthreads();
      if (tid == 0) {
        double acc = 0.0;
        for (int wv = 0; wv < NT / 64; ++wv) acc += red[wv];
        A.partials[blockIdx.x] = acc;
      }
    } else {
      // blocks narrower than a wavefront (tiny test grids): serial sum
      __shared__ double reds[NT];
      reds[tid] = r2;
      __syncthreads();
      if (tid == 0) {
        double acc = 0.0;
        for (int i = 0; i < NT; ++i) acc += reds[i];
        A.partials[blockIdx.x] = acc;
      }
    }
  }
}

}  // namespace msc
