// Wall-bounded kinetic correction (paper Sec. 3.3, Algorithm 2) on the D2Q9
// lid-driven cavity: (I - L) df = r with L = B_Gamma S blkdiag(J^C(x))
// (Eq. wall-global-jacobian).  J^C(x) is the local collision Jacobian of Eq.
// (wall-local-jacobian) at a reference field (m, s): with G of Eq. (wall-G),
// J^C_kk' = (G_k0 + sum_a G_ka c_k'a) / (1 + a/2), i.e. (J^C z)_k =
// sum_b G_kb mu_b with mu = P z / (1 + a/2).  S streams with the periodic
// wrap, B_Gamma replaces the wall rows in the order of Eq. (bounceback-rows)
// (the lid constants have zero derivative).
//
// The paper factors I - L with a sparse direct solver.  Here it is solved by
// restarted GMRES, preconditioned on the right with the periodic full-symbol
// inverse at rest (the transform kernels of msc_fullsym.h in plain mode):
// away from the walls the two operators coincide, so the preconditioned
// operator is the identity plus a perturbation supported on the wall rows.
// The kernels below are the matrix-free operator and the Krylov vector
// operations (FP64, fixed-order block partial sums, so results do not depend
// on scheduling).
#pragma once

#include "msc_fullsym.h"

namespace msc {

// Eq. (wall-G) at omega+- = 1 for direction k (D2Q9): G[0] = dC_k/dp,
// G[1 + b] = dC_k/du_b at the reference moments m and source s.
__device__ inline void wall_G(int k, const double* m, const double* s, double a, double* G) {
  const double cs2 = 1.0 / 3.0, cs4 = cs2 * cs2;
  const double wk = D2Q9::w(k);
  const double c0 = (double)D2Q9::cx(k), c1 = (double)D2Q9::cy(k);
  const double cu = c0 * m[1] + c1 * m[2];
  G[0] = wk * (1.0 - 0.5 * a);
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const double cb = (b == 0) ? c0 : c1, ub = m[1 + b];
    double g = wk * (cb / cs2 + cu * cb / cs4 - ub / cs2);
    double src = 0.0;
#pragma unroll
    for (int al = 0; al < 2; ++al) {
      const double ca_ = (al == 0) ? c0 : c1;
      src += (-(al == b ? 1.0 : 0.0) / cs2 + ca_ * cb / cs4) * s[1 + al];
    }
    src -= a * ((cb - ub) / cs2 + cu * cb / cs4);
    G[1 + b] = g + 0.5 * wk * src;
  }
}

// mu = P z / (1 + a/2) at every site (3 fields).
template <int UNUSED = 0>
__global__ __launch_bounds__(256) void k_wall_mu(const double* __restrict__ z, double* __restrict__ mu, int64_t NS,
                                                 double inv1pa2) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += (int64_t)gridDim.x * blockDim.x) {
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double v = z[k * NS + s];
      m0 += v;
      m1 += (double)D2Q9::cx(k) * v;
      m2 += (double)D2Q9::cy(k) * v;
    }
    mu[s] = m0 * inv1pa2;
    mu[NS + s] = m1 * inv1pa2;
    mu[2 * NS + s] = m2 * inv1pa2;
  }
}

// w = z - L z at every destination node: the streamed rows (J^C(x) z(x))_k
// from the upwind site x = y - c_k (periodic wrap), then the wall rows of the
// node replaced in order.  mref/sref: the reference field ((d+1) x N_sites
// each), or null for the uniform rest reference (m = (1, 0), s = 0).
template <int UNUSED = 0>
__global__ __launch_bounds__(256) void k_wall_apply(const double* __restrict__ z, const double* __restrict__ mu,
                                                    const double* __restrict__ mref,
                                                    const double* __restrict__ sref, double a, int Nx, int Ny,
                                                    double* __restrict__ w) {
  const int64_t NS = (int64_t)Nx * Ny;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(s / Ny), y = (int)(s - (int64_t)x * Ny);
    double Lz[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      int xu = x - D2Q9::cx(k), yu = y - D2Q9::cy(k);
      xu = (xu < 0) ? xu + Nx : (xu >= Nx ? xu - Nx : xu);
      yu = (yu < 0) ? yu + Ny : (yu >= Ny ? yu - Ny : yu);
      const int64_t su = (int64_t)xu * Ny + yu;
      double m[3] = {1.0, 0.0, 0.0}, sv[3] = {0.0, 0.0, 0.0}, G[3];
      if (mref) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          m[b] = mref[b * NS + su];
          sv[b] = sref[b * NS + su];
        }
      }
      wall_G(k, m, sv, a, G);
      Lz[k] = G[0] * mu[su] + G[1] * mu[NS + su] + G[2] * mu[2 * NS + su];
    }
    cavity_rows<double>(Lz, x, y, Nx, Ny, 0.0);
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k * NS + s] = z[k * NS + s] - Lz[k];
  }
}

// Reference field of a refresh (Algorithm 2): the current iterate f = f_T - r
// reconstructed with the unchanged history term, m = (P f + h/2)/(1 + a/2),
// s = h - a m.
template <int UNUSED = 0>
__global__ __launch_bounds__(256) void k_wall_reference(const double* __restrict__ fT, const double* __restrict__ r,
                                                        const double* __restrict__ h, double a, int64_t NS,
                                                        double* __restrict__ mref, double* __restrict__ sref) {
  const double inv = 1.0 / (1.0 + 0.5 * a);
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < NS; s += (int64_t)gridDim.x * blockDim.x) {
    double M[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double f = fT[k * NS + s] - r[k * NS + s];
      M[0] += f;
      M[1] += (double)D2Q9::cx(k) * f;
      M[2] += (double)D2Q9::cy(k) * f;
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double m = (M[b] + 0.5 * h[b * NS + s]) * inv;
      mref[b * NS + s] = m;
      sref[b * NS + s] = h[b * NS + s] - a * m;
    }
  }
}

// ------------------------------------------------------- Krylov helpers --
// The Krylov basis V is stored in VT: double, or float for the loose
// tolerances (the new vector w, the coefficients and every sum stay FP64).
//
// acc[k] += <V_k, w> over this thread's elements of [b0, b1), k < G, with G
// fixed at compile time so that the G + 1 loads of an element issue together.
template <int G, int GMAX, class VT>
__device__ inline void dot_rows(const VT* __restrict__ v, int64_t stride, const double* __restrict__ w, int64_t b0,
                                int64_t b1, double (&acc)[GMAX]) {
#pragma unroll 2
  for (int64_t t = b0 + threadIdx.x; t < b1; t += blockDim.x) {
    const double wt = w[t];
    double x[G];
#pragma unroll
    for (int k = 0; k < G; ++k) x[k] = (double)v[k * stride + t];
#pragma unroll
    for (int k = 0; k < G; ++k) acc[k] += x[k] * wt;
  }
}

template <int G, int GMAX, class VT>
__device__ inline void dot_rows_n(int g, const VT* __restrict__ v, int64_t stride, const double* __restrict__ w,
                                  int64_t b0, int64_t b1, double (&acc)[GMAX]) {
  if constexpr (G > 0) {
    if (g == G)
      dot_rows<G, GMAX, VT>(v, stride, w, b0, b1, acc);
    else
      dot_rows_n<G - 1, GMAX, VT>(g, v, stride, w, b0, b1, acc);
  }
}

// partials[i * gridDim.x + block] = this block's part of <V_i, w>, i < nv
// (V_i = V + i * stride), and with self also <w, w> at i = nv.  The vectors go
// in groups of kDotGroup, so w is read once per group and one block reduction
// serves the whole group.
constexpr int kDotGroup = 16;
__device__ inline void block_sum_store(double acc, double* red4, double* dst) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) red4[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *dst = ((red4[0] + red4[1]) + red4[2]) + red4[3];
  __syncthreads();
}

template <class VT>
__global__ __launch_bounds__(256) void k_dots(const VT* __restrict__ V, int64_t stride, int nv,
                                              const double* __restrict__ w, int64_t n,
                                              double* __restrict__ partials, int self) {
  __shared__ double red[kDotGroup][4];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * chunk;
  const int64_t b1 = (b0 + chunk < n) ? b0 + chunk : n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i0 = 0; i0 < nv; i0 += kDotGroup) {
    const int g = (nv - i0 < kDotGroup) ? nv - i0 : kDotGroup;
    double acc[kDotGroup];
#pragma unroll
    for (int k = 0; k < kDotGroup; ++k) acc[k] = 0.0;
    dot_rows_n<kDotGroup, kDotGroup, VT>(g, V + (int64_t)i0 * stride, stride, w, b0, b1, acc);
#pragma unroll
    for (int k = 0; k < kDotGroup; ++k) {
      if (k < g) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
        if (lane == 0) red[k][wv] = acc[k];
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < g)
      partials[(int64_t)(i0 + threadIdx.x) * gridDim.x + blockIdx.x] =
          ((red[threadIdx.x][0] + red[threadIdx.x][1]) + red[threadIdx.x][2]) + red[threadIdx.x][3];
    __syncthreads();
  }
  if (self) {
    double acc = 0.0;
    for (int64_t t = b0 + threadIdx.x; t < b1; t += blockDim.x) acc += w[t] * w[t];
    block_sum_store(acc, red[0], &partials[(int64_t)nv * gridDim.x + blockIdx.x]);
  }
}

// Blocks of k_dots in the Gram-Schmidt passes (a multiple of 64).
constexpr int kDotBlocks = 512;

// h[i] = sum over the kDotBlocks partials of <V_i, w>, i < nv, by the whole
// block: wave wv takes the vectors i = wv, wv + (waves per block), ...; each
// lane sums its kDotBlocks / 64 strided partials (loaded together), then a
// butterfly over the wave.  The order is fixed, so the sums do not depend on
// scheduling.
__device__ inline void sum_partials(const double* __restrict__ partials, int nv, double* h) {
  constexpr int kPer = kDotBlocks / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = wv; i < nv; i += (int)(blockDim.x >> 6)) {
    const double* p = partials + (int64_t)i * kDotBlocks + lane;
    double x[kPer];
#pragma unroll
    for (int b = 0; b < kPer; ++b) x[b] = p[64 * b];
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < kPer; ++b) acc += x[b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) h[i] = acc;
  }
  __syncthreads();
}

// acc -/+= sum_k coef[k] V_k[t], k < G in order, with G fixed at compile time
// so that the G loads of element t issue together; the _n form dispatches a
// run-time group width g <= G.
template <int G, bool SUB, class VT>
__device__ inline double comb_rows(double acc, const VT* __restrict__ v, int64_t stride,
                                   const double* __restrict__ coef, int64_t t) {
  double x[G];
#pragma unroll
  for (int k = 0; k < G; ++k) x[k] = (double)v[k * stride + t];
#pragma unroll
  for (int k = 0; k < G; ++k) {
    if constexpr (SUB)
      acc -= coef[k] * x[k];
    else
      acc += coef[k] * x[k];
  }
  return acc;
}

template <int G, bool SUB, class VT>
__device__ inline double comb_rows_n(int g, double acc, const VT* __restrict__ v, int64_t stride,
                                     const double* __restrict__ coef, int64_t t) {
  if constexpr (G > 0) {
    if (g == G) return comb_rows<G, SUB, VT>(acc, v, stride, coef, t);
    return comb_rows_n<G - 1, SUB, VT>(g, acc, v, stride, coef, t);
  } else {
    return acc;
  }
}

template <bool SUB, class VT>
__device__ inline double comb_all(double acc, const VT* __restrict__ V, int64_t stride, int nv,
                                  const double* __restrict__ coef, int64_t t) {
  for (int i0 = 0; i0 < nv; i0 += kDotGroup) {
    const int g = (nv - i0 < kDotGroup) ? nv - i0 : kDotGroup;
    acc = comb_rows_n<kDotGroup, SUB, VT>(g, acc, V + (int64_t)i0 * stride, stride, coef + i0, t);
  }
  return acc;
}

// w -= sum_i coef[i] V_i (coef on the device), i < nv.
template <class VT>
__global__ __launch_bounds__(256) void k_axpy_multi(double* __restrict__ w, const VT* __restrict__ V, int64_t stride,
                                                    int nv, const double* __restrict__ coef, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    w[t] = comb_all<true, VT>(w[t], V, stride, nv, coef, t);
}

// the next basis vector: v = (w - sum_i coef[i] V_i) * scale[0], i < nv (coef
// and scale on the device), into out (VT) and its FP64 copy out64 (the
// preconditioner's next input), unless out64 is null.
template <class VT>
__global__ __launch_bounds__(256) void k_axpy_scale(VT* __restrict__ out, double* __restrict__ out64,
                                                    const double* __restrict__ w, const VT* __restrict__ V,
                                                    int64_t stride, int nv, const double* __restrict__ coef,
                                                    const double* __restrict__ scale, int64_t n) {
  const double sc = scale[0];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const double v = comb_all<true, VT>(w[t], V, stride, nv, coef, t) * sc;
    out[t] = (VT)v;
    if (out64) out64[t] = v;
  }
}

// out = alpha x into the basis type (and its FP64 copy out64 unless null).
template <class VT>
__global__ __launch_bounds__(256) void k_scale_to(VT* __restrict__ out, double* __restrict__ out64,
                                                  const double* __restrict__ x, double alpha, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const double v = alpha * x[t];
    out[t] = (VT)v;
    if (out64) out64[t] = v;
  }
}

// Device-side Gram-Schmidt bookkeeping of one GMRES iteration (one block;
// the dot-product partials summed by sum_partials).
//
// k_gs_first: h = <V_i, w> for i < nv -> coef (for the projection) and hcol.
template <int UNUSED = 0>
__global__ __launch_bounds__(1024) void k_gs_first(const double* __restrict__ partials, int nv,
                                                  double* __restrict__ coef, double* __restrict__ hcol) {
  __shared__ double h[72];
  sum_partials(partials, nv, h);
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    coef[i] = h[i];
    hcol[i] = h[i];
  }
}

// k_gs_second: the re-orthogonalisation coefficients h2 = <V_i, w> (i <= j)
// and <w, w> (entry j+1) -> coef; column j of the Hessenberg matrix is
// hcol + h2 with H(j+1, j) = |w - V h2| = sqrt(<w, w> - |h2|^2); the earlier
// Givens rotations are applied to it, a new one zeroes H(j+1, j), g is
// rotated; R(:, j) goes to Hd (row stride m), 1/H(j+1, j) to scale and
// |g(j+1)| to resid[j].
template <int UNUSED = 0>
__global__ __launch_bounds__(1024) void k_gs_second(const double* __restrict__ partials, int j, int m,
                                                   double* __restrict__ coef, const double* __restrict__ hcol,
                                                   double* __restrict__ Hd, double* __restrict__ cs,
                                                   double* __restrict__ sn, double* __restrict__ g,
                                                   double* __restrict__ scale, double* __restrict__ resid) {
  __shared__ double h2[72], col[72], c_s[72], s_s[72];
  sum_partials(partials, j + 2, h2);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    coef[i] = h2[i];
    col[i] = hcol[i] + h2[i];
    if (i < j) {
      c_s[i] = cs[i];
      s_s[i] = sn[i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double hh = 0.0;
    for (int i = 0; i <= j; ++i) hh += h2[i] * h2[i];
    const double ww = h2[j + 1];
    const double hn = sqrt(ww - hh > 0.0 ? ww - hh : 0.0);
    // the earlier rotations; the running entry stays in a register
    double cur = col[0];
    for (int i = 0; i < j; ++i) {
      const double nxt = col[i + 1];
      col[i] = c_s[i] * cur + s_s[i] * nxt;
      cur = -s_s[i] * cur + c_s[i] * nxt;
    }
    const double den = hypot(cur, hn);
    const double cj = den > 0.0 ? cur / den : 1.0;
    const double sj = den > 0.0 ? hn / den : 0.0;
    cs[j] = cj;
    sn[j] = sj;
    col[j] = den;
    const double gj = g[j];
    g[j + 1] = -sj * gj;
    g[j] = cj * gj;
    scale[0] = hn > 0.0 ? 1.0 / hn : 1.0;
    resid[j] = fabs(sj * gj);
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += blockDim.x) Hd[(int64_t)i * m + j] = col[i];
}

// out = sum_i coef[i] V_i, i < nv.
template <class VT>
__global__ __launch_bounds__(256) void k_combine(double* __restrict__ out, const VT* __restrict__ V, int64_t stride,
                                                 int nv, const double* __restrict__ coef, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    out[t] = comb_all<false, VT>(0.0, V, stride, nv, coef, t);
}

// out = alpha * x + beta * y (any of x, y may alias out).
template <int UNUSED = 0>
__global__ __launch_bounds__(256) void k_lincomb(double* out, const double* x, double alpha, const double* y,
                                                 double beta, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    out[t] = alpha * x[t] + (y ? beta * y[t] : 0.0);
}

}  // namespace msc
