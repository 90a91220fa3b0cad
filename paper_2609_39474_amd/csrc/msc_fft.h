// Periodic macroscopic shadow correction (paper Sec. 3.2, Eq. shadow-update):
// dm = F^{-1}[ chi(k) H^{-1}(k) F[P r](k) ] with the transform convention of
// Eq. (fft-convention) (forward unnormalised, inverse 1/N_Omega), the signed
// wavenumbers of Eq. (wavenumbers) and the rectangular mask of Eq.
// (shadow-mask).  Only the masked band |j_alpha| <= N_alpha/4 is ever
// materialised: the residual moments are real, so the contiguous axis keeps
// j = 0..N/4 (the negative half follows by conjugate symmetry) and the other
// axes keep |j| <= N/4.
//
// Transforms are Stockham passes of radix 8 (then one of radix 4 or 2 for the
// remaining factors of two) on complex lines held in LDS, ping-ponging between
// two LDS arrays; the
// twiddle table exp(-2 pi i t/N) is precomputed per axis.  The per-wavevector
// 3x3 (2D) / 4x4 (3D) solve of Eq. (schur) runs in FP64 inside the kernel that
// holds the full spectrum line of the last axis.
#pragma once

#include "msc_kernels.h"

namespace msc {


// Eq. (schur) at one wavevector, FP64.  r[0] = F[r_p], r[1..D] = F[r_m];
// out[0] = dp, out[1..D] = du, each scaled by `scale` (the 1/N_Omega of the
// inverse transform).
template <int D>
__device__ __forceinline__ void schur_solve(const double* kv, const double (*r)[2], double a, double nu,
                                            double scale, double (*out)[2]) {
  const double cs2 = 1.0 / 3.0;
  double kk = 0.0;
  for (int b = 0; b < D; ++b) kk += kv[b] * kv[b];
  const double bc = a + nu * kk;
  // k . r_m
  double kr_re = 0.0, kr_im = 0.0;
  for (int b = 0; b < D; ++b) {
    kr_re += kv[b] * r[1 + b][0];
    kr_im += kv[b] * r[1 + b][1];
  }
  // numerator r_p - i (k.r_m)/b ; -i*(x + iy) = y - ix
  const double num_re = r[0][0] + kr_im / bc;
  const double num_im = r[0][1] - kr_re / bc;
  const double den = a + cs2 * kk / bc;
  const double dp_re = num_re / den, dp_im = num_im / den;
  out[0][0] = dp_re * scale;
  out[0][1] = dp_im * scale;
  for (int b = 0; b < D; ++b) {
    // (r_b - cs2 i k_b dp)/b ; i*dp = (-dp_im, dp_re)
    const double re = (r[1 + b][0] + cs2 * kv[b] * dp_im) / bc;
    const double im = (r[1 + b][1] - cs2 * kv[b] * dp_re) / bc;
    out[1 + b][0] = re * scale;
    out[1 + b][1] = im * scale;
  }
}

// Eq. (schur) conjugate-transposed, for the adjoint of the correction:
// solve H^H y = r, H^H = [[a, -i cs2 k^T], [-i k, b I]], b = a + nu |k|^2:
//   y_p = (r_p + i cs2 (k.r_u)/b) / (a + cs2 |k|^2 / b),  y_u = (r_u + i k y_p)/b.
template <int D>
__device__ __forceinline__ void schur_solve_adjoint(const double* kv, const double (*r)[2], double a, double nu,
                                                    double scale, double (*out)[2]) {
  const double cs2 = 1.0 / 3.0;
  double kk = 0.0;
  for (int b = 0; b < D; ++b) kk += kv[b] * kv[b];
  const double bc = a + nu * kk;
  double kr_re = 0.0, kr_im = 0.0;
  for (int b = 0; b < D; ++b) {
    kr_re += kv[b] * r[1 + b][0];
    kr_im += kv[b] * r[1 + b][1];
  }
  const double den = a + cs2 * kk / bc;
  const double yp_re = (r[0][0] - cs2 * kr_im / bc) / den;
  const double yp_im = (r[0][1] + cs2 * kr_re / bc) / den;
  out[0][0] = yp_re * scale;
  out[0][1] = yp_im * scale;
  for (int b = 0; b < D; ++b) {
    out[1 + b][0] = (r[1 + b][0] - kv[b] * yp_im) / bc * scale;
    out[1 + b][1] = (r[1 + b][1] + kv[b] * yp_re) / bc * scale;
  }
}

// Guard shared by the correction kernels: run only right after sweep ell of
// step n without acceptance (Algorithm 1 mode), or always (diagnostic mode).
struct CorrGuard {
  const DevCtl* ctl;
  int n, ell;
  __device__ bool skip() const { return ctl && !phase_correct(ctl->phase, n, ell); }
};

// ---------------------------------------------------------------- 2D ----
// Pass 1: forward transform along y (contiguous) of the three residual-moment
// rows of each x, keeping j_y = 0..N_y/4.  Rows (r_p, r_x) share one complex
// transform (real/imaginary packing); r_y takes a second one.
template <class CT, class TM>
struct Fft2Args {
  CorrGuard g;
  int do_accept;  // Algorithm 1 mode: the first pass decides acceptance (and reconstructs m^{n+1})
  int decide_only;  // with do_accept: take the decision only (the sweep left P r out)
  int decide;     // the row pass ran inside the sweep: the column pass decides instead
  int adjoint;    // apply chi H^{-H} (transpose of the correction) instead of chi H^{-1}
  int Nx, Ny, lgx, lgy;
  int NBy;      // N_y/4 + 1
  int rows_per_block, cols_per_block;
  const TM* Pr;            // 3 x Nx x Ny
  cpx<CT>* spec;           // 3 x Nx x NBy
  TM* dm;                  // 3 x Nx x Ny
  const cpx<CT>* twx;      // Nx
  const cpx<CT>* twy;      // Ny
  double a, nu, inv_ns;
};

template <class L, class T, class CT, class TM>
__global__ __launch_bounds__(256) void k_fft2_rows_fwd(Fft2Args<CT, TM> A, AcceptArgs<L, T> Ac, FinishArgs Fin) {
  if (A.do_accept) {
    // Algorithm 1: decide on sweep ell of step n here; if accepted,
    // reconstruct m^{n+1} on this block's rows instead of transforming
    __shared__ double red[256];
    const int dec = finish_block(Fin, red);
    if (dec != DEC_RUNNING) {
      if (dec == DEC_ACCEPTED) {
        const int64_t s0 = (int64_t)blockIdx.x * A.rows_per_block * A.Ny;
        accept_sites<L, T>(Ac, s0 + threadIdx.x, s0 + (int64_t)A.rows_per_block * A.Ny, blockDim.x);
      }
      return;
    }
    if (A.decide_only) return;
  } else if (A.g.skip()) {
    return;
  }
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  const int Ny = A.Ny, R = A.rows_per_block;
  cpx<CT>* tmp = buf + 2 * R * Ny;
  const int x0 = blockIdx.x * R;
  const int64_t NS = (int64_t)A.Nx * Ny;
  for (int i = threadIdx.x; i < R * Ny; i += blockDim.x) {
    const int r = i / Ny, y = i - r * Ny;
    const int64_t s = (int64_t)(x0 + r) * Ny + y;
    buf[(2 * r) * Ny + y] = {(CT)A.Pr[s], (CT)A.Pr[NS + s]};
    buf[(2 * r + 1) * Ny + y] = {(CT)A.Pr[2 * NS + s], (CT)0};
  }
  __syncthreads();
  const cpx<CT>* out = lds_fft<CT>(buf, tmp, A.lgy, 2 * R, -1, A.twy);
  const int NB = A.NBy;
  for (int i = threadIdx.x; i < R * NB; i += blockDim.x) {
    const int r = i / NB, j = i - r * NB;
    const cpx<CT> z = out[(2 * r) * Ny + j];
    const cpx<CT> zc = out[(2 * r) * Ny + ((Ny - j) & (Ny - 1))];
    // unpack: F0 = (Z(j) + conj Z(-j))/2, F1 = (Z(j) - conj Z(-j))/(2i)
    const cpx<CT> f0 = {(CT)0.5 * (z.x + zc.x), (CT)0.5 * (z.y - zc.y)};
    const cpx<CT> f1 = {(CT)0.5 * (z.y + zc.y), (CT)0.5 * (zc.x - z.x)};
    const int64_t o = (int64_t)(x0 + r) * NB + j;
    const int64_t FS = (int64_t)A.Nx * NB;
    A.spec[o] = f0;
    A.spec[FS + o] = f1;
    A.spec[2 * FS + o] = out[(2 * r + 1) * Ny + j];
  }
}

// Pass 2: for a group of j_y columns, forward transform along x, the FP64
// Schur solve on the band |j_x| <= N_x/4 (zero elsewhere), and the inverse
// transform along x, in place in the band spectrum array.
template <class L, class T, class CT, class TM>
__global__ __launch_bounds__(512) void k_fft2_cols_solve(Fft2Args<CT, TM> A, AcceptArgs<L, T> Ac, FinishArgs Fin) {
  if (A.decide) {
    // Algorithm 1 with the row pass fused into the sweep: decide here; if
    // accepted, reconstruct m^{n+1} over the whole field instead
    __shared__ double red[4];
    const int dec = finish_block(Fin, red);
    if (dec != DEC_RUNNING) {
      if (dec == DEC_ACCEPTED)
        accept_sites<L, T>(Ac, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, Ac.NS,
                           (int64_t)gridDim.x * blockDim.x);
      return;
    }
  } else if (A.g.skip()) {
    return;
  }
  // XCD-aware column order over the first pad8(column blocks) blocks; the
  // rest (decision mode) only reconstruct
  const int Nx = A.Nx, JB = A.cols_per_block, NB = A.NBy;
  const int GC = pad8((NB + JB - 1) / JB);
  const int cbk = ((int)blockIdx.x < GC) ? xcd_item(blockIdx.x, GC) : (int)blockIdx.x;
  if (cbk * JB >= NB) return;  // padding or reconstruction-only block
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  cpx<CT>* tmp = buf + 3 * JB * Nx;
  const int j0 = cbk * JB;
  const int64_t FS = (int64_t)Nx * NB;
  // transform t = f*JB + c holds column j0 + c of field f
  for (int i = threadIdx.x; i < 3 * JB * Nx; i += blockDim.x) {
    const int c = i % JB;
    const int rest = i / JB;
    const int x = rest % Nx, f = rest / Nx;
    const int j = j0 + c;
    buf[(f * JB + c) * Nx + x] = (j < NB) ? A.spec[f * FS + (int64_t)x * NB + j] : cpx<CT>{0, 0};
  }
  __syncthreads();
  cpx<CT>* F = lds_fft<CT>(buf, tmp, A.lgx, 3 * JB, -1, A.twx);
  cpx<CT>* G = (F == buf) ? tmp : buf;
  const double two_pi = 6.283185307179586476925286766559;
  for (int i = threadIdx.x; i < JB * Nx; i += blockDim.x) {
    const int c = i / Nx, jx = i - c * Nx;
    const int jy = j0 + c;
    const int sjx = signed_index(jx, Nx);
    if (jy < NB && in_band(sjx, Nx)) {
      double kv[2] = {two_pi * sjx / Nx, two_pi * jy / A.Ny};
      double r[3][2], o[3][2];
      for (int f = 0; f < 3; ++f) {
        const cpx<CT> v = F[(f * JB + c) * Nx + jx];
        r[f][0] = (double)v.x;
        r[f][1] = (double)v.y;
      }
      if (A.adjoint)
        schur_solve_adjoint<2>(kv, r, A.a, A.nu, A.inv_ns, o);
      else
        schur_solve<2>(kv, r, A.a, A.nu, A.inv_ns, o);
      for (int f = 0; f < 3; ++f) G[(f * JB + c) * Nx + jx] = {(CT)o[f][0], (CT)o[f][1]};
    } else {
      for (int f = 0; f < 3; ++f) G[(f * JB + c) * Nx + jx] = {(CT)0, (CT)0};
    }
  }
  __syncthreads();
  cpx<CT>* H = lds_fft<CT>(G, F, A.lgx, 3 * JB, +1, A.twx);
  for (int i = threadIdx.x; i < 3 * JB * Nx; i += blockDim.x) {
    const int c = i % JB;
    const int rest = i / JB;
    const int x = rest % Nx, f = rest / Nx;
    const int j = j0 + c;
    if (j < NB) A.spec[f * FS + (int64_t)x * NB + j] = H[(f * JB + c) * Nx + x];
  }
}

// Pass 3: inverse transform along y from the half band to real rows.  The
// band of field f at x is extended by conjugate symmetry (Z(N - j) =
// conj Z(j)); fields 0 and 1 share one complex inverse transform (real and
// imaginary parts), field 2 uses the real part of a second one.
template <class CT, class TM>
__global__ __launch_bounds__(256) void k_fft2_rows_inv(Fft2Args<CT, TM> A) {
  if (A.g.skip()) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  const int Ny = A.Ny, R = A.rows_per_block, NB = A.NBy;
  cpx<CT>* tmp = buf + 2 * R * Ny;
  const int x0 = blockIdx.x * R;
  const int64_t FS = (int64_t)A.Nx * NB;
  for (int i = threadIdx.x; i < R * Ny; i += blockDim.x) {
    const int r = i / Ny, j = i - r * Ny;
    const int64_t o = (int64_t)(x0 + r) * NB;
    cpx<CT> a0 = {0, 0}, a1 = {0, 0}, a2 = {0, 0};
    if (j < NB) {
      a0 = A.spec[o + j];
      a1 = A.spec[FS + o + j];
      a2 = A.spec[2 * FS + o + j];
      if (j == 0) {
        a0.y = 0;
        a1.y = 0;
        a2.y = 0;
      }
    } else if (Ny - j < NB) {
      const int jj = Ny - j;
      a0 = A.spec[o + jj];
      a1 = A.spec[FS + o + jj];
      a2 = A.spec[2 * FS + o + jj];
      a0.y = -a0.y;
      a1.y = -a1.y;
      a2.y = -a2.y;
    }
    // pack a0 + i a1
    buf[(2 * r) * Ny + j] = {a0.x - a1.y, a0.y + a1.x};
    buf[(2 * r + 1) * Ny + j] = a2;
  }
  __syncthreads();
  const cpx<CT>* out = lds_fft<CT>(buf, tmp, A.lgy, 2 * R, +1, A.twy);
  const int64_t NS = (int64_t)A.Nx * Ny;
  for (int i = threadIdx.x; i < R * Ny; i += blockDim.x) {
    const int r = i / Ny, y = i - r * Ny;
    const int64_t s = (int64_t)(x0 + r) * Ny + y;
    const cpx<CT> z = out[(2 * r) * Ny + y];
    A.dm[s] = (TM)z.x;
    A.dm[NS + s] = (TM)z.y;
    A.dm[2 * NS + s] = (TM)out[(2 * r + 1) * Ny + y].x;
  }
}

// ---------------------------------------------------------------- 3D ----
// Five passes over the band |j_alpha| <= N_alpha/4: forward along z (real
// input, keeps j_z = 0..N_z/4), forward along y (keeps the y band), along x
// with the FP64 4x4 Schur solve of Eq. (schur) between the forward and
// inverse transforms, inverse along y, inverse along z to real fields.
// spec1 holds [field][x][y][j_z] (after the z passes), spec2 holds
// [field][x][band_y][j_z] (after the y passes).
template <class CT, class TM>
struct Fft3Args {
  CorrGuard g;
  int do_accept;
  int decide_only;  // with do_accept: take the decision only (the sweep left P r out)
  int adjoint;
  int Nx, Ny, Nz, lgx, lgy, lgz;
  int NBz;  // N_z/4 + 1
  int NBy;  // 2 (N_y/4) + 1 retained y indices
  int pencils_per_block, cols_per_block;
  const TM* Pr;        // 4 x N_sites
  TM* dm;              // 4 x N_sites
  cpx<CT>* spec1;      // 4 x Nx*Ny x NBz
  cpx<CT>* spec2;      // 4 x Nx*NBy x NBz
  const cpx<CT>* twx;
  const cpx<CT>* twy;
  const cpx<CT>* twz;
  double a, nu, inv_ns;
};

__device__ inline int band_to_j(int i, int N, int NB) { return (i <= N / 4) ? i : N - (NB - i); }

// pass 1: forward along z of pencils (x, y); fields (0,1) and (2,3) packed.
// The grid holds as many blocks as the device runs at once and each block
// loops over groups of R pencils, so that the acceptance decision (a chain
// of dependent loads) is taken once per block rather than once per group.
template <class L, class T, class CT, class TM>
__global__ __launch_bounds__(256) void k_fft3_z_fwd(Fft3Args<CT, TM> A, AcceptArgs<L, T> Ac, FinishArgs Fin) {
  const int R = A.pencils_per_block, Nz = A.Nz;
  const int ngrp = (A.Nx * A.Ny) / R;
  if (A.do_accept) {
    __shared__ double red[256];
    const int dec = finish_block(Fin, red);
    if (dec != DEC_RUNNING) {
      if (dec == DEC_ACCEPTED) {
        for (int g = blockIdx.x; g < ngrp; g += gridDim.x) {
          const int64_t s0 = (int64_t)g * R * Nz;
          accept_sites<L, T>(Ac, s0 + threadIdx.x, s0 + (int64_t)R * Nz, blockDim.x);
        }
      }
      return;
    }
    if (A.decide_only) return;
  } else if (A.g.skip()) {
    return;
  }
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  cpx<CT>* tmp = buf + 2 * R * Nz;
  const int64_t NS = (int64_t)A.Nx * A.Ny * Nz;
  const int NB = A.NBz;
  const int64_t FS = (int64_t)A.Nx * A.Ny * NB;
  for (int g = blockIdx.x; g < ngrp; g += gridDim.x) {
    const int64_t p0 = (int64_t)g * R;
    for (int i = threadIdx.x; i < R * Nz; i += blockDim.x) {
      const int r = i / Nz, z = i - r * Nz;
      const int64_t s = (p0 + r) * Nz + z;
      buf[(2 * r) * Nz + z] = {(CT)A.Pr[s], (CT)A.Pr[NS + s]};
      buf[(2 * r + 1) * Nz + z] = {(CT)A.Pr[2 * NS + s], (CT)A.Pr[3 * NS + s]};
    }
    __syncthreads();
    const cpx<CT>* out = lds_fft<CT>(buf, tmp, A.lgz, 2 * R, -1, A.twz);
    for (int i = threadIdx.x; i < R * NB; i += blockDim.x) {
      const int r = i / NB, j = i - r * NB;
      const int64_t o = (p0 + r) * NB + j;
      for (int h = 0; h < 2; ++h) {
        const cpx<CT> z = out[(2 * r + h) * Nz + j];
        const cpx<CT> zc = out[(2 * r + h) * Nz + ((Nz - j) & (Nz - 1))];
        A.spec1[(2 * h) * FS + o] = {(CT)0.5 * (z.x + zc.x), (CT)0.5 * (z.y - zc.y)};
        A.spec1[(2 * h + 1) * FS + o] = {(CT)0.5 * (z.y + zc.y), (CT)0.5 * (zc.x - z.x)};
      }
    }
    __syncthreads();  // buf and tmp are refilled by the next group
  }
}

// pass 2: forward along y for a group of j_z columns at one x; keep the band
template <class CT, class TM>
__global__ __launch_bounds__(256) void k_fft3_y_fwd(Fft3Args<CT, TM> A) {
  if (A.g.skip()) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  const int Ny = A.Ny, JB = A.cols_per_block, NBz = A.NBz;
  cpx<CT>* tmp = buf + 4 * JB * Ny;
  const int ngroups = (NBz + JB - 1) / JB;
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= A.Nx * ngroups) return;  // grid padding
  const int x = item / ngroups, j0 = (item % ngroups) * JB;
  const int64_t FS1 = (int64_t)A.Nx * Ny * NBz, FS2 = (int64_t)A.Nx * A.NBy * NBz;
  for (int i = threadIdx.x; i < 4 * JB * Ny; i += blockDim.x) {
    const int c = i % JB, rest = i / JB;
    const int y = rest % Ny, f = rest / Ny;
    const int j = j0 + c;
    buf[(f * JB + c) * Ny + y] = (j < NBz) ? A.spec1[f * FS1 + ((int64_t)x * Ny + y) * NBz + j] : cpx<CT>{0, 0};
  }
  __syncthreads();
  const cpx<CT>* out = lds_fft<CT>(buf, tmp, A.lgy, 4 * JB, -1, A.twy);
  for (int i = threadIdx.x; i < 4 * JB * A.NBy; i += blockDim.x) {
    const int c = i % JB, rest = i / JB;
    const int bi = rest % A.NBy, f = rest / A.NBy;
    const int j = j0 + c;
    if (j < NBz)
      A.spec2[f * FS2 + ((int64_t)x * A.NBy + bi) * NBz + j] = out[(f * JB + c) * Ny + band_to_j(bi, Ny, A.NBy)];
  }
}

// pass 3: along x for a group of j_z columns at one band-y index: forward,
// FP64 Schur solve on |j_x| <= N_x/4 (zero elsewhere), inverse; in place
template <class CT, class TM>
__global__ __launch_bounds__(256) void k_fft3_x_solve(Fft3Args<CT, TM> A) {
  if (A.g.skip()) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  const int Nx = A.Nx, JB = A.cols_per_block, NBz = A.NBz, NBy = A.NBy;
  cpx<CT>* tmp = buf + 4 * JB * Nx;
  const int ngroups = (NBz + JB - 1) / JB;
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= NBy * ngroups) return;  // grid padding
  const int bi = item / ngroups, j0 = (item % ngroups) * JB;
  const int64_t FS2 = (int64_t)Nx * NBy * NBz;
  for (int i = threadIdx.x; i < 4 * JB * Nx; i += blockDim.x) {
    const int c = i % JB, rest = i / JB;
    const int x = rest % Nx, f = rest / Nx;
    const int j = j0 + c;
    buf[(f * JB + c) * Nx + x] = (j < NBz) ? A.spec2[f * FS2 + ((int64_t)x * NBy + bi) * NBz + j] : cpx<CT>{0, 0};
  }
  __syncthreads();
  cpx<CT>* F = lds_fft<CT>(buf, tmp, A.lgx, 4 * JB, -1, A.twx);
  cpx<CT>* Gb = (F == buf) ? tmp : buf;
  const double two_pi = 6.283185307179586476925286766559;
  const int sjy = signed_index(band_to_j(bi, A.Ny, NBy), A.Ny);
  for (int i = threadIdx.x; i < JB * Nx; i += blockDim.x) {
    const int c = i / Nx, jx = i - c * Nx;
    const int jz = j0 + c;
    const int sjx = signed_index(jx, Nx);
    if (jz < NBz && in_band(sjx, Nx)) {
      double kv[3] = {two_pi * sjx / Nx, two_pi * sjy / A.Ny, two_pi * jz / A.Nz};
      double r[4][2], o[4][2];
      for (int f = 0; f < 4; ++f) {
        const cpx<CT> v = F[(f * JB + c) * Nx + jx];
        r[f][0] = (double)v.x;
        r[f][1] = (double)v.y;
      }
      if (A.adjoint)
        schur_solve_adjoint<3>(kv, r, A.a, A.nu, A.inv_ns, o);
      else
        schur_solve<3>(kv, r, A.a, A.nu, A.inv_ns, o);
      for (int f = 0; f < 4; ++f) Gb[(f * JB + c) * Nx + jx] = {(CT)o[f][0], (CT)o[f][1]};
    } else {
      for (int f = 0; f < 4; ++f) Gb[(f * JB + c) * Nx + jx] = {(CT)0, (CT)0};
    }
  }
  __syncthreads();
  cpx<CT>* H = lds_fft<CT>(Gb, F, A.lgx, 4 * JB, +1, A.twx);
  for (int i = threadIdx.x; i < 4 * JB * Nx; i += blockDim.x) {
    const int c = i % JB, rest = i / JB;
    const int x = rest % Nx, f = rest / Nx;
    const int j = j0 + c;
    if (j < NBz) A.spec2[f * FS2 + ((int64_t)x * NBy + bi) * NBz + j] = H[(f * JB + c) * Nx + x];
  }
}

// pass 4: inverse along y from the band to every y, for a group of j_z at x
template <class CT, class TM>
__global__ __launch_bounds__(256) void k_fft3_y_inv(Fft3Args<CT, TM> A) {
  if (A.g.skip()) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  const int Ny = A.Ny, JB = A.cols_per_block, NBz = A.NBz, NBy = A.NBy;
  cpx<CT>* tmp = buf + 4 * JB * Ny;
  const int ngroups = (NBz + JB - 1) / JB;
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= A.Nx * ngroups) return;  // grid padding
  const int x = item / ngroups, j0 = (item % ngroups) * JB;
  const int64_t FS1 = (int64_t)A.Nx * Ny * NBz, FS2 = (int64_t)A.Nx * NBy * NBz;
  for (int i = threadIdx.x; i < 4 * JB * Ny; i += blockDim.x) {
    const int c = i % JB, rest = i / JB;
    const int jy = rest % Ny, f = rest / Ny;
    const int j = j0 + c;
    cpx<CT> v = {0, 0};
    const int bi = (jy <= Ny / 4) ? jy : ((Ny - jy <= Ny / 4) ? NBy - (Ny - jy) : -1);
    if (j < NBz && bi >= 0) v = A.spec2[f * FS2 + ((int64_t)x * NBy + bi) * NBz + j];
    buf[(f * JB + c) * Ny + jy] = v;
  }
  __syncthreads();
  const cpx<CT>* out = lds_fft<CT>(buf, tmp, A.lgy, 4 * JB, +1, A.twy);
  for (int i = threadIdx.x; i < 4 * JB * Ny; i += blockDim.x) {
    const int c = i % JB, rest = i / JB;
    const int y = rest % Ny, f = rest / Ny;
    const int j = j0 + c;
    if (j < NBz) A.spec1[f * FS1 + ((int64_t)x * Ny + y) * NBz + j] = out[(f * JB + c) * Ny + y];
  }
}

// pass 5: inverse along z from j_z = 0..N_z/4 (conjugate-symmetric
// extension, real part at j_z = 0) to real fields; (0,1) and (2,3) packed
template <class CT, class TM>
__global__ __launch_bounds__(256) void k_fft3_z_inv(Fft3Args<CT, TM> A) {
  if (A.g.skip()) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  const int R = A.pencils_per_block, Nz = A.Nz, NB = A.NBz;
  cpx<CT>* tmp = buf + 2 * R * Nz;
  const int64_t p0 = (int64_t)blockIdx.x * R;
  const int64_t FS = (int64_t)A.Nx * A.Ny * NB;
  for (int i = threadIdx.x; i < R * Nz; i += blockDim.x) {
    const int r = i / Nz, j = i - r * Nz;
    const int64_t o = (p0 + r) * NB;
    cpx<CT> v[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    if (j < NB) {
      for (int f = 0; f < 4; ++f) {
        v[f] = A.spec1[f * FS + o + j];
        if (j == 0) v[f].y = 0;
      }
    } else if (Nz - j < NB) {
      for (int f = 0; f < 4; ++f) {
        v[f] = A.spec1[f * FS + o + (Nz - j)];
        v[f].y = -v[f].y;
      }
    }
    buf[(2 * r) * Nz + j] = {v[0].x - v[1].y, v[0].y + v[1].x};
    buf[(2 * r + 1) * Nz + j] = {v[2].x - v[3].y, v[2].y + v[3].x};
  }
  __syncthreads();
  const cpx<CT>* out = lds_fft<CT>(buf, tmp, A.lgz, 2 * R, +1, A.twz);
  const int64_t NS = (int64_t)A.Nx * A.Ny * Nz;
  for (int i = threadIdx.x; i < R * Nz; i += blockDim.x) {
    const int r = i / Nz, z = i - r * Nz;
    const int64_t s = (p0 + r) * Nz + z;
    const cpx<CT> a = out[(2 * r) * Nz + z];
    const cpx<CT> b = out[(2 * r + 1) * Nz + z];
    A.dm[s] = (TM)a.x;
    A.dm[NS + s] = (TM)a.y;
    A.dm[2 * NS + s] = (TM)b.x;
    A.dm[3 * NS + s] = (TM)b.y;
  }
}

}  // namespace msc
