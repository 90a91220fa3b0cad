// Full-symbol reference correction (paper Sec. 4.1, Eq. full-symbol) on the
// periodic D2Q9 lattice: the sweep linearised about the uniform rest state
// (p, u) = (1, 0) has the per-wavevector symbol Z(k) J, with
// Z(k) = diag(exp(-i k . c_q)) (push streaming under the transform
// convention of Eq. fft-convention) and J the collision Jacobian at rest.  The
// correction solves [I - Z(k) J] df^(k) = r^(k) on all Q population fields
// and every wavevector and sets f <- f + df.
//
// J is taken in closed form (derived from Eq. collision with Eq.
// macro-reconstruct and Eq. source-moments at u = 0, s = 0):
//   J = B + U V,  B = (1 - w+) Pi+ + (1 - w-) Pi-,
//   U = [c+ E0 | c- Eu],  V = [P0 ; Pu],  c+- = [w+- - a (1 - w+-/2)] / (1 + a/2),
// where Pi+- are the even/odd projections over opposite pairs, E0 = w,
// Eu = w c / cs2, P0 = 1, Pu = c.  The paper evaluates J by a forward
// difference of step 1e-7 at rest; the closed form is that derivative
// without the difference's truncation error.
//
// Per wavevector the Q x Q solve uses the Woodbury identity instead of a
// dense factorisation: A = I - Z B couples only the pair (q, opp q) (and the
// rest direction alone), so A^{-1} is explicit; the rank-(d+1) part leaves a
// (d+1) x (d+1) capacitance system S = I - V A^{-1} Z U:
//   y = A^{-1} r^,  S z = V y,  df^ = y + A^{-1} Z U z.
// All of it runs in FP64 in registers.  The pair determinant
// 1 - (b+ + b-) cos(k.c_q) + b+ b-  (b+- = 1 - w+-) is >= w+ w- > 0 for
// w+- in (0, 2).
//
// Data path (the sweep writes the raw residual r = T(f) - f of all Q fields):
//   rows pass   r rows -> forward transform along y, half spectrum j_y <= N_y/2
//               (real rows packed two to a complex line); the first pass also
//               takes the acceptance decision of Algorithm 1;
//   column pass for a group of j_y: forward transform along x, the solve at
//               every (j_x, j_y), output df^ - r^, inverse transform along x;
//   rows pass   inverse transform along y back to real rows and
//               f_{l+1} = f_T + (df - r) = f_l + df in place in the sweep's
//               output buffer, which the next sweep reads.
#pragma once

#include "msc_fft.h"

namespace msc {

template <class T, class CT, class TM>
struct FsArgs {
  CorrGuard g;
  int do_accept;  // the rows pass decides acceptance (Algorithm 1 mode)
  int Nx, Ny, lgx, lgy;
  int NH;  // N_y/2 + 1 retained j_y
  int rows_per_block, cols_per_block;
  const TM* r;             // Q x Nx x Ny residual of the last sweep
  cpx<CT>* spec;           // Q x Nx x NH
  const cpx<CT>* twx;      // Nx
  const cpx<CT>* twy;      // Ny
  double a, wp, wm, inv_ns;
  FBufs<T> fb;             // population buffers (output through the roles) ...
  T* out;                  // ... or this buffer when g.ctl is null
  // plain solve: out = F^{-1}[(I - Z J)^{-1} F[r]] itself (the column pass
  // keeps df^, the inverse rows overwrite out), e.g. as a preconditioner
  int plain;
};

// Eq. (full-symbol) at one wavevector, FP64: y holds r^ on entry and
// df^ = (I - Z J)^{-1} r^ on return.  kpi[b] = k_b / pi = 2 j_b / N_b (signed
// index j_b), so that exp(-i k_b) comes from sincospi without a large-argument
// reduction and the Q phase factors z_q = exp(-i k . c_q) are products of the
// d axis factors (c_q components are -1, 0, 1).
template <class L>
__device__ inline void fs_solve(const double* kpi, double (*y)[2], double a, double wp, double wm) {
  constexpr int Q = L::Q, D = L::D, D1 = D + 1;
  const double bp = 1.0 - wp, bm = 1.0 - wm;
  const double beta = 0.5 * (bp + bm), gam = 0.5 * (bp - bm);
  const double cpl = (wp - a * (1.0 - 0.5 * wp)) / (1.0 + 0.5 * a);
  const double cmi = (wm - a * (1.0 - 0.5 * wm)) / (1.0 + 0.5 * a);
  double er[D], ei[D];  // exp(-i k_b)
#pragma unroll
  for (int b = 0; b < D; ++b) {
    double sn, cs;
    sincospi(kpi[b], &sn, &cs);
    er[b] = cs;
    ei[b] = -sn;
  }
  double zr[Q], zi[Q];  // z_q = exp(-i k . c_q)
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double pr = 1.0, pi = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const int cb = ca<L>(q, b);
      if (cb == 0) continue;
      const double fr = er[b], fi = (cb > 0) ? ei[b] : -ei[b];
      const double tr = pr * fr - pi * fi;
      pi = pr * fi + pi * fr;
      pr = tr;
    }
    zr[q] = pr;
    zi[q] = pi;
  }
  // 1/det of each opposite pair's 2 x 2 block of A (indexed by the pair's
  // lower direction)
  double invd[Q];
#pragma unroll
  for (int q = 1; q < Q; ++q)
    invd[q] = (L::opp(q) > q) ? 1.0 / (1.0 - 2.0 * beta * zr[q] + beta * beta - gam * gam) : 0.0;
  const double iwp = 1.0 / wp;
  // v <- A^{-1} v in place (A = I - Z B)
  auto apply_Ainv = [&](double (*v)[2]) {
    v[0][0] *= iwp;  // rest direction: 1 - b+ = w+
    v[0][1] *= iwp;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      const int p = L::opp(q);
      if (p < q) continue;
      const double id = invd[q];
      // [[1 - conj(z) beta, z gam], [conj(z) gam, 1 - z beta]] / det
      const double ar = 1.0 - beta * zr[q], ai = beta * zi[q];   // 1 - conj(z) beta
      const double br = gam * zr[q], bi = gam * zi[q];           // z gam
      const double cr = gam * zr[q], ci = -gam * zi[q];          // conj(z) gam
      const double dr = 1.0 - beta * zr[q], di = -beta * zi[q];  // 1 - z beta
      const double xr = v[q][0], xi = v[q][1], yr = v[p][0], yi = v[p][1];
      v[q][0] = (ar * xr - ai * xi + br * yr - bi * yi) * id;
      v[q][1] = (ar * xi + ai * xr + br * yi + bi * yr) * id;
      v[p][0] = (cr * xr - ci * xi + dr * yr - di * yi) * id;
      v[p][1] = (cr * xi + ci * xr + dr * yi + di * yr) * id;
    }
  };
  // U column j at direction q (real): c+ w_q (j = 0), c- w_q c_{q,j-1} / cs2
  auto Ucol = [&](int q, int j) -> double {
    return (j == 0) ? cpl * L::w(q) : cmi * L::w(q) * 3.0 * (double)ca<L>(q, j - 1);
  };
  auto Vrow = [&](int i, int q) -> double { return (i == 0) ? 1.0 : (double)ca<L>(q, i - 1); };

  // capacitance S = I - V A^{-1} Z U, column by column
  double S[D1][D1][2];
  double tmp[Q][2];
#pragma unroll
  for (int j = 0; j < D1; ++j) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const double u = Ucol(q, j);
      tmp[q][0] = zr[q] * u;
      tmp[q][1] = zi[q] * u;
    }
    apply_Ainv(tmp);
#pragma unroll
    for (int i = 0; i < D1; ++i) {
      double sr = (i == j) ? 1.0 : 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        sr -= Vrow(i, q) * tmp[q][0];
        si -= Vrow(i, q) * tmp[q][1];
      }
      S[i][j][0] = sr;
      S[i][j][1] = si;
    }
  }
  // y = A^{-1} r, t = V y
  apply_Ainv(y);
  double t[D1][2];
#pragma unroll
  for (int i = 0; i < D1; ++i) {
    t[i][0] = 0.0;
    t[i][1] = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      t[i][0] += Vrow(i, q) * y[q][0];
      t[i][1] += Vrow(i, q) * y[q][1];
    }
  }
  // S z = t: Gaussian elimination with partial pivoting on the small system
#pragma unroll
  for (int c = 0; c < D1; ++c) {
    int piv = c;
    double best = S[c][c][0] * S[c][c][0] + S[c][c][1] * S[c][c][1];
#pragma unroll
    for (int rr = c + 1; rr < D1; ++rr) {
      const double m2 = S[rr][c][0] * S[rr][c][0] + S[rr][c][1] * S[rr][c][1];
      if (m2 > best) {
        best = m2;
        piv = rr;
      }
    }
#pragma unroll
    for (int rr = c + 1; rr < D1; ++rr) {
      if (rr == piv) {
#pragma unroll
        for (int cc = 0; cc < D1; ++cc) {
          const double s0 = S[c][cc][0], s1 = S[c][cc][1];
          S[c][cc][0] = S[rr][cc][0];
          S[c][cc][1] = S[rr][cc][1];
          S[rr][cc][0] = s0;
          S[rr][cc][1] = s1;
        }
        const double t0 = t[c][0], t1 = t[c][1];
        t[c][0] = t[rr][0];
        t[c][1] = t[rr][1];
        t[rr][0] = t0;
        t[rr][1] = t1;
      }
    }
    const double pr = S[c][c][0], pi = S[c][c][1];
    const double pn = 1.0 / (pr * pr + pi * pi);
#pragma unroll
    for (int rr = c + 1; rr < D1; ++rr) {
      // fac = S[rr][c] / S[c][c]
      const double fr = (S[rr][c][0] * pr + S[rr][c][1] * pi) * pn;
      const double fi = (S[rr][c][1] * pr - S[rr][c][0] * pi) * pn;
#pragma unroll
      for (int cc = c; cc < D1; ++cc) {
        S[rr][cc][0] -= fr * S[c][cc][0] - fi * S[c][cc][1];
        S[rr][cc][1] -= fr * S[c][cc][1] + fi * S[c][cc][0];
      }
      t[rr][0] -= fr * t[c][0] - fi * t[c][1];
      t[rr][1] -= fr * t[c][1] + fi * t[c][0];
    }
  }
  double zz[D1][2];
#pragma unroll
  for (int rr = D1 - 1; rr >= 0; --rr) {
    double ar = t[rr][0], ai = t[rr][1];
#pragma unroll
    for (int cc = rr + 1; cc < D1; ++cc) {
      ar -= S[rr][cc][0] * zz[cc][0] - S[rr][cc][1] * zz[cc][1];
      ai -= S[rr][cc][0] * zz[cc][1] + S[rr][cc][1] * zz[cc][0];
    }
    const double pr = S[rr][rr][0], pi = S[rr][rr][1];
    const double pn = 1.0 / (pr * pr + pi * pi);
    zz[rr][0] = (ar * pr + ai * pi) * pn;
    zz[rr][1] = (ai * pr - ar * pi) * pn;
  }
  // df = y + A^{-1} Z (U z)
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double ur = 0.0, ui = 0.0;
#pragma unroll
    for (int j = 0; j < D1; ++j) {
      const double u = Ucol(q, j);
      ur += u * zz[j][0];
      ui += u * zz[j][1];
    }
    tmp[q][0] = zr[q] * ur - zi[q] * ui;
    tmp[q][1] = zr[q] * ui + zi[q] * ur;
  }
  apply_Ainv(tmp);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    y[q][0] += tmp[q][0];
    y[q][1] += tmp[q][1];
  }
}

// Pass 1: forward transform along y of the Q residual rows of each x
// (fields 2p and 2p+1 packed in one complex line; the last odd field alone),
// half spectrum j_y = 0 .. N_y/2 kept.
template <class L, class T, class CT, class TM>
__global__ __launch_bounds__(256) void k_fs_rows_fwd(FsArgs<T, CT, TM> A, AcceptArgs<L, T> Ac, FinishArgs Fin) {
  constexpr int Q = L::Q, NL = (Q + 1) / 2;
  if (A.do_accept) {
    __shared__ double red[256];
    const int dec = finish_block(Fin, red);
    if (dec != DEC_RUNNING) {
      if (dec == DEC_ACCEPTED) {
        const int64_t s0 = (int64_t)blockIdx.x * A.rows_per_block * A.Ny;
        accept_sites<L, T>(Ac, s0 + threadIdx.x, s0 + (int64_t)A.rows_per_block * A.Ny, blockDim.x);
      }
      return;
    }
  } else if (A.g.skip()) {
    return;
  }
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  const int Ny = A.Ny, R = A.rows_per_block;
  cpx<CT>* tmp = buf + NL * R * Ny;
  const int x0 = blockIdx.x * R;
  const int64_t NS = (int64_t)A.Nx * Ny;
  for (int i = threadIdx.x; i < R * Ny; i += blockDim.x) {
    const int rr = i / Ny, y = i - rr * Ny;
    const int64_t s = (int64_t)(x0 + rr) * Ny + y;
#pragma unroll
    for (int p = 0; p < NL; ++p) {
      const CT re = (CT)A.r[(2 * p) * NS + s];
      const CT im = (2 * p + 1 < Q) ? (CT)A.r[(2 * p + 1) * NS + s] : (CT)0;
      buf[(NL * rr + p) * Ny + y] = {re, im};
    }
  }
  __syncthreads();
  const cpx<CT>* out = lds_fft<CT>(buf, tmp, A.lgy, NL * R, -1, A.twy);
  const int NH = A.NH;
  const int64_t FS = (int64_t)A.Nx * NH;
  for (int i = threadIdx.x; i < R * NH; i += blockDim.x) {
    const int rr = i / NH, j = i - rr * NH;
    const int64_t o = (int64_t)(x0 + rr) * NH + j;
#pragma unroll
    for (int p = 0; p < NL; ++p) {
      const cpx<CT> z = out[(NL * rr + p) * Ny + j];
      if (2 * p + 1 < Q) {
        const cpx<CT> zc = out[(NL * rr + p) * Ny + ((Ny - j) & (Ny - 1))];
        // F_a = (Z(j) + conj Z(-j))/2, F_b = (Z(j) - conj Z(-j))/(2i)
        A.spec[(2 * p) * FS + o] = {(CT)0.5 * (z.x + zc.x), (CT)0.5 * (z.y - zc.y)};
        A.spec[(2 * p + 1) * FS + o] = {(CT)0.5 * (z.y + zc.y), (CT)0.5 * (zc.x - z.x)};
      } else {
        A.spec[(2 * p) * FS + o] = z;
      }
    }
  }
}

// Pass 2: for a group of j_y columns, forward transform along x, the solve of
// Eq. (full-symbol) at every wavevector of the group, inverse transform
// along x, in place in the half spectrum.
template <class L, class T, class CT, class TM>
__global__ __launch_bounds__(256) void k_fs_cols_solve(FsArgs<T, CT, TM> A) {
  constexpr int Q = L::Q;
  if (A.g.skip()) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  const int Nx = A.Nx, JB = A.cols_per_block, NH = A.NH;
  cpx<CT>* tmp = buf + Q * JB * Nx;
  const int cbk = xcd_item(blockIdx.x, gridDim.x);
  if (cbk * JB >= NH) return;  // grid padding
  const int j0 = cbk * JB;
  const int64_t FS = (int64_t)Nx * NH;
  // transform t = q*JB + c holds column j0 + c of field q
  for (int i = threadIdx.x; i < Q * JB * Nx; i += blockDim.x) {
    const int c = i % JB;
    const int rest = i / JB;
    const int x = rest % Nx, q = rest / Nx;
    const int j = j0 + c;
    buf[(q * JB + c) * Nx + x] = (j < NH) ? A.spec[q * FS + (int64_t)x * NH + j] : cpx<CT>{0, 0};
  }
  __syncthreads();
  cpx<CT>* F = lds_fft<CT>(buf, tmp, A.lgx, Q * JB, -1, A.twx);
  cpx<CT>* G = (F == buf) ? tmp : buf;
  for (int i = threadIdx.x; i < JB * Nx; i += blockDim.x) {
    const int c = i / Nx, jx = i - c * Nx;
    const int jy = j0 + c;
    if (jy < NH) {
      const double kpi[2] = {2.0 * signed_index(jx, Nx) / Nx, 2.0 * jy / A.Ny};
      double v[Q][2];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const cpx<CT> z = F[(q * JB + c) * Nx + jx];
        v[q][0] = (double)z.x;
        v[q][1] = (double)z.y;
      }
      fs_solve<L>(kpi, v, A.a, A.wp, A.wm);
      // df^ - r^ (r^ read again from LDS), or df^ for a plain solve, with
      // the 1/N_sites of the inverse
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const cpx<CT> z = F[(q * JB + c) * Nx + jx];
        const double sr = A.plain ? 0.0 : (double)z.x, si = A.plain ? 0.0 : (double)z.y;
        G[(q * JB + c) * Nx + jx] = {(CT)((v[q][0] - sr) * A.inv_ns), (CT)((v[q][1] - si) * A.inv_ns)};
      }
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) G[(q * JB + c) * Nx + jx] = {(CT)0, (CT)0};
    }
  }
  __syncthreads();
  cpx<CT>* H = lds_fft<CT>(G, F, A.lgx, Q * JB, +1, A.twx);
  for (int i = threadIdx.x; i < Q * JB * Nx; i += blockDim.x) {
    const int c = i % JB;
    const int rest = i / JB;
    const int x = rest % Nx, q = rest / Nx;
    const int j = j0 + c;
    if (j < NH) A.spec[q * FS + (int64_t)x * NH + j] = H[(q * JB + c) * Nx + x];
  }
}

// Split form of pass 2 (more parallel at N <= 512, where one block per
// retained column leaves most compute units idle): the x transforms of LB
// (field, j_y) lines per block, then the solve with one wavevector per thread,
// then the inverse x transforms.  Same arithmetic as the fused pass.
template <class L, class T, class CT, class TM>
__global__ __launch_bounds__(256) void k_fs_cols_fft(FsArgs<T, CT, TM> A, int sign) {
  constexpr int Q = L::Q;
  if (A.g.skip()) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  const int Nx = A.Nx, NH = A.NH, LB = A.cols_per_block;
  cpx<CT>* tmp = buf + LB * Nx;
  const int t0 = xcd_item(blockIdx.x, gridDim.x) * LB, nlines = Q * NH;
  if (t0 >= nlines) return;  // grid padding
  const int64_t FS = (int64_t)Nx * NH;
  // line t = q * NH + j: element x at spec[q][x][j]
  for (int i = threadIdx.x; i < LB * Nx; i += blockDim.x) {
    const int c = i % LB, x = i / LB;
    const int t = t0 + c;
    cpx<CT> v = {0, 0};
    if (t < nlines) v = A.spec[(t / NH) * FS + (int64_t)x * NH + (t % NH)];
    buf[c * Nx + x] = v;
  }
  __syncthreads();
  const cpx<CT>* out = lds_fft<CT>(buf, tmp, A.lgx, LB, sign, A.twx);
  for (int i = threadIdx.x; i < LB * Nx; i += blockDim.x) {
    const int c = i % LB, x = i / LB;
    const int t = t0 + c;
    if (t < nlines) A.spec[(t / NH) * FS + (int64_t)x * NH + (t % NH)] = out[c * Nx + x];
  }
}

template <class L, class T, class CT, class TM>
__global__ __launch_bounds__(64) void k_fs_solve_k(FsArgs<T, CT, TM> A) {
  constexpr int Q = L::Q;
  if (A.g.skip()) return;
  const int Nx = A.Nx, NH = A.NH;
  const int64_t FS = (int64_t)Nx * NH;
  const int64_t nk = FS;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (int64_t)gridDim.x * blockDim.x) {
    const int jx = (int)(i / NH), jy = (int)(i - (int64_t)jx * NH);
    const double kpi[2] = {2.0 * signed_index(jx, Nx) / Nx, 2.0 * jy / A.Ny};
    double v[Q][2];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const cpx<CT> z = A.spec[q * FS + i];
      v[q][0] = (double)z.x;
      v[q][1] = (double)z.y;
    }
    fs_solve<L>(kpi, v, A.a, A.wp, A.wm);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const cpx<CT> z = A.spec[q * FS + i];
      const double sr = A.plain ? 0.0 : (double)z.x, si = A.plain ? 0.0 : (double)z.y;
      A.spec[q * FS + i] = {(CT)((v[q][0] - sr) * A.inv_ns), (CT)((v[q][1] - si) * A.inv_ns)};
    }
  }
}

// Pass 3: inverse transform along y from the half spectrum to real rows
// (Z(N_y - j) = conj Z(j); the j = 0 and j = N_y/2 terms of a real row are
// real) and f <- f_T + (df - r) in place in the sweep's output buffer.
template <class L, class T, class CT, class TM>
__global__ __launch_bounds__(256) void k_fs_rows_inv(FsArgs<T, CT, TM> A) {
  constexpr int Q = L::Q, NL = (Q + 1) / 2;
  if (A.g.skip()) return;
  T* __restrict__ dst = A.out;
  if (A.g.ctl) dst = A.fb.p[A.g.ctl->roles[A.g.n & 1].slot_w[A.g.ell & 1]];
  extern __shared__ unsigned char smem_raw[];
  cpx<CT>* buf = reinterpret_cast<cpx<CT>*>(smem_raw);
  const int Ny = A.Ny, R = A.rows_per_block, NH = A.NH;
  cpx<CT>* tmp = buf + NL * R * Ny;
  const int x0 = blockIdx.x * R;
  const int64_t FS = (int64_t)A.Nx * NH;
  for (int i = threadIdx.x; i < R * Ny; i += blockDim.x) {
    const int rr = i / Ny, j = i - rr * Ny;
    const int64_t o = (int64_t)(x0 + rr) * NH;
    const bool lower = j < NH;
    const int jj = lower ? j : Ny - j;
    const bool real_term = (j == 0) || (2 * j == Ny);
#pragma unroll
    for (int p = 0; p < NL; ++p) {
      cpx<CT> a0 = A.spec[(2 * p) * FS + o + jj];
      cpx<CT> a1 = (2 * p + 1 < Q) ? A.spec[(2 * p + 1) * FS + o + jj] : cpx<CT>{0, 0};
      if (real_term) {
        a0.y = 0;
        a1.y = 0;
      } else if (!lower) {
        a0.y = -a0.y;
        a1.y = -a1.y;
      }
      // pack a0 + i a1
      buf[(NL * rr + p) * Ny + j] = {a0.x - a1.y, a0.y + a1.x};
    }
  }
  __syncthreads();
  const cpx<CT>* out = lds_fft<CT>(buf, tmp, A.lgy, NL * R, +1, A.twy);
  const int64_t NS = (int64_t)A.Nx * Ny;
  for (int i = threadIdx.x; i < R * Ny; i += blockDim.x) {
    const int rr = i / Ny, y = i - rr * Ny;
    const int64_t s = (int64_t)(x0 + rr) * Ny + y;
#pragma unroll
    for (int p = 0; p < NL; ++p) {
      const cpx<CT> z = out[(NL * rr + p) * Ny + y];
      const int64_t ia = (2 * p) * NS + s;
      dst[ia] = A.plain ? (T)z.x : (T)((CT)dst[ia] + z.x);
      if (2 * p + 1 < Q) {
        const int64_t ib = (2 * p + 1) * NS + s;
        dst[ib] = A.plain ? (T)z.y : (T)((CT)dst[ib] + z.y);
      }
    }
  }
}

}  // namespace msc
