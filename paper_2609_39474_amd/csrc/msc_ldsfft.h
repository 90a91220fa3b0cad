// Complex arithmetic and the Stockham transform (radix 8, 4, 2) of lines held in
// LDS, shared by the transform passes of the shadow correction and by the
// sweep's fused forward row transform.
#pragma once

#include <hip/hip_runtime.h>

namespace msc {

template <class CT>
struct cpx {
  CT x, y;
};

template <class CT>
__device__ __forceinline__ cpx<CT> cmul(cpx<CT> a, cpx<CT> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class CT>
__device__ __forceinline__ cpx<CT> cadd(cpx<CT> a, cpx<CT> b) {
  return {a.x + b.x, a.y + b.y};
}
template <class CT>
__device__ __forceinline__ cpx<CT> csub(cpx<CT> a, cpx<CT> b) {
  return {a.x - b.x, a.y - b.y};
}
// multiply by +i (s > 0) or -i (s < 0)
template <class CT>
__device__ __forceinline__ cpx<CT> cmuli(cpx<CT> a, int s) {
  return s > 0 ? cpx<CT>{-a.y, a.x} : cpx<CT>{a.y, -a.x};
}

// XCD-aware order of the column passes: a grid of G blocks, G a multiple of 8
// (the host pads it), is dealt to the 8 XCDs round-robin; block b takes work
// item (b mod 8) G/8 + b/8, so that each XCD gets a contiguous range of items
// (adjacent columns, whose values share cache lines) and its L2 serves them.
__device__ __forceinline__ int xcd_item(int b, int G) { return (G & 7) ? b : (b & 7) * (G >> 3) + (b >> 3); }
__host__ __device__ constexpr int pad8(int n) { return (n + 7) / 8 * 8; }

// Bank swizzle of the intermediate stages: element i of a line is stored at
// i with its position inside a 128-byte row XORed with the row number, so the
// strided writes of the early stages (stride 8 or 4 Ns elements) fall on
// different banks; a bijection within every aligned row group, so a line of
// N >= G elements keeps its footprint.
template <class CT>
__device__ __forceinline__ int lds_swz(int i) {
  constexpr int G = 128 / (int)sizeof(cpx<CT>);  // elements per 128-byte row: 8 (FP64), 16 (FP32)
  return i ^ ((i / G) & (G - 1));
}

// 4-point DFT (sign as in lds_fft) of c0..c3, stored at q0 + q*st, q = 0..3
// (swizzled if ws).
template <class CT>
__device__ __forceinline__ void dft4_store(cpx<CT>* y, int q0, int st, bool ws, int sign, cpx<CT> c0, cpx<CT> c1,
                                           cpx<CT> c2, cpx<CT> c3) {
  const cpx<CT> s02 = cadd(c0, c2), d02 = csub(c0, c2);
  const cpx<CT> s13 = cadd(c1, c3), d13 = cmuli(csub(c1, c3), sign);
  y[ws ? lds_swz<CT>(q0) : q0] = cadd(s02, s13);
  y[ws ? lds_swz<CT>(q0 + st) : q0 + st] = cadd(d02, d13);
  y[ws ? lds_swz<CT>(q0 + 2 * st) : q0 + 2 * st] = csub(s02, s13);
  y[ws ? lds_swz<CT>(q0 + 3 * st) : q0 + 3 * st] = csub(d02, d13);
}

// nt independent transforms of length N = 2^lg stored contiguously at
// buf + t*N.  sign = -1 forward, +1 inverse (no scaling).  The caller has
// synchronised after filling buf; returns the array holding the result (buf
// or tmp), synchronised.  Stockham stages of radix 8 while three factors of
// two remain, then one of radix 4 or 2 (N = 128: 8, 8, 2; N = 256: 8, 8, 4).
// The first stage reads and the last stage writes in the plain layout (both
// contiguous); the stages in between keep their outputs swizzled (lds_swz)
// when lines hold at least G elements.
template <class CT>
__device__ __forceinline__ cpx<CT>* lds_fft(cpx<CT>* buf, cpx<CT>* tmp, int lg, int nt, int sign,
                            const cpx<CT>* __restrict__ tw) {
  constexpr int G = 128 / (int)sizeof(cpx<CT>);
  const int N = 1 << lg;
  const int tid = threadIdx.x, nth = blockDim.x;
  const bool swz = N >= G;
  const int n8 = lg / 3, rem = lg - 3 * n8;
  const int nst = n8 + (rem ? 1 : 0);  // stages
  cpx<CT>* a = buf;
  cpx<CT>* b = tmp;
  int Ns = 1;
  for (int p = 0; p < n8; ++p) {
    const int lnb = lg - 3, nb = 1 << lnb;
    const int tstride = N / (8 * Ns);
    const bool rs = swz && p > 0, ws = swz && p + 1 < nst;
    for (int j = tid; j < (nt << lnb); j += nth) {
      const int t = j >> lnb, jj = j & (nb - 1);
      const cpx<CT>* x = a + t * N;
      cpx<CT>* y = b + t * N;
      const int k = jj & (Ns - 1);
      // inputs m = 0..7 at stride N/8, times the twiddles w^(m k)
      cpx<CT> v[8];
      v[0] = x[rs ? lds_swz<CT>(jj) : jj];
#pragma unroll
      for (int m = 1; m < 8; ++m) {
        cpx<CT> w = tw[m * k * tstride];
        if (sign > 0) w.y = -w.y;
        v[m] = cmul(x[rs ? lds_swz<CT>(jj + m * nb) : jj + m * nb], w);
      }
      // 8-point DFT: the even outputs are the 4-point DFT of v_m + v_{m+4},
      // the odd ones that of (v_m - v_{m+4}) e^(sign 2 pi i m / 8)
      cpx<CT> e[4], o[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        e[m] = cadd(v[m], v[m + 4]);
        o[m] = csub(v[m], v[m + 4]);
      }
      const CT r = (CT)0.70710678118654752440;
      const CT sg = (CT)sign;
      o[1] = cpx<CT>{r * (o[1].x - sg * o[1].y), r * (o[1].y + sg * o[1].x)};
      o[2] = cmuli(o[2], sign);
      o[3] = cpx<CT>{r * (-o[3].x - sg * o[3].y), r * (-o[3].y + sg * o[3].x)};
      const int base = ((jj - k) << 3) + k;
      dft4_store(y, base, 2 * Ns, ws, sign, e[0], e[1], e[2], e[3]);       // outputs 0, 2, 4, 6
      dft4_store(y, base + Ns, 2 * Ns, ws, sign, o[0], o[1], o[2], o[3]);  // outputs 1, 3, 5, 7
    }
    __syncthreads();
    cpx<CT>* sw = a;
    a = b;
    b = sw;
    Ns <<= 3;
  }
  if (rem == 2) {
    const int lnb = lg - 2, nb = 1 << lnb;
    const int tstride = N / (4 * Ns);
    const bool rs = swz && n8 > 0;
    for (int j = tid; j < (nt << lnb); j += nth) {
      const int t = j >> lnb, jj = j & (nb - 1);
      const cpx<CT>* x = a + t * N;
      cpx<CT>* y = b + t * N;
      const int k = jj & (Ns - 1);
      cpx<CT> w1 = tw[k * tstride], w2 = tw[2 * k * tstride], w3 = tw[3 * k * tstride];
      if (sign > 0) {
        w1.y = -w1.y;
        w2.y = -w2.y;
        w3.y = -w3.y;
      }
      const cpx<CT> v0 = x[rs ? lds_swz<CT>(jj) : jj];
      const cpx<CT> v1 = cmul(x[rs ? lds_swz<CT>(jj + nb) : jj + nb], w1);
      const cpx<CT> v2 = cmul(x[rs ? lds_swz<CT>(jj + 2 * nb) : jj + 2 * nb], w2);
      const cpx<CT> v3 = cmul(x[rs ? lds_swz<CT>(jj + 3 * nb) : jj + 3 * nb], w3);
      const cpx<CT> s02 = cadd(v0, v2), d02 = csub(v0, v2);
      const cpx<CT> s13 = cadd(v1, v3), d13 = cmuli(csub(v1, v3), sign);
      const int base = ((jj - k) << 2) + k;
      y[base] = cadd(s02, s13);
      y[base + Ns] = cadd(d02, d13);
      y[base + 2 * Ns] = csub(s02, s13);
      y[base + 3 * Ns] = csub(d02, d13);
    }
    __syncthreads();
    a = b;
  } else if (rem == 1) {
    const int lnb = lg - 1, nb = 1 << lnb;
    const int tstride = N / (2 * Ns);
    const bool rs = swz && n8 > 0;
    for (int j = tid; j < (nt << lnb); j += nth) {
      const int t = j >> lnb, jj = j & (nb - 1);
      const cpx<CT>* x = a + t * N;
      cpx<CT>* y = b + t * N;
      const int k = jj & (Ns - 1);
      cpx<CT> w1 = tw[k * tstride];
      if (sign > 0) w1.y = -w1.y;
      const cpx<CT> v0 = x[rs ? lds_swz<CT>(jj) : jj];
      const cpx<CT> v1 = cmul(x[rs ? lds_swz<CT>(jj + nb) : jj + nb], w1);
      const int base = ((jj - k) << 1) + k;
      y[base] = cadd(v0, v1);
      y[base + Ns] = csub(v0, v1);
    }
    __syncthreads();
    a = b;
  }
  return a;
}

}  // namespace msc
