// Shared definitions of the HIP library: lattice traits, the device control
// block that sequences Algorithm 1 on the GPU, and kernel argument records.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msc {

// ------------------------------------------------------------- lattices --
// Discrete velocities, weights and opposites of App. A (Eq. d2q9, d3q19).
// The sweep walks planes along x; a plane is addressed by (p1, p2) with p2
// the contiguous index: (p1, p2) = (-, y) in 2D and (y, z) in 3D.  c1/c2 are
// the velocity components along p1/p2.
struct D2Q9 {
  static constexpr int D = 2, Q = 9;
  __host__ __device__ static constexpr int cx(int k) {
    return (k == 1 || k == 5 || k == 8) ? 1 : ((k == 3 || k == 6 || k == 7) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cy(int k) {
    return (k == 2 || k == 5 || k == 6) ? 1 : ((k == 4 || k == 7 || k == 8) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr int c1(int) { return 0; }
  __host__ __device__ static constexpr int c2(int k) { return cy(k); }
  __host__ __device__ static constexpr int opp(int k) {
    return k == 0 ? 0 : (k <= 4 ? ((k + 1) % 4) + 1 : ((k - 5 + 2) % 4) + 5);
  }
  __host__ __device__ static constexpr double w(int k) {
    return k == 0 ? 4.0 / 9.0 : (k <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

struct D3Q19 {
  static constexpr int D = 3, Q = 19;
  __host__ __device__ static constexpr int cx(int k) {
    return (k == 1 || k == 7 || k == 9 || k == 11 || k == 13)
               ? 1
               : ((k == 2 || k == 8 || k == 10 || k == 12 || k == 14) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cy(int k) {
    return (k == 3 || k == 7 || k == 10 || k == 15 || k == 17)
               ? 1
               : ((k == 4 || k == 8 || k == 9 || k == 16 || k == 18) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cz(int k) {
    return (k == 5 || k == 11 || k == 14 || k == 15 || k == 18)
               ? 1
               : ((k == 6 || k == 12 || k == 13 || k == 16 || k == 17) ? -1 : 0);
  }
  __host__ __device__ static constexpr int c1(int k) { return cy(k); }
  __host__ __device__ static constexpr int c2(int k) { return cz(k); }
  __host__ __device__ static constexpr int opp(int k) { return k == 0 ? 0 : (k % 2 == 1 ? k + 1 : k - 1); }
  __host__ __device__ static constexpr double w(int k) {
    return k == 0 ? 1.0 / 3.0 : (k <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

template <class L>
__host__ __device__ constexpr int ca(int k, int a) {
  return a == 0 ? L::cx(k) : (a == 1 ? L::cy(k) : L::cz(k));
}

// ------------------------------------------------------- control block --
// Algorithm 1 runs as a sequence of kernels enqueued ahead by the host.  The
// device decides acceptance; every kernel launched for (step n, iteration
// ell) first reads one 64-bit phase word and returns at once unless the march
// is exactly at that point.  Only single-block kernels write the phase, so
// the word every block of a grid reads is the same.
enum : uint32_t { PH_RUNNING = 1, PH_ACCEPTED = 2, PH_FAILED = 3 };

__host__ __device__ inline uint64_t make_phase(int n, int ell, uint32_t st) {
  return ((uint64_t)(uint32_t)(n + 1) << 32) | ((uint64_t)(uint32_t)ell << 8) | st;
}
__host__ __device__ inline int phase_n(uint64_t p) { return (int)(uint32_t)(p >> 32) - 1; }
__host__ __device__ inline int phase_ell(uint64_t p) { return (int)((p >> 8) & 0xFFFFFF); }
__host__ __device__ inline uint32_t phase_state(uint64_t p) { return (uint32_t)(p & 0xFF); }

// Before iteration ell of step n (setup of step n counts as "before ell = 1").
__host__ __device__ inline bool phase_ready(uint64_t p, int n, int ell) {
  if (ell == 1) return phase_state(p) == PH_ACCEPTED && phase_n(p) == n - 1;
  return phase_state(p) == PH_RUNNING && phase_n(p) == n && phase_ell(p) == ell - 1;
}
// After sweep ell of step n, not accepted: the correction of ell runs.
__host__ __device__ inline bool phase_correct(uint64_t p, int n, int ell) {
  return phase_state(p) == PH_RUNNING && phase_n(p) == n && phase_ell(p) == ell;
}
// Step n accepted at sweep ell.
__host__ __device__ inline bool phase_accepted(uint64_t p, int n, int ell) {
  return phase_state(p) == PH_ACCEPTED && phase_n(p) == n && phase_ell(p) == ell;
}

struct StepStat {
  int32_t q, iters;
  double R_first, R_final, rho_obs;
  int32_t converged, fail;
};

// Buffer roles during one physical step.
struct Roles {
  int32_t slot_hist[3];  // population buffer index of f^n, f^{n-1}, f^{n-2}
  int32_t slot_w[2];     // the two working buffers of the inner iteration
  int32_t slot_m[3];     // moment buffer index of m^n, m^{n-1} and the spare
};

// The roles of step n live in roles[n & 1]: the acceptance of step n writes
// the rotated roles of step n + 1 into the other copy, so the kernel that
// decides the acceptance can still read step n's roles in every block.
struct DevCtl {
  uint64_t phase;
  int32_t fail_code;
  int32_t pad;
  Roles roles[2];
};

// D2Q9 lid-driven cavity (Sec. 3.3, Eq. bounceback-rows): the wall rows of
// the streamed values v of node (x, y), overwritten in the printed order
// y = 0, y = N_y - 1 (lid moving along +x at ulid), x = 0, x = N_x - 1; each
// copies the current value of another direction of the same node, so the
// side walls own the corners.  With ulid = 0 it is the row replacement of the
// linearised map (the lid constants have no derivative).
template <class CT>
__device__ __forceinline__ void cavity_rows(CT* v, int x, int y, int Nx, int Ny, CT ulid) {
  const CT u6 = ulid / (CT)6;
  if (y == 0) {
    v[2] = v[4];
    v[5] = v[7];
    v[6] = v[8];
  }
  if (y == Ny - 1) {
    v[4] = v[2];
    v[7] = v[5] - u6;
    v[8] = v[6] + u6;
  }
  if (x == 0) {
    v[1] = v[3];
    v[5] = v[7];
    v[8] = v[6];
  }
  if (x == Nx - 1) {
    v[3] = v[1];
    v[6] = v[8];
    v[7] = v[5];
  }
}

// Population buffers (five, roles assigned through DevCtl slots).
template <class T>
struct FBufs {
  T* p[5];
};

// ------------------------------------------- FP16 deviation storage --
// A buffer of element type _Float16 holds populations as their deviation
// from equilibrium: g[k*NS + s] = (f_k - feq_k(M)) / sigma in FP16, followed
// by the moments M = P f as FP32, M[b*NS + s] (starting at element Q*NS).
// sigma is a power of two fixed per state.  The rebuild projects the FP16
// rounding of g out of the conserved moments, so that P f = M exactly:
// g' = g - w_k (sum g + 3 c_k . sum c g) (sum w = 1, sum w c = 0,
// sum w c c = I/3).
template <class T>
struct PopDev {
  static constexpr bool value = false;
};
template <>
struct PopDev<_Float16> {
  static constexpr bool value = true;
};

template <class T>
__host__ __device__ inline float* dev_moments(T* p, int Q, int64_t NS) {
  return reinterpret_cast<float*>(p + (int64_t)Q * NS);
}
template <class T>
__host__ __device__ inline const float* dev_moments(const T* p, int Q, int64_t NS) {
  return reinterpret_cast<const float*>(p + (int64_t)Q * NS);
}

// Equilibrium (Eq. feq) in FP32 from moments M = (p, u).
template <class L>
__device__ inline float feq_f32(int k, const float* M) {
  float cu = 0.f, uu = 0.f;
#pragma unroll
  for (int b = 0; b < L::D; ++b) {
    cu += (float)ca<L>(k, b) * M[1 + b];
    uu += M[1 + b] * M[1 + b];
  }
  return (float)L::w(k) * (M[0] + 3.f * cu + 4.5f * cu * cu - 1.5f * uu);
}

// f from (g, M).
template <class L>
__device__ inline void dev_rebuild(const _Float16* g, const float* M, float sig, float* f) {
  float gs[L::Q], s0 = 0.f, s1[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    gs[k] = (float)g[k];
    s0 += gs[k];
#pragma unroll
    for (int b = 0; b < L::D; ++b)
      if (ca<L>(k, b) != 0) s1[b] += (float)ca<L>(k, b) * gs[k];
  }
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    float cs = 0.f;
#pragma unroll
    for (int b = 0; b < L::D; ++b)
      if (ca<L>(k, b) != 0) cs += (float)ca<L>(k, b) * s1[b];
    f[k] = feq_f32<L>(k, M) + sig * (gs[k] - (float)L::w(k) * (s0 + 3.f * cs));
  }
}

// (g, M) from f.  The moments are summed in AT and rounded to FP32 once: in
// the dual-time sweeps AT = double, because the inner fixed point amplifies a
// systematic rounding of the conserved moments by about dt (as for the
// collision's arithmetic); the explicit map sums in FP32.
template <class L, class AT = float>
__device__ inline void dev_split(const float* f, float isig, _Float16* g, float* M) {
  AT acc[L::D + 1];
#pragma unroll
  for (int b = 0; b <= L::D; ++b) acc[b] = 0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    acc[0] += (AT)f[k];
#pragma unroll
    for (int b = 0; b < L::D; ++b) {
      if (ca<L>(k, b) > 0)
        acc[1 + b] += (AT)f[k];
      else if (ca<L>(k, b) < 0)
        acc[1 + b] -= (AT)f[k];
    }
  }
#pragma unroll
  for (int b = 0; b <= L::D; ++b) M[b] = (float)acc[b];
#pragma unroll
  for (int k = 0; k < L::Q; ++k) g[k] = (_Float16)((f[k] - feq_f32<L>(k, M)) * isig);
}

}  // namespace msc
