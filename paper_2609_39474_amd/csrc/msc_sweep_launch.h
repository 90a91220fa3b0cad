// Launch shapes and dispatch of the fused sweep kernel: the tile table per
// lattice, the automatic choice of tile and strip length, and the switch from
// a run-time tile index to the kernel instantiation.  Shared by the solver and
// by the context-free sweep entry point, so both launch the same kernel on
// the same grid.
#pragma once

#include <hip/hip_ext.h>

#include <algorithm>

#include "msc_solver.h"
#include "msc_sweep.h"

namespace msc {

// ----------------------------------------------------------- sweep dispatch --
// Available tiles (T1 x T2 sites of the (p1, p2) plane, NT threads).
struct TileCfg {
  int T1, T2, NT;
};

template <class L>
struct TileSet;
template <>
struct TileSet<D2Q9> {
  static constexpr int count = 7;
  static TileCfg get(int i) {
    const TileCfg t[7] = {{1, 4, 4},     {1, 8, 8},     {1, 16, 16},  {1, 32, 32},
                          {1, 64, 64},   {1, 128, 128}, {1, 256, 256}};
    return t[i];
  }
};
template <>
struct TileSet<D3Q19> {
  static constexpr int count = 7;
  static TileCfg get(int i) {
    const TileCfg t[7] = {{4, 4, 16}, {8, 8, 64}, {16, 16, 256}, {8, 32, 256}, {4, 64, 256}, {2, 128, 256},
                          {1, 256, 256}};
    return t[i];
  }
};

// With ev0/ev1 the launch carries its own start/stop timestamps (kernel
// timing), which adds no packets between this launch and its neighbours.
template <class L, class T, class TM, int NT, int T1, int T2, int MODE>
void launch_sweep_mode(const SweepArgs<T, TM>& A, int grid, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0)
    hipExtLaunchKernelGGL((k_sweep<L, T, TM, NT, T1, T2, MODE>), dim3(grid), dim3(NT), 0, st, ev0, ev1, 0, A);
  else
    hipLaunchKernelGGL((k_sweep<L, T, TM, NT, T1, T2, MODE>), dim3(grid), dim3(NT), 0, st, A);
}

template <class L, class T, class TM, int NT, int T1, int T2>
void launch_sweep_tile(int mode, const SweepArgs<T, TM>& A, int grid, hipStream_t st, hipEvent_t ev0,
                       hipEvent_t ev1) {
  if (mode == SW_EXPLICIT)
    launch_sweep_mode<L, T, TM, NT, T1, T2, SW_EXPLICIT>(A, grid, st, ev0, ev1);
  else if (mode == SW_DTS)
    launch_sweep_mode<L, T, TM, NT, T1, T2, SW_DTS>(A, grid, st, ev0, ev1);
  else if (mode == SW_DTS_LIFT)
    launch_sweep_mode<L, T, TM, NT, T1, T2, SW_DTS_LIFT>(A, grid, st, ev0, ev1);
  else if (mode == SW_DTS_SETUP && A.order <= 1 &&
           (!setup_halo_prefetch<L, T, SW_DTS_SETUP1>() || tile_halo_sites(T1, T2, A.N1, A.N2) <= NT))
    launch_sweep_mode<L, T, TM, NT, T1, T2, SW_DTS_SETUP1>(A, grid, st, ev0, ev1);
  else if (mode == SW_DTS_SETUP)
    launch_sweep_mode<L, T, TM, NT, T1, T2, SW_DTS_SETUP>(A, grid, st, ev0, ev1);
  else if constexpr (T1 == 1 && NT == T2 && L::D == 2)
    launch_sweep_mode<L, T, TM, NT, T1, T2, SW_DTS_LIFT_ROWS>(A, grid, st, ev0, ev1);
  else
    throw DeviceError{hipErrorInvalidValue, "inverse-row lift requested for a tile that does not span rows"};
}


template <class T, class TM>
void launch_sweep_d2(int tile, int mode, const SweepArgs<T, TM>& A, int grid, hipStream_t st,
                     hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
  switch (tile) {
    case 0: launch_sweep_tile<D2Q9, T, TM, 4, 1, 4>(mode, A, grid, st, ev0, ev1); break;
    case 1: launch_sweep_tile<D2Q9, T, TM, 8, 1, 8>(mode, A, grid, st, ev0, ev1); break;
    case 2: launch_sweep_tile<D2Q9, T, TM, 16, 1, 16>(mode, A, grid, st, ev0, ev1); break;
    case 3: launch_sweep_tile<D2Q9, T, TM, 32, 1, 32>(mode, A, grid, st, ev0, ev1); break;
    case 4: launch_sweep_tile<D2Q9, T, TM, 64, 1, 64>(mode, A, grid, st, ev0, ev1); break;
    case 5: launch_sweep_tile<D2Q9, T, TM, 128, 1, 128>(mode, A, grid, st, ev0, ev1); break;
    default: launch_sweep_tile<D2Q9, T, TM, 256, 1, 256>(mode, A, grid, st, ev0, ev1); break;
  }
}
template <class T, class TM>
void launch_sweep_d3(int tile, int mode, const SweepArgs<T, TM>& A, int grid, hipStream_t st,
                     hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
  switch (tile) {
    case 0: launch_sweep_tile<D3Q19, T, TM, 16, 4, 4>(mode, A, grid, st, ev0, ev1); break;
    case 1: launch_sweep_tile<D3Q19, T, TM, 64, 8, 8>(mode, A, grid, st, ev0, ev1); break;
    case 2: launch_sweep_tile<D3Q19, T, TM, 256, 16, 16>(mode, A, grid, st, ev0, ev1); break;
    case 3: launch_sweep_tile<D3Q19, T, TM, 256, 8, 32>(mode, A, grid, st, ev0, ev1); break;
    case 4: launch_sweep_tile<D3Q19, T, TM, 256, 4, 64>(mode, A, grid, st, ev0, ev1); break;
    case 5: launch_sweep_tile<D3Q19, T, TM, 256, 2, 128>(mode, A, grid, st, ev0, ev1); break;
    default: launch_sweep_tile<D3Q19, T, TM, 256, 1, 256>(mode, A, grid, st, ev0, ev1); break;
  }
}

// D3Q19 sweeps after the first of a step (SW_DTS, SW_DTS_LIFT) at N_z = 128:
// a 4 x 128 tile of 512 threads, one halo row per two owned rows instead of
// one per owned row; one block of eight waves per CU (the FP64 rings take
// 148 KB of LDS), the occupancy of two 2 x 128 blocks.  The first sweep keeps
// the 2 x 128 tile (its registers allow one wave per SIMD only).
constexpr TileCfg kWideDualTile3 = {4, 128, 512};
template <class T, class TM>
void launch_sweep_dual_wide(int mode, const SweepArgs<T, TM>& A, int grid, hipStream_t st, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr) {
  if (mode == SW_DTS)
    launch_sweep_mode<D3Q19, T, TM, 512, 4, 128, SW_DTS>(A, grid, st, ev0, ev1);
  else if (mode == SW_DTS_LIFT)
    launch_sweep_mode<D3Q19, T, TM, 512, 4, 128, SW_DTS_LIFT>(A, grid, st, ev0, ev1);
  else
    throw DeviceError{hipErrorInvalidValue, "the wide dual-time tile serves SW_DTS and SW_DTS_LIFT only"};
}

// Automatic tile: the largest tile that fits (measured best at every size;
// the strip length supplies the parallelism).  3D: at N_z = 128 the 2 x 128
// tile, which spans z and so has no z halo (measured at N = 128: 5% per step
// over 4 x 64); otherwise 4 x 64 tiles where they fit (fewer partial-line halo
// columns than 8 x 32 or 16 x 16; measured best at N = 256, where the 1 x 256
// tile's two halo rows per row cost more), else 8 x 32.
template <class L>
int auto_sweep_tile(int N1, int N2) {
  const int n = TileSet<L>::count;
  bool wide_fits = false;  // some tile with a full wavefront fits
  for (int i = 0; i < n; ++i) {
    const TileCfg t = TileSet<L>::get(i);
    if (t.T1 <= N1 && t.T2 <= N2 && t.NT >= 64) wide_fits = true;
  }
  int best = 0;
  for (int i = 0; i < n; ++i) {
    const TileCfg t = TileSet<L>::get(i);
    if (t.T1 > N1 || t.T2 > N2) continue;
    if (wide_fits && t.NT < 64) continue;
    if (L::D == 3) {
      if (N2 == 128 && N1 >= 2) {
        if (!(t.T1 == 2 && t.T2 == 128)) continue;
      } else if (N2 >= 64 && N1 >= 4) {
        if (!(t.T1 == 4 && t.T2 == 64)) continue;
      } else {
        if (t.T1 == 16 && N2 >= 32 && N1 >= 8) continue;
        if (t.T1 < 4) continue;
      }
    }
    best = i;
  }
  return best;
}

// Strip length: the requested one, or the longest strip (at most 64 planes in
// 2D, 32 in 3D) that keeps a target block count: short strips cut the
// per-block chain of plane steps, which bounds small grids; long ones cut the
// two halo planes per strip.  Always a divisor of N0.  Targets by kind:
//
// STRIP_EXPLICIT (the tiled explicit sweep): >= 1024 blocks (2D) or 512 (3D,
// more work per site), the measured optimum at N = 256 ... 4096 (2D) and
// N = 64 ... 256 (3D; with FP64 populations, two blocks per CU with the
// two-barrier rings, 512 blocks against 256: explicit sweep 10% faster).
//
// STRIP_DUAL (the dual-time sweeps after the first of a step): >= 512 blocks
// in 2D, strips twice as long as the explicit sweep's, whose extra halo planes
// weigh more there (each re-collided site also re-reads the history term and
// the correction): 2D corrected march N = 512 FP32 95 -> 84 us per step,
// N = 1024 FP32 191 -> 182 us, FP64 387 -> 333 us (N = 256 and 2048
// unchanged); 3D as the explicit sweep.
//
// STRIP_SETUP (the first sweep of a step): as STRIP_DUAL, except that with FP64
// D3Q19 populations it holds three history states and runs one block per CU;
// one wave of 256 blocks then keeps every tile of a strip resident on its XCD,
// so the halo rows a block re-collides are its neighbours' rows in that XCD's
// L2 (the setup sweep read 2.0x its algorithmic bytes with 512 blocks).
//
// STRIP_DUAL_WIDE (the 512-thread dual-time tile, one block per CU): 256 blocks.
enum StripKind { STRIP_EXPLICIT = 0, STRIP_DUAL = 1, STRIP_SETUP = 2, STRIP_DUAL_WIDE = 3 };

template <class L, class T>
int sweep_strip_for(const TileCfg& tile, int N0, int N1, int N2, int requested, StripKind kind) {
  const int64_t tiles = (int64_t)(N1 / tile.T1) * (N2 / tile.T2);
  int Lp = requested;
  if (Lp <= 0) {
    int64_t target;
    if (L::D == 2)
      target = (kind == STRIP_EXPLICIT) ? 1024 : 512;
    else
      target = ((kind == STRIP_SETUP && sizeof(T) == 8) || kind == STRIP_DUAL_WIDE) ? 256 : 512;
    const int Lmax = (L::D == 2) ? 64 : 32;
    Lp = 1;
    while (Lp < Lmax && tiles * (N0 / (Lp * 2)) >= target) Lp *= 2;
  }
  Lp = std::min(Lp, N0);
  while (N0 % Lp) Lp >>= 1;
  return std::max(Lp, 1);
}

}  // namespace msc
