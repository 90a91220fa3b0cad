// One evaluation of the sweep T_{q,h}(f) (Eq. sweep) with its raw residual
// (Eq. residual) on caller-owned device buffers, for callers that cannot
// allocate device memory.  It launches the same fused sweep kernel, tile and
// strip as a context's msc_sweep; the one device buffer of its own, the
// per-block partial sums of r^2, is a fixed array in device memory shared by
// every call on a GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/msc.h"
#include "msc_sweep_launch.h"

namespace {
// one FP64 partial sum of r^2 per sweep block
constexpr int kScratchDoubles = 65536;
}  // namespace

// Held by each GPU the library runs on until the process ends.  Host code
// never passes this name to a kernel: it takes the array's device address per
// GPU (scratch_on_device) and passes that.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double* scratch_dev[kMaxDevices] = {};

// Device address of this GPU's copy of the scratch array, looked up once per
// device with that device current.
msc_status scratch_on_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MSC_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MSC_ERR_DEVICE;
    scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = scratch_dev[dev];
  return MSC_OK;
}

// R = sqrt(sum of the partials / (Q N_sites)) in one block, folded in a fixed
// order (strided per thread, shuffles within each wavefront, then the
// wavefronts in order), so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_noalloc_rms(const double* __restrict__ partials, int n, double inv_count,
                                                     double* __restrict__ R) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += partials[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) R[0] = sqrt((red[0] + red[1] + red[2] + red[3]) * inv_count);
}

// the dual-time sweep (SW_DTS) for a run-time tile index of the table
template <class T>
void launch_dts(int d, int tile, const msc::SweepArgs<T, T>& A, int grid, hipStream_t st) {
  using namespace msc;
  if (d == 2) {
    switch (tile) {
      case 0: launch_sweep_mode<D2Q9, T, T, 4, 1, 4, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      case 1: launch_sweep_mode<D2Q9, T, T, 8, 1, 8, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      case 2: launch_sweep_mode<D2Q9, T, T, 16, 1, 16, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      case 3: launch_sweep_mode<D2Q9, T, T, 32, 1, 32, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      case 4: launch_sweep_mode<D2Q9, T, T, 64, 1, 64, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      case 5: launch_sweep_mode<D2Q9, T, T, 128, 1, 128, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      default: launch_sweep_mode<D2Q9, T, T, 256, 1, 256, SW_DTS>(A, grid, st, nullptr, nullptr); break;
    }
  } else {
    switch (tile) {
      case 0: launch_sweep_mode<D3Q19, T, T, 16, 4, 4, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      case 1: launch_sweep_mode<D3Q19, T, T, 64, 8, 8, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      case 2: launch_sweep_mode<D3Q19, T, T, 256, 16, 16, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      case 3: launch_sweep_mode<D3Q19, T, T, 256, 8, 32, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      case 4: launch_sweep_mode<D3Q19, T, T, 256, 4, 64, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      case 5: launch_sweep_mode<D3Q19, T, T, 256, 2, 128, SW_DTS>(A, grid, st, nullptr, nullptr); break;
      default: launch_sweep_mode<D3Q19, T, T, 256, 1, 256, SW_DTS>(A, grid, st, nullptr, nullptr); break;
    }
  }
}

template <class L, class T>
msc_status run(const int* n, double tau_plus, double tau_minus, const T* f, const double* h, double a, T* fT,
               T* Pr, double* R, hipStream_t st) {
  using namespace msc;
  const int N0 = n[0];
  const int N1 = (L::D == 2) ? 1 : n[1];
  const int N2 = (L::D == 2) ? n[1] : n[2];
  const int64_t NS = (int64_t)N0 * N1 * N2;
  const int tile_id = auto_sweep_tile<L>(N1, N2);
  const TileCfg base = TileSet<L>::get(tile_id);
  // the wide dual-time tile where a context takes it (D3Q19, N_z = 128)
  const bool wide = L::D == 3 && base.T1 == 2 && base.T2 == 128 && N2 == 128 && N1 >= 4;
  const TileCfg tile = wide ? kWideDualTile3 : base;
  const int strip = sweep_strip_for<L, T>(tile, N0, N1, N2, 0, wide ? STRIP_DUAL_WIDE : STRIP_DUAL);
  const int64_t grid = (int64_t)(N1 / tile.T1) * (N2 / tile.T2) * (N0 / strip);
  if (grid > kScratchDoubles) return MSC_ERR_INVALID_ARG;
  double* parts = nullptr;
  const msc_status ss = scratch_on_device(&parts);
  if (ss != MSC_OK) return ss;
  SweepArgs<T, T> S{};
  S.N0 = N0;
  S.N1 = N1;
  S.N2 = N2;
  S.L = strip;
  S.ntile1 = N1 / tile.T1;
  S.ntile2 = N2 / tile.T2;
  S.nstrip = N0 / strip;
  S.NS = NS;
  S.ctl = nullptr;
  S.src = f;
  S.dst = fT;
  S.h = const_cast<double*>(h);
  S.Pr = Pr;
  S.partials = parts;
  S.a = a;
  S.inv1pa2 = 1.0 / (1.0 + a / 2.0);
  S.wp = 1.0 / tau_plus;
  S.wm = 1.0 / tau_minus;
  S.sig = 1.0f;
  S.isig = 1.0f;
  if constexpr (L::D == 3) {
    if (wide)
      launch_sweep_dual_wide<T, T>(SW_DTS, S, (int)grid, st);
    else
      launch_dts<T>(L::D, tile_id, S, (int)grid, st);
  } else {
    launch_dts<T>(L::D, tile_id, S, (int)grid, st);
  }
  if (hipGetLastError() != hipSuccess) return MSC_ERR_DEVICE;
  if (R) {
    hipLaunchKernelGGL(k_noalloc_rms, dim3(1), dim3(256), 0, st, parts, (int)grid, 1.0 / ((double)L::Q * (double)NS),
                       R);
    if (hipGetLastError() != hipSuccess) return MSC_ERR_DEVICE;
  }
  return MSC_OK;
}

bool pow2_ok(int v) { return v >= 4 && (v & (v - 1)) == 0; }

}  // namespace

extern "C" {

msc_status msc_sweep_noalloc(int32_t lattice, const int32_t* n, double tau_plus, double tau_minus,
                             int32_t storage, const void* f, const double* h, double a, void* fT, void* Pr,
                             double* R, void* stream) {
  const int d = (lattice == MSC_D2Q9) ? 2 : (lattice == MSC_D3Q19 ? 3 : 0);
  if (!d || !n || !f || !h || !fT || !Pr) return MSC_ERR_INVALID_ARG;
  for (int i = 0; i < d; ++i)
    if (!pow2_ok(n[i])) return MSC_ERR_INVALID_ARG;
  if (!(tau_plus > 0.5) || !(tau_minus > 0.5) || !(a >= 0.0) || !std::isfinite(a) || !std::isfinite(tau_plus) ||
      !std::isfinite(tau_minus))
    return MSC_ERR_INVALID_ARG;
  if (storage != MSC_STORAGE_FP64 && storage != MSC_STORAGE_FP32)
    return (storage == MSC_STORAGE_FP16_DEV) ? MSC_ERR_UNSUPPORTED : MSC_ERR_INVALID_ARG;
  const int nn[3] = {n[0], n[1], d == 3 ? n[2] : 1};
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (storage == MSC_STORAGE_FP64) {
    if (d == 2)
      return run<msc::D2Q9, double>(nn, tau_plus, tau_minus, (const double*)f, h, a, (double*)fT, (double*)Pr, R, st);
    return run<msc::D3Q19, double>(nn, tau_plus, tau_minus, (const double*)f, h, a, (double*)fT, (double*)Pr, R, st);
  }
  if (d == 2)
    return run<msc::D2Q9, float>(nn, tau_plus, tau_minus, (const float*)f, h, a, (float*)fT, (float*)Pr, R, st);
  return run<msc::D3Q19, float>(nn, tau_plus, tau_minus, (const float*)f, h, a, (float*)fT, (float*)Pr, R, st);
}

}  // extern "C"
