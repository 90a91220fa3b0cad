// Host runtime of the library: one Solver<L, T> per (lattice, storage type)
// owns the device buffers and sequences the kernels.  The C ABI in
// msc_api.cpp validates arguments and forwards to the SolverBase interface.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/msc.h"

namespace msc {

struct DeviceError {
  hipError_t err;
  std::string what;
};

struct Geometry {
  int d, Q;
  int n[3];       // user extents (x, y, z)
  int N0, N1, N2; // sweep frame: x, p1, p2
  int64_t NS;
};

struct Tuning {
  int sweep_tile = 0;     // 0 = automatic
  int sweep_strip = 0;    // planes per strip, 0 = automatic
  int batch_steps = 32;   // physical steps enqueued between host synchronisations
  int spec_extra = 0;     // speculative iterations beyond the last step's count
  int use_graph = 1;      // capture explicit chunks in hipGraphs
  int fuse_rows = 2;      // 2D, tiles spanning rows: 1 = forward row transform inside the sweep,
                          // 2 = also the inverse row transform (one-plane strips)
  int sweep_tile_index = 0;  // 1-based entry of the tile table, 0 = automatic
  int fft3_pencils = 0;      // 3D transform passes: z pencils per block, 0 = automatic
  int fft3_cols = 0;         // 3D transform passes: j_z columns per block, 0 = automatic
  int fs_split = 0;          // full-symbol column pass: 0 = automatic, 1 = three kernels
                             // (transforms, solve, transforms), 2 = one fused kernel
  int explicit_aa = 1;       // explicit march in place by the AA pattern where available
  int wide_dual = 1;         // D3Q19 at N_z = 128: the 4 x 128 tile of 512 threads for the
                             // dual-time sweeps after the first of a step
  int skip_pr = 1;           // the lift sweep enqueued last for a step leaves P r out (3D;
                             // 2D with the row transforms as passes of their own)
};

class SolverBase {
 public:
  virtual ~SolverBase() {}
  virtual msc_status init(const double* phat0, const double* u0, bool on_device) = 0;
  virtual msc_status bdf2_step(int32_t nsteps, msc_step_stats* stats) = 0;
  virtual msc_status explicit_step(int64_t nsteps) = 0;
  virtual msc_status moments(double* phat, double* u, bool on_device) = 0;
  virtual msc_status export_tables(int32_t* nbr, int32_t* sidx, uint8_t* mask) = 0;
  virtual msc_status get_populations(double* f) = 0;
  virtual msc_status set_populations(const double* f) = 0;
  virtual msc_status sweep(const double* f, const double* h, double a, double* fT, double* Pr,
                           double* R) = 0;
  virtual msc_status correct(const double* f, const double* h, double a, double* fnext, double* dm,
                             double* R) = 0;
  virtual msc_status set_schedule(const int32_t* K, int32_t nsteps) = 0;
  virtual int64_t state_size() const = 0;
  virtual msc_status get_state(double* state, int64_t* bdf_count) = 0;
  virtual msc_status set_state(const double* state, int64_t bdf_count) = 0;
  virtual msc_status set_kernel_timing(int enable) = 0;
  virtual msc_status kernel_time(int kind, double* seconds, int64_t* launches, double* bytes) = 0;
  virtual msc_status set_recording(int enable) = 0;
  virtual int32_t recorded_steps() const = 0;
  virtual msc_status bdf2_adjoint(int32_t nsteps, double* lam, bool on_device) = 0;
  virtual msc_status init_adjoint(const double* phat0, const double* u0, const double* lam, double* lam_phat0,
                                  double* lam_u0, bool on_device) = 0;
  virtual void krylov_stats(int64_t* solves, int64_t* iters, int64_t* refreshes, double* worst) const = 0;
  virtual Tuning& tuning() = 0;
  virtual msc_status reconfigure() = 0;  // re-pick launch shapes after a tuning change

  std::string last_error;
  bool broken = false;
};

// Factory per (lattice, storage); each lives in its own translation unit.
SolverBase* make_solver_d2_fp64(const msc_params& p, const Geometry& g, hipStream_t s);
SolverBase* make_solver_d2_fp32(const msc_params& p, const Geometry& g, hipStream_t s);
SolverBase* make_solver_d3_fp64(const msc_params& p, const Geometry& g, hipStream_t s);
SolverBase* make_solver_d3_fp32(const msc_params& p, const Geometry& g, hipStream_t s);
SolverBase* make_solver_d2_fp16dev(const msc_params& p, const Geometry& g, hipStream_t s);
SolverBase* make_solver_d3_fp16dev(const msc_params& p, const Geometry& g, hipStream_t s);

}  // namespace msc
