// C ABI of the library (declarations and contracts in include/msc.h).
// Validates arguments, owns the stream, and forwards to the Solver for the
// context's lattice and storage type.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/msc.h"
#include "msc_solver.h"

struct msc_ctx {
  msc_params p;
  msc::Geometry g;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  msc::SolverBase* s = nullptr;
  std::string err;
};

namespace {

bool pow2_ok(int v) { return v >= 4 && (v & (v - 1)) == 0; }

msc_status fail(msc_ctx* c, msc_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

// Forward the status of a solver call and keep its message.
msc_status fwd(msc_ctx* c, msc_status st) {
  if (st != MSC_OK && c && c->s) c->err = c->s->last_error;
  return st;
}

}  // namespace

extern "C" {

msc_status msc_params_default(msc_params* p, int32_t lattice, int32_t n, double dt, double eps) {
  if (!p || (lattice != MSC_D2Q9 && lattice != MSC_D3Q19)) return MSC_ERR_INVALID_ARG;
  std::memset(p, 0, sizeof(*p));
  p->lattice = lattice;
  p->n[0] = p->n[1] = n;
  p->n[2] = (lattice == MSC_D3Q19) ? n : 1;
  p->tau_plus = 1.0;   // nu = 1/6
  p->tau_minus = 1.0;  // Lambda = 1/4
  p->dt = dt;
  p->eps = eps;
  p->k_max = 300;
  p->n_min = (lattice == MSC_D2Q9) ? 2 : 1;
  p->corrector = MSC_CORRECTOR_SHADOW;
  p->storage = MSC_STORAGE_FP64;
  p->boundary = MSC_BOUNDARY_PERIODIC;
  p->wall_operator = MSC_WALL_FROZEN;
  return MSC_OK;
}

msc_status msc_init(const msc_params* p, const double* phat0, const double* u0, msc_ctx** out) {
  if (!out) return MSC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!p || !phat0 || !u0) return MSC_ERR_INVALID_ARG;
  const int d = (p->lattice == MSC_D2Q9) ? 2 : (p->lattice == MSC_D3Q19 ? 3 : 0);
  if (!d) return MSC_ERR_INVALID_ARG;
  for (int a = 0; a < d; ++a)
    if (!pow2_ok(p->n[a])) return MSC_ERR_INVALID_ARG;
  if (!(p->tau_plus > 0.5) || !(p->tau_minus > 0.5) || !(p->dt > 0.0) || !(p->eps > 0.0) ||
      !std::isfinite(p->dt) || p->k_max < 1 || p->n_min < 1)
    return MSC_ERR_INVALID_ARG;
  if (p->corrector != MSC_CORRECTOR_PICARD && p->corrector != MSC_CORRECTOR_SHADOW &&
      p->corrector != MSC_CORRECTOR_FULL_SYMBOL && p->corrector != MSC_CORRECTOR_WALL_KINETIC)
    return MSC_ERR_INVALID_ARG;
  if (p->boundary != MSC_BOUNDARY_PERIODIC && p->boundary != MSC_BOUNDARY_CAVITY) return MSC_ERR_INVALID_ARG;
  if (p->boundary == MSC_BOUNDARY_CAVITY) {
    // the cavity of Sec. 3.3 is D2Q9; the Fourier correctors need periodic axes
    if (d != 2 || !std::isfinite(p->u_lid)) return MSC_ERR_INVALID_ARG;
    if (p->corrector != MSC_CORRECTOR_PICARD && p->corrector != MSC_CORRECTOR_WALL_KINETIC)
      return MSC_ERR_INVALID_ARG;
  } else if (p->corrector == MSC_CORRECTOR_WALL_KINETIC) {
    return MSC_ERR_INVALID_ARG;
  }
  if (p->wall_operator != MSC_WALL_FROZEN && p->wall_operator != MSC_WALL_ADAPTIVE) return MSC_ERR_INVALID_ARG;
  if (p->wall_forced < 0 || p->wall_restart < 0 || p->wall_restart > 64 || !(p->krylov_tol >= 0.0))
    return MSC_ERR_INVALID_ARG;
  if (p->extrap_states < 0 || p->extrap_states > 3) return MSC_ERR_INVALID_ARG;
  if (p->storage != MSC_STORAGE_FP64 && p->storage != MSC_STORAGE_FP32 &&
      p->storage != MSC_STORAGE_FP16_DEV)
    return MSC_ERR_INVALID_ARG;

  msc_ctx* c = new (std::nothrow) msc_ctx();
  if (!c) return MSC_ERR_OUT_OF_MEMORY;
  c->p = *p;
  msc::Geometry& g = c->g;
  g.d = d;
  g.Q = (d == 2) ? 9 : 19;
  g.n[0] = p->n[0];
  g.n[1] = p->n[1];
  g.n[2] = (d == 3) ? p->n[2] : 1;
  g.N0 = g.n[0];
  if (d == 2) {
    g.N1 = 1;
    g.N2 = g.n[1];
  } else {
    g.N1 = g.n[1];
    g.N2 = g.n[2];
  }
  g.NS = (int64_t)g.n[0] * g.n[1] * g.n[2];
  if (p->stream) {
    c->stream = (hipStream_t)p->stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return MSC_ERR_DEVICE;
    }
    c->own_stream = true;
  }
  if (d == 2) {
    if (p->storage == MSC_STORAGE_FP64)
      c->s = msc::make_solver_d2_fp64(*p, g, c->stream);
    else if (p->storage == MSC_STORAGE_FP32)
      c->s = msc::make_solver_d2_fp32(*p, g, c->stream);
    else
      c->s = msc::make_solver_d2_fp16dev(*p, g, c->stream);
  } else {
    if (p->storage == MSC_STORAGE_FP64)
      c->s = msc::make_solver_d3_fp64(*p, g, c->stream);
    else if (p->storage == MSC_STORAGE_FP32)
      c->s = msc::make_solver_d3_fp32(*p, g, c->stream);
    else
      c->s = msc::make_solver_d3_fp16dev(*p, g, c->stream);
  }
  if (!c->s) {
    msc_free(c);
    return MSC_ERR_OUT_OF_MEMORY;
  }
  msc_status st = c->s->init(phat0, u0, p->inputs_on_device != 0);
  if (st != MSC_OK) {
    msc_free(c);
    return st;
  }
  *out = c;
  return MSC_OK;
}

msc_status msc_bdf2_step(msc_ctx* c, int32_t nsteps, msc_step_stats* stats) {
  if (!c) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  if (nsteps < 0) return fail(c, MSC_ERR_INVALID_ARG, "nsteps < 0");
  return fwd(c, c->s->bdf2_step(nsteps, stats));
}

msc_status msc_explicit_step(msc_ctx* c, int64_t nsteps) {
  if (!c) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  if (nsteps < 0) return fail(c, MSC_ERR_INVALID_ARG, "nsteps < 0");
  return fwd(c, c->s->explicit_step(nsteps));
}

msc_status msc_moments(msc_ctx* c, double* phat, double* u) {
  if (!c) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->moments(phat, u, c->p.inputs_on_device != 0));
}

void msc_free(msc_ctx* c) {
  if (!c) return;
  delete c->s;
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* msc_status_string(msc_status s) {
  switch (s) {
    case MSC_OK: return "ok";
    case MSC_ERR_INVALID_ARG: return "invalid argument";
    case MSC_ERR_OUT_OF_MEMORY: return "out of device memory";
    case MSC_ERR_DEVICE: return "HIP runtime error";
    case MSC_ERR_STATE: return "context unusable after an earlier device error";
    case MSC_ERR_NONCONVERGED: return "inner iteration reached K_max without acceptance";
    case MSC_ERR_NONFINITE: return "non-finite raw residual";
    case MSC_ERR_UNSUPPORTED: return "not supported by this library";
  }
  return "unknown status";
}

const char* msc_last_error(const msc_ctx* c) { return c ? c->err.c_str() : ""; }

msc_status msc_export_tables(msc_ctx* c, int32_t* nbr, int32_t* signed_idx, uint8_t* mask) {
  if (!c) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->export_tables(nbr, signed_idx, mask));
}

msc_status msc_get_populations(msc_ctx* c, double* f) {
  if (!c || !f) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->get_populations(f));
}

msc_status msc_set_populations(msc_ctx* c, const double* f) {
  if (!c || !f) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->set_populations(f));
}

msc_status msc_sweep(msc_ctx* c, const double* f, const double* h, double a, double* fT, double* Pr,
                     double* R) {
  if (!c || !f || !(a >= 0.0)) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->sweep(f, h, a, fT, Pr, R));
}

msc_status msc_correct(msc_ctx* c, const double* f, const double* h, double a, double* f_next,
                       double* dm, double* R) {
  if (!c || !f || !(a > 0.0)) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->correct(f, h, a, f_next, dm, R));
}

msc_status msc_set_schedule(msc_ctx* c, const int32_t* K, int32_t nsteps) {
  if (!c || nsteps < 0) return MSC_ERR_INVALID_ARG;
  return fwd(c, c->s->set_schedule(K, nsteps));
}

msc_status msc_state_size(const msc_ctx* c, int64_t* n_doubles) {
  if (!c || !n_doubles) return MSC_ERR_INVALID_ARG;
  *n_doubles = c->s->state_size();
  return MSC_OK;
}

msc_status msc_get_state(msc_ctx* c, double* state, int64_t* bdf_count) {
  if (!c || !state) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->get_state(state, bdf_count));
}

msc_status msc_set_state(msc_ctx* c, const double* state, int64_t bdf_count) {
  if (!c || !state || bdf_count < 0) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->set_state(state, bdf_count));
}

msc_status msc_set_recording(msc_ctx* c, int32_t enable) {
  if (!c) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->set_recording(enable));
}

msc_status msc_recorded_steps(const msc_ctx* c, int32_t* count) {
  if (!c || !count) return MSC_ERR_INVALID_ARG;
  *count = c->s->recorded_steps();
  return MSC_OK;
}

msc_status msc_bdf2_adjoint(msc_ctx* c, int32_t nsteps, double* lam, int32_t on_device) {
  if (!c || !lam) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->bdf2_adjoint(nsteps, lam, on_device != 0));
}

msc_status msc_init_adjoint(msc_ctx* c, const double* phat0, const double* u0, const double* lam,
                            double* lam_phat0, double* lam_u0, int32_t on_device) {
  if (!c || !phat0 || !u0 || !lam || !lam_phat0 || !lam_u0) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->init_adjoint(phat0, u0, lam, lam_phat0, lam_u0, on_device != 0));
}

msc_status msc_set_kernel_timing(msc_ctx* c, int32_t enable) {
  if (!c) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->set_kernel_timing(enable));
}

msc_status msc_krylov_stats(msc_ctx* c, int64_t* solves, int64_t* iters, int64_t* refreshes,
                            double* worst_rel) {
  if (!c) return MSC_ERR_INVALID_ARG;
  c->s->krylov_stats(solves, iters, refreshes, worst_rel);
  return MSC_OK;
}

msc_status msc_kernel_time(msc_ctx* c, int32_t kind, double* seconds, int64_t* launches,
                           double* bytes_per_launch) {
  if (!c) return MSC_ERR_INVALID_ARG;
  if (c->s->broken) return MSC_ERR_STATE;
  return fwd(c, c->s->kernel_time(kind, seconds, launches, bytes_per_launch));
}

// Launch-shape knobs (declared in msc.h): key 0 = sweep tile size in sites,
// 1 = planes per strip, 2 = physical steps enqueued per host synchronisation,
// 3 = speculative extra iterations, 4 = graph capture of explicit chunks,
// 5 = tile by table index, 6 = row transforms inside the sweep (0/1/2),
// 7 / 8 = pencils / columns per block of the 3D transform passes, 9 = the
// full-symbol column pass split in three kernels (0 auto / 1 split / 2 fused),
// 10 = the in-place (AA) explicit march, 11 = the 512-thread D3Q19 dual-time
// tile at N_z = 128, 12 = the last lift sweep enqueued for a step leaving P r
// out (3D, and 2D with row passes of their own; formed afterwards only if the
// step goes on).
// Keys 0, 1 and 5-8 re-pick the launch shapes at once; the others apply
// from the next call.
msc_status msc_set_tuning(msc_ctx* c, int32_t key, int32_t value) {
  if (!c) return MSC_ERR_INVALID_ARG;
  msc::Tuning& t = c->s->tuning();
  switch (key) {
    case 0: t.sweep_tile = value < 0 ? 0 : value; break;
    case 1: t.sweep_strip = value < 0 ? 0 : value; break;
    case 2: t.batch_steps = value < 1 ? 1 : value; break;
    case 3: t.spec_extra = value < 0 ? 0 : value; break;
    case 4: t.use_graph = value != 0; break;
    case 5: t.sweep_tile_index = value < 0 ? 0 : value; break;
    case 6:
      if (value < 0 || value > 2) return MSC_ERR_INVALID_ARG;
      t.fuse_rows = value;
      break;
    case 7: t.fft3_pencils = value < 0 ? 0 : value; break;
    case 8: t.fft3_cols = value < 0 ? 0 : value; break;
    case 9:
      if (value < 0 || value > 2) return MSC_ERR_INVALID_ARG;
      t.fs_split = value;
      break;
    case 10:
      if (value < 0 || value > 1) return MSC_ERR_INVALID_ARG;
      t.explicit_aa = value;
      break;
    case 11:
      if (value < 0 || value > 1) return MSC_ERR_INVALID_ARG;
      t.wide_dual = value;
      break;
    case 12:
      if (value < 0 || value > 1) return MSC_ERR_INVALID_ARG;
      t.skip_pr = value;
      break;
    default: return MSC_ERR_INVALID_ARG;
  }
  if (key <= 1 || key >= 5) return fwd(c, c->s->reconfigure());
  return MSC_OK;
}

}  // extern "C"
