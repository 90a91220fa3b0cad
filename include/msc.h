/*
 * msc.h -- C ABI of the MI355X (gfx950) MSC-LBM library.
 *
 * The library advances the fully discrete lattice Boltzmann population
 * equation on a periodic D2Q9 or D3Q19 lattice by BDF dual-time stepping,
 * where every physical step solves the population fixed point
 * T_{q,h_q}(f) = f (paper Sec. 2.1, Eq. fixed-point-problem) with the
 * macroscopic-shadow-corrected inner iteration of Algorithm 1, and also runs
 * the explicit collide-stream march that uses the same sweep kernel
 * (Sec. 4.1, last paragraph).
 *
 * Conventions shared by every entry point
 *  - All calls return msc_status; MSC_OK is 0.  No C++ exception crosses this
 *    interface.
 *  - Field layout is the canonical site order: site(x, y) = x*Ny + y in 2D and
 *    ((x*Ny) + y)*Nz + z in 3D (last index fastest).  Population arrays are
 *    direction-major, f[k*N_sites + site], with the direction ordering of
 *    App. A (Eq. d2q9, d3q19).  Hydrodynamic fields m = (p_hat, u_1..u_d) are
 *    stored as m[b*N_sites + site], b = 0 the pressure-like variable.
 *  - Host arrays are FP64 regardless of the storage precision the context
 *    computes in; they are converted at the boundary.  With
 *    params.inputs_on_device set, msc_init's initial fields and
 *    msc_moments's outputs are device pointers instead.
 *  - All device work is ordered on params.stream (a hipStream_t, or NULL for
 *    a stream the context creates).  Calls that return host-visible data
 *    synchronise that stream.
 *  - A context is not thread-safe; separate contexts are independent.
 *  - After a HIP runtime error the context is unusable: every later call
 *    returns MSC_ERR_STATE until msc_free.
 *  - Nothing here allocates on the host side on behalf of the caller; all
 *    buffers passed in are owned by the caller and only read or written for
 *    the duration of the call.
 */
#ifndef MSC_H_
#define MSC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum msc_status {
  MSC_OK = 0,
  MSC_ERR_INVALID_ARG = 1,   /* a parameter or size outside the supported range */
  MSC_ERR_OUT_OF_MEMORY = 2, /* device allocation failed */
  MSC_ERR_DEVICE = 3,        /* a HIP runtime call failed (context now unusable) */
  MSC_ERR_STATE = 4,         /* context unusable after an earlier device error */
  MSC_ERR_NONCONVERGED = 5,  /* K_max inner iterations without acceptance (Alg. 1, last line) */
  MSC_ERR_NONFINITE = 6,     /* a non-finite raw residual (never accepted, Sec. 4.1) */
  MSC_ERR_UNSUPPORTED = 7    /* valid request the library does not implement */
} msc_status;

typedef enum msc_lattice { MSC_D2Q9 = 2, MSC_D3Q19 = 3 } msc_lattice;

typedef enum msc_corrector {
  MSC_CORRECTOR_PICARD = 0, /* plain fixed-point iteration f <- T(f) */
  MSC_CORRECTOR_SHADOW = 1, /* periodic macroscopic shadow correction (Alg. 1) */
  /* Off-design reference corrector (Sec. 4.1, Eq. full-symbol): the sweep
   * linearised about the rest state (p, u) = (1, 0) has the per-wavevector
   * symbol Z(k) J (Z(k) = diag(exp(-i k.c_q)), J the collision Jacobian at
   * rest for the case's omega+-, a); each inner iteration solves
   * [I - Z(k) J] df^ = r^ on all Q fields and every wavevector and sets
   * f <- f + df, with the raw-residual test of Algorithm 1.  D2Q9 only, FP64
   * or FP32 storage, extents up to 512 (FP32) / 256 (FP64); J in closed
   * form (the paper forms it by a forward difference of step 1e-7). */
  MSC_CORRECTOR_FULL_SYMBOL = 2,
  /* Wall-bounded kinetic correction (Sec. 3.3, Algorithm 2) for
   * MSC_BOUNDARY_CAVITY: each inner iteration solves (I - L) df = r with
   * L = B_Gamma S blkdiag(J^C(x)) (Eq. wall-global-jacobian; J^C of Eq.
   * wall-local-jacobian at a reference field) and sets f <- f + df.  The
   * operator is frozen at rest (p = 1, u = 0, s = 0, assembled with the BDF2
   * coefficient) or, with MSC_WALL_ADAPTIVE, re-linearised at the current
   * iterate under the residual guard of Algorithm 2.  The library solves the
   * system by restarted GMRES preconditioned with the periodic full-symbol
   * inverse at rest (the paper factors it with a sparse direct solver), to
   * the relative residual krylov_tol.  D2Q9, omega+ = omega- = 1 (Eq.
   * wall-G holds there), FP64 storage, extents up to 256. */
  MSC_CORRECTOR_WALL_KINETIC = 3
} msc_corrector;

typedef enum msc_boundary {
  MSC_BOUNDARY_PERIODIC = 0, /* every axis periodic (the Fourier correctors) */
  /* D2Q9 lid-driven cavity (Sec. 3.3): after streaming (with the periodic
   * wrap) the wall rows of Eq. (bounceback-rows) are overwritten in the
   * printed order y = 0, y = N_y - 1 (the lid, moving along +x at u_lid),
   * x = 0, x = N_x - 1, so the side walls own the corners.  Correctors:
   * MSC_CORRECTOR_PICARD or MSC_CORRECTOR_WALL_KINETIC; the explicit march
   * and the diagnostic sweep apply the same rows. */
  MSC_BOUNDARY_CAVITY = 1
} msc_boundary;

typedef enum msc_wall_operator {
  MSC_WALL_FROZEN = 0,  /* Algorithm 2, frozen branch: the initial operator for the whole run */
  MSC_WALL_ADAPTIVE = 1 /* Algorithm 2, adaptive branch: residual-guarded refresh (<= 3 per step) */
} msc_wall_operator;

typedef enum msc_storage {
  MSC_STORAGE_FP64 = 0, /* FP64 populations, FP64 arithmetic */
  MSC_STORAGE_FP32 = 1, /* FP32 populations and arithmetic; FP64 BDF history
                           combination, collision temporaries, residual reductions and
                           per-wavevector solve */
  MSC_STORAGE_FP16_DEV = 2 /* populations as g = (f - feq(P f))/sigma in FP16 plus P f in
                              FP32, sigma a power of two chosen from the data when a state
                              is set (msc_init, msc_set_populations, msc_set_state); FP32
                              arithmetic as MSC_STORAGE_FP32.  The rebuild keeps P f equal
                              to the stored moments; the raw residual is taken against the
                              stored output.  A deviation beyond the FP16 range becomes
                              non-finite and fails the step (MSC_ERR_NONFINITE) */
} msc_storage;

typedef struct msc_params {
  int32_t lattice;   /* msc_lattice */
  int32_t n[3];      /* extents (x, y, z); powers of two >= 4; n[2] ignored in 2D */
  double tau_plus;   /* TRT relaxation times (Eq. trt); both > 1/2.  nu = (tau_plus - 1/2)/3 */
  double tau_minus;
  double dt;         /* physical BDF step, > 0, in lattice time units */
  double eps;        /* raw-residual RMS acceptance tolerance, > 0 (Eq. residual) */
  int32_t k_max;     /* inner iteration cap, >= 1 */
  int32_t n_min;     /* minimum inner count before acceptance, >= 1 */
  int32_t corrector; /* msc_corrector */
  int32_t storage;   /* msc_storage */
  int32_t inputs_on_device; /* see conventions */
  /* Population states used for the initial trial of a physical step.  0 (the
   * default) is the paper's rule (Sec. 3.1): f^n, then 2 f^n - f^{n-1}, then
   * 3 f^n - 3 f^{n-1} + f^{n-2} once enough accepted states exist.  1, 2, 3
   * cap it at constant, linear, cubic.  A cap below 3 is a deviation from the
   * paper; it changes iteration counts only, never the fixed point. */
  int32_t extrap_states;
  void* stream;      /* hipStream_t, or NULL */
  /* Optional device allocator (e.g. a framework's caching allocator).  When
   * alloc_fn is NULL the library uses hipMalloc/hipFree. */
  void* (*alloc_fn)(size_t bytes, void* user);
  void (*free_fn)(void* ptr, void* user);
  void* alloc_user;
  int32_t boundary;      /* msc_boundary (default MSC_BOUNDARY_PERIODIC) */
  int32_t wall_operator; /* msc_wall_operator (MSC_CORRECTOR_WALL_KINETIC) */
  double u_lid;          /* lid velocity along +x (MSC_BOUNDARY_CAVITY) */
  int32_t wall_forced;   /* Algorithm 2's forced refresh interval N_forced, 0 = off (the paper's setting) */
  int32_t wall_restart;  /* GMRES restart length of the wall corrector, 0 = 50, at most 64 */
  double krylov_tol;     /* relative residual of the wall corrector's solve, 0 = 1e-12 */
} msc_params;

/* Per physical step record (Alg. 1; Eq. rho-observed for rho_obs). */
typedef struct msc_step_stats {
  int32_t q;         /* BDF order used: 1 on the first step after a reset, else 2 */
  int32_t iters;     /* inner sweeps performed (the accepted one included) */
  double R_first;    /* raw residual RMS of the first sweep */
  double R_final;    /* raw residual RMS of the last sweep */
  double rho_obs;    /* tail geometric-mean contraction, NaN if fewer than 3 residuals */
  int32_t converged; /* 1 if accepted */
  int32_t refreshes; /* Algorithm 2: operator refreshes in this step (wall-kinetic corrector), else 0 */
} msc_step_stats;

typedef struct msc_ctx msc_ctx;

/* Fill *p with the paper's operating point (nu = 1/6, Lambda = 1/4 so
 * tau+ = tau- = 1; K_max = 300; n_min = 2 in 2D, 1 in 3D; shadow corrector;
 * FP64 storage) for a cubic/square grid of side n and the given dt and eps
 * (Sec. 4.1, Tab. 1).  Returns MSC_ERR_INVALID_ARG for an unknown lattice. */
msc_status msc_params_default(msc_params* p, int32_t lattice, int32_t n, double dt, double eps);

/* Create a context (paper Sec. 4.1 initial state).
 * phat0: N_sites FP64, u0: d*N_sites FP64, canonical order (see top).
 * Sets f^0 = feq(phat0, u0) (Eq. feq) and m^0 = P f^0 (Eq. moments); the next
 * BDF step is BDF1 (Eq. bdf2).  Inputs are copied during the call.
 * Errors: MSC_ERR_INVALID_ARG (extent not a power of two or < 4, tau <= 1/2,
 * dt <= 0, eps <= 0, k_max < 1, n_min < 1, unknown lattice/storage/corrector,
 * NULL pointers); MSC_ERR_OUT_OF_MEMORY; MSC_ERR_DEVICE; MSC_ERR_UNSUPPORTED
 * with the shadow corrector for a grid larger than the transform kernels
 * support (2D: x extent up to 2048 in FP32 and 1024 in FP64, y extent up to
 * 4096 and 2048; 3D: every extent up to 2048 and 1024), and with the
 * full-symbol corrector outside D2Q9, FP64/FP32 storage and extents up to
 * 512 (FP32) / 256 (FP64).  *out is owned by the library until msc_free. */
msc_status msc_init(const msc_params* p, const double* phat0, const double* u0, msc_ctx** out);

/* Advance nsteps physical steps by Algorithm 1 (or Picard with
 * MSC_CORRECTOR_PICARD): BDF1 on the first step after a reset, BDF2 after
 * (Eq. bdf2); initial trial by population-history extrapolation; acceptance
 * when the inner count >= n_min and the raw residual RMS < eps; on acceptance
 * m^{n+1} = R(f_T) with the step's histories, then the histories rotate
 * (Sec. 3.1).  stats: NULL or an array of nsteps records (caller-owned).
 * Errors: MSC_ERR_NONCONVERGED (K_max reached) or MSC_ERR_NONFINITE: the
 * context stays at the last accepted step and stats are filled up to and
 * including the failing step.  MSC_ERR_INVALID_ARG for nsteps < 0. */
msc_status msc_bdf2_step(msc_ctx* c, int32_t nsteps, msc_step_stats* stats);

/* Advance nsteps lattice steps of the source-free TRT map (the sweep with
 * a = 0, h = 0: m = P f, no source; Sec. 4.1: the explicit baseline uses the
 * same collision and streaming).  With periodic boundaries and FP64 or FP32
 * storage the march runs in place by the AA access pattern (pairs of steps on
 * one population array; an odd count ends with one step of the two-buffer
 * sweep), otherwise on the two-buffer sweep; both give identical results
 * (msc_set_tuning key 10).  Resets the BDF history: the next
 * msc_bdf2_step is BDF1 from the current state with m^n = P f^n.
 * Errors: MSC_ERR_INVALID_ARG (nsteps < 0); MSC_ERR_NONFINITE when the final
 * state holds a non-finite value (checked once at the end). */
msc_status msc_explicit_step(msc_ctx* c, int64_t nsteps);

/* Current hydrodynamic field: after BDF steps m^n = R(f^n) with that step's
 * histories (Alg. 1); after explicit steps or msc_set_populations, P f.
 * phat: N_sites FP64, u: d*N_sites FP64 (host, or device if flagged). */
msc_status msc_moments(msc_ctx* c, double* phat, double* u);

/* Release everything; NULL-safe. */
void msc_free(msc_ctx* c);

const char* msc_status_string(msc_status s);
/* Message of the last failure on this context; valid until the next call. */
const char* msc_last_error(const msc_ctx* c);

/* ------------------------------------------------------------------------ */
/* Diagnostic and test entry points.  Same conventions and error codes.      */

/* Canonical index tables computed by the device with the index arithmetic
 * the kernels use.  nbr: Q*N_sites int32, nbr[k*N_sites + s] = site of
 * (x + c_k) mod N (push target, Eq. sweep); signed_idx: n[0] + n[1] (+ n[2])
 * int32, the signed wavenumber index of Eq. (wavenumbers) per axis; mask:
 * N_sites uint8, chi of Eq. (shadow-mask) (1 where 4|j_alpha| <= N for every
 * alpha).  Any pointer may be NULL to skip that table.  Host buffers. */
msc_status msc_export_tables(msc_ctx* c, int32_t* nbr, int32_t* signed_idx, uint8_t* mask);

/* Copy the current populations f^n to / from a host FP64 array
 * (Q*N_sites).  msc_set_populations rounds to the storage precision, sets
 * m^n = P f and resets the BDF history (next step BDF1). */
msc_status msc_get_populations(msc_ctx* c, double* f);
msc_status msc_set_populations(msc_ctx* c, const double* f);

/* One evaluation of the sweep T_{q,h}(f) (Eq. sweep) with its raw residual
 * (Eq. residual), on the device.  f: Q*N_sites, h: (d+1)*N_sites (NULL
 * means h = 0), a: the BDF coefficient a_q (0 for the source-free map).
 * Outputs (any may be NULL): fT (Q*N_sites), Pr ((d+1)*N_sites, the residual
 * moments P r), R (scalar RMS).  Host FP64 arrays.  Does not change the
 * context's march state. */
msc_status msc_sweep(msc_ctx* c, const double* f, const double* h, double a, double* fT,
                     double* Pr, double* R);

/* One corrected iteration (Alg. 1 body): fT = T(f), r = fT - f,
 * dm = F^{-1}[chi H^{-1} F[P r]] (Eq. schur, shadow-update) and
 * f_next = fT + E dm (Eq. lift).  With MSC_CORRECTOR_FULL_SYMBOL instead
 * f_next = f + F^{-1}[(I - Z J)^{-1} F[r]] (Eq. full-symbol) and dm is set
 * to zero.  Outputs (any may be NULL): f_next, dm ((d+1)*N_sites), R.  Host
 * FP64.  Does not change the march state. */
msc_status msc_correct(msc_ctx* c, const double* f, const double* h, double a, double* f_next,
                       double* dm, double* R);

/* Replay a recorded inner schedule: the next nsteps BDF steps accept at
 * exactly K[i] sweeps regardless of eps (K[i] >= 1).  K == NULL or
 * nsteps == 0 clears it.  The schedule is consumed by msc_bdf2_step. */
msc_status msc_set_schedule(msc_ctx* c, const int32_t* K, int32_t nsteps);

/* Checkpoint of the march state: f^n, f^{n-1}, f^{n-2} (3*Q*N_sites),
 * m^n, m^{n-1} (2*(d+1)*N_sites) as FP64 host arrays, and the number of BDF
 * steps accepted since the last reset.  msc_state_size gives the FP64 count
 * of the array part. */
msc_status msc_state_size(const msc_ctx* c, int64_t* n_doubles);
msc_status msc_get_state(msc_ctx* c, double* state, int64_t* bdf_count);
msc_status msc_set_state(msc_ctx* c, const double* state, int64_t bdf_count);

/* Discrete adjoint of the march (the transpose of the unrolled computation:
 * inner iterations of Alg. 1 at their accepted counts, Eq. sweep, schur,
 * shadow-update, lift, macro-reconstruct, bdf2 and the trial
 * extrapolation).  It is an extension of the method, which defines no
 * adjoint; it differentiates the discrete map, acceptance counts held fixed.
 *
 * msc_set_recording(c, 1) clears earlier records and makes every later
 * msc_bdf2_step keep, per accepted step, a device checkpoint of the state at
 * the step's start (the five arrays of msc_get_state in the storage
 * precision, m in FP64), its BDF count and its inner count K_n.  While
 * recording, msc_bdf2_step synchronises once per physical step.  A step that
 * fails is not recorded.  msc_set_recording(c, 0) stops and frees the
 * records; a new context does not record.  msc_recorded_steps returns their
 * number. */
msc_status msc_set_recording(msc_ctx* c, int32_t enable);
msc_status msc_recorded_steps(const msc_ctx* c, int32_t* count);

/* Backward pass over the last nsteps recorded steps (1 <= nsteps <= the
 * recorded count), which are consumed, so successive calls walk further back.
 * lam holds msc_state_size FP64 values in the msc_get_state layout: on entry
 * the adjoint (gradient) of a scalar loss with respect to the state after
 * the last of those steps, on return its adjoint with respect to the state
 * before the first of them.  Each step's inner iterates are recomputed in
 * FP64 from its checkpoint, and all adjoint arithmetic (transforms included)
 * is FP64, whatever the storage precision.  lam is a device pointer when
 * on_device is nonzero.  MSC_ERR_INVALID_ARG for nsteps outside that range;
 * MSC_ERR_UNSUPPORTED with the shadow corrector where the FP64 transforms do
 * not fit (2D: x extent > 1024 or y extent > 2048; 3D: an extent > 1024),
 * and with the full-symbol corrector.
 * The march state is not changed. */
msc_status msc_bdf2_adjoint(msc_ctx* c, int32_t nsteps, double* lam, int32_t on_device);

/* Adjoint of msc_init's map from (p_hat0, u0) to the initial state
 * (f0, f0, f0, P f0, P f0) with f0 = feq(p_hat0, u0) (Eq. feq, moments):
 * given lam (msc_state_size values), writes lam_phat0 (N_sites) and lam_u0
 * (d*N_sites).  All five arrays are host FP64 unless on_device is nonzero.
 * Does not change the march state. */
msc_status msc_init_adjoint(msc_ctx* c, const double* phat0, const double* u0, const double* lam,
                            double* lam_phat0, double* lam_u0, int32_t on_device);

/* Kernel timing for roofline reports: when enabled, every launch of the
 * population sweep kernel is bracketed by HIP events on the context's stream
 * and its duration accumulated.  msc_kernel_time returns the total seconds,
 * launch count and algorithmic bytes per launch of the sweep (explicit and
 * dual-time launches counted separately: kind 0 = dual-time sweep, 1 =
 * explicit sweep).  Enabling resets the counters. */
msc_status msc_set_kernel_timing(msc_ctx* c, int32_t enable);

/* Counters of the wall corrector's linear solves since msc_init (Sec. 3.3):
 * solves = corrected inner iterations, iters = GMRES iterations over them,
 * refreshes = operator re-linearisations (adaptive branch); worst_rel = the
 * largest final relative residual ||(I - L) df - r|| / ||r|| reached.  Any
 * output may be NULL.  Zero for the other correctors. */
msc_status msc_krylov_stats(msc_ctx* c, int64_t* solves, int64_t* iters, int64_t* refreshes,
                            double* worst_rel);
msc_status msc_kernel_time(msc_ctx* c, int32_t kind, double* seconds, int64_t* launches,
                           double* bytes_per_launch);

/* Launch-shape knobs for tuning sweeps: key 0 = sweep tile size in sites
 * (0 = automatic; must match an available tile), key 1 = planes per strip of
 * the sweep (0 = automatic), key 2 = physical steps enqueued per
 * host synchronisation (>= 1, default 32), 3 = speculative inner iterations
 * enqueued beyond the previous step's count (>= 0, default 0), 4 = capture
 * explicit-march chunks in HIP graphs (0/1, default 1), 5 = sweep tile by
 * its 1-based position in the library's tile table (0 = automatic; overrides
 * key 0), 6 = in 2D with tiles spanning whole rows, do the correction's row
 * transforms inside the sweep: 0 = neither, 1 = the forward one, 2 = the
 * forward one and, with one-plane strips, the inverse one before the lift
 * (default 2), 7 / 8 = z pencils / j_z columns per block of the 3D
 * transform passes (0 = automatic; capped by the LDS), 9 = the full-symbol
 * corrector's column pass as three kernels (x transforms, per-wavevector
 * solve, inverse transforms): 0 = automatic (split from N_x = 512), 1 =
 * split, 2 = one fused kernel, 10 = march msc_explicit_step in place by the
 * AA pattern (pairs of steps on one population array; periodic boundaries
 * with FP64 or FP32 storage; 0/1, default 1), 11 = D3Q19 with N_z = 128: run
 * the dual-time sweeps after the first of a step on 4 x 128 tiles of 512
 * threads (0/1, default 1), 12 = with the shadow corrector and FP64 or FP32
 * storage, in 3D and in 2D where the row transforms run as passes of their
 * own (N_y above 256): the lift sweep enqueued as the last of its step (the
 * step is predicted to accept there) leaves out the residual moments P r, which are
 * formed afterwards from that sweep's input and output only if the step goes
 * on (0/1, default 1).  Results do not depend on these beyond rounding order
 * (keys 6 = 1 and 2 give identical results; keys 10, 11 and 12 give identical
 * populations).  MSC_ERR_INVALID_ARG for an unknown key or value. */
msc_status msc_set_tuning(msc_ctx* c, int32_t key, int32_t value);

/* ------------------------------------------------------------------------ */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * evaluation of the sweep, as msc_sweep computes it, on caller-owned device
 * buffers, with no context and no allocation.  It launches the same kernel,
 * tile and strip length as a context's msc_sweep with automatic launch shapes,
 * so fT and Pr are bit-identical to msc_sweep's and R agrees to rounding.
 *
 * lattice: MSC_D2Q9 or MSC_D3Q19.  n: extents (2 or 3 int32, powers of two
 * >= 4).  tau_plus, tau_minus > 1/2 (Eq. trt).  storage: MSC_STORAGE_FP64
 * (T = double) or MSC_STORAGE_FP32 (T = float).  Device arrays in canonical
 * site order (x slowest), direction- or field-major: f (in) and fT (out)
 * Q*N_sites of T; h (in) (d+1)*N_sites FP64, required (zeros give the
 * source-free map); Pr (out) (d+1)*N_sites of T, the residual moments P r;
 * R (out) one FP64 on the device, the RMS raw residual, or NULL.  a: the BDF
 * coefficient a_q (>= 0).  stream: a hipStream_t (NULL = the default
 * stream); the call only enqueues work and returns without synchronising.
 * The caller keeps ownership of every buffer.
 *
 * Device memory of its own: the per-block partial sums of r^2 live in a
 * fixed array of 65536 doubles (512 KiB) that each GPU holds from the first
 * call on it until the process ends; grids with more sweep blocks than that
 * (far beyond N = 16384^2 in 2D) return MSC_ERR_INVALID_ARG.  Every call on
 * one GPU uses that one array, so calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 *
 * Errors: MSC_ERR_INVALID_ARG (unknown lattice, extents, rates, a, storage,
 * NULL buffers other than R, or a grid beyond the fixed array);
 * MSC_ERR_UNSUPPORTED (MSC_STORAGE_FP16_DEV); MSC_ERR_DEVICE (a launch
 * failed). */
msc_status msc_sweep_noalloc(int32_t lattice, const int32_t* n, double tau_plus, double tau_minus,
                             int32_t storage, const void* f, const double* h, double a, void* fT, void* Pr,
                             double* R, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MSC_H_ */
