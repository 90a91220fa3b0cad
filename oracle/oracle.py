"""Python binding of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the bench's CPU-baseline leg import this
module.  It wraps ``liboracle.so`` (built from ``msc_oracle.cpp`` by
``build()`` below) with numpy arrays in the canonical layout: populations are
direction-major ``f[k, x, y(, z)]`` and moment fields ``m[b, x, y(, z)]`` with
``b = 0`` the pressure-like variable and ``b = 1..d`` the velocity (Eq.
(moments), Eq. (unknowns) of the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "msc_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle with plain g++ (no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("tau_plus", ctypes.c_double),
        ("tau_minus", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("kmax", ctypes.c_int),
        ("nmin", ctypes.c_int),
        ("corrector", ctypes.c_int),
        ("extrap_states", ctypes.c_int),
        ("fd_step", ctypes.c_double),
    ]


class OrcStepStats(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int),
        ("iters", ctypes.c_int),
        ("R_first", ctypes.c_double),
        ("R_final", ctypes.c_double),
        ("rho_obs", ctypes.c_double),
        ("converged", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_lattice.argtypes = [ctypes.c_int, _ip, _ip, _dp, _ip]
        L.orc_feq_site.argtypes = [ctypes.c_int, _dp, _dp]
        L.orc_phi_site.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.orc_collide_site.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _dp, _dp, _dp]
        L.orc_sweep.argtypes = [ctypes.c_int, _ip, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, _dp, _dp, _dp]
        L.orc_shadow.argtypes = [ctypes.c_int, _ip, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_corrected_iteration.argtypes = [ctypes.c_int, _ip, _dp, _dp, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                              _dp, _dp, _dp, _dp, _dp]
        L.orc_fft.argtypes = [ctypes.c_int, _ip, _dp, _dp, ctypes.c_int]
        L.orc_tables.argtypes = [ctypes.c_int, _ip, _ip, _ip, ctypes.POINTER(ctypes.c_uint8)]
        L.orc_init_populations.argtypes = [ctypes.c_int, _ip, _dp, _dp, _dp]
        L.orc_moments.argtypes = [ctypes.c_int, _ip, _dp, _dp]
        L.orc_explicit.argtypes = [ctypes.c_int, _ip, ctypes.c_double, ctypes.c_double, _dp,
                                   ctypes.c_int64]
        L.orc_march.argtypes = [ctypes.POINTER(OrcParams), _dp, _dp, ctypes.c_int, _ip,
                                ctypes.POINTER(OrcStepStats), _dp, _dp, _dp, _ip]
        L.orc_march_state.argtypes = [ctypes.POINTER(OrcParams), _dp, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_int, _ip, ctypes.POINTER(OrcStepStats), _dp, _ip]
        L.orc_initial_state.argtypes = [ctypes.c_int, _ip, _dp, _dp, _dp]
        L.orc_sweep_adjoint.argtypes = [ctypes.c_int, _ip, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, _dp, _dp, _dp]
        L.orc_shadow_adjoint.argtypes = [ctypes.c_int, _ip, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_march_adjoint.argtypes = [ctypes.POINTER(OrcParams), _dp, ctypes.c_int64, ctypes.c_int, _ip, _dp]
        L.orc_initial_state_adjoint.argtypes = [ctypes.c_int, _ip, _dp, _dp, _dp, _dp, _dp]
        L.orc_sweep_cavity.argtypes = [_ip, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, _dp, _dp]
        L.orc_cavity_local_jacobians.argtypes = [ctypes.c_int64, ctypes.c_double, _dp, _dp, _dp]
        L.orc_collision_jacobian.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, _dp]
        L.orc_full_symbol.argtypes = [ctypes.c_int, _ip, _dp, _dp, _dp]
        L.orc_full_symbol_iteration.argtypes = [ctypes.c_int, _ip, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
        for name in ("orc_sweep_cavity", "orc_cavity_local_jacobians", "orc_collision_jacobian", "orc_full_symbol", "orc_full_symbol_iteration", "orc_sweep_adjoint", "orc_shadow_adjoint", "orc_march_adjoint", "orc_initial_state_adjoint",
                     "orc_march_state", "orc_initial_state", "orc_lattice", "orc_sweep", "orc_shadow", "orc_corrected_iteration", "orc_fft",
                     "orc_tables", "orc_init_populations", "orc_moments", "orc_explicit",
                     "orc_march"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(shape_n):
    n = list(shape_n) + [1] * (3 - len(shape_n))
    return (ctypes.c_int32 * 3)(*n)


# ------------------------------------------------------------------ lattice --
def lattice(d: int):
    """(c[Q,3] int, w[Q], opp[Q]) from App. A."""
    Q = ctypes.c_int32()
    c = np.zeros(19 * 3, dtype=np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    rc = lib().orc_lattice(d, ctypes.byref(Q), c.ctypes.data_as(_ip), _p(w), opp.ctypes.data_as(_ip))
    assert rc == 0
    q = Q.value
    return c[: 3 * q].reshape(q, 3).copy(), w[:q].copy(), opp[:q].copy()


def feq_site(d, m):
    m = _c64(m)
    _, w, _ = lattice(d)
    out = np.zeros(len(w))
    lib().orc_feq_site(d, _p(m), _p(out))
    return out


def phi_site(d, m, s):
    m, s = _c64(m), _c64(s)
    _, w, _ = lattice(d)
    out = np.zeros(len(w))
    lib().orc_phi_site(d, _p(m), _p(s), _p(out))
    return out


def collide_site(d, f, h, a, wp, wm):
    f = _c64(f)
    Q = f.shape[0]
    C = np.zeros(Q)
    m = np.zeros(d + 1)
    s = np.zeros(d + 1)
    hh = _c64(h) if h is not None else None
    lib().orc_collide_site(d, _p(f), _p(hh) if hh is not None else None, a, wp, wm, _p(C), _p(m),
                           _p(s))
    return C, m, s


# ---------------------------------------------------------------- operators --
def sweep(f, h, a, wp, wm):
    """One evaluation of T: returns (fT, Pr, R)."""
    f = _c64(f)
    Q = f.shape[0]
    d = f.ndim - 1
    n = _dims(f.shape[1:])
    fT = np.zeros_like(f)
    Pr = np.zeros((d + 1,) + f.shape[1:])
    R = ctypes.c_double()
    hh = _c64(h) if h is not None else None
    rc = lib().orc_sweep(d, n, _p(f), _p(hh) if hh is not None else None, a, wp, wm, _p(fT), _p(Pr),
                         ctypes.byref(R))
    assert rc == 0 and Q in (9, 19)
    return fT, Pr, R.value


def shadow(Pr, a, nu):
    Pr = _c64(Pr)
    d = Pr.ndim - 1
    dm = np.zeros_like(Pr)
    rc = lib().orc_shadow(d, _dims(Pr.shape[1:]), _p(Pr), a, nu, _p(dm))
    assert rc == 0
    return dm


def corrected_iteration(f, h, a, wp, wm, nu):
    """fT = T(f); dm from P r; returns (f_next, fT, Pr, dm, R)."""
    f = _c64(f)
    d = f.ndim - 1
    fn = np.zeros_like(f)
    fT = np.zeros_like(f)
    Pr = np.zeros((d + 1,) + f.shape[1:])
    dm = np.zeros_like(Pr)
    R = ctypes.c_double()
    hh = _c64(h) if h is not None else None
    rc = lib().orc_corrected_iteration(d, _dims(f.shape[1:]), _p(f),
                                       _p(hh) if hh is not None else None, a, wp, wm, nu, _p(fn),
                                       _p(fT), _p(Pr), _p(dm), ctypes.byref(R))
    assert rc == 0
    return fn, fT, Pr, dm, R.value


def fft(z, inverse=False):
    z = np.asarray(z, dtype=np.complex128)
    re = np.ascontiguousarray(z.real)
    im = np.ascontiguousarray(z.imag)
    rc = lib().orc_fft(z.ndim, _dims(z.shape), _p(re), _p(im), 1 if inverse else 0)
    assert rc == 0
    return re + 1j * im


def tables(d, shape):
    """(nbr[Q, NS] int32, signed index per axis (concatenated), mask[NS] uint8)."""
    Q = 9 if d == 2 else 19
    NS = int(np.prod(shape))
    nbr = np.zeros(Q * NS, dtype=np.int32)
    sidx = np.zeros(int(sum(shape)), dtype=np.int32)
    mask = np.zeros(NS, dtype=np.uint8)
    rc = lib().orc_tables(d, _dims(shape), nbr.ctypes.data_as(_ip), sidx.ctypes.data_as(_ip),
                          mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    assert rc == 0
    return nbr.reshape(Q, NS), sidx, mask


def init_populations(p0, u0):
    p0, u0 = _c64(p0), _c64(u0)
    d = u0.shape[0]
    Q = 9 if d == 2 else 19
    f = np.zeros((Q,) + p0.shape)
    rc = lib().orc_init_populations(d, _dims(p0.shape), _p(p0), _p(u0), _p(f))
    assert rc == 0
    return f


def moments(f):
    f = _c64(f)
    d = f.ndim - 1
    M = np.zeros((d + 1,) + f.shape[1:])
    lib().orc_moments(d, _dims(f.shape[1:]), _p(f), _p(M))
    return M


def explicit(f, nsteps, wp=1.0, wm=1.0):
    f = _c64(f).copy()
    d = f.ndim - 1
    rc = lib().orc_explicit(d, _dims(f.shape[1:]), wp, wm, _p(f), int(nsteps))
    assert rc == 0
    return f


@dataclass
class MarchResult:
    status: int
    steps_done: int
    f: np.ndarray
    m: np.ndarray
    stats: list
    Rhist: np.ndarray | None


def initial_state(p0, u0):
    """Full march state (f^n, f^{n-1}, f^{n-2}, m^n, m^{n-1}) flattened, as
    the library's msc_get_state lays it out, at the initial condition."""
    p0, u0 = _c64(p0), _c64(u0)
    d = u0.shape[0]
    Q = 9 if d == 2 else 19
    NS = p0.size
    st = np.zeros(3 * Q * NS + 2 * (d + 1) * NS)
    rc = lib().orc_initial_state(d, _dims(p0.shape), _p(p0), _p(u0), _p(st))
    assert rc == 0
    return st


def _params(d, shape, dt, eps, kmax, nmin, corrector, tau_plus, tau_minus, extrap_states=0, fd_step=0.0):
    P = OrcParams()
    P.extrap_states = extrap_states
    P.fd_step = fd_step
    P.d = d
    P.n = (ctypes.c_int * 3)(*(list(shape) + [1] * (3 - len(shape))))
    P.tau_plus, P.tau_minus, P.dt, P.eps = tau_plus, tau_minus, dt, eps
    P.kmax, P.nmin, P.corrector = kmax, nmin, corrector
    return P


def march_state(state, bdf_count, shape, *, dt, nsteps, eps=1e-10, kmax=300, nmin=2, corrector=1,
                tau_plus=1.0, tau_minus=1.0, schedule=None, extrap_states=0, fd_step=0.0):
    """Advance a full march state; returns (status, new_state, bdf_count, stats)."""
    d = len(shape)
    P = _params(d, shape, dt, eps, kmax, nmin, corrector, tau_plus, tau_minus, extrap_states, fd_step)
    st = np.array(state, dtype=np.float64, copy=True)
    bc = ctypes.c_int64(int(bdf_count))
    stats = (OrcStepStats * max(nsteps, 1))()
    sched = np.ascontiguousarray(schedule, dtype=np.int32) if schedule is not None else None
    done = ctypes.c_int32()
    rc = lib().orc_march_state(ctypes.byref(P), _p(st), ctypes.byref(bc), nsteps,
                               sched.ctypes.data_as(_ip) if sched is not None else None, stats, None,
                               ctypes.byref(done))
    out = [dict(q=s.q, iters=s.iters, R_first=s.R_first, R_final=s.R_final, rho_obs=s.rho_obs,
                converged=s.converged) for s in stats[:nsteps]]
    return rc, st, bc.value, out


def march(p0, u0, *, dt, nsteps, eps=1e-10, kmax=300, nmin=2, corrector=1, tau_plus=1.0,
          tau_minus=1.0, schedule=None, keep_rhist=False, extrap_states=0, fd_step=0.0) -> MarchResult:
    """Dual-time march by Algorithm 1 (corrector=1), Picard (corrector=0) or
    with the full-symbol reference corrector of Eq. (full-symbol)
    (corrector=2; fd_step 0 = exact Jacobian at rest, > 0 = the paper's
    forward difference of that step)."""
    p0, u0 = _c64(p0), _c64(u0)
    d = u0.shape[0]
    shape = p0.shape
    Q = 9 if d == 2 else 19
    P = OrcParams()
    P.d = d
    P.n = (ctypes.c_int * 3)(*(list(shape) + [1] * (3 - len(shape))))
    P.tau_plus, P.tau_minus, P.dt, P.eps = tau_plus, tau_minus, dt, eps
    P.kmax, P.nmin, P.corrector = kmax, nmin, corrector
    P.extrap_states = extrap_states
    P.fd_step = fd_step
    st = (OrcStepStats * max(nsteps, 1))()
    f = np.zeros((Q,) + shape)
    m = np.zeros((d + 1,) + shape)
    sched = None
    if schedule is not None:
        sched = np.ascontiguousarray(schedule, dtype=np.int32)
    Rh = np.full(nsteps * kmax, np.nan) if keep_rhist else None
    done = ctypes.c_int32()
    rc = lib().orc_march(ctypes.byref(P), _p(p0), _p(u0), nsteps,
                         sched.ctypes.data_as(_ip) if sched is not None else None, st,
                         _p(Rh) if Rh is not None else None, _p(f), _p(m), ctypes.byref(done))
    stats = [dict(q=s.q, iters=s.iters, R_first=s.R_first, R_final=s.R_final, rho_obs=s.rho_obs,
                  converged=s.converged) for s in st[: nsteps]]
    return MarchResult(rc, done.value, f, m, stats,
                       Rh.reshape(nsteps, kmax) if Rh is not None else None)


# -------------------------------------------------------- full symbol --
def collision_jacobian(d, a, wp, wm, fd_step=0.0):
    """Q x Q collision Jacobian dC/df at the rest state (p, u) = (1, 0), h = a m
    (Sec. 4.1): exact (central differences of the quadratic map) for
    fd_step <= 0, else the one-sided forward difference of that step."""
    Q = 9 if d == 2 else 19
    J = np.zeros((Q, Q))
    assert lib().orc_collision_jacobian(d, a, wp, wm, fd_step, _p(J)) == 0
    return J


def full_symbol(r, J):
    """df = F^{-1}[(I - Z(k) J)^{-1} F[r]] on all fields and wavevectors (Eq. full-symbol)."""
    r = _c64(r)
    d = r.ndim - 1
    df = np.zeros_like(r)
    assert lib().orc_full_symbol(d, _dims(r.shape[1:]), _p(_c64(J)), _p(r), _p(df)) == 0
    return df


def full_symbol_iteration(f, h, a, wp, wm, fd_step=0.0):
    """One full-symbol corrected iteration: returns (f_next, fT, R)."""
    f = _c64(f)
    d = f.ndim - 1
    hh = _c64(h) if h is not None else None
    fn = np.zeros_like(f)
    fT = np.zeros_like(f)
    R = ctypes.c_double()
    assert lib().orc_full_symbol_iteration(d, _dims(f.shape[1:]), _p(f), _p(hh) if hh is not None else None, a,
                                           wp, wm, fd_step, _p(fn), _p(fT), ctypes.byref(R)) == 0
    return fn, fT, R.value


# ---------------------------------------------------- wall-bounded cavity --
# Sec. 3.3 and Algorithm 2: D2Q9 lid-driven cavity, boundary-node modified
# bounce-back rows of Eq. (bounceback-rows) in the printed order (y = 0,
# y = N_y - 1 with the moving lid along +x, x = 0, x = N_x - 1), and the
# kinetic correction (I - L) df = r with L = B_Gamma S blkdiag(J^C(x)) of
# Eq. (wall-global-jacobian), factorised by a sparse LU (the paper uses a
# sparse direct solver; scipy's SuperLU here).
_CAV_WALLS = (
    ("y0", ((2, 4), (5, 7), (6, 8))),
    ("y1", ((4, 2), (7, 5), (8, 6))),
    ("x0", ((1, 3), (5, 7), (8, 6))),
    ("x1", ((3, 1), (6, 8), (7, 5))),
)


def cavity_sweep(f, h, a, ulid, wp=1.0, wm=1.0):
    """(f_T, R) of the cavity sweep T_{q,h,Gamma} (h None means h = 0)."""
    f = _c64(f)
    fT = np.zeros_like(f)
    R = ctypes.c_double()
    hh = _c64(h) if h is not None else None
    assert lib().orc_sweep_cavity(_dims(f.shape[1:]), _p(f), _p(hh) if hh is not None else None, a, wp, wm,
                                  ulid, _p(fT), ctypes.byref(R)) == 0
    return fT, R.value


def cavity_local_jacobians(mref, sref, a):
    """J^C(x) of Eq. (wall-local-jacobian) at every site: (N_sites, Q, Q)."""
    mref, sref = _c64(mref), _c64(sref)
    NS = int(np.prod(mref.shape[1:]))
    Jc = np.zeros((NS, 9, 9))
    assert lib().orc_cavity_local_jacobians(NS, a, _p(mref), _p(sref), _p(Jc)) == 0
    return Jc


def cavity_row_sources(shape):
    """lab[k, x, y]: the streamed direction whose row ends in row (k, x, y)
    after the wall assignments, in their order (copies of copies follow)."""
    Nx, Ny = shape
    lab = np.broadcast_to(np.arange(9).reshape(9, 1, 1), (9, Nx, Ny)).copy()
    for wall, pairs in _CAV_WALLS:
        sl = {"y0": (slice(None), 0), "y1": (slice(None), Ny - 1), "x0": (0, slice(None)),
              "x1": (Nx - 1, slice(None))}[wall]
        for kR, kS in pairs:
            lab[(kR,) + sl] = lab[(kS,) + sl]
    return lab


def cavity_operator(Jc, shape):
    """Sparse L = B_Gamma S blkdiag(J^C) (Eq. wall-stream-row, the row copies
    of Eq. bounceback-rows, Eq. wall-global-jacobian), rows and columns in
    the canonical order iota(k, x, y) = (k N_x + x) N_y + y."""
    import scipy.sparse as sp
    Nx, Ny = shape
    NS = Nx * Ny
    c, _, _ = lattice(2)
    lab = cavity_row_sources(shape).reshape(9, NS)
    X, Y = np.meshgrid(np.arange(Nx), np.arange(Ny), indexing="ij")
    X, Y = X.ravel(), Y.ravel()
    rows, cols, vals = [], [], []
    for k in range(9):
        src = lab[k]
        xu = (X - c[src, 0]) % Nx  # upwind site of the streamed source row
        yu = (Y - c[src, 1]) % Ny
        su = xu * Ny + yu
        for kp in range(9):
            rows.append(k * NS + np.arange(NS))
            cols.append(kp * NS + su)
            vals.append(Jc[su, src, kp])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(9 * NS, 9 * NS))


def _reconstruct(f, h, a):
    m = moments(f)
    return (m + (h if h is not None else 0.0) / 2.0) / (1.0 + a / 2.0)


def cavity_march(p0, u0, *, ulid, dt, nsteps, eps, kmax=300, nmin=1, corrector="frozen", n_forced=0,
                 max_refresh=3, schedule=None, extrap_states=0):
    """Algorithm 2 (corrector "frozen" or "adaptive"), or the Picard
    iteration with the same walls (corrector "picard"), from f^0 = feq(p0, u0).
    Returns dict(status, f, m, stats) with per-step q, iters, R list,
    refresh count and the inner indices at which the operator was refreshed."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    p0, u0 = _c64(p0), _c64(u0)
    shape = p0.shape
    NS = int(np.prod(shape))
    n = 9 * NS
    f0 = init_populations(p0, u0)
    fn = f0.copy(); fn1 = f0.copy(); fn2 = f0.copy()
    mn = moments(f0); mn1 = mn.copy()
    bc = 0
    eye = sp.identity(n, format="csc")

    def factor(a_A, mref, sref):
        Jc = cavity_local_jacobians(mref, sref, a_A)
        return spl.splu((eye - cavity_operator(Jc, shape)).tocsc())

    lu = None
    if corrector != "picard":
        # Algorithm 2: the initial operator at rest (p = 1, u = 0, h_2 = a_2 m,
        # s = 0), assembled with q_A = 2
        a2 = 3.0 / (2.0 * dt)
        mref = np.zeros((3,) + shape); mref[0] = 1.0
        lu = factor(a2, mref, np.zeros((3,) + shape))
    stats = []
    status = 0
    for step in range(nsteps):
        q = 1 if bc == 0 else 2
        a = 1.0 / dt if q == 1 else 3.0 / (2.0 * dt)
        h = mn / dt if q == 1 else (4.0 * mn - mn1) / (2.0 * dt)
        cap = 2 if extrap_states == 0 else extrap_states - 1
        order = min(bc, cap)
        f = fn.copy() if order == 0 else (2 * fn - fn1 if order == 1 else 3 * fn - 3 * fn1 + fn2)
        Rl, refreshed = [], []
        n_grow, n_ref, Rref = 0, 0, None
        accepted = False
        for ell in range(1, kmax + 1):
            fT, R = cavity_sweep(f, h, a, ulid)
            Rl.append(R)
            if ell == 1:
                Rref = R
            ok = (ell == schedule[step]) if schedule is not None else (ell >= nmin and np.isfinite(R) and R < eps)
            if ok:
                mnew = _reconstruct(fT, h, a)
                fn2, fn1, fn = fn1, fn, fT
                mn1, mn = mn, mnew
                accepted = True
                break
            if not np.isfinite(R):
                status = 6
                break
            if ell == kmax:
                break
            n_grow = n_grow + 1 if (ell > 1 and R > Rl[-2]) else 0
            if corrector == "adaptive" and n_ref < max_refresh:
                if n_grow >= 2 or R > 10.0 * Rref or (n_forced > 0 and ell % n_forced == 0):
                    mref = _reconstruct(f, h, a)  # the current iterate, unchanged histories
                    lu = factor(a, mref, h - a * mref)
                    n_ref += 1
                    n_grow = 0
                    Rref = R
                    refreshed.append(ell)
            r = fT - f
            if corrector == "picard":
                f = fT
            else:
                f = f + lu.solve(r.ravel()).reshape(f.shape)
        stats.append(dict(q=q, iters=len(Rl), R=Rl, refreshes=len(refreshed), refreshed_at=refreshed,
                          converged=accepted))
        if not accepted:
            status = status or 5
            break
        bc += 1
    return dict(status=status, f=fn, m=mn, stats=stats)


def cavity_explicit(f, nsteps, ulid, wp=1.0, wm=1.0):
    """Explicit TRT march with the cavity walls (a = 0, h = 0)."""
    f = _c64(f).copy()
    for _ in range(int(nsteps)):
        f, _ = cavity_sweep(f, None, 0.0, ulid, wp, wm)
    return f


# ------------------------------------------------------------------ adjoint --
def sweep_adjoint(f, h, a, wp, wm, lamT):
    """(lam_f, lam_h) = transposes of dT/df and dT/dh applied to lamT."""
    f, lamT = _c64(f), _c64(lamT)
    d = f.ndim - 1
    lf = np.zeros_like(f)
    lh = np.zeros((d + 1,) + f.shape[1:])
    hh = _c64(h) if h is not None else None
    rc = lib().orc_sweep_adjoint(d, _dims(f.shape[1:]), _p(f), _p(hh) if hh is not None else None, a, wp, wm,
                                 _p(lamT), _p(lf), _p(lh))
    assert rc == 0
    return lf, lh


def shadow_adjoint(y, a, nu):
    y = _c64(y)
    d = y.ndim - 1
    out = np.zeros_like(y)
    rc = lib().orc_shadow_adjoint(d, _dims(y.shape[1:]), _p(y), a, nu, _p(out))
    assert rc == 0
    return out


def march_adjoint(state0, bdf_count0, shape, lam_final, *, dt, schedule, eps=1e-10, kmax=300, nmin=2,
                  corrector=1, tau_plus=1.0, tau_minus=1.0, extrap_states=0):
    """Adjoint of the state map of march_state at the given inner counts."""
    d = len(shape)
    P = _params(d, shape, dt, eps, kmax, nmin, corrector, tau_plus, tau_minus, extrap_states)
    lam = np.array(lam_final, dtype=np.float64, copy=True)
    sched = np.ascontiguousarray(schedule, dtype=np.int32)
    st = _c64(state0)
    rc = lib().orc_march_adjoint(ctypes.byref(P), _p(st), int(bdf_count0), len(sched),
                                 sched.ctypes.data_as(_ip), _p(lam))
    assert rc == 0, rc
    return lam


def initial_state_adjoint(p0, u0, lam_state):
    p0, u0, lam = _c64(p0), _c64(u0), _c64(lam_state)
    d = u0.shape[0]
    lp = np.zeros_like(p0)
    lu = np.zeros_like(u0)
    rc = lib().orc_initial_state_adjoint(d, _dims(p0.shape), _p(p0), _p(u0), _p(lam), _p(lp), _p(lu))
    assert rc == 0
    return lp, lu
