"""Seeded synthetic workloads (initial fields and analytic references).

This module holds no arithmetic of the method itself: it only builds the
initial hydrodynamic fields ``(p0, u0)`` that both the HIP library and the CPU
oracle receive as data, the analytic Taylor-Green reference used for error
gates, and the horizon rule.  Arrays use the canonical site order
``[x, y]`` / ``[x, y, z]`` (last index fastest); velocities are stacked as
``u[alpha, ...]``.

Workloads (paper Sec. 4.1):
  * 2D Taylor-Green vortex, Eq. (tgv2d) with the zero-mean pressure gauge of
    Eq. (tgv2d-pressure-init); ``U = Re nu / N``.
  * 3D Taylor-Green initial field, Eq. (tgv3d-ic), zero initial pressure,
    optionally plus a seeded divergence-free perturbation.
  * Random divergence-free 2D field: a seeded Fourier stream function with a
    ``|k|^-3`` energy spectrum over ``1 <= |j| <= jmax`` (integer index
    vectors), velocity by analytic differentiation, rescaled so that
    ``max |u| = U``.  This stands in for a generic smooth decaying flow; the
    paper itself only uses Taylor-Green fields.
  * Vorticity control fields for the differentiable march (curl of the random
    field above).
"""
from __future__ import annotations

import math

import numpy as np

CS2 = 1.0 / 3.0


def nint(x: float) -> int:
    """Nearest integer with halves rounded up, floor(x + 1/2) (Sec. 4.1)."""
    return int(math.floor(x + 0.5))


def horizon(c: float, N: int, nu: float, dt_nominal: float):
    """(T_end, S, dt) with T_end = nint(c N^2 / nu), S = nint(T_end / dt_nom),
    dt = T_end / S (integer step counts set dt, Tab. 1)."""
    T_end = nint(c * N * N / nu)
    S = max(1, nint(T_end / dt_nominal))
    return T_end, S, T_end / S


# ------------------------------------------------------------ Taylor-Green --
def tgv2d(N: int, U: float, nu: float = 1.0 / 6.0, t: float = 0.0, rho0: float = 1.0):
    """2D Taylor-Green vortex at time t (Eq. tgv2d); returns (p_hat, u[2])."""
    k0 = 2.0 * math.pi / N
    x = np.arange(N, dtype=np.float64)[:, None]
    y = np.arange(N, dtype=np.float64)[None, :]
    du = math.exp(-2.0 * nu * k0 * k0 * t)
    dp = math.exp(-4.0 * nu * k0 * k0 * t)
    ux = -U * np.cos(k0 * x) * np.sin(k0 * y) * du
    uy = U * np.sin(k0 * x) * np.cos(k0 * y) * du
    p = -(rho0 * U * U / (4.0 * CS2)) * (np.cos(2 * k0 * x) + np.cos(2 * k0 * y)) * dp
    return p, np.stack([ux, uy])


def tgv3d(N: int, U: float):
    """3D Taylor-Green initial velocity (Eq. tgv3d-ic), zero pressure."""
    k0 = 2.0 * math.pi / N
    x = np.arange(N, dtype=np.float64)[:, None, None]
    y = np.arange(N, dtype=np.float64)[None, :, None]
    z = np.arange(N, dtype=np.float64)[None, None, :]
    ux = U * np.sin(k0 * x) * np.cos(k0 * y) * np.cos(k0 * z)
    uy = -U * np.cos(k0 * x) * np.sin(k0 * y) * np.cos(k0 * z)
    uz = np.zeros((N, N, N))
    return np.zeros((N, N, N)), np.stack([ux, uy, uz])


# ---------------------------------------------------------- random fields --
def _half_space_modes(d: int, jmax: int):
    """Integer index vectors j with 1 <= |j| <= jmax in a half space
    (first nonzero component positive), in a fixed lexicographic order."""
    rng = range(-jmax, jmax + 1)
    out = []
    if d == 2:
        for jx in rng:
            for jy in rng:
                r2 = jx * jx + jy * jy
                if r2 == 0 or r2 > jmax * jmax:
                    continue
                if jx > 0 or (jx == 0 and jy > 0):
                    out.append((jx, jy))
    else:
        for jx in rng:
            for jy in rng:
                for jz in rng:
                    r2 = jx * jx + jy * jy + jz * jz
                    if r2 == 0 or r2 > jmax * jmax:
                        continue
                    first = jx if jx != 0 else (jy if jy != 0 else jz)
                    if first > 0:
                        out.append((jx, jy, jz))
    return out


def _spectral_potential(shape, modes, amp, phases):
    """Coefficient array S with psi(x) = Re sum_j amp_j e^{i(2 pi j.x/N + phi_j)}
    = Re(N_Omega * ifftn(S))."""
    S = np.zeros(shape, dtype=np.complex128)
    for j, a, ph in zip(modes, amp, phases):
        idx = tuple(int(jj) % n for jj, n in zip(j, shape))
        S[idx] += a * np.exp(1j * ph)
    return S


def _deriv(S, axis, shape):
    """Spectral coefficients of d/dx_axis for coefficients placed at j mod N."""
    n = shape[axis]
    j = np.fft.fftfreq(n, d=1.0 / n)  # signed integer index
    kk = 2.0 * math.pi * j / n
    bshape = [1] * len(shape)
    bshape[axis] = n
    return S * (1j * kk.reshape(bshape))


def _real_field(S):
    return np.real(np.fft.ifftn(S)) * S.size


def random_field_2d(N: int, U: float, seed: int = 1, jmax: int = 16):
    """Divergence-free random 2D velocity (|k|^-3 energy spectrum), p_hat = 0.

    psi = sum_j |j|^-3 cos(2 pi j.x/N + phi_j) with phi_j ~ U[0, 2pi) drawn
    from numpy PCG64(seed) in the fixed mode order; u = (d_y psi, -d_x psi);
    rescaled so that max |u| = U.
    """
    modes = _half_space_modes(2, jmax)
    rng = np.random.Generator(np.random.PCG64(seed))
    phases = rng.uniform(0.0, 2.0 * math.pi, size=len(modes))
    amp = [math.hypot(*j) ** -3 for j in modes]
    shape = (N, N)
    S = _spectral_potential(shape, modes, amp, phases)
    ux = _real_field(_deriv(S, 1, shape))
    uy = -_real_field(_deriv(S, 0, shape))
    u = np.stack([ux, uy])
    scale = U / np.sqrt((u * u).sum(axis=0)).max()
    return np.zeros(shape), u * scale


def random_perturbation_3d(N: int, amplitude: float, seed: int = 1, jmax: int = 8):
    """Divergence-free 3D perturbation u' = curl A, each component of A a
    seeded |j|^-3 spectral sum over 1 <= |j| <= jmax; max |u'| = amplitude."""
    modes = _half_space_modes(3, jmax)
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (N, N, N)
    amp = [math.sqrt(j[0] ** 2 + j[1] ** 2 + j[2] ** 2) ** -3 for j in modes]
    A = []
    for _ in range(3):
        phases = rng.uniform(0.0, 2.0 * math.pi, size=len(modes))
        A.append(_spectral_potential(shape, modes, amp, phases))
    ux = _real_field(_deriv(A[2], 1, shape) - _deriv(A[1], 2, shape))
    uy = _real_field(_deriv(A[0], 2, shape) - _deriv(A[2], 0, shape))
    uz = _real_field(_deriv(A[1], 0, shape) - _deriv(A[0], 1, shape))
    u = np.stack([ux, uy, uz])
    return u * (amplitude / np.sqrt((u * u).sum(axis=0)).max())


def tgv3d_perturbed(N: int, U: float, seed: int = 1, rel_amp: float = 1e-2, jmax: int = 8):
    p, u = tgv3d(N, U)
    return p, u + random_perturbation_3d(N, rel_amp * U, seed=seed, jmax=jmax)


def vorticity_2d(u):
    """Spectral vorticity w = d_x u_y - d_y u_x of a periodic 2D field."""
    shape = u.shape[1:]
    Ux = np.fft.fftn(u[0])
    Uy = np.fft.fftn(u[1])
    return np.real(np.fft.ifftn(_deriv(Uy, 0, shape) - _deriv(Ux, 1, shape)))


def random_vorticity_2d(N: int, U: float, seed: int):
    """Control field for the differentiable march: the vorticity of the
    seeded random field."""
    _, u = random_field_2d(N, U, seed=seed)
    return vorticity_2d(u)


def config(name: str):
    """Named workloads with their sizes (nu = 1/6, Lambda = 1/4)."""
    nu = 1.0 / 6.0
    if name == "tgv2d_n64_fp64":
        N, Re = 64, 1.0
        T_end, S, dt = horizon(0.1, N, nu, 64.0)
        return dict(name=name, d=2, N=N, Re=Re, U=Re * nu / N, nu=nu, T_end=T_end, S=S, dt=dt,
                    eps=1e-10, nmin=2, storage="fp64", kind="tgv2d")
    if name == "rand2d_n256_fp32":
        N, Re = 256, 1.0
        T_end, S, dt = horizon(0.25, N, nu, 256.0)
        return dict(name=name, d=2, N=N, Re=Re, U=Re * nu / N, nu=nu, T_end=T_end, S=S, dt=dt,
                    eps=1e-8, nmin=2, storage="fp32", kind="rand2d", seed=1)
    if name == "rand2d_n1024_fp32":
        N, Re = 1024, 1.0
        T_end, S, dt = horizon(0.1, N, nu, 9830.4)
        return dict(name=name, d=2, N=N, Re=Re, U=Re * nu / N, nu=nu, T_end=T_end, S=S, dt=dt,
                    eps=1e-8, nmin=2, storage="fp32", kind="rand2d", seed=1)
    if name == "tgv3d_n128_fp32":
        N, Re = 128, 1.0
        T_end, S, dt = horizon(0.1, N, nu, 64.0)
        # n_min = 2 (the paper's 3D control is 1): over this horizon the field
        # decays by about five decades and one-sweep acceptances under the
        # absolute tolerance lose the solution
        return dict(name=name, d=3, N=N, Re=Re, U=Re * nu / N, nu=nu, T_end=T_end, S=S, dt=dt,
                    eps=1e-8, nmin=2, storage="fp32", kind="tgv3d_pert", seed=1)
    if name == "tgv3d_n128_fp64":
        # the same D3Q19 run in FP64 storage and arithmetic (the paper's
        # precision); eps is the tightest of the candidate tolerances, the
        # benchmark selects among them by the accuracy gates
        N, Re = 128, 1.0
        T_end, S, dt = horizon(0.1, N, nu, 64.0)
        return dict(name=name, d=3, N=N, Re=Re, U=Re * nu / N, nu=nu, T_end=T_end, S=S, dt=dt,
                    eps=1e-10, nmin=2, storage="fp64", kind="tgv3d_pert", seed=1)
    if name == "vort2d_n256_adjoint":
        # differentiable march: vorticity control (seed 1), target from the
        # march of the seed-2 control, 20 steps of dt = 64
        N, Re = 256, 1.0
        return dict(name=name, d=2, N=N, Re=Re, U=Re * nu / N, nu=nu, nsteps=20, dt=64.0, T_end=20 * 64.0,
                    eps=1e-8, nmin=2, storage="fp32", kind="vort2d", seed=1, target_seed=2)
    raise KeyError(name)


def initial_fields(cfg):
    N, U = cfg["N"], cfg["U"]
    if cfg["kind"] == "tgv2d":
        return tgv2d(N, U, cfg["nu"])
    if cfg["kind"] == "rand2d":
        return random_field_2d(N, U, seed=cfg.get("seed", 1))
    if cfg["kind"] == "tgv3d":
        return tgv3d(N, U)
    if cfg["kind"] == "tgv3d_pert":
        return tgv3d_perturbed(N, U, seed=cfg.get("seed", 1))
    raise KeyError(cfg["kind"])
