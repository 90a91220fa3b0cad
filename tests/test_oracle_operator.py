"""Pins of the oracle's sweep, transforms and shadow correction on tiny grids.

* Eq. (symbol) / Sec. 2.4.1: the Frechet derivative of one sweep about a
  uniform rest state is translation invariant; in Fourier space each block is
  Z(theta) J with Z = diag(exp(-i theta.c_k)) and the local Jacobian
  J = (1-w+) Pi+ + (1-w-) Pi- + c+ E0 P0 + c- Eu Pu,
  c+- = [w+- - a (1 - w+-/2)] / (1 + a/2), derived from Eq. (collision) with
  Eq. (macro-reconstruct) and Eq. (source-moments).  At w = 1, J = gamma_q E P
  (Eq. local-linear-response).  T is quadratic in f, so a central difference
  gives its Jacobian exactly up to rounding: brute force vs closed form.
* Corrected iteration (Eq. shadow-update): blocks
  Z J + chi E H^-1 P (Z J - I); at theta = 0 and w = 1 this is
  -(a/2)/(1 + a/2) E P (Eq. zero-mode-scale).
* Eq. (schur) equals a direct complex solve of H(k) (Eq. shadow-cont/mom).
* The oracle's radix-2 FFT equals numpy's FFT (an independent library) and the
  naive DFT; inverse(forward) = identity; Parseval (Eq. fft-convention).
"""
import itertools
import math

import numpy as np
import pytest

CS2 = 1.0 / 3.0


def _lat(orc, d):
    c, w, opp = orc.lattice(d)
    return c[:, :d].astype(float), w, opp


def _thetas(shape):
    axes = [2 * np.pi * np.array([j if j <= n // 2 else j - n for j in range(n)]) / n for n in shape]
    return list(itertools.product(*[list(enumerate(a)) for a in axes]))


def _fourier_blocks(Jd, nblock, shape):
    """B(theta) = U^H Jd U with U = I_nblock (x) exp(i theta.x)/sqrt(NS)."""
    NS = int(np.prod(shape))
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    out = {}
    for combo in _thetas(shape):
        th = np.array([t for _, t in combo])
        phase = np.exp(1j * sum(th[a] * grids[a] for a in range(len(shape)))).ravel() / math.sqrt(NS)
        U = np.zeros((nblock * NS, nblock), dtype=complex)
        for b in range(nblock):
            U[b * NS:(b + 1) * NS, b] = phase
        out[tuple(j for j, _ in combo)] = (th, U.conj().T @ Jd @ U)
    return out


def _local_J(c, w, opp, a, wp, wm):
    Q, d = c.shape
    I = np.eye(Q)
    Pi_p = 0.5 * (I + I[opp])
    Pi_m = 0.5 * (I - I[opp])
    E0 = w[:, None]
    Eu = (w[:, None] * c) / CS2
    P0 = np.ones((1, Q))
    Pu = c.T
    cp = (wp - a * (1 - wp / 2)) / (1 + a / 2)
    cm = (wm - a * (1 - wm / 2)) / (1 + a / 2)
    return (1 - wp) * Pi_p + (1 - wm) * Pi_m + cp * E0 @ P0 + cm * Eu @ Pu


def _E_P(c, w):
    E = np.hstack([w[:, None], w[:, None] * c / CS2])
    P = np.vstack([np.ones(len(w)), c.T])
    return E, P


def _H(th, a, nu):
    d = len(th)
    kk = float(th @ th)
    H = np.zeros((d + 1, d + 1), dtype=complex)
    H[0, 0] = a
    H[0, 1:] = 1j * th
    H[1:, 0] = CS2 * 1j * th
    H[1:, 1:] = (a + nu * kk) * np.eye(d)
    return H


def _dense_jacobian(fun, f0, step):
    n = f0.size
    J = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = step
        J[:, i] = (fun((f0.ravel() + e).reshape(f0.shape)).ravel()
                   - fun((f0.ravel() - e).reshape(f0.shape)).ravel()) / (2 * step)
    return J


CASES = [
    (2, (4, 4), 1.0, 1.0, 3.0 / 128.0),
    (2, (8, 8), 1.0, 1.0, 1.0 / 38.9),
    (2, (4, 4), 1 / 0.77, 1 / (0.5 + 1 / 1.08), 3.0 / 128.0),
    (2, (8, 4), 1 / 1.3, 1 / 0.9, 0.2),
    (3, (4, 4, 4), 1.0, 1.0, 3.0 / 128.0),
]


@pytest.mark.parametrize("d,shape,wp,wm,a", CASES)
def test_sweep_symbol_blocks_and_spectrum(orc, d, shape, wp, wm, a):
    c, w, opp = _lat(orc, d)
    Q = len(w)
    pbar = 0.37
    fbar = np.broadcast_to((w * pbar).reshape((Q,) + (1,) * d), (Q,) + shape).copy()
    h = np.zeros((d + 1,) + shape)
    h[0] = a * pbar  # s = 0 at the base state, so fbar is a fixed point
    fT, _, R = orc.sweep(fbar, h, a, wp, wm)
    assert R < 1e-16
    Jd = _dense_jacobian(lambda f: orc.sweep(f, h, a, wp, wm)[0], fbar, 1e-4)
    J = _local_J(c, w, opp, a, wp, wm)
    blocks = _fourier_blocks(Jd, Q, shape)
    allev = []
    for key, (th, B) in blocks.items():
        Z = np.diag(np.exp(-1j * (c @ th)))
        np.testing.assert_allclose(B, Z @ J, rtol=0, atol=1e-10)
        allev.append(np.linalg.eigvals(Z @ J))
    # spectrum of the dense Jacobian = union over theta of eig(Z J)
    ev_dense = np.linalg.eigvals(Jd)
    ev_sym = np.concatenate(allev)
    # match eigenvalues greedily (both multisets have Q*NS entries)
    remaining = list(ev_sym)
    for ev in sorted(ev_dense, key=lambda z: (-abs(z), z.real, z.imag)):
        j = int(np.argmin([abs(ev - r) for r in remaining]))
        assert abs(ev - remaining[j]) < 1e-5
        remaining.pop(j)
    if wp == 1.0 and wm == 1.0:
        # J = gamma_q E P (Eq. local-linear-response)
        E, P = _E_P(c, w)
        gamma = (1 - a / 2) / (1 + a / 2)
        np.testing.assert_allclose(J, gamma * E @ P, atol=1e-15)
        # theta = 0: gamma (x d+1), 0 elsewhere (Q-d-1 ghost directions removed)
        ev0 = np.sort(np.abs(np.linalg.eigvals(J)))
        np.testing.assert_allclose(ev0[-(d + 1):], gamma, atol=1e-13)
        np.testing.assert_allclose(ev0[: Q - d - 1], 0.0, atol=1e-13)
    else:
        ev0 = np.linalg.eigvals(J)
        nplus = {9: 4, 19: 9}[Q]
        nminus = {9: 2, 19: 6}[Q]
        assert np.sum(np.abs(ev0 - (1 - wp)) < 1e-10) >= nplus
        assert np.sum(np.abs(ev0 - (1 - wm)) < 1e-10) >= nminus


CORR_CASES = [
    (2, (8, 8), 1.0, 1.0, 3.0 / 128.0),
    (2, (4, 8), 1.0, 1.0, 1.0 / 64.0),
    (2, (8, 8), 1 / 0.8, 1 / 1.3, 3.0 / 128.0),
    (3, (4, 4, 4), 1.0, 1.0, 3.0 / 128.0),
]


@pytest.mark.parametrize("d,shape,wp,wm,a", CORR_CASES)
def test_corrected_iteration_blocks(orc, d, shape, wp, wm, a):
    c, w, opp = _lat(orc, d)
    Q = len(w)
    nu = CS2 * (1 / wp - 0.5)
    pbar = 0.21
    fbar = np.broadcast_to((w * pbar).reshape((Q,) + (1,) * d), (Q,) + shape).copy()
    h = np.zeros((d + 1,) + shape)
    h[0] = a * pbar
    fun = lambda f: orc.corrected_iteration(f, h, a, wp, wm, nu)[0]
    Jd = _dense_jacobian(fun, fbar, 1e-4)
    J = _local_J(c, w, opp, a, wp, wm)
    E, P = _E_P(c, w)
    for key, (th, B) in _fourier_blocks(Jd, Q, shape).items():
        Z = np.diag(np.exp(-1j * (c @ th)))
        chi = all(4 * abs(j if j <= n // 2 else j - n) <= n for j, n in zip(key, shape))
        M = Z @ J
        if chi:
            M = M + E @ np.linalg.solve(_H(th, a, nu), P @ (Z @ J - np.eye(Q)))
        np.testing.assert_allclose(B, M, rtol=0, atol=1e-10)
        if all(j == 0 for j in key) and wp == 1.0 and wm == 1.0:
            # Eq. (zero-mode-scale) consequence: -(a/2)/(1+a/2) E P
            np.testing.assert_allclose(B, -(a / 2) / (1 + a / 2) * E @ P, atol=1e-10)


def test_zero_mode_value_printed():
    """k = 0 block coefficient at dt = 64, BDF2: -0.01158."""
    a = 3 / (2 * 64)
    assert abs(-(a / 2) / (1 + a / 2) - (-0.01158)) < 5e-6


@pytest.mark.parametrize("d,shape", [(2, (8, 8)), (2, (16, 8)), (3, (8, 4, 8))])
def test_shadow_blocks_equal_direct_solve(orc, d, shape):
    """The shadow operator P r -> dm is the Fourier multiplier chi H^{-1}
    (Eq. schur vs a Gaussian-elimination solve of H, masks per Eq. shadow-mask)."""
    a = 3.0 / 128.0
    nu = 1.0 / 6.0
    NS = int(np.prod(shape))
    n = (d + 1) * NS
    Jd = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        Jd[:, i] = orc.shadow(e.reshape((d + 1,) + shape), a, nu).ravel()
    for key, (th, B) in _fourier_blocks(Jd, d + 1, shape).items():
        sj = [j if j <= m // 2 else j - m for j, m in zip(key, shape)]
        chi = all(4 * abs(s) <= m for s, m in zip(sj, shape))
        ref = np.linalg.inv(_H(th, a, nu)) if chi else np.zeros((d + 1, d + 1))
        np.testing.assert_allclose(B, ref, rtol=0, atol=1e-10)


def test_mask_boundary_and_nyquist(orc):
    """|k| = pi/2 retained, Nyquist (k = pi) excluded: integer index table."""
    _, sidx, mask = orc.tables(2, (16, 8))
    np.testing.assert_array_equal(sidx[:16], [0, 1, 2, 3, 4, 5, 6, 7, 8, -7, -6, -5, -4, -3, -2, -1])
    np.testing.assert_array_equal(sidx[16:], [0, 1, 2, 3, 4, -3, -2, -1])
    m = mask.reshape(16, 8)
    keepx = np.array([abs(s) * 4 <= 16 for s in sidx[:16]])
    keepy = np.array([abs(s) * 4 <= 8 for s in sidx[16:]])
    np.testing.assert_array_equal(m, np.outer(keepx, keepy).astype(np.uint8))
    assert m[4, 2] == 1 and m[12, 6] == 1 and m[8, 0] == 0 and m[0, 4] == 0


@pytest.mark.parametrize("shape", [(8,), (16, 8), (4, 8, 16), (64, 32)])
def test_fft_against_numpy_and_dft(orc, shape):
    rng = np.random.default_rng(4)
    z = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    F = orc.fft(z)
    np.testing.assert_allclose(F, np.fft.fftn(z), rtol=0, atol=1e-12 * np.abs(F).max())
    zi = orc.fft(F, inverse=True)
    np.testing.assert_allclose(zi, z, rtol=0, atol=1e-14 * np.abs(z).max() * 10)
    # Parseval for the unnormalised forward transform
    assert abs(np.sum(np.abs(F) ** 2) / z.size - np.sum(np.abs(z) ** 2)) < 1e-10 * np.sum(np.abs(z) ** 2)
    if z.size <= 128:
        grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
        for jj in [tuple(0 for _ in shape), tuple(1 for _ in shape), tuple(n - 1 for n in shape)]:
            ph = sum(2 * np.pi * j * g / n for j, g, n in zip(jj, grids, shape))
            ref = np.sum(z * np.exp(-1j * ph))
            assert abs(F[jj] - ref) < 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("d,shape", [(2, (8, 4)), (3, (4, 8, 4))])
def test_neighbour_table_is_push_permutation(orc, d, shape):
    """nbr[k][x] = index of (x + c_k) mod N; each direction's map is a bijection."""
    c, w, _ = _lat(orc, d)
    nbr, _, _ = orc.tables(d, shape)
    NS = int(np.prod(shape))
    idx = np.arange(NS).reshape(shape)
    for k in range(len(w)):
        shifted = idx
        for ax in range(d):
            shifted = np.roll(shifted, int(c[k, ax]), axis=ax)
        # np.roll moves the entry at x to x + c; so shifted[x + c] = x
        inv = np.empty(NS, dtype=np.int64)
        inv[shifted.ravel()] = np.arange(NS)
        np.testing.assert_array_equal(nbr[k], inv)
        assert len(set(nbr[k].tolist())) == NS
