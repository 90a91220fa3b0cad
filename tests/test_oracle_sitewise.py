"""Pins of the oracle's sitewise algebra against closed forms and identities.

Each check is something the paper or textbook lattice algebra fixes
independently of the oracle's own formulas:
  * App. A lattice tables: quadrature identities of D2Q9/D3Q19 up to 4th order.
  * Eq. (feq): sum feq = p, sum c feq = u (quadrature identities, Sec. 2.2.1).
  * Eq. (source-moments-check): sum Phi = s0, sum c Phi = s_u.
  * Eq. (macro-reconstruct): m = P f + s/2 after reconstruction.
  * Post-collision moments: P C = m + s/2 (collision conserves P(f - feq),
    adds the source with weight 1/2 on each parity).
  * Eq. (collision-operating): C = feq + Phi/2 exactly at omega+- = 1.
  * Equal rates reduce TRT to the BGK map C = f - w(f - feq) + (1 - w/2) Phi
    (Sec. 4.1).
  * Ghost elimination and survival (Sec. 2.4.1-2.4.2, Eq. eta).
"""
import itertools
import math

import numpy as np
import pytest

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("d", [2, 3])
def test_lattice_quadrature(orc, d):
    c, w, opp = orc.lattice(d)
    Q = 9 if d == 2 else 19
    assert c.shape == (Q, 3)
    c = c[:, :d].astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose((w[:, None] * c).sum(0), 0.0, atol=1e-16)
    second = np.einsum("k,ka,kb->ab", w, c, c)
    np.testing.assert_allclose(second, CS2 * np.eye(d), atol=1e-16)
    third = np.einsum("k,ka,kb,kc->abc", w, c, c, c)
    np.testing.assert_allclose(third, 0.0, atol=1e-16)
    fourth = np.einsum("k,ka,kb,kc,kd->abcd", w, c, c, c, c)
    I = np.eye(d)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
                      + np.einsum("ad,bc->abcd", I, I))
    np.testing.assert_allclose(fourth, iso, atol=1e-16)
    # opposite-direction table: c_kbar = -c_k, an involution
    np.testing.assert_array_equal(c[opp], -c)
    np.testing.assert_array_equal(opp[opp], np.arange(Q))
    # App. A orderings (exact listing)
    if d == 2:
        np.testing.assert_array_equal(c[:, 0], [0, 1, 0, -1, 0, 1, -1, -1, 1])
        np.testing.assert_array_equal(c[:, 1], [0, 0, 1, 0, -1, 1, 1, -1, -1])
        np.testing.assert_array_equal(opp, [0, 3, 4, 1, 2, 7, 8, 5, 6])
    else:
        np.testing.assert_array_equal(opp, [0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17])


def _rand_m(rng, d, scale=1e-2):
    return rng.normal(size=d + 1) * scale


@pytest.mark.parametrize("d", [2, 3])
def test_equilibrium_and_source_moments(orc, d):
    c, w, _ = orc.lattice(d)
    c = c[:, :d].astype(float)
    rng = np.random.default_rng(5)
    for _ in range(20):
        m = _rand_m(rng, d)
        s = _rand_m(rng, d, 1e-3)
        fe = orc.feq_site(d, m)
        assert abs(fe.sum() - m[0]) <= 1e-15
        np.testing.assert_allclose(c.T @ fe, m[1:], atol=1e-17, rtol=1e-13)
        ph = orc.phi_site(d, m, s)
        assert abs(ph.sum() - s[0]) <= 1e-16
        np.testing.assert_allclose(c.T @ ph, s[1:], atol=1e-18, rtol=1e-12)
        # the linear lift E of Eq. (linear-lift): feq linear part at u = 0
        fe_lin = orc.feq_site(d, np.concatenate([[m[0]], np.zeros(d)]))
        np.testing.assert_allclose(fe_lin, w * m[0], rtol=1e-15)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("taus", [(1.0, 1.0), (0.8, 1.4), (1.7, 0.6)])
def test_reconstruction_and_collision_moments(orc, d, taus):
    c, w, _ = orc.lattice(d)
    c = c[:, :d].astype(float)
    P = np.vstack([np.ones(len(w)), c.T])
    rng = np.random.default_rng(11)
    wp, wm = 1.0 / taus[0], 1.0 / taus[1]
    for a in (0.0, 1.0 / 64.0, 3.0 / 128.0, 0.7):
        f = w * (1.0 + rng.normal(size=len(w)) * 1e-2)
        h = rng.normal(size=d + 1) * 1e-2
        C, m, s = orc.collide_site(d, f, h, a, wp, wm)
        # Eq. (macro-reconstruct): m = P f + s/2 and s = h - a m
        np.testing.assert_allclose(m, P @ f + s / 2, rtol=0, atol=1e-15)
        np.testing.assert_allclose(s, h - a * m, rtol=0, atol=1e-16)
        # post-collision moments: P C = m + s/2
        np.testing.assert_allclose(P @ C, m + s / 2, rtol=0, atol=2e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_operating_point_reduction(orc, d):
    """Eq. (collision-operating): C = feq(m) + Phi(m, s)/2 at omega+- = 1."""
    c, w, _ = orc.lattice(d)
    rng = np.random.default_rng(3)
    for _ in range(10):
        f = w * (0.3 + rng.normal(size=len(w)) * 0.1)
        h = rng.normal(size=d + 1) * 1e-2
        a = 3.0 / (2 * 64.0)
        C, m, s = orc.collide_site(d, f, h, a, 1.0, 1.0)
        ref = orc.feq_site(d, m) + 0.5 * orc.phi_site(d, m, s)
        np.testing.assert_allclose(C, ref, rtol=0, atol=4e-17)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("omega", [1.0, 0.7, 1.6])
def test_trt_equals_bgk_at_equal_rates(orc, d, omega):
    """Equal TRT rates give the BGK map (Sec. 4.1); paper bound 2e-14 per step."""
    c, w, _ = orc.lattice(d)
    rng = np.random.default_rng(7)
    for _ in range(10):
        f = w * (1.0 + rng.normal(size=len(w)) * 1e-2)
        h = rng.normal(size=d + 1) * 1e-3
        a = 1.0 / 50.0
        C, m, s = orc.collide_site(d, f, h, a, omega, omega)
        bgk = f - omega * (f - orc.feq_site(d, m)) + (1 - omega / 2) * orc.phi_site(d, m, s)
        assert np.max(np.abs(C - bgk)) < 2e-14


def _ghost_basis(orc, d):
    """Orthonormal basis of ker P (population perturbations with no moments)."""
    c, w, _ = orc.lattice(d)
    P = np.vstack([np.ones(len(w)), c[:, :d].T.astype(float)])
    _, _, vt = np.linalg.svd(P)
    return vt[d + 1:]


@pytest.mark.parametrize("d", [2, 3])
def test_ghost_elimination_and_survival(orc, d):
    """At omega+- = 1 a ghost perturbation (P g = 0) does not change C at all
    (nonlinear statement, Sec. 2.4.1).  Off design the collision output changes
    by exactly (1 - w+) g+ + (1 - w-) g- (Sec. 2.4.2)."""
    c, w, opp = orc.lattice(d)
    G = _ghost_basis(orc, d)
    assert G.shape[0] == len(w) - d - 1  # six ghost directions in D2Q9
    rng = np.random.default_rng(2)
    f = w * (1.0 + rng.normal(size=len(w)) * 1e-2)
    h = rng.normal(size=d + 1) * 1e-3
    a = 3.0 / 128.0
    C0, _, _ = orc.collide_site(d, f, h, a, 1.0, 1.0)
    for g in G:
        g = g * 1e-3
        C1, _, _ = orc.collide_site(d, f + g, h, a, 1.0, 1.0)
        assert np.max(np.abs(C1 - C0)) < 1e-15  # a few ulps of f ~ 0.3
    for wp, wm in ((0.8, 1.3), (1.5, 0.6)):
        C0, _, _ = orc.collide_site(d, f, h, a, wp, wm)
        for g in G:
            g = g * 1e-3
            C1, _, _ = orc.collide_site(d, f + g, h, a, wp, wm)
            gp, gm = 0.5 * (g + g[opp]), 0.5 * (g - g[opp])
            np.testing.assert_allclose(C1 - C0, (1 - wp) * gp + (1 - wm) * gm, rtol=0, atol=1e-15)
    # on the Lambda = 1/4 line every ghost survives one collision with the
    # common amplitude eta(nu) of Eq. (eta)
    for nu in (0.09, 0.12, 0.25):
        tp = 0.5 + 3 * nu
        tm = 0.5 + 1 / (12 * nu)
        eta = abs(6 * nu - 1) / (6 * nu + 1)
        C0, _, _ = orc.collide_site(d, f, h, a, 1 / tp, 1 / tm)
        for g in G:
            g = g * 1e-3
            C1, _, _ = orc.collide_site(d, f + g, h, a, 1 / tp, 1 / tm)
            ratio = np.linalg.norm(C1 - C0) / np.linalg.norm(g)
            assert abs(ratio - eta) < 1e-9


@pytest.mark.parametrize("nu", [0.05, 0.09, 1.0 / 6.0, 0.3, 1.2])
def test_eta_on_lambda_quarter_line(nu):
    """Eq. (eta): on Lambda = 1/4 the two survival amplitudes are equal."""
    tp = 0.5 + nu / CS2
    tm = 0.5 + 0.25 / (tp - 0.5)
    eta = abs(6 * nu - 1) / (6 * nu + 1)
    assert abs(abs(1 - 1 / tp) - eta) < 1e-15
    assert abs(abs(1 - 1 / tm) - eta) < 1e-15
    assert abs((tp - 0.5) * (tm - 0.5) - 0.25) < 1e-15


def test_eta_value_printed():
    """Sec. 4.6: eta(0.09) = 0.2987 (about 0.30)."""
    eta = abs(6 * 0.09 - 1) / (6 * 0.09 + 1)
    assert abs(eta - 0.2987) < 5e-5


def test_gamma_dt_printed():
    """Eq. (slowrate) and Sec. 4.3: gamma_dt = 0.9622 at dt = 38.9."""
    dt = 38.9
    g = (1 - 3 / (4 * dt)) / (1 + 3 / (4 * dt))
    assert abs(g - 0.962169) < 1e-6
