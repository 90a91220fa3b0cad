"""Pins of the oracle's full-symbol reference corrector (Sec. 4.1, Eq.
full-symbol) on tiny grids.

* The collision Jacobian at rest equals the closed form derived from Eq.
  (collision) with Eq. (macro-reconstruct) and Eq. (source-moments):
  J = (1-w+) Pi+ + (1-w-) Pi- + c+ E0 P0 + c- Eu Pu,
  c+- = [w+- - a (1 - w+-/2)] / (1 + a/2).  The paper's forward difference
  of step 1e-7 lies within its truncation error of it.
* The full-symbol correction is the exact Newton step of the sweep
  linearised at rest: on tiny grids the dense Jacobian of T (central
  differences, exact for the quadratic T) gives df = (I - dT/df)^-1 r by a
  dense solve, independent of the transforms, Z(k) and J.
* Near rest the corrected iteration converges quadratically (the residual
  after one step is second order in the distance from rest).
* Off the collision operating point the full-symbol reference keeps a small
  contraction where the shadow correction diverges (Sec. 4.6).
"""
import numpy as np
import pytest

from paper_2609_39474_amd import workloads as W

CS2 = 1.0 / 3.0


def _closed_J(orc, d, a, wp, wm):
    c, w, opp = orc.lattice(d)
    c = c[:, :d].astype(float)
    Q = len(w)
    I = np.eye(Q)
    Pi_p = 0.5 * (I + I[opp])
    Pi_m = 0.5 * (I - I[opp])
    E0 = w[:, None]
    Eu = (w[:, None] * c) / CS2
    cp = (wp - a * (1 - wp / 2)) / (1 + a / 2)
    cm = (wm - a * (1 - wm / 2)) / (1 + a / 2)
    return (1 - wp) * Pi_p + (1 - wm) * Pi_m + cp * E0 @ np.ones((1, Q)) + cm * Eu @ c.T


J_CASES = [(2, 3.0 / 128.0, 1.0, 1.0), (2, 1.0 / 64.0, 1 / 0.8, 1 / 1.3), (2, 0.2, 1 / 1.4, 1 / 0.6),
           (3, 3.0 / 128.0, 1.0, 1.0), (3, 0.05, 1 / 0.9, 1 / 1.2)]


@pytest.mark.parametrize("d,a,wp,wm", J_CASES)
def test_jacobian_at_rest_closed_form(orc, d, a, wp, wm):
    J = orc.collision_jacobian(d, a, wp, wm)
    np.testing.assert_allclose(J, _closed_J(orc, d, a, wp, wm), rtol=0, atol=2e-15)
    # the paper's construction: forward difference of step 1e-7
    Jf = orc.collision_jacobian(d, a, wp, wm, 1e-7)
    err = np.abs(Jf - J).max()
    assert 1e-12 < err < 2e-6


def _dense_T_jacobian(orc, fbar, h, a, wp, wm):
    n = fbar.size
    Jd = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        fp = orc.sweep((fbar.ravel() + e).reshape(fbar.shape), h, a, wp, wm)[0]
        fm = orc.sweep((fbar.ravel() - e).reshape(fbar.shape), h, a, wp, wm)[0]
        Jd[:, i] = (fp - fm).ravel() / 2.0
    return Jd


NEWTON_CASES = [
    (2, (4, 4), 1.0, 1.0, 3.0 / 128.0),
    (2, (8, 4), 1 / 0.8, 1 / 1.3, 1.0 / 64.0),
    (2, (4, 8), 1 / 1.4, 1 / 0.6, 0.2),
    (3, (4, 4, 2), 1 / 0.9, 1 / 1.2, 3.0 / 128.0),
]


@pytest.mark.parametrize("d,shape,wp,wm,a", NEWTON_CASES)
def test_full_symbol_is_dense_newton_step(orc, d, shape, wp, wm, a):
    c, w, _ = orc.lattice(d)
    Q = len(w)
    fbar = np.broadcast_to(w.reshape((Q,) + (1,) * d), (Q,) + shape).copy()  # feq(1, 0)
    h = np.zeros((d + 1,) + shape)
    h[0] = a  # h = a m at rest, s = 0
    Jd = _dense_T_jacobian(orc, fbar, h, a, wp, wm)
    rng = np.random.default_rng(Q + sum(shape))
    r = rng.normal(size=(Q,) + shape)
    dense = np.linalg.solve(np.eye(Jd.shape[0]) - Jd, r.ravel()).reshape(r.shape)
    df = orc.full_symbol(r, orc.collision_jacobian(d, a, wp, wm))
    assert np.abs(df - dense).max() <= 1e-11 * np.abs(dense).max()


@pytest.mark.parametrize("d,shape,wp,wm", [(2, (16, 16), 1.0, 1.0), (2, (16, 8), 1 / 0.8, 1 / 1.3),
                                           (3, (8, 8, 8), 1 / 0.9, 1 / 1.2)])
def test_quadratic_convergence_near_rest(orc, d, shape, wp, wm):
    """From rest plus a perturbation of size delta, one corrected iteration
    leaves a residual of order delta^2 (the sweep is quadratic)."""
    c, w, _ = orc.lattice(d)
    Q = len(w)
    a = 3.0 / 128.0
    rng = np.random.default_rng(7)
    wq = w.reshape((Q,) + (1,) * d)
    h = np.zeros((d + 1,) + shape)
    h[0] = a
    ratios = []
    for delta in (1e-3, 1e-4):
        f = wq * (1.0 + delta * rng.normal(size=(Q,) + shape))
        f1, _, R0 = orc.full_symbol_iteration(f, h, a, wp, wm)
        _, _, R1 = orc.sweep(f1, h, a, wp, wm)
        ratios.append(R1 / R0)
        assert R1 / R0 < 50 * delta
    # the contraction itself scales with delta (second order)
    assert ratios[1] < 0.2 * ratios[0]


def test_contraction_off_design(orc):
    """Taylor-Green at Re = 1, N = 32, one interior BDF2 step at dt = 64: the
    shadow correction diverges at nu = 0.05 on Lambda = 1/4 and barely
    contracts at Lambda = 1/64; the full-symbol reference converges at both."""
    N = 32
    for nu, lam in ((0.05, 0.25), (1 / 6, 1 / 64)):
        tp = 0.5 + 3 * nu
        tm = 0.5 + lam / (tp - 0.5)
        p0, u0 = W.tgv2d(N, nu / N, nu)
        sh = orc.march(p0, u0, dt=64.0, nsteps=2, eps=1e-10, kmax=400, nmin=2, corrector=1, tau_plus=tp,
                       tau_minus=tm)
        fs = orc.march(p0, u0, dt=64.0, nsteps=2, eps=1e-10, kmax=400, nmin=2, corrector=2, tau_plus=tp,
                       tau_minus=tm)
        assert fs.status == 0 and fs.stats[-1]["iters"] <= 4
        assert fs.stats[-1]["rho_obs"] < 0.01
        assert sh.status != 0 or sh.stats[-1]["rho_obs"] > 0.5
