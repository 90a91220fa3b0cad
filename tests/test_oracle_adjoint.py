"""Pins of the oracle's discrete adjoint (the transpose of the unrolled march).

* Per stage, the dot-product (transpose) test <J v, w> = <v, J^T w>:
  the sweep with respect to f and to h (T is quadratic in both, so a central
  difference gives J v exactly up to rounding), and the shadow operator
  (linear) with respect to its input.
* The whole march at replayed inner counts and the initial-state map:
  directional central finite differences of a scalar loss against the adjoint
  inner product.
"""
import numpy as np
import pytest

from paper_2609_39474_amd import workloads as W

NU = 1.0 / 6.0


def _state(orc, d, shape, seed):
    rng = np.random.default_rng(seed)
    c, w, _ = orc.lattice(d)
    Q = len(w)
    f = w.reshape((Q,) + (1,) * d) * (1 + 1e-2 * rng.normal(size=(Q,) + shape))
    h = 1e-3 * rng.normal(size=(d + 1,) + shape)
    return f, h, rng


@pytest.mark.parametrize("d,shape,wp,wm", [(2, (8, 4), 1.0, 1.0), (2, (4, 8), 1 / 0.8, 1 / 1.3),
                                           (3, (4, 4, 4), 1.0, 1.0), (3, (4, 2, 4), 1 / 1.2, 1 / 0.9)])
def test_sweep_adjoint_dot_product(orc, d, shape, wp, wm):
    f, h, rng = _state(orc, d, shape, 3)
    a = 3 / 128
    v = rng.normal(size=f.shape)
    vh = rng.normal(size=h.shape)
    w = rng.normal(size=f.shape)
    eps = 1e-5
    Jv = (orc.sweep(f + eps * v, h, a, wp, wm)[0] - orc.sweep(f - eps * v, h, a, wp, wm)[0]) / (2 * eps)
    Jhv = (orc.sweep(f, h + eps * vh, a, wp, wm)[0] - orc.sweep(f, h - eps * vh, a, wp, wm)[0]) / (2 * eps)
    lf, lh = orc.sweep_adjoint(f, h, a, wp, wm, w)
    lhs, rhs = np.sum(Jv * w), np.sum(v * lf)
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
    lhs, rhs = np.sum(Jhv * w), np.sum(vh * lh)
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


@pytest.mark.parametrize("d,shape", [(2, (16, 8)), (3, (8, 4, 8))])
def test_shadow_adjoint_dot_product(orc, d, shape):
    rng = np.random.default_rng(5)
    x = rng.normal(size=(d + 1,) + shape)
    y = rng.normal(size=(d + 1,) + shape)
    a = 3 / 128
    lhs = np.sum(orc.shadow(x, a, NU) * y)
    rhs = np.sum(x * orc.shadow_adjoint(y, a, NU))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def _loss(orc, m_final, ustar):
    return 0.5 * np.sum((m_final[1:] - ustar) ** 2)


@pytest.mark.parametrize("corrector,extrap", [(1, 0), (0, 0), (1, 2)])
def test_march_adjoint_vs_finite_differences(orc, corrector, extrap):
    N = 8
    shape = (N, N)
    p0, u0 = W.random_field_2d(N, NU / N, seed=2, jmax=3)
    st0 = orc.initial_state(p0, u0)
    kw = dict(dt=24.0, eps=1e-10, nmin=2, corrector=corrector, extrap_states=extrap, kmax=400)
    rc, st, _, stats = orc.march_state(st0, 0, shape, nsteps=4, **kw)
    assert rc == 0
    K = [s["iters"] for s in stats]
    Q, NS = 9, N * N
    FQ = Q * NS
    ustar = 0.7 * st[3 * FQ + NS:3 * FQ + 3 * NS].reshape(2, N, N)

    def L(state):
        _, s1, _, _ = orc.march_state(state, 0, shape, nsteps=4, schedule=K, **kw)
        return _loss(orc, s1[3 * FQ:3 * FQ + 3 * NS].reshape(3, N, N), ustar)

    lam = np.zeros_like(st)
    lam[3 * FQ + NS:3 * FQ + 3 * NS] = (st[3 * FQ + NS:3 * FQ + 3 * NS].reshape(2, N, N) - ustar).ravel()
    lam0 = orc.march_adjoint(st0, 0, shape, lam, schedule=K, **kw)
    rng = np.random.default_rng(8)
    v = rng.normal(size=st0.shape) * np.abs(st0).max()
    h = 1e-4
    fd = (L(st0 + h * v) - L(st0 - h * v)) / (2 * h)
    ad = np.sum(lam0 * v)
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)


def test_initial_state_adjoint(orc):
    N = 8
    p0, u0 = W.random_field_2d(N, NU / N, seed=4, jmax=3)
    rng = np.random.default_rng(1)
    lam = rng.normal(size=orc.initial_state(p0, u0).shape)
    lp, lu = orc.initial_state_adjoint(p0, u0, lam)
    vp, vu = rng.normal(size=p0.shape) * 1e-3, rng.normal(size=u0.shape) * 1e-3
    eps = 1e-3
    fd = (np.sum(orc.initial_state(p0 + eps * vp, u0 + eps * vu) * lam)
          - np.sum(orc.initial_state(p0 - eps * vp, u0 - eps * vu) * lam)) / (2 * eps)
    ad = np.sum(lp * vp) + np.sum(lu * vu)
    assert abs(fd - ad) <= 1e-9 * abs(ad)
