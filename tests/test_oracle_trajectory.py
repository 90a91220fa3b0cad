"""Trajectory-level pins of the oracle: values the paper prints for worked
runs, exact solutions, conservation invariants and closed-form rates.

* Tab. 2 (Sec. 4.2): temporal self-convergence of the corrected method, 2D and
  3D, reproduced to about three significant figures (fixture
  tests/golden/tab2_temporal_order.json, with the normalisation reading).
* Eq. (tgv2d): the explicit march follows the analytic decay; the corrected
  method passes the matched gate e_abs <= 3 e_explicit (Sec. 4.1) on the
  paper's horizon T_end = nint(0.15 N^2) at N = 64 with S = 32.
* Eq. (symbol) and Sec. 4.3: the plain Picard tail contraction equals the
  slowest symbol eigenvalue of the excited Taylor-Green mode; the paper's
  gamma_dt = 0.9622 bounds it and its measured 0.958-0.960 sits just below.
* Sec. 4.2: the corrected and Picard iterations reach the same fixed point.
* Sec. 4.3: mean inner counts at the Taylor-Green protocol lie in the printed
  2.0-3.2 (loose); Sec. 3.1: the trial extrapolation is exact for population
  histories polynomial in time (closed form).
* Sec. 4.6: stability points (N = 128, Re = 100, T_end = 2458: S = 32
  stable, S = 16 diverges).
* Conservation: the explicit map conserves sum f and sum c f; one DTS sweep
  returns sum_x P T(f) = sum_x (m + s/2) (post-collision moments, Eq.
  macro-reconstruct, Eq. source-moments-check); streaming is a permutation.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2609_39474_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tab2_temporal_order.json")
NU = 1.0 / 6.0


def _rms_components(a, b):
    return math.sqrt(float(((a - b) ** 2).mean()))


def _tab2(orc, key, tgv, eps):
    g = json.load(open(GOLD))[key]
    N = g["N"]
    U = g["Re"] * NU / N
    p0, u0 = tgv(N, U)
    us = {}
    for dt in g["dt"]:
        S = int(round(g["T_end"] / dt))
        r = orc.march(p0, u0, dt=float(dt), nsteps=S, eps=eps, kmax=20000, nmin=g["nmin"],
                      corrector=1)
        assert r.status == 0 and r.steps_done == S
        assert max(s["R_final"] for s in r.stats) < eps
        us[dt] = r.m[1:]
    dts = g["dt"]
    D = [_rms_components(us[dts[i]], us[dts[i + 1]]) for i in range(3)]
    p = [math.log2(D[i] / D[i + 1]) for i in range(2)]
    return g, D, p


def test_tab2_2d(orc):
    g, D, p = _tab2(orc, "2d", lambda N, U: W.tgv2d(N, U, NU), 1e-13)
    for got, ref in zip(D, g["D"]):
        assert abs(got / ref - 1) < 1e-3, (D, g["D"])
    for got, ref in zip(p, g["p"]):
        assert abs(got - ref) < 2e-3, (p, g["p"])


@pytest.mark.slow
def test_tab2_3d(orc):
    g, D, p = _tab2(orc, "3d", lambda N, U: W.tgv3d(N, U), 1e-12)
    for got, ref in zip(D, g["D"]):
        assert abs(got / ref - 1) < 2e-3, (D, g["D"])
    for got, ref in zip(p, g["p"]):
        assert abs(got - ref) < 3e-3, (p, g["p"])


def test_explicit_tgv_decay_and_conservation(orc):
    N = 64
    U = NU / N
    T = W.nint(0.1 * N * N / NU)
    p0, u0 = W.tgv2d(N, U, NU)
    f0 = orc.init_populations(p0, u0)
    fe = orc.explicit(f0, T)
    M = orc.moments(fe)
    _, uref = W.tgv2d(N, U, NU, t=T)
    err = math.sqrt(((M[1:] - uref) ** 2).sum(0).mean())
    amp = math.sqrt((uref ** 2).sum(0).mean())
    assert err / amp < 1e-2  # O(k0^2) lattice error, about 0.6 % here
    # conservation to round-off: sum f and sum c f
    M0 = orc.moments(f0)
    assert abs(M[0].sum() - M0[0].sum()) < 1e-14
    assert np.all(np.abs(M[1:].sum(axis=(1, 2)) - M0[1:].sum(axis=(1, 2))) < 1e-14)


def test_matched_gate_tgv_n64(orc):
    """Tab. 4 reports a matched-gate pass at (N, Re) = (64, 1)."""
    N = 64
    U = NU / N
    T = W.nint(0.15 * N * N)
    p0, u0 = W.tgv2d(N, U, NU)
    fe = orc.explicit(orc.init_populations(p0, u0), T)
    _, uref = W.tgv2d(N, U, NU, t=T)
    e_exp = math.sqrt(((orc.moments(fe)[1:] - uref) ** 2).sum(0).mean())
    S = 32
    r = orc.march(p0, u0, dt=T / S, nsteps=S, eps=1e-10, nmin=2)
    assert r.status == 0
    e_dts = math.sqrt(((r.m[1:] - uref) ** 2).sum(0).mean())
    assert e_dts <= 3 * e_exp, (e_dts, e_exp)


def test_picard_tail_factor(orc):
    N = 128
    dt = 38.9
    p0, u0 = W.tgv2d(N, NU / N, NU)
    r = orc.march(p0, u0, dt=dt, nsteps=2, eps=1e-10, nmin=2, corrector=0, kmax=2000)
    assert r.status == 0
    rho = r.stats[1]["rho_obs"]
    # slowest symbol eigenvalue of gamma P Z(theta) E at theta = 2 pi (1, 1)/N
    cs2 = 1 / 3
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1.0])
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1.0])
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    c = np.stack([cx, cy], 1)
    E = np.hstack([w[:, None], w[:, None] * c / cs2])
    P = np.vstack([np.ones(9), c.T])
    a = 3 / (2 * dt)
    g = (1 - a / 2) / (1 + a / 2)
    th = 2 * np.pi * np.array([1, 1]) / N
    lam = np.abs(np.linalg.eigvals(g * P @ np.diag(np.exp(-1j * (c @ th))) @ E)).max()
    assert abs(rho - lam) < 1e-4, (rho, lam)
    assert 0.955 < rho < 0.9622  # paper: gamma 0.9622 predicted, 0.958-0.960 measured


def test_msc_and_picard_share_fixed_point(orc):
    """Sec. 4.2: 3.57e-11 abs / 4.15e-10 rel at N = 128, Re = 100, dt = 38.9."""
    N = 128
    U = 100 * NU / N
    p0, u0 = W.tgv2d(N, U, NU)
    a = orc.march(p0, u0, dt=38.9, nsteps=2, eps=1e-12, nmin=2, corrector=1, kmax=3000)
    b = orc.march(p0, u0, dt=38.9, nsteps=2, eps=1e-12, nmin=2, corrector=0, kmax=3000)
    assert a.status == 0 and b.status == 0
    diff = math.sqrt(((a.m[1:] - b.m[1:]) ** 2).sum(0).mean())
    ref = math.sqrt((a.m[1:] ** 2).sum(0).mean())
    assert diff < 3.57e-10 and diff / ref < 4.15e-9  # within 10x of the printed values
    # and the corrector needs far fewer iterations than Picard
    assert sum(s["iters"] for s in a.stats) * 5 < sum(s["iters"] for s in b.stats)


def test_stability_points(orc):
    N = 128
    U = 100 * NU / N
    p0, u0 = W.tgv2d(N, U, NU)
    ok = orc.march(p0, u0, dt=2458 / 32, nsteps=32, eps=1e-8, nmin=2)
    assert ok.status == 0 and ok.steps_done == 32
    assert np.isfinite(ok.m).all() and np.abs(ok.m[1:]).max() < U
    bad = orc.march(p0, u0, dt=2458 / 16, nsteps=16, eps=1e-8, nmin=2)
    assert bad.status != 0 and bad.steps_done < 16


@pytest.mark.parametrize("N,S", [(64, 16), (128, 16), (128, 8), (256, 32)])
def test_inner_counts_tab4_protocol(orc, N, S):
    """Sec. 4.3: along the refinement sequence the corrected method needs 2.0 to
    3.2 inner iterations per physical step on average.  The Taylor-Green
    protocol (Re = 1, T_end = nint(0.15 N^2), the paper's trial rule, n_min =
    2) at the (S, eps = 1e-6) cells that pass the matched and 1% gates must
    land in that range.  A loose check: at these tolerances the counts do not
    distinguish the trial rules (constant, linear and up to cubic give 2.0 to
    2.6), so the extrapolation itself is pinned by the test below."""
    U = NU / N
    T = W.nint(0.15 * N * N)
    p0, u0 = W.tgv2d(N, U, NU)
    r = orc.march(p0, u0, dt=T / S, nsteps=S, eps=1e-6, nmin=2)
    assert r.status == 0
    mean = float(np.mean([s["iters"] for s in r.stats]))
    assert 2.0 <= mean <= 3.2, mean


@pytest.mark.parametrize("bc,extrap,degree", [(0, 0, 0), (1, 0, 1), (2, 0, 2), (7, 0, 2), (7, 2, 1), (7, 1, 0)])
def test_trial_extrapolation_exact_for_polynomial_histories(orc, bc, extrap, degree):
    """Sec. 3.1: the first trial of a physical step extrapolates the accepted
    population states (f^n on the first step, 2 f^n - f^{n-1} on the second,
    3 f^n - 3 f^{n-1} + f^{n-2} after that, or a cap on the number of states).
    Each rule is the next value of the polynomial through the states it uses,
    so for histories sampled at t = 0, 1, 2 from a polynomial of that degree in
    time the trial equals the polynomial at t = 3 (the slots a rule must not
    read hold unrelated values).  One Picard sweep accepted at
    a replayed count of one returns T(trial), which must equal the sweep of that
    value; a rule of the wrong degree (or the wrong states) misses it by O(1)."""
    shape = (16, 8)
    Q, NS = 9, 16 * 8
    rng = np.random.default_rng(100 + bc + 10 * extrap)
    c, w, _ = orc.lattice(2)
    coef = [w.reshape(Q, 1, 1) * 1e-3 * rng.normal(size=(Q,) + shape) for _ in range(3)]
    for j in range(degree + 1, 3):
        coef[j] = np.zeros_like(coef[j])

    def f_at(t):
        return coef[0] + t * coef[1] + t * t * coef[2]

    mn = 1e-4 * rng.normal(size=(3,) + shape)
    mp = 1e-4 * rng.normal(size=(3,) + shape)
    # slots the rule must not read hold unrelated values
    order = min(bc, 2 if extrap == 0 else extrap - 1)
    hist = [f_at(2.0), f_at(1.0), f_at(0.0)]
    for j in range(order + 1, 3):
        hist[j] = w.reshape(Q, 1, 1) * 1e-3 * rng.normal(size=(Q,) + shape)
    state = np.concatenate([hist[0].ravel(), hist[1].ravel(), hist[2].ravel(), mn.ravel(), mp.ravel()])
    dt = 40.0
    rc, st, _, stats = orc.march_state(state, bc, shape, dt=dt, nsteps=1, schedule=[1], nmin=1, corrector=0,
                                       extrap_states=extrap)
    assert rc == 0 and stats[0]["iters"] == 1
    q = 1 if bc == 0 else 2
    a = 1.0 / dt if q == 1 else 1.5 / dt
    h = mn / dt if q == 1 else (4 * mn - mp) / (2 * dt)
    want, _, _ = orc.sweep(f_at(3.0), h, a, 1.0, 1.0)
    got = st[:Q * NS].reshape(want.shape)
    err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    assert err <= 1e-13, err
    # the next-lower degree rule misses (guards against a test that cannot fail)
    if degree > 0:
        lower, _, _ = orc.sweep(f_at(2.0) if degree == 1 else 2 * f_at(2.0) - f_at(1.0), h, a, 1.0, 1.0)
        assert float(np.max(np.abs(got - lower)) / np.max(np.abs(want))) > 1e-3


@pytest.mark.parametrize("d,shape", [(2, (16, 8)), (3, (8, 4, 8))])
def test_dts_sweep_conservation(orc, d, shape):
    rng = np.random.default_rng(9)
    c, w, _ = orc.lattice(d)
    Q = len(w)
    f = (w.reshape((Q,) + (1,) * d) * (1 + 1e-2 * rng.normal(size=(Q,) + shape)))
    h = 1e-3 * rng.normal(size=(d + 1,) + shape)
    a = 3 / 128
    fT, Pr, R = orc.sweep(f, h, a, 1.0, 1.0)
    M = orc.moments(f)
    m = (M + h / 2) / (1 + a / 2)
    s = h - a * m
    MT = orc.moments(fT)
    np.testing.assert_allclose(MT.sum(axis=tuple(range(1, d + 1))),
                               (m + s / 2).sum(axis=tuple(range(1, d + 1))), rtol=0, atol=1e-13)
    # residual moments: P r = P fT - P f
    np.testing.assert_allclose(Pr, MT - M, rtol=0, atol=1e-15)
    # RMS definition of Eq. (residual)
    assert abs(R - math.sqrt(((fT - f) ** 2).mean())) < 1e-16


def test_march_conserves_totals(orc):
    """At the fixed point sum_x s = 0, so totals of m carry over; zero-mean
    pressure gauge and zero net momentum persist (drift of order eps)."""
    N = 32
    p0, u0 = W.random_field_2d(N, NU / N, seed=3, jmax=6)
    r = orc.march(p0, u0, dt=32.0, nsteps=6, eps=1e-12, nmin=2)
    assert r.status == 0
    assert abs(r.m[0].sum()) < 1e-9 and np.all(np.abs(r.m[1:].sum(axis=(1, 2))) < 1e-9)


def test_failure_modes(orc):
    N = 16
    p0, u0 = W.tgv2d(N, NU / N, NU)
    r = orc.march(p0, u0, dt=64.0, nsteps=3, eps=1e-30, kmax=2, nmin=1)
    assert r.status == 5 and r.steps_done == 0  # nonconvergent at K_max
    # schedule replay accepts at the given counts regardless of eps
    r2 = orc.march(p0, u0, dt=64.0, nsteps=3, eps=1e-30, kmax=10, nmin=1, schedule=[3, 2, 4])
    assert r2.status == 0 and [s["iters"] for s in r2.stats] == [3, 2, 4]


def test_march_state_composes(orc):
    """Stepping the full state one step at a time reproduces the one-shot march
    bit for bit (same arithmetic, same order)."""
    N = 16
    p0, u0 = W.random_field_2d(N, NU / N, seed=5, jmax=4)
    full = orc.march(p0, u0, dt=48.0, nsteps=4, eps=1e-12, nmin=2)
    st, bc = orc.initial_state(p0, u0), 0
    for n in range(4):
        rc, st, bc, _ = orc.march_state(st, bc, (N, N), dt=48.0, nsteps=1, eps=1e-12, nmin=2,
                                        schedule=[full.stats[n]["iters"]])
        assert rc == 0
    Q = 9
    NS = N * N
    np.testing.assert_array_equal(st[:Q * NS].reshape(full.f.shape), full.f)
    np.testing.assert_array_equal(st[3 * Q * NS:3 * Q * NS + 3 * NS].reshape(full.m.shape), full.m)
    assert bc == 4
