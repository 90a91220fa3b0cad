"""Pins of the oracle's wall-bounded kinetic correction (Sec. 3.3,
Algorithm 2) on small lid-driven cavities.

* Eq. (wall-G) and Eq. (wall-local-jacobian) equal the central-difference
  Jacobian of the oracle's collision at omega+- = 1 (exact: C is quadratic).
* The assembled L = B_Gamma S blkdiag(J^C) (Eq. wall-global-jacobian) equals
  the central-difference Jacobian of the whole cavity sweep, at rest and at
  a random state, on square and rectangular grids: this is the paper's own
  check of the analytic assembly (Sec. 4, verification).
* The wall rows follow the printed order: from a zero state with only the
  lid moving, the sweep leaves -u/6 and +u/6 on the lid rows and the corner
  values that the side walls copy last.
* Algorithm 2 with the frozen or adaptive operator reaches the fixed point
  of the Picard iteration (the corrector changes the convergence, not the
  solution); near rest one correction leaves a residual of second order;
  the forced refresh interval refreshes at the stated inner indices.
"""
import numpy as np
import pytest

NU = 1.0 / 6.0


def _rand_state(orc, shape, seed, amp=1e-2):
    rng = np.random.default_rng(seed)
    c, w, _ = orc.lattice(2)
    wq = w.reshape((9, 1, 1))
    f = wq * (1.0 + amp * rng.normal(size=(9,) + shape))
    h = 0.05 * (1.0 + amp * rng.normal(size=(3,) + shape))
    return f, h


@pytest.mark.parametrize("a", [3.0 / 128.0, 1.0 / 16.0, 0.3])
def test_wall_G_is_collision_derivative(orc, a):
    rng = np.random.default_rng(11)
    c, w, _ = orc.lattice(2)
    for _ in range(4):
        f = w * (1.0 + 0.2 * rng.normal(size=9)) + 0.01 * rng.normal(size=9)
        h = 0.1 * rng.normal(size=3)
        M = np.array([f.sum(), (c[:9, 0] * f).sum(), (c[:9, 1] * f).sum()])
        m = (M + h / 2) / (1 + a / 2)
        s = h - a * m
        Jc = orc.cavity_local_jacobians(m.reshape(3, 1, 1), s.reshape(3, 1, 1), a)[0]
        Jd = np.zeros((9, 9))
        for j in range(9):
            e = np.zeros(9)
            e[j] = 1.0
            Cp = orc.collide_site(2, f + e, h, a, 1.0, 1.0)[0]
            Cm = orc.collide_site(2, f - e, h, a, 1.0, 1.0)[0]
            Jd[:, j] = (Cp - Cm) / 2.0
        np.testing.assert_allclose(Jc, Jd, rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape,state", [((4, 4), "rest"), ((6, 4), "rest"), ((4, 4), "random"),
                                         ((4, 6), "random")])
def test_assembled_operator_is_sweep_jacobian(orc, shape, state):
    a = 3.0 / 64.0
    ulid = 0.05
    if state == "rest":
        c, w, _ = orc.lattice(2)
        f = np.broadcast_to(w.reshape(9, 1, 1), (9,) + shape).copy()
        h = np.zeros((3,) + shape)
        h[0] = a
    else:
        f, h = _rand_state(orc, shape, seed=sum(shape))
    m = (orc.moments(f) + h / 2) / (1 + a / 2)
    Jc = orc.cavity_local_jacobians(m, h - a * m, a)
    L = orc.cavity_operator(Jc, shape).toarray()
    n = f.size
    Jd = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        fp = orc.cavity_sweep((f.ravel() + e).reshape(f.shape), h, a, ulid)[0]
        fm = orc.cavity_sweep((f.ravel() - e).reshape(f.shape), h, a, ulid)[0]
        Jd[:, i] = (fp - fm).ravel() / 2.0
    np.testing.assert_allclose(L, Jd, rtol=0, atol=1e-12)
    # at most nine nonzeros per row (Sec. 3.3)
    assert max(np.count_nonzero(row) for row in L) <= 9


def test_wall_rows_and_corner_order(orc):
    N = 4
    u = 0.12
    f = np.zeros((9, N, N))
    fT, _ = orc.cavity_sweep(f, None, 0.0, u)
    top = N - 1
    for x in range(1, N - 1):  # lid interior: f7 = f5 - u/6, f8 = f6 + u/6
        assert fT[7, x, top] == pytest.approx(-u / 6) and fT[8, x, top] == pytest.approx(u / 6)
    # top-left corner: the left wall copies last (f5 <- f7, f8 <- f6)
    assert fT[5, 0, top] == pytest.approx(-u / 6) and fT[8, 0, top] == 0.0 and fT[7, 0, top] == pytest.approx(-u / 6)
    # top-right corner: the right wall copies last (f6 <- f8, f7 <- f5)
    assert fT[6, N - 1, top] == pytest.approx(u / 6) and fT[7, N - 1, top] == 0.0
    assert fT[8, N - 1, top] == pytest.approx(u / 6)
    # no other population moves
    mask = np.zeros_like(fT, dtype=bool)
    mask[[5, 6, 7, 8], :, top] = True
    assert np.all(fT[~mask] == 0.0)


def test_kinetic_correction_same_fixed_point_as_picard(orc):
    N = 16
    ulid = 10 * NU / N
    p0 = np.zeros((N, N))
    u0 = np.zeros((2, N, N))
    out = {}
    for corr in ("picard", "frozen", "adaptive"):
        r = orc.cavity_march(p0, u0, ulid=ulid, dt=16.0, nsteps=3, eps=1e-12, kmax=1000, corrector=corr)
        assert r["status"] == 0
        out[corr] = r
    iters = {k: [s["iters"] for s in v["stats"]] for k, v in out.items()}
    assert all(a < b / 5 for a, b in zip(iters["frozen"], iters["picard"]))
    for corr in ("frozen", "adaptive"):
        assert np.abs(out[corr]["m"] - out["picard"]["m"]).max() <= 1e-9 * np.abs(out["picard"]["m"]).max()


def test_quadratic_convergence_near_rest(orc):
    """Without the lid the rest state is a fixed point and the frozen operator
    is the exact linearisation there: one correction from rest + delta leaves
    a residual of order delta^2."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    shape = (8, 8)
    dt = 32.0
    a = 3.0 / (2 * dt)
    c, w, _ = orc.lattice(2)
    mref = np.zeros((3,) + shape)
    mref[0] = 1.0
    L = orc.cavity_operator(orc.cavity_local_jacobians(mref, np.zeros_like(mref), a), shape)
    lu = spl.splu((sp.identity(L.shape[0], format="csc") - L).tocsc())
    h = a * mref
    rng = np.random.default_rng(3)
    ratios = []
    for delta in (1e-3, 1e-4):
        f = w.reshape(9, 1, 1) * (1.0 + delta * rng.normal(size=(9,) + shape))
        fT, R0 = orc.cavity_sweep(f, h, a, 0.0)
        f1 = f + lu.solve((fT - f).ravel()).reshape(f.shape)
        _, R1 = orc.cavity_sweep(f1, h, a, 0.0)
        ratios.append(R1 / R0)
        assert R1 / R0 < 20 * delta
    assert ratios[1] < 0.2 * ratios[0]


def test_forced_refresh_schedule(orc):
    N = 16
    r = orc.cavity_march(np.zeros((N, N)), np.zeros((2, N, N)), ulid=10 * NU / N, dt=16.0, nsteps=2, eps=1e-12,
                         kmax=400, corrector="adaptive", n_forced=2)
    assert r["status"] == 0
    for s in r["stats"]:
        K = s["iters"]
        expect = [e for e in (2, 4, 6) if e < K]
        assert s["refreshed_at"] == expect
