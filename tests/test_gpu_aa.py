"""GPU parity of the in-place (AA) explicit march.

The explicit march (Eq. sweep with a = 0 and h = 0, the map of Sec. 4.1) runs
in place by the AA access pattern where the storage holds full populations
and the boundaries are periodic.  Bars: the AA march against the library's
two-buffer sweep on the same state, bit-exact (the collision is the same
code; only the memory access pattern differs), and against the FP64 oracle,
max |gpu - oracle| / max |oracle| <= 1e-12 with FP64 storage.  Step counts
cover a single step, one AA pair, odd counts (a two-buffer step after the
pairs) and graph-captured chunks.  Inputs are seeded random population
fields (equilibrium-scale density perturbations and non-equilibrium parts)
with distinct even and odd relaxation rates, so that every direction pair
and both TRT rates enter.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KEY_USE_GRAPH = 4
KEY_EXPLICIT_AA = 10
TAU = (0.8, 1.3)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


@pytest.fixture(scope="module")
def M():
    from paper_2609_39474_amd import msc
    msc.lib()
    return msc


def _solver(M, shape, storage):
    d = len(shape)
    p = M.make_params(d, shape[0], dt=1.0, eps=1e-10, storage=storage, corrector="picard",
                      tau_plus=TAU[0], tau_minus=TAU[1])
    for a in range(d):
        p.n[a] = shape[a]
    return M.Solver(p, np.zeros(shape), np.zeros((d,) + shape))


def _rand_f(orc, shape, seed):
    d = len(shape)
    _, w, _ = orc.lattice(d)
    Q = len(w)
    rng = np.random.default_rng(seed)
    wb = w.reshape((Q,) + (1,) * d)
    f = wb * (1.0 + 0.02 * rng.normal(size=shape))
    f = f + wb * 1e-3 * rng.normal(size=(Q,) + shape)
    return f


def _march(M, shape, storage, f0, steps, aa, graph):
    s = _solver(M, shape, storage)
    s.set_tuning(KEY_EXPLICIT_AA, 1 if aa else 0)
    s.set_tuning(KEY_USE_GRAPH, 1 if graph else 0)
    s.set_populations(f0)
    s.explicit_step(steps)
    f = s.populations()
    s.close()
    return f


SHAPES = [(64, 32), (32, 16, 8)]
STEPS = [1, 2, 7, 131]


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_aa_matches_two_buffer_bit_exact(M, orc, shape, storage):
    f0 = _rand_f(orc, shape, 11)
    for steps in STEPS:
        for graph in (False, True):
            say("aa vs two-buffer", shape, storage, "steps", steps, "graph", graph)
            fa = _march(M, shape, storage, f0, steps, True, graph)
            fb = _march(M, shape, storage, f0, steps, False, graph)
            np.testing.assert_array_equal(fa, fb)


@pytest.mark.parametrize("shape", SHAPES)
def test_aa_vs_oracle_fp64(M, orc, shape):
    f0 = _rand_f(orc, shape, 12)
    wp, wm = 1.0 / TAU[0], 1.0 / TAU[1]
    for steps in (2, 7, 131):
        say("aa vs oracle", shape, "steps", steps)
        fa = _march(M, shape, "fp64", f0, steps, True, True)
        of = orc.explicit(f0, steps, wp, wm)
        assert rel(fa, of) <= 1e-12


def test_aa_sequence_of_calls(M, orc):
    """Consecutive calls on one context (odd, even, odd counts) leave the
    population roles consistent: the result equals one call of the total."""
    shape = (32, 16, 8)
    f0 = _rand_f(orc, shape, 13)
    s = _solver(M, shape, "fp64")
    s.set_populations(f0)
    for n in (3, 64, 5):
        s.explicit_step(n)
    f = s.populations()
    s.close()
    of = orc.explicit(f0, 72, 1.0 / TAU[0], 1.0 / TAU[1])
    say("aa call sequence: rel", rel(f, of))
    assert rel(f, of) <= 1e-12


def test_aa_kernel_timing(M, orc):
    """Timed AA launches are counted as explicit-march launches with 2 Q
    values per site of traffic."""
    shape = (32, 16, 8)
    s = _solver(M, shape, "fp32")
    s.set_populations(_rand_f(orc, shape, 14))
    s.set_kernel_timing(True)
    s.explicit_step(10)
    sec, n, b = s.kernel_time(1)
    s.close()
    say("aa timing", sec, n, b)
    assert n == 10
    assert b == 2 * 19 * 32 * 16 * 8 * 4
    assert sec > 0


@pytest.mark.parametrize("storage,aa", [("fp32", 1), ("fp32", 0), ("fp16dev", 1), ("fp64", 1)])
@pytest.mark.parametrize("shape", [(64, 64), (16, 16, 16)])
def test_explicit_march_conserves_mass_and_momentum(M, orc, shape, storage, aa):
    """Periodic explicit march (Eq. collision conserves p-hat and j exactly;
    streaming permutes): over 20000 steps the totals of p-hat and of each
    momentum component stay within 5e-6 of their start, relative to the
    total momentum (the unbiased rounding of the stores walks randomly: FP32
    4e-8, FP16 deviation with FP32 moments 7e-7).  A collision whose equilibrium is built with rounded
    weights (sum w != 1, 3 sum w c^2 != 1 by ~1e-8) drifts by ~1e-8 per step
    of one sign, a few 1e-4 here."""
    d = len(shape)
    rng = np.random.default_rng(15)
    U = 1e-3
    p0 = 1e-2 * U * rng.normal(size=shape)
    u0 = np.stack([U * (1.0 + 0.5 * a) + 0.1 * U * rng.normal(size=shape) for a in range(d)])
    p = M.make_params(d, shape[0], dt=1.0, eps=1e-10, storage=storage, corrector="picard")
    for a in range(d):
        p.n[a] = shape[a]
    s = M.Solver(p, p0, u0)
    s.set_tuning(KEY_EXPLICIT_AA, aa)
    m0 = s.moments().reshape(d + 1, -1).sum(axis=1)
    s.explicit_step(20000)
    m1 = s.moments().reshape(d + 1, -1).sum(axis=1)
    s.close()
    scale = float(np.max(np.abs(m0[1:])))
    drift = float(np.max(np.abs(m1 - m0))) / scale
    say("conservation", shape, storage, "aa", aa, "drift", drift)
    assert drift <= 5e-6
