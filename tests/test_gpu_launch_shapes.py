"""GPU parity of the launch-shape variants (through the C ABI, FP64 storage,
against the FP64 oracle at 1e-12 per field, or ten times the oracle's own
one-ulp sensitivity of the field where that is larger): the row transforms of the correction fused
into the sweep (forward only, or forward and inverse) or run as their own
passes, sweep tiles and strip lengths other than the automatic choice, the
folded-partials path of large sweep grids, every D3Q19 tile of the library's
table, the 512-thread tile of the D3Q19 dual-time sweeps at N_z = 128, and
the pencils and columns per block of the 3D transform passes.  Results must not depend on these choices beyond rounding
order; the two fused variants run the same arithmetic and agree bit for bit.
"""
import sys

import numpy as np
import pytest

from paper_2609_39474_amd import workloads as W

import parity_bars as PB

pytestmark = pytest.mark.gpu

NU = 1.0 / 6.0
KEY_TILE, KEY_STRIP, KEY_TILE_INDEX, KEY_FUSE_ROWS = 0, 1, 5, 6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def rel_fields(a, b):
    """rel() of each moment field (p-hat, u_x, u_y[, u_z]) at its own scale."""
    return max(rel(np.asarray(a)[i], np.asarray(b)[i]) for i in range(np.asarray(b).shape[0]))


def check_vs_oracle(m, ref_m, alt_m, what):
    """Every moment field within max(1e-12, 10x the oracle's one-ulp
    sensitivity of that field) of the oracle."""
    errs = PB.field_rels(m, ref_m)
    say(what, "per-field rel", errs)
    PB.check_fields(errs, PB.sensitivity_bars(PB.field_rels(alt_m, ref_m)), what)


@pytest.fixture(scope="module")
def M():
    from paper_2609_39474_amd import msc
    msc.lib()
    return msc


def _solver(M, shape, p0, u0, *, dt, eps=1e-10, n_min=2):
    d = len(shape)
    p = M.make_params(d, shape[0], dt=dt, eps=eps, n_min=n_min)
    for a in range(d):
        p.n[a] = shape[a]
    return M.Solver(p, p0, u0)


@pytest.mark.parametrize("fuse", [0, 1, 2])
def test_fused_row_transform_on_off(M, orc, fuse):
    """2D TGV N = 64: twelve steps at the oracle's inner counts."""
    cfg = W.config("tgv2d_n64_fp64")
    N = cfg["N"]
    p0, u0 = W.initial_fields(cfg)
    ref = orc.march(p0, u0, dt=cfg["dt"], nsteps=12, eps=cfg["eps"], nmin=2)
    K = [st["iters"] for st in ref.stats]
    alt = orc.march(p0, PB.ulp_perturbed(u0), dt=cfg["dt"], nsteps=12, eps=cfg["eps"], nmin=2, schedule=K)
    s = _solver(M, (N, N), p0, u0, dt=cfg["dt"], eps=cfg["eps"])
    s.set_tuning(KEY_FUSE_ROWS, fuse)
    s.set_schedule(K)
    rc, stats = s.bdf2_step(12)
    assert rc == 0 and [x["iters"] for x in stats] == K
    check_vs_oracle(s.moments(), ref.m, alt.m, f"fuse_rows {fuse}")
    s.close()


@pytest.mark.parametrize("storage", ["fp32", "fp16dev"])
def test_inverse_rows_in_sweep_bit_exact(M, storage):
    """The random-field workload at N = 256 (dt = 256, eps = 1e-8, six free
    running steps): inverse row transform inside the sweep (key 6 = 2) and as
    its own pass (key 6 = 1) give identical counts and identical moments."""
    N = 256
    p0, u0 = W.random_field_2d(N, NU / N, seed=1)
    out = {}
    for fuse in (1, 2):
        p = M.make_params(2, N, dt=256.0, eps=1e-8, storage=storage, extrap_states=2)
        s = M.Solver(p, p0, u0)
        s.set_tuning(KEY_FUSE_ROWS, fuse)
        rc, stats = s.bdf2_step(6)
        assert rc == 0
        out[fuse] = ([x["iters"] for x in stats], s.moments())
        s.close()
    say(storage, "inverse rows in the sweep: counts", out[2][0], "separate:", out[1][0])
    assert out[1][0] == out[2][0]
    assert np.array_equal(out[1][1], out[2][1])


SHAPES_2D = [
    # (tile sites, strip planes): the automatic shape (fused row transform,
    # one plane per strip); 4-site tiles with one-plane strips (16384 sweep
    # blocks: the partials are folded by a separate kernel first); 64-site
    # tiles (row transform as its own pass); whole rows with four-plane
    # strips (fused, four row transforms per block)
    (0, 0), (4, 1), (64, 2), (256, 4),
]


@pytest.fixture(scope="module")
def ref256(orc):
    N = 256
    p0, u0 = W.random_field_2d(N, NU / N, seed=3)
    ref = orc.march(p0, u0, dt=256.0, nsteps=3, eps=1e-10, nmin=2, extrap_states=2)
    K = [st["iters"] for st in ref.stats]
    alt = orc.march(p0, PB.ulp_perturbed(u0), dt=256.0, nsteps=3, eps=1e-10, nmin=2, extrap_states=2, schedule=K)
    return p0, u0, ref, alt


@pytest.mark.parametrize("tile,strip", SHAPES_2D)
def test_march_launch_shapes_2d(M, ref256, tile, strip):
    p0, u0, ref, alt = ref256
    K = [st["iters"] for st in ref.stats]
    p = M.make_params(2, 256, dt=256.0, eps=1e-10, extrap_states=2)
    s = M.Solver(p, p0, u0)
    s.set_tuning(KEY_TILE, tile)
    s.set_tuning(KEY_STRIP, strip)
    s.set_schedule(K)
    rc, stats = s.bdf2_step(3)
    assert rc == 0 and [x["iters"] for x in stats] == K
    for a, b in zip(stats, ref.stats):
        assert abs(a["R_final"] - b["R_final"]) <= 1e-9 * b["R_final"]
    check_vs_oracle(s.moments(), ref.m, alt.m, f"2D tile {tile} strip {strip}")
    s.close()


@pytest.mark.parametrize("idx", [1, 2, 3, 4, 5, 6, 7])
def test_d3q19_tiles(M, orc, idx):
    """Every D3Q19 tile of the table on a grid they all fit (8 x 16 x 256):
    one corrected iteration and one BDF step at the oracle's count."""
    shape = (8, 16, 256)
    rng = np.random.default_rng(idx)
    c, w, _ = orc.lattice(3)
    wq = w.reshape((19, 1, 1, 1))
    f = wq * (1e-3 * rng.normal(size=(19,) + shape)) + wq * 0.01 * rng.normal(size=shape)
    h = 1e-4 * rng.normal(size=(4,) + shape)
    a = 3.0 / 128.0
    p0 = np.zeros(shape)
    u0 = np.zeros((3,) + shape)
    s = _solver(M, shape, p0, u0, dt=16.0, n_min=1)
    s.set_tuning(KEY_TILE_INDEX, idx)
    fn, dm, R = s.correct(f, h, a)
    ofn, _, _, odm, oR = orc.corrected_iteration(f, h, a, 1.0, 1.0, NU)
    assert rel_fields(dm, odm) <= 1e-12 and rel(fn, ofn) <= 1e-12 and abs(R - oR) <= 1e-12 * oR
    # one BDF step from a smooth state
    u1 = W.random_perturbation_3d(8, 1e-3, seed=idx, jmax=2)
    u1 = np.tile(u1, (1, 1, 2, 32))
    st0 = orc.initial_state(p0, u1)
    rc, st1, bc1, ost = orc.march_state(st0, 0, shape, dt=16.0, nsteps=1, eps=1e-10, nmin=1)
    s.set_state(st0, 0)
    s.set_schedule([ost[0]["iters"]])
    rc, gst = s.bdf2_step(1)
    assert rc == 0 and gst[0]["iters"] == ost[0]["iters"]
    g, _ = s.get_state()
    say("3D tile index", idx, "correct", rel(fn, ofn), "step", rel(g, st1))
    assert rel(g, st1) <= 1e-12
    s.close()


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_wide_dual_tile(M, orc, storage):
    """D3Q19 at N_z = 128: the sweeps after the first of a step on 4 x 128
    tiles of 512 threads (key 11 = 1, the default) and on the 2 x 128 tiles
    (key 11 = 0) give the same counts and bit-identical states over three
    steps (the per-site arithmetic is the same; only the halo rows each block
    re-collides differ); with FP64 storage one corrected iteration on the wide
    tile matches the oracle at 1e-12."""
    shape = (16, 8, 128)
    u1 = np.tile(W.random_perturbation_3d(8, 1e-3, seed=5, jmax=2), (1, 2, 1, 16))
    p0 = np.zeros(shape)
    states, counts = {}, {}
    for wide in (0, 1):
        p = M.make_params(3, shape[0], dt=32.0, eps=1e-10, storage=storage, n_min=2, extrap_states=2)
        for a in range(3):
            p.n[a] = shape[a]
        s = M.Solver(p, p0, u1)
        s.set_tuning(11, wide)
        if wide == 1:
            s.set_schedule(counts[0])
        rc, st = s.bdf2_step(3)
        assert rc == 0
        counts[wide] = [x["iters"] for x in st]
        states[wide], _ = s.get_state()
        if wide == 1 and storage == "fp64":
            rng = np.random.default_rng(7)
            c, w, _ = orc.lattice(3)
            wq = w.reshape((19, 1, 1, 1))
            f = wq * (1e-3 * rng.normal(size=(19,) + shape)) + wq * 0.01 * rng.normal(size=shape)
            h = 1e-4 * rng.normal(size=(4,) + shape)
            fn, dm, R = s.correct(f, h, 3.0 / 64.0)
            ofn, _, _, odm, oR = orc.corrected_iteration(f, h, 3.0 / 64.0, 1.0, 1.0, NU)
            say("wide tile correct: rel f", rel(fn, ofn), "dm", rel_fields(dm, odm))
            assert rel_fields(dm, odm) <= 1e-12 and rel(fn, ofn) <= 1e-12 and abs(R - oR) <= 1e-12 * oR
        s.close()
    say(storage, "wide dual tile: counts", counts[1], "2 x 128:", counts[0])
    assert counts[0] == counts[1]
    assert np.array_equal(states[0], states[1])


KEY_FFT3_PENCILS, KEY_FFT3_COLS = 7, 8


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_transform_shapes_3d(M, orc, storage):
    """The 3D correction's launch shapes: z pencils per block (key 7; the
    forward z pass loops over pencil groups on a grid of resident blocks) and
    j_z columns per block of the y and x passes (key 8, widths that divide the
    9 band columns of N_z = 32 unevenly and evenly) leave the corrected
    iteration bit-identical; with FP64 storage the automatic shape matches the
    oracle at 1e-12 per field."""
    shape = (16, 32, 32)
    rng = np.random.default_rng(21)
    c, w, _ = orc.lattice(3)
    wq = w.reshape((19, 1, 1, 1))
    f = wq * (1e-3 * rng.normal(size=(19,) + shape)) + wq * 0.01 * rng.normal(size=shape)
    h = 1e-4 * rng.normal(size=(4,) + shape)
    a = 3.0 / 64.0
    p = M.make_params(3, shape[0], dt=32.0, eps=1e-10, storage=storage, n_min=2)
    for ax in range(3):
        p.n[ax] = shape[ax]
    s = M.Solver(p, np.zeros(shape), np.zeros((3,) + shape))
    ref = None
    for pencils, cols in [(0, 0), (1, 1), (2, 3), (4, 4), (4, 8), (1, 5), (2, 2)]:
        s.set_tuning(KEY_FFT3_PENCILS, pencils)
        s.set_tuning(KEY_FFT3_COLS, cols)
        fn, dm, R = s.correct(f, h, a)
        say(storage, "3D transform shape: pencils", pencils, "cols", cols, "R", R)
        if ref is None:
            ref = (fn, dm, R)
            if storage == "fp64":
                ofn, _, _, odm, oR = orc.corrected_iteration(f, h, a, 1.0, 1.0, NU)
                say("  vs oracle: rel f", rel(fn, ofn), "dm", rel_fields(dm, odm))
                assert rel_fields(dm, odm) <= 1e-12 and rel(fn, ofn) <= 1e-12 and abs(R - oR) <= 1e-12 * oR
        else:
            assert np.array_equal(fn, ref[0]) and np.array_equal(dm, ref[1]) and R == ref[2]
    s.close()


@pytest.mark.parametrize("shape,storage", [((4, 4, 128), "fp64"), ((4, 4, 128), "fp32"), ((4, 8, 128), "fp64")])
def test_small_y_extent_at_nz128(M, orc, shape, storage):
    """D3Q19 at N_z = 128 with the smallest y extents: N_y = 4, where the 4 x
    128 tile of the dual-time sweeps after the first spans y as well (no halo
    rows, streaming wraps inside the tile) and the first sweep's two 2 x 128
    tiles take their halo rows from each other, and N_y = 8.  Four corrected
    BDF steps against the oracle's march with the same inner counts.  FP64:
    the final populations and moments per field within 1e-12 or ten times the
    oracle's own one-ulp sensitivity; FP32: the RMS error of each velocity
    component within 1e-5 of that component's RMS."""
    # every component dominated by slow modes along z (|k| = 2 pi/128, 4 pi/128)
    # with smaller parts along x and y: on 4-site extents those sit at |k| =
    # pi/2, decay by ~e^-52 over the four steps and would leave a relative
    # error measured against a vanished field
    x, y, z = np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")
    tp = 2.0 * np.pi
    u1 = 1e-3 * np.stack([np.sin(tp * z) + 0.2 * np.cos(tp * x) * np.sin(tp * z),
                          0.5 * np.cos(tp * z) + 0.2 * np.sin(tp * y),
                          0.3 * np.sin(2 * tp * z) + 0.2 * np.sin(tp * x)])
    p0 = np.zeros(shape)
    p = M.make_params(3, shape[0], dt=32.0, eps=1e-10 if storage == "fp64" else 1e-8, storage=storage,
                      n_min=2, extrap_states=2)
    for a in range(3):
        p.n[a] = shape[a]
    st0 = orc.initial_state(p0, u1)
    kw = dict(dt=32.0, nsteps=4, eps=1e-10, nmin=2, extrap_states=2)
    rc, ref, _, ost = orc.march_state(st0, 0, shape, **kw)
    assert rc == 0
    K = [x["iters"] for x in ost]
    s = M.Solver(p, p0, u1)
    s.set_schedule(K)
    rc, st = s.bdf2_step(4)
    assert rc == 0 and [x["iters"] for x in st] == K
    state, _ = s.get_state()
    s.close()
    NS = int(np.prod(shape))
    FQ, FM = 19 * NS, 4 * NS
    say(storage, shape, "small y extent at N_z = 128: counts", K)
    if storage == "fp64":
        _, alt, _, _ = orc.march_state(PB.ulp_perturbed(st0, 0), 0, shape, schedule=K, **kw)
        for lo, hi, nf, what in ((0, FQ, 1, "f^n"), (3 * FQ, 3 * FQ + FM, 4, "m^n")):
            errs = PB.field_rels(state[lo:hi], ref[lo:hi], nf)
            say("  vs oracle:", what, errs)
            PB.check_fields(errs, PB.sensitivity_bars(PB.field_rels(alt[lo:hi], ref[lo:hi], nf)), what)
    else:
        u = state[3 * FQ + NS:3 * FQ + FM].reshape(3, -1)
        uref = ref[3 * FQ + NS:3 * FQ + FM].reshape(3, -1)
        # RMS error of each velocity component relative to the reference
        # component's RMS (the FP32 precision bar's measure), worst component
        err = max(float(np.sqrt(np.mean((u[i] - uref[i]) ** 2) / np.mean(uref[i] ** 2))) for i in range(3))
        say("  fp32 velocity error", err, "max-norm", max(rel(u[i], uref[i]) for i in range(3)))
        assert err <= 1e-5


KEY_SKIP_PR = 12


@pytest.mark.parametrize("shape", [(16, 8, 128), (8, 8, 32)])
@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_last_lift_sweep_without_pr(M, orc, storage, shape):
    """3D: the lift sweep enqueued as the last of its step leaves P r out
    (key 12 = 1, the default); when the step goes on, P r is formed from that
    sweep's input, the correction it lifted and its output before the
    correction runs.  A free-running march (no replayed counts: the first step
    needs far more sweeps than predicted, so P r is formed several times)
    gives the same counts, the same residuals and bit-identical states as
    with P r always stored (key 12 = 0)."""
    reps = (1, shape[0] // 8, shape[1] // 8, shape[2] // 8)
    u1 = np.tile(W.random_perturbation_3d(8, 1e-3, seed=5, jmax=2), reps)
    p0 = np.zeros(shape)
    states, counts, stats = {}, {}, {}
    for skip in (0, 1):
        p = M.make_params(3, shape[0], dt=32.0, eps=1e-10, storage=storage, n_min=2, extrap_states=2)
        for a in range(3):
            p.n[a] = shape[a]
        s = M.Solver(p, p0, u1)
        s.set_tuning(KEY_SKIP_PR, skip)
        rc, st = s.bdf2_step(5)
        assert rc == 0
        counts[skip] = [x["iters"] for x in st]
        stats[skip] = st
        states[skip], _ = s.get_state()
        s.close()
    say(storage, shape, "last lift sweep without P r: counts", counts[1], "with P r:", counts[0])
    assert counts[0] == counts[1]
    assert counts[1][0] > 4 + 8  # the first step outran two predictions
    for a, b in zip(stats[0], stats[1]):
        assert a["R_final"] == b["R_final"] and a["R_first"] == b["R_first"]
    assert np.array_equal(states[0], states[1])


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_last_lift_sweep_without_pr_2d(M, orc, storage):
    """2D at N_y = 512, Re = 100 (the row transforms run as passes of their
    own; the forward row pass takes the decision): the last lift sweep enqueued for a
    step leaving P r out (key 12 = 1) and P r always stored (key 12 = 0) give
    the same counts, the same residuals and bit-identical states over a
    free-running march whose first step outruns its prediction."""
    N = 512
    # Re = 100: the first step needs 10 (FP32) to 17 (FP64) sweeps against a
    # prediction of 4
    p0, u0 = W.random_field_2d(N, 100.0 * NU / N, seed=3)
    states, counts, stats = {}, {}, {}
    for skip in (0, 1):
        p = M.make_params(2, N, dt=256.0, eps=1e-10 if storage == "fp64" else 1e-8, storage=storage, n_min=2,
                          extrap_states=2)
        s = M.Solver(p, p0, u0)
        s.set_tuning(KEY_SKIP_PR, skip)
        rc, st = s.bdf2_step(5)
        assert rc == 0
        counts[skip] = [x["iters"] for x in st]
        stats[skip] = st
        states[skip], _ = s.get_state()
        s.close()
    say(storage, "2D last lift sweep without P r: counts", counts[1], "with P r:", counts[0])
    assert counts[0] == counts[1]
    assert counts[1][0] > 4  # the first step outran its prediction
    for a, b in zip(stats[0], stats[1]):
        assert a["R_final"] == b["R_final"] and a["R_first"] == b["R_first"]
    assert np.array_equal(states[0], states[1])
