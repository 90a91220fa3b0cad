"""GPU parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (the library's automatic tile, strip and
transform shapes, the dual-time march through msc_bdf2_step): the FP64
oracle marches the same seeded inputs with the same parameters and its inner
counts are replayed on the GPU.

* D2Q9 N = 256, FP32 storage, dt = 256, eps = 1e-8, linear trial (the
  benchmark's headline configuration);
* D2Q9 N = 1024, FP32 and FP16-deviation storage, dt = 9830.4, eps = 1e-8;
* D3Q19 N = 128, FP32 storage, dt = 63.83, eps = 1e-8, n_min = 2.

Bar: RMS velocity error relative to the FP64 oracle, and the replayed counts
are reached.  For FP32 (and FP16-deviation, whose moments are FP32) storage
the error is set by FP32 rounding of the populations and of the sweep's
arithmetic, amplified by the dual-time system: a rounding perturbation of a
sweep output moves the inner fixed point by about dt times as much (the slow
hydrodynamic modes of I - T have eigenvalues near a = 3/(2 dt)), and the S
steps add it up like a random walk.  Measured: 0.5 eps32 dt sqrt(S) (eps32 =
2^-24) at dt = 64 and 256, N = 128 and 256; so the bar here is
max(1e-5, 2 eps32 dt sqrt(S)): 1e-5 (the FP32 bar of the other parity tests)
up to dt ~ 100, growing linearly beyond.
"""
import math
import sys

import numpy as np
import pytest

from paper_2609_39474_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    from paper_2609_39474_amd import msc
    msc.lib()
    return msc


def _vel_err(m, ref):
    return math.sqrt(((m[1:] - ref[1:]) ** 2).sum(0).mean()) / math.sqrt((ref[1:] ** 2).sum(0).mean())


def _replay(M, orc, name, storage, nsteps, extrap):
    cfg = W.config(name)
    d, N = cfg["d"], cfg["N"]
    p0, u0 = W.initial_fields(cfg)
    say(f"{name} {storage}: oracle march of {nsteps} steps at N = {N}")
    ref = orc.march(p0, u0, dt=cfg["dt"], nsteps=nsteps, eps=cfg["eps"], nmin=cfg["nmin"], extrap_states=extrap)
    assert ref.status == 0
    K = [st["iters"] for st in ref.stats]
    p = M.make_params(d, N, dt=cfg["dt"], eps=cfg["eps"], storage=storage, corrector="shadow", n_min=cfg["nmin"],
                      extrap_states=extrap)
    s = M.Solver(p, p0, u0)
    s.set_schedule(K)
    rc, stats = s.bdf2_step(nsteps)
    assert rc == 0 and [x["iters"] for x in stats] == K
    err = _vel_err(s.moments(), ref.m)
    bar = max(1e-5, 2.0 * 2.0 ** -24 * cfg["dt"] * math.sqrt(nsteps))
    say(f"  counts {K}, RMS velocity error relative to the oracle {err:.3e}, bar {bar:.3e}")
    s.close()
    return err, bar


def test_headline_config_n256_fp32(M, orc):
    err, bar = _replay(M, orc, "rand2d_n256_fp32", "fp32", 8, 2)
    assert err <= bar


@pytest.mark.parametrize("storage", ["fp32", "fp16dev"])
def test_n1024(M, orc, storage):
    err, bar = _replay(M, orc, "rand2d_n1024_fp32", storage, 3, 2)
    assert err <= bar


def test_d3q19_n128_fp32(M, orc):
    err, bar = _replay(M, orc, "tgv3d_n128_fp32", "fp32", 2, 2)
    assert err <= bar
