"""msc_sweep_noalloc (one sweep on caller-owned device buffers, no context
and no device allocation) against msc_sweep of a context: two calls in a row
per lattice and storage, the second on a smaller grid (the fixed partial-sum
array keeps the first call's contents).  f_T and P r bit-identical (same
kernel, tile and strip), R within rounding of the summation order."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NU = 1.0 / 6.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    from paper_2609_39474_amd import msc
    msc.lib()
    return msc


def _state(d, shape, seed):
    rng = np.random.default_rng(seed)
    Q = 9 if d == 2 else 19
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4) if d == 2 else \
        np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    f = w.reshape((Q,) + (1,) * d) * (1e-3 * rng.normal(size=(Q,) + shape) + 0.01 * rng.normal(size=shape))
    h = 1e-4 * rng.normal(size=(d + 1,) + shape)
    return f, h


CASES = [
    (2, "fp64", (128, 64), (32, 16)),
    (2, "fp32", (256, 256), (64, 32)),
    (3, "fp64", (16, 16, 32), (8, 8, 8)),
    (3, "fp32", (32, 32, 64), (8, 16, 8)),
    # N_z = 128: the wide dual-time tile (4 x 128 sites, 512 threads)
    (3, "fp64", (8, 8, 128), (4, 4, 16)),
    (3, "fp32", (16, 4, 128), (8, 8, 128)),
]


@pytest.mark.parametrize("d,storage,big,small", CASES)
def test_noalloc_matches_context_sweep(M, d, storage, big, small):
    import torch

    dev = torch.device("cuda:0")
    tdt = torch.float64 if storage == "fp64" else torch.float32
    stream = torch.cuda.current_stream().cuda_stream
    for call, shape in enumerate((big, small)):
        say(f"noalloc sweep: lattice d={d} {storage} shape {shape} call {call + 1}")
        f, h = _state(d, shape, seed=7 + call + sum(shape))
        a = 3.0 / 128.0 if call == 0 else 1.0 / 40.0
        p = M.make_params(d, shape[0], dt=64.0, eps=1e-10, storage=storage, corrector="picard")
        for i in range(d):
            p.n[i] = shape[i]
        s = M.Solver(p, np.zeros(shape), np.zeros((d,) + shape), stream=stream)
        fT_ref, Pr_ref, R_ref = s.sweep(f, h, a)
        s.close()
        Q = f.shape[0]
        fd = torch.tensor(f, dtype=tdt, device=dev).contiguous()
        hd = torch.tensor(h, dtype=torch.float64, device=dev).contiguous()
        fT = torch.empty_like(fd)
        Pr = torch.empty((d + 1,) + shape, dtype=tdt, device=dev)
        R = torch.empty(1, dtype=torch.float64, device=dev)
        M.sweep_noalloc(d, shape, storage, fd.data_ptr(), hd.data_ptr(), a, fT.data_ptr(), Pr.data_ptr(),
                        R.data_ptr(), stream)
        torch.cuda.synchronize()
        fT_h = fT.double().cpu().numpy().reshape((Q,) + shape)
        Pr_h = Pr.double().cpu().numpy()
        R_h = float(R.cpu()[0])
        say(f"  max |dfT| {np.max(np.abs(fT_h - fT_ref)):.3e}  max |dPr| {np.max(np.abs(Pr_h - Pr_ref)):.3e}  "
            f"R {R_h:.17e} vs {R_ref:.17e}")
        np.testing.assert_array_equal(fT_h, fT_ref)
        np.testing.assert_array_equal(Pr_h, Pr_ref)
        assert abs(R_h - R_ref) <= 1e-13 * R_ref


def test_noalloc_refusals(M):
    import torch

    say("noalloc refusals")
    x = torch.zeros(64, dtype=torch.float64, device="cuda:0")
    ptr = x.data_ptr()
    # FP16 deviation storage is not offered
    with pytest.raises(M.MscError) as e:
        M.sweep_noalloc(2, (8, 8), "fp16dev", ptr, ptr, 0.1, ptr, ptr)
    assert e.value.status == M.MSC_ERR_UNSUPPORTED
    # extents that are not powers of two, and a grid with more sweep blocks
    # than the fixed partial-sum array (rejected before any launch)
    for n in ((12, 8), (1 << 23, 4)):
        with pytest.raises(M.MscError) as e:
            M.sweep_noalloc(2, n, "fp64", ptr, ptr, 0.1, ptr, ptr)
        assert e.value.status == M.MSC_ERR_INVALID_ARG
    # h is required
    with pytest.raises(M.MscError) as e:
        M.sweep_noalloc(2, (8, 8), "fp64", ptr, None, 0.1, ptr, ptr)
    assert e.value.status == M.MSC_ERR_INVALID_ARG
