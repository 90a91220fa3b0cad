"""Bars shared by the GPU parity tests.

Fields are compared one at a time (the populations; the pressure-like moment
and each velocity component), each by max |a - b| / max |b|.  The FP64 bar is
1e-12, or ten times the oracle's own sensitivity to a one-ulp perturbation of
its input where that is larger: the pressure-like moment is O(U^2) but is
summed from O(U) populations, so rounding in a different order moves it by
about eps64 U / |p| relative per operation, and a march carries that forward;
the oracle run twice from inputs one ulp apart shows how far any FP64
implementation can land from it.
"""
import numpy as np


def rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def field_rels(a, b, nf=None):
    """rel() of each field along the leading axis, or of nf equal parts of a
    flat array."""
    a = np.asarray(a)
    b = np.asarray(b)
    if nf is not None:
        a = a.reshape(nf, -1)
        b = b.reshape(nf, -1)
    return [rel(a[i], b[i]) for i in range(b.shape[0])]


def ulp_perturbed(x, seed=0):
    """x with every entry moved by about one unit in the last place."""
    x = np.asarray(x, dtype=np.float64)
    return x * (1.0 + 1e-16 * np.random.default_rng(seed).normal(size=x.shape))


def sensitivity_bars(sens, floor=1e-12, factor=10.0):
    return [max(floor, factor * s) for s in sens]


def check_fields(errs, bars, what=""):
    bad = [(i, e, b) for i, (e, b) in enumerate(zip(errs, bars)) if not e <= b]
    assert not bad, f"{what}: field, error, bar: {bad}"
