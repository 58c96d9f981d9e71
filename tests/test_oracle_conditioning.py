"""Pins of the oracle's rounding-sensitivity estimate (oracle/conditioning.py).

The estimate is pinned against what it claims to measure, not against itself:
  * brute force: on a tiny truncating lattice every entry of every
    intermediate is perturbed on its own (central differences); the exact
    root-mean-square of the estimator's random directional derivative follows
    from those derivatives, and the estimate must lie within a small factor
    of it (for the evaluation's outputs and for the exchange ratios of the
    transverse correlations);
  * two backward-stable LAPACK SVD drivers (gesdd, gesvd) applied to the same
    sample must agree within twice the per-evaluation bound;
  * an evaluation with a planted relative error of 1e-7 in one block must
    fall outside the bound (the bound does not hide real mistakes).
"""
import numpy as np
import pytest

from oracle import conditioning as cond
from oracle import peps
from paper_1611_09467_amd import workloads as wl


class _Record:
    def __init__(self):
        self.sizes = []

    def __call__(self, X):
        self.sizes.append(X.size)
        return X


class _OneEntry:
    """Perturb entry e of the k-th intermediate by h ||X||_F, leave the rest."""

    def __init__(self, k, e, h):
        self.k, self.e, self.h, self.i = k, e, h, 0

    def __call__(self, X):
        if self.i == self.k:
            X = X.copy()
            X.flat[self.e] += self.h * np.linalg.norm(X)
        self.i += 1
        return X


def test_estimate_matches_brute_force_derivatives():
    # 3x4 D=2 Dc=2 truncates the middle blocks (4 x 4 cut to 2)
    N, M, D, Dc = 3, 4, 2, 2
    T = wl.make_peps(N, M, D, seed=11)
    S = wl.chain_configs(N, M, 1, 1, 12)[0]
    rec = _Record()
    base = peps.evaluate(T, S, Dc, 1.0, 0.5, perturb=rec)
    assert base["flags"] == 0 and len(rec.sizes) > 20
    h = 1e-7
    var = np.zeros(2)
    for k, m in enumerate(rec.sizes):
        g2 = np.zeros(2)
        for e in range(m):
            a = peps.evaluate(T, S, Dc, 1.0, 0.5, want_grad=False, perturb=_OneEntry(k, e, h))
            b = peps.evaluate(T, S, Dc, 1.0, 0.5, want_grad=False, perturb=_OneEntry(k, e, -h))
            gp = (a["logabs"] - b["logabs"]) / (2 * h)
            ge = (a["eloc"] - b["eloc"]) / (2 * h) / max(1.0, abs(base["eloc"]))
            g2 += np.array([gp * gp, ge * ge])
        # a uniformly random unit direction in R^m sees |g|^2 / m on average
        var += g2 / m
    rms = np.sqrt(var)
    _, kap = cond.kappa(T, S, Dc, 1.0, 0.5)
    ratio = kap[:2] / rms
    assert np.all(ratio > 0.3) and np.all(ratio < 4.0), (kap, rms)


@pytest.mark.parametrize("b", [0, 1200, 2496, 3248])
def test_lapack_drivers_agree_within_bound(b):
    T, S = wl.workload_inputs("8x8_D4_Dc8")
    D, Dc = 4, 8
    base, kap = cond.kappa(T, S[b], Dc, 1.0, 0.5)
    other = peps.evaluate(T, S[b], Dc, 1.0, 0.5, svd_driver="gesvd")
    d = cond.differences(other, base)
    assert np.all(d <= 2 * cond.bound(kap, D, Dc)), (d, cond.bound(kap, D, Dc))


def test_planted_error_exceeds_bound():
    T, S = wl.workload_inputs("8x8_D4_Dc8")
    D, Dc = 4, 8
    base, kap = cond.kappa(T, S[7], Dc, 1.0, 0.5)
    # a relative error of 1e-7 in one entry of the 5th truncated block
    planted = peps.evaluate(T, S[7], Dc, 1.0, 0.5, perturb=_OneEntry(4, 3, 1e-7))
    d = cond.differences(planted, base)
    assert d[0] > cond.bound(kap, D, Dc)[0], (d, cond.bound(kap, D, Dc))


def test_ratio_estimate_matches_brute_force_derivatives():
    # the same check for the exchange ratios of the transverse correlations:
    # a column window of a truncating 3x4 lattice, pairs across rows
    from oracle import correlations
    N, M, D, Dc = 3, 4, 2, 2
    T = wl.make_peps(N, M, D, seed=13)
    window = (0, 1, 3, 1)
    S = np.array([0, 1, 0, 1, 1, 0, 1, 0, 0, 1, 0, 1], dtype=np.uint8)
    rec = _Record()
    R0, _, fl = correlations.ratio_matrix(T, S, Dc, window, perturb=rec)
    assert fl == 0 and len(rec.sizes) > 10
    mask = ~np.isnan(R0)
    assert mask.sum() >= 2
    h = 1e-7
    var = np.zeros_like(R0)
    for k, m in enumerate(rec.sizes):
        g2 = np.zeros_like(R0)
        for e in range(m):
            a, _, _ = correlations.ratio_matrix(T, S, Dc, window, perturb=_OneEntry(k, e, h))
            b, _, _ = correlations.ratio_matrix(T, S, Dc, window, perturb=_OneEntry(k, e, -h))
            g = np.where(mask, (a - b) / (2 * h) / np.maximum(1.0, np.abs(R0)), 0.0)
            g2 += g * g
        var += g2 / m
    rms = np.sqrt(var[mask])
    _, kap = cond.kappa_ratios(T, S, Dc, window)
    ratio = kap[mask] / rms
    assert np.all(ratio > 0.3) and np.all(ratio < 4.0), (kap[mask], rms)
