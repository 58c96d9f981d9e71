"""Pins of the transverse correlation oracle (oracle/correlations.py).

  * exact regime (nothing truncated): every exchange ratio, at any distance,
    equals W(S^{pq})/W(S) with both W by brute-force contraction;
  * exact enumeration: averaging S^z S^z + O_pq over every S^z = 0
    configuration with weight W^2 gives <psi|S_p . S_q|psi>/<psi|psi> from the
    spin operators applied to the brute-force state vector;
  * under truncation: on row-decoupled PEPS the ratios have a closed form
    (products of 1-D matrix chains), for every Dc; neighbours in a row give
    the horizontal exchange ratios of the local energy; R_pq(S) R_pq(S^{pq}) = 1
    (each ratio's numerator is the other's denominator: both are the same
    truncated contraction of one configuration); the error against the
    untruncated ratios shrinks as Dc grows.
"""
import math

import numpy as np
import pytest

from oracle import brute, correlations, observables
from oracle import peps as op
from paper_1611_09467_amd import workloads as wl


def _swap(S, p, q):
    X = S.copy().reshape(-1)
    X[p], X[q] = X[q], X[p]
    return X


@pytest.mark.parametrize("N,M,D,window", [(3, 3, 2, (0, 0, 3, 3)), (4, 3, 2, (0, 0, 4, 3)),
                                          (3, 4, 2, (1, 1, 2, 3))])
def test_exact_regime_ratios_are_brute_force_ratios(N, M, D, window):
    T = wl.make_peps(N, M, D, seed=71, bias=0.1)
    Dc = D ** ((M + 1) // 2 + 1)
    sites = correlations.window_sites(N, M, window)
    checked = 0
    for S in wl.random_sz0_configs(N, M, 3, 72):
        R, tie, fl = correlations.ratio_matrix(T, S, Dc, window)
        assert fl == 0 and not tie.any()
        w0 = brute.amplitude(T, S.reshape(N, M))
        for x, p in enumerate(sites):
            assert math.isnan(R[x, x])
            for y, q in enumerate(sites):
                if x == y:
                    continue
                if S[p] == S[q]:
                    assert math.isnan(R[x, y])
                    continue
                want = brute.amplitude(T, _swap(S, p, q).reshape(N, M)) / w0
                assert R[x, y] == pytest.approx(want, rel=1e-10, abs=1e-12), (p, q)
                checked += 1
    assert checked > 20


def _operator_expectation(vec, n, p, q):
    """<S_p . S_q> on a state vector (bit k of the index = label of site k)."""
    idx = np.arange(vec.size)
    bp, bq = (idx >> p) & 1, (idx >> q) & 1
    zz = np.where(bp == bq, 0.25, -0.25)
    norm = float(vec @ vec)
    if p == q:
        return 0.75
    diff = bp != bq
    flipped = idx ^ ((1 << p) | (1 << q))
    off = 0.5 * float(np.sum(vec[diff] * vec[flipped[diff]]))
    return (float(np.sum(zz * vec * vec)) + off) / norm


def test_enumeration_equals_spin_operator_expectation():
    N, M, D = 3, 4, 2
    T = wl.make_peps(N, M, D, seed=73)
    Dc = 16
    n = N * M
    vec = brute.state_vector(T, N, M)
    idx = np.arange(vec.size)
    pop = np.array([bin(k).count("1") for k in idx])
    vec0 = np.where(pop == n // 2, vec, 0.0)            # the S^z = 0 sector
    configs = [np.array([(k >> s) & 1 for s in range(n)], dtype=np.uint8)
               for k in idx[pop == n // 2]]
    w2 = np.array([vec0[k] ** 2 for k in idx[pop == n // 2]])
    window = (0, 0, N, M)
    same, wsum = observables.same_counts(configs, N, M, *window, weights=w2)
    ratios = [correlations.ratio_matrix(T, S, Dc, window) for S in configs]
    trans = np.zeros((n, n))
    for (R, _, fl), wt in zip(ratios, w2):
        assert fl == 0
        trans += wt * np.where(np.isnan(R), 0.0, 0.5 * R)
    trans[np.arange(n), np.arange(n)] += 0.5 * w2.sum()
    C = correlations.spin_correlations(same, wsum, trans, w2.sum())
    for p in range(n):
        for q in range(n):
            assert C[p, q] == pytest.approx(_operator_expectation(vec0, n, p, q), abs=1e-12)
    # the diagonal-only shortcut is not the answer for this state
    zz3 = 3 * observables.szsz(same, wsum)
    assert np.abs(zz3 - C).max() > 1e-2


def _row_weight(T, i, row_spins):
    v = np.ones((1,))
    for j, s in enumerate(row_spins):
        v = v @ T[i][j][s][:, :, 0, 0]
    return v.item()


@pytest.mark.parametrize("Dc", [1, 3, 8])
def test_row_decoupled_closed_form(Dc):
    N, M, D = 6, 5, 3
    T = wl.row_decoupled_peps(N, M, D, seed=74)
    window = (1, 1, 4, 3)
    sites = correlations.window_sites(N, M, window)
    for S in wl.random_sz0_configs(N, M, 2, 75):
        R, tie, fl = correlations.ratio_matrix(T, S, Dc, window)
        assert fl & ~op.FLAG_NEAR_TIE == 0
        G = S.reshape(N, M)
        for x, p in enumerate(sites):
            for y, q in enumerate(sites):
                if x == y or S[p] == S[q]:
                    continue
                X = _swap(S, p, q).reshape(N, M)
                a, b = p // M, q // M
                want = 1.0
                for i in {a, b}:
                    want *= _row_weight(T, i, X[i]) / _row_weight(T, i, G[i])
                assert R[x, y] == pytest.approx(want, rel=1e-10), (p, q)


def test_row_neighbours_equal_local_energy_ratios_under_truncation():
    N, M, D, Dc = 5, 5, 3, 4
    T = wl.make_peps(N, M, D, seed=76, bias=0.1)
    window = (0, 0, N, M)
    for S in wl.random_sz0_configs(N, M, 2, 77):
        R, _, fl = correlations.ratio_matrix(T, S, Dc, window)
        ev = op.evaluate(T, S, Dc, 1.0, 0.0, want_grad=False)
        for i in range(N):
            for j in range(M - 1):
                p, q = i * M + j, i * M + j + 1
                if S[p] == S[q]:
                    continue
                want = ev["ratios"][("h", (i, j), (i, j + 1))]
                assert R[p, q] == pytest.approx(want, rel=1e-12)


def test_reciprocity_under_truncation():
    N, M, D, Dc = 6, 5, 3, 3
    T = wl.make_peps(N, M, D, seed=82, bias=0.1)
    window = (1, 0, 4, 4)
    sites = correlations.window_sites(N, M, window)
    S = wl.random_sz0_configs(N, M, 1, 83)[0]
    R, _, _ = correlations.ratio_matrix(T, S, Dc, window)
    checked = 0
    for x, p in enumerate(sites):
        for y, q in enumerate(sites):
            if y <= x or S[p] == S[q] or p // M == q // M:
                continue
            Rb, _, _ = correlations.ratio_matrix(T, _swap(S, p, q), Dc, window)
            assert R[x, y] * Rb[x, y] == pytest.approx(1.0, rel=1e-10), (p, q)
            checked += 1
            if checked >= 12:
                return
    assert checked >= 12


def test_truncation_error_shrinks_with_dc():
    N, M, D = 6, 5, 2
    T = wl.make_peps(N, M, D, seed=78, bias=0.2)
    window = (1, 1, 4, 3)
    S = wl.random_sz0_configs(N, M, 1, 79)[0]
    exact, _, _ = correlations.ratio_matrix(T, S, D ** 3, window)
    errs = []
    for Dc in (1, 2, 4):
        R, _, _ = correlations.ratio_matrix(T, S, Dc, window)
        m = ~np.isnan(exact)
        errs.append(float(np.max(np.abs(R[m] - exact[m]) / np.maximum(1.0, np.abs(exact[m])))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-2 * errs[0]


def test_transverse_sums_skip_flagged_samples_and_count_the_diagonal():
    N, M, D, Dc = 4, 4, 2, 4
    T = wl.make_peps(N, M, D, seed=80)
    window = (1, 1, 2, 2)
    configs = list(wl.random_sz0_configs(N, M, 3, 81))
    tot, n = correlations.transverse_sums(T, configs, Dc, window)
    assert n == 3
    assert np.allclose(np.diag(tot), 1.5)
    assert np.allclose(tot, tot.T)
    # Neel product PEPS: W = 0 for every configuration but the Neel one
    Tn = wl.neel_product_peps(N, M)
    neel = wl.neel_config(N, M)
    other = _swap(neel, 0, 1)                    # W(other) = 0: flagged, left out
    tot2, n2 = correlations.transverse_sums(Tn, [neel, other], Dc, window)
    assert n2 == 1
    off = tot2 - np.diag(np.diag(tot2))
    assert np.all(off == 0.0)                   # every exchange leaves the Neel state
