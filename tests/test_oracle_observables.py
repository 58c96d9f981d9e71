"""Pins of the correlation estimator (oracle.observables).

* Neel configuration: every <S^z_i S^z_j> = +-1/4 staggered, so the staggered
  structure factor is 3/4 exactly (1/4 from S^z S^z, times 3).
* All 2^n configurations with equal weight: spins are independent,
  <S^z_i S^z_j> = delta_ij / 4, so m_s^2(k) = 3 / (4 N) at every k.
* Counting against plain loops over random configurations.
* The factor 3: on the exact 4x4 Heisenberg ground state (a singlet) the
  operator expectation <S_a . S_b> from the sparse Hamiltonian blocks equals
  3 <S^z_a S^z_b> of the |psi|^2-weighted counts, for near and far pairs.
"""
import math

import numpy as np
import pytest

from oracle import ed, observables as ob


def test_neel_structure_factor():
    N, M = 6, 6
    S = np.array([[(i + j) % 2 for j in range(M)] for i in range(N)], dtype=np.uint8)[None]
    for (r0, c0, h, w) in [(1, 1, 4, 4), (2, 2, 2, 2), (0, 0, 6, 6)]:
        same, n = ob.same_counts(S, N, M, r0, c0, h, w)
        C = ob.szsz(same, n)
        assert ob.structure_factor(C, h, w, math.pi, math.pi, 3.0) == pytest.approx(0.75, abs=1e-15)
        assert ob.structure_factor(C, h, w, 0.0, 0.0, 3.0) == pytest.approx(0.0, abs=1e-15)


def test_uniform_ensemble():
    N, M = 3, 3
    n = N * M
    S = np.array([[(st >> k) & 1 for k in range(n)] for st in range(1 << n)], dtype=np.uint8)
    same, cnt = ob.same_counts(S, N, M, 0, 0, N, M)
    C = ob.szsz(same, cnt)
    assert np.array_equal(C, np.eye(n) / 4)
    for k in [(0.0, 0.0), (math.pi, math.pi), (0.7, -1.9)]:
        assert ob.structure_factor(C, N, M, *k, 3.0) == pytest.approx(3 / (4 * n), abs=1e-15)


def test_counts_against_loops():
    rng = np.random.default_rng(4)
    N, M = 5, 6
    S = rng.integers(0, 2, size=(40, N, M)).astype(np.uint8)
    keep = rng.random(40) > 0.3
    r0, c0, h, w = 1, 2, 3, 4
    same, n = ob.same_counts(S, N, M, r0, c0, h, w, keep=keep)
    ref = np.zeros((h * w, h * w), dtype=np.int64)
    cells = [(r0 + a, c0 + b) for a in range(h) for b in range(w)]
    for b in range(40):
        if not keep[b]:
            continue
        for p, (i1, j1) in enumerate(cells):
            for q, (i2, j2) in enumerate(cells):
                ref[p, q] += int(S[b, i1, j1] == S[b, i2, j2])
    assert n == keep.sum()
    assert np.array_equal(same, ref)


def test_singlet_factor_three():
    N, M = 4, 4
    e0, vec, states = ed.ground_state(N, M, 1.0, 0.0)
    cfg = np.array([ed.config_of_state(int(st), N, M) for st in states], dtype=np.uint8)
    same, n = ob.same_counts(cfg, N, M, 0, 0, N, M, weights=vec * vec)
    C = ob.szsz(same, n)
    for a, b in [(0, 1), (0, 5), (0, 15), (5, 10), (3, 12)]:
        op = ed._bond_operator(states, [(a, b)])
        ss = float(vec @ (op @ vec))
        assert ss == pytest.approx(3 * C[a, b], abs=1e-9)
