"""Exact diagonalisation against the exact energies printed in the paper's Table I,
and the local-energy assembly E(S) against the zero-variance property."""
import math
import os

import numpy as np
import pytest

from oracle import ed, hamiltonian

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_exact_energies.txt")


def table1():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        n, m, j2, e = line.split()
        out[(int(n), int(m), float(j2))] = float(e)
    return out


def test_ed_4x4_heisenberg_table1():
    E, _, _ = ed.ground_state(4, 4, 1.0, 0.0)
    assert E / 16 == pytest.approx(table1()[(4, 4, 0.0)], abs=6e-9)


@pytest.fixture(scope="module")
def blocks_4x6():
    return ed.hamiltonian_blocks(4, 6)


@pytest.mark.slow
def test_ed_4x6_j2_half_table1(blocks_4x6):
    # pins the next-nearest-neighbour (plaquette diagonal) convention and the J2 term
    E, _, _ = ed.ground_state(4, 6, 1.0, 0.5, blocks=blocks_4x6)
    assert E / 24 == pytest.approx(table1()[(4, 6, 0.5)], abs=6e-9)


@pytest.mark.slow
@pytest.mark.parametrize("J2", [0.0, 0.56])
def test_ed_4x6_other_rows_table1(blocks_4x6, J2):
    E, _, _ = ed.ground_state(4, 6, 1.0, J2, blocks=blocks_4x6)
    assert E / 24 == pytest.approx(table1()[(4, 6, J2)], abs=6e-9)


def test_ed_two_routes_agree_3x4():
    # ARPACK and dense LAPACK on the same sector (independent eigensolvers)
    a, _, _ = ed.ground_state(3, 4, 1.0, 0.5)
    b, _, _ = ed.ground_state(3, 4, 1.0, 0.5, method="dense")
    assert a == pytest.approx(b, abs=1e-10)


def test_bond_counts():
    for N, M in [(4, 4), (4, 6), (10, 10)]:
        kinds = [k for k, _, _ in hamiltonian.bonds(N, M)]
        assert sum(k in ("h", "v") for k in kinds) == 2 * N * M - N - M
        assert sum(k in ("d1", "d2") for k in kinds) == 2 * (N - 1) * (M - 1)


@pytest.mark.parametrize("J2", [0.0, 0.5])
def test_local_energy_zero_variance_4x4(J2):
    # with exact eigenvector amplitudes E(S) equals E0 for every S (Eq. (2) and the
    # definition of E(S)); pins the pair list, the 1/2 exchange element and Sz Sz
    N, M = 4, 4
    E0, vec, states = ed.ground_state(N, M, 1.0, J2)
    index = {int(s): k for k, s in enumerate(states)}
    rng = np.random.default_rng(0)
    picks = rng.choice(states.size, 40, replace=False)
    for p in picks:
        st = int(states[p])
        if abs(vec[p]) < 1e-6:
            continue
        S = ed.config_of_state(st, N, M)

        def ratio(kind, a, b):
            S2 = hamiltonian.swapped(S, a, b)
            st2 = sum(int(S2.ravel()[k]) << k for k in range(N * M))
            return vec[index[st2]] / vec[p]

        assert hamiltonian.local_energy(S, 1.0, J2, ratio) == pytest.approx(E0, abs=1e-7)
