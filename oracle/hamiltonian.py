"""J1-J2 Heisenberg model on an open N x M square lattice and the local energy E(S).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper, Sec. IV, Eq. (7): H = J1 sum_<ij> S_i.S_j + J2 sum_<<ij>> S_i.S_j over
nearest-neighbour and next-nearest-neighbour (plaquette diagonal) pairs, with
S_i.S_i = 3/4.  In the S^z basis, S_a.S_b = Sz_a Sz_b + (S+_a S-_b + S-_a S+_b)/2:
its diagonal element is +1/4 for parallel and -1/4 for antiparallel spins, and
it connects an antiparallel configuration to the one with the two spins
exchanged with element 1/2.

Sec. II (the equation after Eq. (2)): E(S) = sum_{S'} W(S')/W(S) <S'|H|S>.  With
H real symmetric, <S'|H|S> = <S|H|S'>.

Pins: the bond lists and the assembly are pinned by exact diagonalisation
against the energies printed in Table I (tests/test_oracle_ed.py) and by the
zero-variance property of E(S) fed with exact eigenvector amplitudes.
"""
from __future__ import annotations

import numpy as np


def sz(s: int) -> float:
    """S^z of a spin label: s = 0 -> +1/2, s = 1 -> -1/2."""
    return 0.5 - float(s)


def bonds(N: int, M: int):
    """All interacting pairs on the open lattice, as (kind, (i1, j1), (i2, j2)).

    kind is 'h' (horizontal nearest neighbour), 'v' (vertical nearest
    neighbour), 'd1' (diagonal (i,j)-(i+1,j+1)) or 'd2' (anti-diagonal
    (i,j+1)-(i+1,j)).  Counts: 2NM - N - M nearest-neighbour and 2(N-1)(M-1)
    next-nearest-neighbour pairs.
    """
    out = []
    for i in range(N):
        for j in range(M - 1):
            out.append(("h", (i, j), (i, j + 1)))
    for i in range(N - 1):
        for j in range(M):
            out.append(("v", (i, j), (i + 1, j)))
    for i in range(N - 1):
        for j in range(M - 1):
            out.append(("d1", (i, j), (i + 1, j + 1)))
            out.append(("d2", (i, j + 1), (i + 1, j)))
    return out


def coupling(kind: str, J1: float, J2: float) -> float:
    return J1 if kind in ("h", "v") else J2


def local_energy(S: np.ndarray, J1: float, J2: float, ratio) -> float:
    """E(S) = sum_pairs J [Sz_a Sz_b + (1/2) [s_a != s_b] R_ab].

    ``S`` is an (N, M) integer array.  ``ratio(kind, a, b)`` returns
    R_ab = W(S_ab)/W(S) for the configuration S_ab with the (antiparallel) spins
    at sites a and b exchanged; it is called only for antiparallel pairs.
    """
    N, M = S.shape
    e = 0.0
    for kind, a, b in bonds(N, M):
        J = coupling(kind, J1, J2)
        if J == 0.0:
            continue
        sa, sb = S[a], S[b]
        e += J * sz(sa) * sz(sb)
        if sa != sb:
            e += J * 0.5 * ratio(kind, a, b)
    return e


def swapped(S: np.ndarray, a, b) -> np.ndarray:
    S2 = S.copy()
    S2[a], S2[b] = S[b], S[a]
    return S2
