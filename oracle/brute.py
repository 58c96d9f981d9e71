"""Exact contractions of a fixed-spin PEPS on tiny lattices.

TEST INFRASTRUCTURE ONLY (see the package header).

W(S) = Tr(A_11^{s_11} ... A_NM^{s_NM}) (paper, Sec. II, Eq. (1) and the weight
W(S) after Eq. (2)): the contraction of every virtual bond of the network of
fixed-spin slices.  This module writes that definition out with numpy.einsum
over the whole network, and the full state vector by contracting rows while
keeping every physical index open.  It is the plain definition; it is pinned by
closed forms (product states, decoupled rows) in the tests.
"""
from __future__ import annotations

import string

import numpy as np

from . import hamiltonian


def _labels(N: int, M: int):
    """Distinct einsum labels for every bond of an N x M lattice."""
    pool = iter(string.ascii_letters)
    h = [[next(pool) for _ in range(M - 1)] for _ in range(N)]
    v = [[next(pool) for _ in range(M)] for _ in range(N - 1)]
    return h, v


def amplitude(T, S: np.ndarray) -> float:
    """W(S) by one einsum over the whole single-layer network (N*M <= ~20 sites)."""
    N, M = S.shape
    h, v = _labels(N, M)
    operands, subs = [], []
    for i in range(N):
        for j in range(M):
            A = T[i][j][S[i, j]]  # [l, r, u, d]
            idx = []
            for leg, lab in (("l", h[i][j - 1] if j > 0 else None),
                             ("r", h[i][j] if j < M - 1 else None),
                             ("u", v[i - 1][j] if i > 0 else None),
                             ("d", v[i][j] if i < N - 1 else None)):
                idx.append(lab)
            keep = [k for k, lab in enumerate(idx) if lab is not None]
            # squeeze the edge legs (dimension 1)
            A = A.reshape([A.shape[k] for k in keep]) if keep else A.reshape(())
            operands.append(A)
            subs.append("".join(idx[k] for k in keep))
    expr = ",".join(subs) + "->"
    return float(np.einsum(expr, *operands, optimize="greedy"))


def state_vector(T, N: int, M: int) -> np.ndarray:
    """All amplitudes W(S), indexed by the integer whose bit (i*M+j) is s_ij.

    One einsum over the whole network with every physical index left open
    (tiny lattices only: at most 52 labels, 2^(N*M) outputs).
    """
    h, v = _labels(N, M)
    used = {c for row in h for c in row} | {c for row in v for c in row}
    pool = iter(c for c in string.ascii_letters if c not in used)
    phys = [[next(pool) for _ in range(M)] for _ in range(N)]
    operands, subs = [], []
    for i in range(N):
        for j in range(M):
            t = T[i][j]  # [s, l, r, u, d]
            idx = [phys[i][j],
                   h[i][j - 1] if j > 0 else None,
                   h[i][j] if j < M - 1 else None,
                   v[i - 1][j] if i > 0 else None,
                   v[i][j] if i < N - 1 else None]
            keep = [k for k, lab in enumerate(idx) if lab is not None]
            operands.append(t.reshape([t.shape[k] for k in keep]))
            subs.append("".join(idx[k] for k in keep))
    # most significant output axis = last site, so the flat index has bit k = s of site k
    out = "".join(phys[k // M][k % M] for k in reversed(range(N * M)))
    vec = np.einsum(",".join(subs) + "->" + out, *operands, optimize="greedy")
    return np.asarray(vec).reshape(-1)


def local_energy_exact(T, S: np.ndarray, J1: float, J2: float) -> float:
    """E(S) with every W(S') contracted exactly and independently (tiny lattices)."""
    w0 = amplitude(T, S)

    def ratio(kind, a, b):
        return amplitude(T, hamiltonian.swapped(S, a, b)) / w0

    return hamiltonian.local_energy(S, J1, J2, ratio)


def environment_exact(T, S: np.ndarray, i: int, j: int, eps: float = 1e-6) -> np.ndarray:
    """B_ij = dW/dA_ij as the exact network with site (i, j) removed (Eq. (5)).

    W is linear in the slice A_ij, so B_ij[l,r,u,d] is read off as W with A_ij
    replaced by a unit tensor at (l,r,u,d).
    """
    A = T[i][j][S[i, j]]
    B = np.zeros_like(A)
    for idx in np.ndindex(A.shape):
        Tm = [list(r) for r in T]
        t = T[i][j].copy()
        t[S[i, j]] = 0.0
        t[(S[i, j],) + idx] = 1.0
        Tm[i][j] = t
        B[idx] = amplitude(Tm, S)
    return B
