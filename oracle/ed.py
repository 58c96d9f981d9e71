"""Exact diagonalisation of the open-boundary J1-J2 Heisenberg model.

TEST INFRASTRUCTURE ONLY (see the package header).

Builds H of Eq. (7) (paper, Sec. IV) as a sparse matrix in one S^z sector of
the computational basis (bit k of a basis integer is the spin label s of site
k = i*M + j, s = 1 meaning S^z = -1/2) and finds its lowest eigenpair with
ARPACK (scipy.sparse.linalg.eigsh) or, for small sectors, LAPACK (eigh).

Pinned by the exact energies printed in Table I (4x4 and 4x6, open boundaries).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import hamiltonian


def sector_states(n_sites: int, n_down: int) -> np.ndarray:
    """Sorted basis integers with exactly ``n_down`` bits set."""
    if n_sites <= 20:
        allst = np.arange(1 << n_sites, dtype=np.int64)
        pc = np.zeros_like(allst)
        for k in range(n_sites):
            pc += (allst >> k) & 1
        return allst[pc == n_down]
    out = []
    for comb in itertools.combinations(range(n_sites), n_down):
        v = 0
        for k in comb:
            v |= 1 << k
        out.append(v)
    return np.sort(np.asarray(out, dtype=np.int64))


def _pair_sites(N: int, M: int):
    nn, nnn = [], []
    for kind, a, b in hamiltonian.bonds(N, M):
        ka, kb = a[0] * M + a[1], b[0] * M + b[1]
        (nn if kind in ("h", "v") else nnn).append((ka, kb))
    return nn, nnn


def _bond_operator(states: np.ndarray, pairs) -> sp.csr_matrix:
    """sum over pairs of S_a.S_b restricted to the sector spanned by ``states``."""
    n = states.size
    diag = np.zeros(n)
    rows, cols = [], []
    for a, b in pairs:
        sa = (states >> a) & 1
        sb = (states >> b) & 1
        anti = sa != sb
        diag += np.where(anti, -0.25, 0.25)
        src = np.nonzero(anti)[0]
        dst = np.searchsorted(states, states[src] ^ ((1 << a) | (1 << b)))
        rows.append(dst)
        cols.append(src)
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    off = sp.csr_matrix((np.full(rows.size, 0.5), (rows, cols)), shape=(n, n))
    return off + sp.diags(diag)


def hamiltonian_blocks(N: int, M: int, n_down: int | None = None):
    """(states, H_nn, H_nnn) so that H = J1 * H_nn + J2 * H_nnn on the sector."""
    n = N * M
    if n_down is None:
        n_down = n // 2
    states = sector_states(n, n_down)
    nn, nnn = _pair_sites(N, M)
    return states, _bond_operator(states, nn), _bond_operator(states, nnn)


def ground_state(N: int, M: int, J1: float = 1.0, J2: float = 0.0, n_down=None,
                 method: str = "arpack", blocks=None):
    """(E0, vector, states) of the lowest eigenpair in the sector (total energy)."""
    states, Hnn, Hnnn = blocks if blocks is not None else hamiltonian_blocks(N, M, n_down)
    H = (J1 * Hnn + J2 * Hnnn).tocsr()
    if method == "dense":
        w, v = np.linalg.eigh(H.toarray())
        return float(w[0]), v[:, 0], states
    rng = np.random.Generator(np.random.PCG64(7))
    v0 = rng.standard_normal(states.size)
    w, v = spla.eigsh(H, k=1, which="SA", v0=v0, tol=1e-12, maxiter=5000)
    return float(w[0]), v[:, 0], states


def config_of_state(st: int, N: int, M: int) -> np.ndarray:
    return np.asarray([(st >> k) & 1 for k in range(N * M)], dtype=np.int64).reshape(N, M)
