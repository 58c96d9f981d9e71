"""Imaginary-time evolution with the simple update (the initialiser of Sec. III).

TEST INFRASTRUCTURE ONLY (see the package header).  Plain numpy/LAPACK in
float64, one bond at a time, no QR reduction.

What is computed (paper, Sec. I and Sec. III, "Computational details"):
the PEPS is held as site tensors Gamma_ij [s, l, r, u, d] with a diagonal
weight vector lambda on every internal bond; the environment of a bond is
approximated by the weights of the bonds around its two sites.  One
imaginary-time step applies exp(-dtau h_b) to every bond b, in groups of
mutually commuting bonds (first-order Suzuki-Trotter), and truncates each
bond back to D by an SVD.

Readings where the paper is silent (each is listed in the design notes):
  SU1 only the nearest-neighbour J1 terms are evolved (the paper quotes the
      O(D^5) cost for NN interactions only); J2 is left to the gradient step.
  SU2 the bond groups, in this order: horizontal bonds (i, j)-(i, j+1) with
      j even, then j odd; vertical bonds (i, j)-(i+1, j) with i even, then i
      odd.  Bonds of one group share no site, so their order does not matter.
  SU3 the new weights are the kept singular values divided by their 2-norm;
      when fewer than D are non-zero the rest are 0.
  SU4 removing a weight from a tensor divides by it, and by nothing (the
      entry is set to 0) where the weight is <= 1e-12 times the largest
      weight of that bond.
  SU5 the PEPS handed to the evaluation carries sqrt(lambda) on both sides of
      every bond: T = Gamma * prod over the legs of sqrt(lambda_leg).

The reduction of the cost to O(D^5) by QR factors of the two site tensors is
an exact rewriting of the same step and is not used here: the full two-site
matrix [(s_a, other legs of a), (s_b, other legs of b)] is decomposed directly.
"""
from __future__ import annotations

import numpy as np

# the two spin-1/2 operators, basis index s = 0, 1 (S^z = +1/2, -1/2)
_SX = 0.5 * np.array([[0.0, 1.0], [1.0, 0.0]])
_SY_IM = 0.5 * np.array([[0.0, -1.0], [1.0, 0.0]])  # S^y = i * _SY_IM
_SZ = 0.5 * np.array([[1.0, 0.0], [0.0, -1.0]])


def bond_hamiltonian(J1: float) -> np.ndarray:
    """J1 S_a.S_b as a 4x4 matrix, row index 2 s_a' + s_b', column 2 s_a + s_b."""
    # S^y S^y = (i A)(i A) = -A A for the real matrix A = _SY_IM
    return J1 * (np.kron(_SX, _SX) - np.kron(_SY_IM, _SY_IM) + np.kron(_SZ, _SZ))


def gate(J1: float, dtau: float) -> np.ndarray:
    """exp(-dtau J1 S_a.S_b) from the eigen-decomposition of the bond term."""
    w, v = np.linalg.eigh(bond_hamiltonian(J1))
    return (v * np.exp(-dtau * w)) @ v.T


def bond_groups(N: int, M: int):
    """The four groups of commuting NN bonds in evolution order (reading SU2)."""
    hb = [[(("h", i, j)) for i in range(N) for j in range(M - 1) if j % 2 == par]
          for par in (0, 1)]
    vb = [[(("v", i, j)) for i in range(N - 1) for j in range(M) if i % 2 == par]
          for par in (0, 1)]
    return hb + vb


def initial_weights(N: int, M: int, D: int):
    """All-ones weights: lam['h'][i][j] on (i,j)-(i,j+1), lam['v'][i][j] on (i,j)-(i+1,j)."""
    return {"h": [[np.ones(D) for _ in range(M - 1)] for _ in range(N)],
            "v": [[np.ones(D) for _ in range(M)] for _ in range(N - 1)]}


def _leg_weights(lam, N, M, i, j):
    """The weight vector on each leg (l, r, u, d) of site (i, j); None on an open edge."""
    return (lam["h"][i][j - 1] if j > 0 else None,
            lam["h"][i][j] if j < M - 1 else None,
            lam["v"][i - 1][j] if i > 0 else None,
            lam["v"][i][j] if i < N - 1 else None)


def _scale_legs(t, weights, power: float, skip: int):
    """Multiply leg k (of l, r, u, d) of t [s, l, r, u, d] by weight**power, except leg ``skip``."""
    out = t.copy()
    for k, w in enumerate(weights):
        if w is None or k == skip:
            continue
        if power >= 0:
            f = w ** power
        else:  # reading SU4
            f = np.where(w > 1e-12 * w.max(), 1.0 / np.where(w > 0, w, 1.0), 0.0) ** (-power)
        shape = [1, 1, 1, 1, 1]
        shape[k + 1] = w.size
        out = out * f.reshape(shape)
    return out


def update_bond(G, lam, bond, g: np.ndarray, D: int):
    """Apply the two-site gate g (4x4) to one bond and truncate it to D (in place)."""
    kind, i, j = bond
    N, M = len(G), len(G[0])
    if kind == "h":
        ia, ja, ib, jb, la, lb = i, j, i, j + 1, 1, 0      # bond leg: r of a, l of b
    else:
        ia, ja, ib, jb, la, lb = i, j, i + 1, j, 3, 2      # bond leg: d of a, u of b
    lam_ab = lam[kind][i][j]
    A = _scale_legs(G[ia][ja], _leg_weights(lam, N, M, ia, ja), 1.0, la)
    B = _scale_legs(G[ib][jb], _leg_weights(lam, N, M, ib, jb), 1.0, lb)
    # move the bond leg last in A and first in B: A[s, oa..., x], B[s, x, ob...]
    A = np.moveaxis(A, la + 1, -1)
    B = np.moveaxis(B, lb + 1, 1)
    sa, xa = A.shape[1:-1], A.shape[-1]
    sb = B.shape[2:]
    Am = A.reshape(2, -1, xa)                       # [s_a, a, x]
    Bm = B.reshape(2, xa, -1)                       # [s_b, x, b]
    theta = np.einsum("pax,x,qxb->paqb", Am, lam_ab, Bm)
    g4 = g.reshape(2, 2, 2, 2)                      # [s_a', s_b', s_a, s_b]
    theta = np.einsum("PQpq,paqb->PaQb", g4, theta)
    na, nb = theta.shape[1], theta.shape[3]
    mat = theta.reshape(2 * na, 2 * nb)
    U, s, Vt = np.linalg.svd(mat, full_matrices=False)
    k = min(D, s.size)
    keep = np.zeros(D)
    keep[:k] = s[:k]
    norm = np.linalg.norm(keep)
    new_lam = keep / norm
    Uk = np.zeros((2 * na, D))
    Uk[:, :k] = U[:, :k]
    Vk = np.zeros((D, 2 * nb))
    Vk[:k, :] = Vt[:k, :]
    An = Uk.reshape((2,) + sa + (D,))               # [s, oa..., x]
    Bn = Vk.reshape((D, 2) + sb)                    # [x, s, ob...]
    Bn = np.moveaxis(Bn, 0, 1)                      # [s, x, ob...]
    An = np.moveaxis(An, -1, la + 1)
    Bn = np.moveaxis(Bn, 1, lb + 1)
    lam[kind][i][j] = new_lam
    G[ia][ja] = _scale_legs(An, _leg_weights(lam, N, M, ia, ja), -1.0, la)
    G[ib][jb] = _scale_legs(Bn, _leg_weights(lam, N, M, ib, jb), -1.0, lb)


def evolve(G, lam, J1: float, dtau: float, nsteps: int, D: int):
    """nsteps first-order Trotter steps over the four bond groups (copies; inputs untouched)."""
    N, M = len(G), len(G[0])
    G = [[t.copy() for t in row] for row in G]
    lam = {k: [[w.copy() for w in row] for row in v] for k, v in lam.items()}
    g = gate(J1, dtau)
    for _ in range(nsteps):
        for grp in bond_groups(N, M):
            for b in grp:
                update_bond(G, lam, b, g, D)
    return G, lam


def grow(G, lam, D_new: int):
    """The same state at a larger bond dimension (the D-ramp of Sec. III): every
    internal leg of every Gamma and every weight vector is padded with zeros."""
    N, M = len(G), len(G[0])
    D_old = lam["h"][0][0].size if M > 1 else lam["v"][0][0].size
    assert D_new >= D_old
    out = []
    for i in range(N):
        row = []
        for j in range(M):
            t = G[i][j]
            inner = (j > 0, j < M - 1, i > 0, i < N - 1)  # l, r, u, d
            pad = [(0, 0)] + [(0, D_new - n if k else 0) for n, k in zip(t.shape[1:], inner)]
            row.append(np.pad(t, pad))
        out.append(row)
    lam2 = {k: [[np.concatenate([w, np.zeros(D_new - w.size)]) for w in r] for r in v]
            for k, v in lam.items()}
    return out, lam2


def to_peps(G, lam):
    """Tensors with sqrt(lambda) on both sides of every bond (reading SU5)."""
    N, M = len(G), len(G[0])
    return [[_scale_legs(G[i][j], _leg_weights(lam, N, M, i, j), 0.5, -1) for j in range(M)]
            for i in range(N)]
