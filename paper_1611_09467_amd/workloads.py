"""Seeded synthetic inputs shared by the HIP path, its tests, the benchmark and the oracle.

This module draws random numbers and arranges them; it holds none of the
method's arithmetic (no contraction, no truncation, no amplitude).  Both the
GPU library and the CPU oracle receive exactly the arrays built here.

Lattice conventions (paper, Sec. II, Eq. (1)):
  * N rows x M columns, open boundaries; site (i, j) is 0-based, i counts rows
    top to bottom and j columns left to right.
  * site tensor T_ij[s, l, r, u, d]: physical index s in {0, 1}, virtual legs
    left/right/up/down; a leg on an open edge has dimension 1.
  * a configuration S is an (N, M) array of spins in {0, 1}; s = 0 is read as
    S^z = +1/2.

Packed layout handed to the C-ABI: sites in row-major order, each site stored
contiguously as [s][l][r][u][d] (C order), float64.
"""
from __future__ import annotations

from pathlib import Path

import numpy as np

PHYS_DIM = 2


def site_dims(N: int, M: int, D: int, i: int, j: int) -> tuple[int, int, int, int]:
    """(Dl, Dr, Du, Dd) of site (i, j): D inside, 1 on an open edge (paper, Eq. (1))."""
    return (1 if j == 0 else D, 1 if j == M - 1 else D,
            1 if i == 0 else D, 1 if i == N - 1 else D)


def site_sizes(N: int, M: int, D: int, d: int = PHYS_DIM) -> list[int]:
    out = []
    for i in range(N):
        for j in range(M):
            dl, dr, du, dd = site_dims(N, M, D, i, j)
            out.append(d * dl * dr * du * dd)
    return out


def make_peps(N: int, M: int, D: int, seed: int = 0, bias: float = 0.0,
              scale: float = 1.0, d: int = PHYS_DIM) -> list[list[np.ndarray]]:
    """Random PEPS: every entry iid N(0,1)/sqrt(D), drawn site by site in row-major order.

    ``bias`` adds an identity-like term ``bias * [l == r] * [u == d]`` (for every
    index pair valid on both legs, both spin values); ``scale`` multiplies every
    entry afterwards.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    T = []
    for i in range(N):
        row = []
        for j in range(M):
            dl, dr, du, dd = site_dims(N, M, D, i, j)
            t = rng.standard_normal((d, dl, dr, du, dd)) / np.sqrt(D)
            if bias:
                for a in range(min(dl, dr)):
                    for b in range(min(du, dd)):
                        t[:, a, a, b, b] += bias
            row.append(t * scale)
        T.append(row)
    return T


def pack_peps(T: list[list[np.ndarray]]) -> np.ndarray:
    """Concatenate site tensors (row-major sites, each [s][l][r][u][d]) into one float64 vector."""
    return np.ascontiguousarray(np.concatenate([t.ravel() for row in T for t in row]),
                                dtype=np.float64)


def unpack_peps(flat: np.ndarray, N: int, M: int, D: int, d: int = PHYS_DIM):
    T, off = [], 0
    for i in range(N):
        row = []
        for j in range(M):
            dl, dr, du, dd = site_dims(N, M, D, i, j)
            n = d * dl * dr * du * dd
            row.append(np.asarray(flat[off:off + n], dtype=np.float64).reshape(d, dl, dr, du, dd))
            off += n
        T.append(row)
    return T


def random_sz0_configs(N: int, M: int, count: int, seed: int) -> np.ndarray:
    """``count`` uniform configurations with floor(N*M/2) spins s=1 (S^z = 0 for even N*M).

    Returns uint8 array [count][N*M] (row-major sites).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = N * M
    base = np.zeros(n, dtype=np.uint8)
    base[: n // 2] = 1
    out = np.empty((count, n), dtype=np.uint8)
    for c in range(count):
        out[c] = rng.permutation(base)
    return out


def nn_bonds(N: int, M: int) -> np.ndarray:
    """Nearest-neighbour bonds (site index pairs), horizontal first then vertical."""
    b = []
    for i in range(N):
        for j in range(M - 1):
            b.append((i * M + j, i * M + j + 1))
    for i in range(N - 1):
        for j in range(M):
            b.append((i * M + j, (i + 1) * M + j))
    return np.asarray(b, dtype=np.int64)


def chain_draws(N: int, M: int, chains: int, steps: int, seed: int):
    """Every random number of the exchange chains: (starts, picks, uniforms).

    starts[c] is chain c's uniform S^z = 0 start configuration, picks[c, t]
    the nearest-neighbour bond (index into ``nn_bonds``) proposed at step t,
    uniforms[c, t] in [0, 1) the number its acceptance test compares with.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    starts = random_sz0_configs(N, M, chains, seed + 1000)
    picks = rng.integers(0, len(nn_bonds(N, M)), size=(chains, steps))
    uniforms = rng.random((chains, steps))
    return starts, picks, uniforms


def chain_configs(N: int, M: int, chains: int, steps: int, seed: int) -> np.ndarray:
    """Configurations recorded along random nearest-neighbour-exchange chains.

    Each chain starts from a uniform S^z = 0 configuration; a step picks a
    uniformly random nearest-neighbour bond and exchanges its two spins when
    they differ (an S^z-conserving move).  The configuration is recorded after
    every step, giving ``chains * steps`` samples ordered chain by chain.
    Every exchange is kept (no amplitude is computed here); the weighted
    chains of the named workloads are stored files (``metropolis_configs``).
    """
    starts, picks, _ = chain_draws(N, M, chains, steps, seed)
    bonds = nn_bonds(N, M)
    out = np.empty((chains * steps, N * M), dtype=np.uint8)
    for c in range(chains):
        s = starts[c].copy()
        for t in range(steps):
            a, b = bonds[picks[c, t]]
            if s[a] != s[b]:
                s[a], s[b] = s[b], s[a]
            out[c * steps + t] = s
    return out


DATA_DIR = Path(__file__).resolve().parent / "data"


def metropolis_file(name: str) -> Path:
    return DATA_DIR / f"metropolis_{name}.npz"


def metropolis_configs(name: str) -> np.ndarray:
    """Stored Metropolis-chain configurations of a named workload, [chains*steps][N*M].

    The chains sample with weight W(S)^2 from the draws of ``chain_draws``;
    the acceptance needs amplitudes, so the file was written once by the
    float64 CPU reference implementation and is only read here.
    """
    w = WORKLOADS[name]
    f = metropolis_file(name)
    if not f.exists():
        raise FileNotFoundError(f"{f} is missing; it is written by `python -m oracle.make_chains {name}`")
    with np.load(f, allow_pickle=False) as z:
        nb, ns = int(z["count"]), int(z["sites"])
        S = np.unpackbits(z["bits"])[: nb * ns].reshape(nb, ns).astype(np.uint8)
    assert ns == w["N"] * w["M"] and nb == w["chains"] * w["steps"], f
    return S


def neel_config(N: int, M: int) -> np.ndarray:
    """Checkerboard configuration: s = (i + j) mod 2."""
    return np.asarray([[(i + j) % 2 for j in range(M)] for i in range(N)], dtype=np.uint8).ravel()


def neel_product_peps(N: int, M: int) -> list[list[np.ndarray]]:
    """D = 1 product PEPS whose only nonzero amplitude is the Neel configuration."""
    T = []
    for i in range(N):
        row = []
        for j in range(M):
            t = np.zeros((PHYS_DIM, 1, 1, 1, 1))
            t[(i + j) % 2, 0, 0, 0, 0] = 1.0
            row.append(t)
        T.append(row)
    return T


def row_decoupled_peps(N: int, M: int, D: int, seed: int, scale: float = 1.0):
    """PEPS whose vertical legs carry only index 0: T = delta_{u0} delta_{d0} t[s, l, r].

    Entries of t are iid N(0,1)/sqrt(D) times ``scale``; every other entry is 0.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    T = []
    for i in range(N):
        row = []
        for j in range(M):
            dl, dr, du, dd = site_dims(N, M, D, i, j)
            t = np.zeros((PHYS_DIM, dl, dr, du, dd))
            t[:, :, :, 0, 0] = rng.standard_normal((PHYS_DIM, dl, dr)) / np.sqrt(D) * scale
            row.append(t)
        T.append(row)
    return T


def column_decoupled_peps(N: int, M: int, D: int, seed: int, scale: float = 1.0):
    """PEPS whose horizontal legs carry only index 0: T = delta_{l0} delta_{r0} t[s, u, d]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T = []
    for i in range(N):
        row = []
        for j in range(M):
            dl, dr, du, dd = site_dims(N, M, D, i, j)
            t = np.zeros((PHYS_DIM, dl, dr, du, dd))
            t[:, 0, 0, :, :] = rng.standard_normal((PHYS_DIM, du, dd)) / np.sqrt(D) * scale
            row.append(t)
        T.append(row)
    return T


def tied_cut_peps(eps: float = 0.0, seed: int = 3):
    """3 x 2 lattice, D = 2, whose first truncated block (top zip, column 0) is
    X = [[1 + eps, 0, 0, 0], [0, 0, 0, 1]] up to signs: its two singular values
    1 + eps and 1 tie exactly at eps = 0, so a cut to Dc = 1 keeps an
    ill-defined subspace.

    Site (0,0): t[s, 0, r, 0, d] = [r == d]; site (0,1): t[s, l, 0, 0, d] = [l == d]
    (identity, so the right-canonical sweep only changes signs); site (1,0):
    t[s, 0, r, u, p] = [r == u == p], entry (r, u, p) = (0, 0, 0) set to 1 + eps.
    Both spin slices are equal on these three sites; the other sites are
    iid N(0,1)/sqrt(2) drawn with ``seed``.
    """
    N, M, D = 3, 2, 2
    T = make_peps(N, M, D, seed=seed)
    T[0][0] = np.zeros((PHYS_DIM, 1, D, 1, D))
    T[0][1] = np.zeros((PHYS_DIM, D, 1, 1, D))
    T[1][0] = np.zeros((PHYS_DIM, 1, D, D, D))
    for a in range(D):
        T[0][0][:, 0, a, 0, a] = 1.0
        T[0][1][:, a, 0, 0, a] = 1.0
        T[1][0][:, 0, a, a, a] = 1.0
    T[1][0][:, 0, 0, 0, 0] = 1.0 + eps
    return T


def orthogonal_matrix(n: int, seed: int) -> np.ndarray:
    """Haar-like random orthogonal matrix (QR of a Gaussian matrix, sign-fixed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


# Workload shapes (the per-sample evaluation at the paper's lattice sizes).
WORKLOADS = {
    "4x4_D2_Dc4": dict(N=4, M=4, D=2, Dc=4, seed=0, bias=0.0, kind="uniform", count=1000,
                       J2=0.5),
    "8x8_D4_Dc8": dict(N=8, M=8, D=4, Dc=8, seed=0, bias=0.1, kind="metropolis", chains=256,
                       steps=16, J2=0.5),
    "10x10_D6_Dc12": dict(N=10, M=10, D=6, Dc=12, seed=0, bias=0.0, kind="metropolis",
                          chains=1024, steps=16, J2=0.5),
    "16x16_D8_Dc16": dict(N=16, M=16, D=8, Dc=16, seed=0, bias=0.0, kind="metropolis",
                          chains=512, steps=16, J2=0.5),
}


def workload_inputs(name: str, count: int | None = None):
    """(T, configs) for a named workload; ``count`` keeps only the first samples."""
    w = WORKLOADS[name]
    T = make_peps(w["N"], w["M"], w["D"], seed=w["seed"], bias=w["bias"])
    if w["kind"] == "uniform":
        S = random_sz0_configs(w["N"], w["M"], w["count"], w["seed"] + 1000)
    elif w["kind"] == "metropolis":
        S = metropolis_configs(name)
    else:
        chains = w["chains"]
        if count is not None:
            chains = min(chains, max(1, -(-count // w["steps"])))
        S = chain_configs(w["N"], w["M"], chains, w["steps"], w["seed"] + 1000)
    if count is not None:
        S = S[:count]
    return T, S
