"""Spin-spin correlations and the structure factor m_s^2(k) (Sec. IV, square lattice).

TEST INFRASTRUCTURE ONLY (see the package header).

m_s^2(k) = (1/N^2) sum_{ij} <S_i . S_j> exp(i k.(r_i - r_j)) over the N sites of a
central bulk window ((L-2)^2 or (L-4)^2 sites in the paper), with the average
taken over configurations drawn with weight W^2.

Reading (listed in the design notes): only the diagonal part S^z_i S^z_j is
estimated from the configurations; <S_i . S_j> = 3 <S^z_i S^z_j>, which holds
for a spin-rotation-invariant (singlet) state such as the ground state of the
Heisenberg model on an even open lattice.  The estimator of the diagonal part
is exact counting: S^z_i S^z_j = +1/4 when s_i = s_j, -1/4 otherwise.
"""
from __future__ import annotations

import numpy as np


def window_sites(N: int, M: int, r0: int, c0: int, h: int, w: int):
    """Row-major site indices k = i*M + j of the window rows r0..r0+h-1, columns c0..c0+w-1."""
    assert 0 <= r0 and r0 + h <= N and 0 <= c0 and c0 + w <= M
    return np.array([(r0 + a) * M + (c0 + b) for a in range(h) for b in range(w)])


def same_counts(configs, N: int, M: int, r0: int, c0: int, h: int, w: int, keep=None,
                weights=None):
    """Per pair of window sites, the number of samples with s_i = s_j, and the sample count
    (with ``weights``: the weighted sums instead, e.g. |psi|^2 for an exact average)."""
    S = np.asarray(configs).reshape(len(configs), N * M)
    wt = None if weights is None else np.asarray(weights, dtype=np.float64)
    if keep is not None:
        sel = np.asarray(keep, dtype=bool)
        S = S[sel]
        wt = None if wt is None else wt[sel]
    X = S[:, window_sites(N, M, r0, c0, h, w)].astype(np.int64)   # spin labels 0/1
    if wt is None:
        ones = X.T @ X                     # samples with both labels 1
        zeros = (1 - X).T @ (1 - X)        # samples with both labels 0
        return ones + zeros, X.shape[0]
    ones = X.T @ (X * wt[:, None])
    zeros = (1 - X).T @ ((1 - X) * wt[:, None])
    return ones + zeros, float(wt.sum())


def szsz(same, n: int):
    """<S^z_i S^z_j> = (same - (n - same)) / (4 n)."""
    return (2.0 * np.asarray(same, dtype=np.float64) - n) / (4.0 * n)


def structure_factor(C, h: int, w: int, kx: float, ky: float, factor: float = 1.0):
    """factor / N^2 * sum_ij C_ij cos(k.(r_i - r_j)), r = (column, row) within the window.

    With C = <S_i . S_j> (factor 1) this is m_s^2(k) of Sec. IV; with
    C = <S^z_i S^z_j> and factor 1 it is the zz structure factor, and factor 3
    turns that into m_s^2(k) only for a spin-rotation-invariant state.
    """
    Nw = h * w
    y, x = np.divmod(np.arange(Nw), w)
    phase = kx * (x[:, None] - x[None, :]) + ky * (y[:, None] - y[None, :])
    return factor * float(np.sum(np.asarray(C) * np.cos(phase))) / (Nw * Nw)
