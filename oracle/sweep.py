"""One Metropolis sweep over every nearest-neighbour bond, reusing environments.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper samples configurations with weight W(S)^2 by sweeps (Sec. I, Sec. II);
it does not state the update.  Reading (listed in the design notes): a sweep
proposes, in a fixed order, the exchange of the two spins of every
nearest-neighbour bond, row by row from the top:

    for row i = 0 .. N-1:
        horizontal bonds (i, j)-(i, j+1), j = 0 .. M-2
        vertical bonds (i, j)-(i+1, j), j = 0 .. M-1      (i < N-1)

A bond whose spins are equal is skipped; otherwise the exchange is accepted
when u < min(1, R^2), u the bond's uniform (one per bond, in this order,
passed in) and R = W(S')/W(S) the shared-environment ratio of the current
configuration (the reading of the local energy: the row-i sandwich between
U_{i-1} and Dn_{i+1} for a horizontal bond, the two-row strip between
U_{i-1} and Dn_{i+2} for a vertical one).  R is the ratio of the two
contractions that differ only in the exchanged column(s), both taken with the
same left and right environments of the row or strip.

Environment reuse: the bottom environments Dn_k are built once per sweep
(rows below i do not move before row i's turn); U_{i-1} is rebuilt from the
rows as they stand after their moves; along a row (strip) the right
environments are built once before its proposals and the left environment is
extended column by column with the spins as they stand after each decision.
"""
from __future__ import annotations

import math

import numpy as np

from . import peps as op


def bond_order(N: int, M: int):
    """Site index pairs (a, b) of one sweep, in proposal order."""
    out = []
    for i in range(N):
        for j in range(M - 1):
            out.append((i * M + j, i * M + j + 1))
        if i < N - 1:
            for j in range(M):
                out.append((i * M + j, (i + 1) * M + j))
    return out


def _accept(num: float, den: float, u: float) -> bool:
    if den == 0.0:
        return num != 0.0  # leave a zero-weight configuration at the first nonzero proposal
    r = num / den
    return u < min(1.0, r * r)


def _row_sweep(T, s, i, Ut, Dt, uniforms, k0, ratios, accepted):
    """Horizontal proposals of row i; s (N x M) is updated in place."""
    M = s.shape[1]
    row = [T[i][j][s[i, j]] for j in range(M)]
    RE = [None] * (M + 1)
    RE[M] = np.ones((1, 1, 1))
    for j in range(M - 1, -1, -1):
        RE[j], _ = op._normalise(op._col1_right(RE[j + 1], Ut[j], row[j], Dt[j]))
    LE = np.ones((1, 1, 1))
    for j in range(M):
        if j < M - 1 and s[i, j] != s[i, j + 1]:
            a, b = int(s[i, j]), int(s[i, j + 1])
            e_num = op._col1(LE, Ut[j], T[i][j][b], Dt[j])
            num = float(np.sum(op._col1(e_num, Ut[j + 1], T[i][j + 1][a], Dt[j + 1]) * RE[j + 2]))
            e_den = op._col1(LE, Ut[j], T[i][j][a], Dt[j])
            den = float(np.sum(op._col1(e_den, Ut[j + 1], T[i][j + 1][b], Dt[j + 1]) * RE[j + 2]))
            ok = _accept(num, den, uniforms[k0 + j])
            ratios[k0 + j] = num / den if den != 0.0 else math.inf
            accepted[k0 + j] = ok
            if ok:
                s[i, j], s[i, j + 1] = b, a
            LE = e_num if ok else e_den
        else:
            LE = op._col1(LE, Ut[j], T[i][j][s[i, j]], Dt[j])
        LE, _ = op._normalise(LE)


def _strip_sweep(T, s, i, Ut, Dt, uniforms, k0, ratios, accepted):
    """Vertical proposals between rows i and i+1; s is updated in place."""
    M = s.shape[1]
    RE = [None] * (M + 1)
    RE[M] = np.ones((1, 1, 1, 1))
    for j in range(M - 1, -1, -1):
        RE[j], _ = op._normalise(op._col2_right(RE[j + 1], Ut[j], T[i][j][s[i, j]],
                                                T[i + 1][j][s[i + 1, j]], Dt[j]))
    LE = np.ones((1, 1, 1, 1))
    for j in range(M):
        a, b = int(s[i, j]), int(s[i + 1, j])
        if a != b:
            e_num = op._col2(LE, Ut[j], T[i][j][b], T[i + 1][j][a], Dt[j])
            num = float(np.sum(e_num * RE[j + 1]))
            e_den = op._col2(LE, Ut[j], T[i][j][a], T[i + 1][j][b], Dt[j])
            den = float(np.sum(e_den * RE[j + 1]))
            ok = _accept(num, den, uniforms[k0 + j])
            ratios[k0 + j] = num / den if den != 0.0 else math.inf
            accepted[k0 + j] = ok
            if ok:
                s[i, j], s[i + 1, j] = b, a
            LE = e_num if ok else e_den
        else:
            LE = op._col2(LE, Ut[j], T[i][j][a], T[i + 1][j][b], Dt[j])
        LE, _ = op._normalise(LE)


def sweep(T, Dc: int, S, uniforms):
    """One sweep of one chain.

    ``uniforms`` has one entry per bond of ``bond_order``.  Returns (new
    configuration (flat uint8), accepted (bool per bond), ratios (R per
    proposed bond, NaN where the spins were equal)).
    """
    N, M = len(T), len(T[0])
    s = np.array(S, dtype=np.uint8).reshape(N, M)
    nb = N * (M - 1) + (N - 1) * M
    accepted = np.zeros(nb, dtype=bool)
    ratios = np.full(nb, math.nan)
    # bottom environments of the configuration at the start of the sweep
    A = op.slices(T, s)
    bot = {N: op.trivial_mps(M), N - 1: op.row_as_mps(A[N - 1], "u")}
    for k in range(N - 2, 0, -1):
        bot[k], _, _ = op.zip_row(bot[k + 1], 0.0, op.flip_row(A[k]), Dc)
        if bot[k] is None:
            return s.reshape(-1), accepted, ratios
    top = op.trivial_mps(M)  # U_{i-1}
    k0 = 0
    for i in range(N):
        _row_sweep(T, s, i, top, bot[i + 1], uniforms, k0, ratios, accepted)
        k0 += M - 1
        if i < N - 1:
            _strip_sweep(T, s, i, top, bot[i + 2], uniforms, k0, ratios, accepted)
            k0 += M
        if i < N - 1:
            row = [T[i][j][s[i, j]] for j in range(M)]
            if i == 0:
                top = op.row_as_mps(row, "d")
            else:
                top, _, _ = op.zip_row(top, 0.0, row, Dc)
                if top is None:
                    return s.reshape(-1), accepted, ratios
    return s.reshape(-1), accepted, ratios
