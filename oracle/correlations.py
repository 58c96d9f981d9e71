"""Transverse spin correlations from configurations drawn with weight W(S)^2.

TEST INFRASTRUCTURE ONLY (see the package header).

m_s^2(k) of Sec. IV sums <S_p . S_q> over the pairs of a bulk window, and
S_p . S_q = S^z_p S^z_q + (S^+_p S^-_q + S^-_p S^+_q) / 2.  With samples drawn
with weight W(S)^2 (Sec. II) the expectation of an operator O is the average
of its local value sum_{S'} <S|O|S'> W(S')/W(S), as for the energy (Eq. (7)).
For the transverse part the only S' is S^{pq} (the spins at p and q
exchanged), reached with matrix element 1/2 when s_p != s_q:

    O_pq(S) = 1/2 [s_p != s_q] W(S^{pq}) / W(S)        (p != q)
    O_pp(S) = 1/2                                      (spin 1/2: S^+S^- + S^-S^+ = 1)

Reading OBS2 (listed in the design notes; the paper does not say how the
ratio is contracted for a pair at any distance).  With p in row a and q in
row b >= a, p before q in row-major order:

    W(S^{pq}) ~ <U_{a-1}(S)| rows a .. b-1 of S^{pq}, each zipped in top-down
                with truncation to Dc | row b of S^{pq} |Dn_{b+1}(S)>
    W(S)      ~ psi_b(S) = <U_{b-1}(S)| row b of S |Dn_{b+1}(S)>

Both contractions share the environments of the rows that do not change:
U_{a-1} above and Dn_{b+1} below, the shared-environment reading of the
nearest-neighbour ratios (R5) carried to rows apart.  For b = a this is the
horizontal ratio of R5 (the row-a sandwich).  Without truncation both are W
exactly.

Parity status: pinned (exact regime against brute-force W ratios; exact
enumeration against the expectation of the spin operators on the state
vector; row-decoupled closed forms under truncation; R5's horizontal ratios).
"""
from __future__ import annotations

import math

import numpy as np

from . import observables
from . import peps as op


def window_sites(N: int, M: int, window):
    r0, c0, h, w = window
    return observables.window_sites(N, M, r0, c0, h, w)


def _row_value(Ut, Uls, row, Dt, Dls, perturb=None):
    """(ln|v|, sign v) of the exact contraction <Ut| row |Dt> (no gradients)."""
    M = len(row)
    E = np.ones((1, 1, 1))
    lg = Uls + Dls
    for j in range(M - 1, -1, -1):
        E, m = op._normalise(op._col1_right(E, Ut[j], row[j], Dt[j]), perturb)
        if m == 0.0:
            return -math.inf, 0
        if not np.isfinite(m):
            return math.nan, 0
        lg += math.log(m)
    v = float(E.reshape(()))
    if v == 0.0:
        return -math.inf, 0
    return lg + math.log(abs(v)), (1 if v > 0 else -1)


def ratio_matrix(T, S, Dc: int, window, perturb=None):
    """Exchange ratios R_pq = W(S^{pq})/W(S) of one sample by reading OBS2.

    Returns (R, tie, flags): R is (n, n) over the window sites in row-major
    order, symmetric, NaN on the diagonal and where s_p = s_q; ``tie`` marks
    pairs whose numerator passed a near-tie truncation; ``flags`` are the
    sample's own flags (peps.FLAG_*) from its environments and row sandwiches,
    with NONFINITE also when a counted ratio is not finite.  ``perturb`` (used
    only to measure conditioning) is applied to every intermediate.
    """
    N, M = len(T), len(T[0])
    S = np.asarray(S, dtype=np.uint8).reshape(N, M)
    sites = window_sites(N, M, window)
    n = len(sites)
    R = np.full((n, n), math.nan)
    tie = np.zeros((n, n), dtype=bool)
    A = op.slices(T, S)
    top, bot, info = op.environments(A, Dc, perturb=perturb)
    flags = op.FLAG_NEAR_TIE if info["near_tie"] else 0
    if info["nonfinite"]:
        return R, tie, flags | op.FLAG_NONFINITE
    if info["zero"]:
        return R, tie, flags | op.FLAG_ZERO_PSI
    rows = sorted({int(k) // M for k in sites})
    den = {}
    for b in rows:
        Ut, Uls = top[b - 1]
        Dt, Dls = bot[b + 1]
        lg, sg = _row_value(Ut, Uls, A[b], Dt, Dls, perturb)
        if sg == 0:
            return R, tie, flags | (op.FLAG_NONFINITE if math.isnan(lg) else op.FLAG_ZERO_PSI)
        den[b] = (lg, sg)
    for x in range(n):
        a, ca = divmod(int(sites[x]), M)
        for y in range(x + 1, n):
            b, cb = divmod(int(sites[y]), M)
            if S[a, ca] == S[b, cb]:
                continue
            Sx = S.copy()
            Sx[a, ca], Sx[b, cb] = S[b, cb], S[a, ca]
            Ax = op.slices(T, Sx)
            # rows a .. b-1 of S^{pq} zipped into U_{a-1}(S)
            Ut, Uls = top[a - 1]
            tied = False
            for i in range(a, b):
                if i == 0:
                    Ut, Uls = op.row_as_mps(Ax[0], "d"), 0.0
                    continue
                Ut, Uls, zi = op.zip_row(Ut, Uls, Ax[i], Dc, perturb=perturb)
                tied |= zi["near_tie"]
                if Ut is None:
                    break
            if Ut is None:
                val = (math.nan, 0) if zi["nonfinite"] else (-math.inf, 0)
            else:
                Dt, Dls = bot[b + 1]
                val = _row_value(Ut, Uls, Ax[b], Dt, Dls, perturb)
            lg, sg = val
            r = sg * den[b][1] * math.exp(lg - den[b][0]) if sg != 0 else (
                math.nan if math.isnan(lg) else 0.0)
            R[x, y] = R[y, x] = r
            tie[x, y] = tie[y, x] = tied
            if not math.isfinite(r):
                flags |= op.FLAG_NONFINITE
    return R, tie, flags


def transverse_sums(T, configs, Dc: int, window, ratios=None):
    """Sum over samples of O_pq(S) = 1/2 [s_p != s_q] R_pq (1/2 on the diagonal).

    Samples flagged ZERO_PSI or NONFINITE are left out.  ``ratios`` may hold
    the ratio matrices already computed for ``configs``.  Returns (sums, n).
    """
    N, M = len(T), len(T[0])
    sites = window_sites(N, M, window)
    nw = len(sites)
    tot = np.zeros((nw, nw))
    count = 0
    for k, S in enumerate(configs):
        R, _, fl = ratios[k] if ratios is not None else ratio_matrix(T, S, Dc, window)
        if fl & (op.FLAG_ZERO_PSI | op.FLAG_NONFINITE):
            continue
        count += 1
        tot += np.where(np.isnan(R), 0.0, 0.5 * R)
        tot[np.arange(nw), np.arange(nw)] += 0.5
    return tot, count


def spin_correlations(same, n_z, trans, n_t):
    """<S_p . S_q> = <S^z_p S^z_q> (from equal-spin counts) + the transverse average."""
    return observables.szsz(same, n_z) + np.asarray(trans, dtype=np.float64) / n_t
