"""Boundary-MPS evaluation of one configuration of a finite open-boundary PEPS.

TEST INFRASTRUCTURE ONLY (see the package header).  Plain numpy/LAPACK in
float64, one sample at a time, no blocking or fusion.

What is computed (paper, Sec. II):
  * W(S) (the weight after Eq. (2)) of the single-layer network of fixed-spin
    slices A_ij = T_ij[s_ij] (Eq. (1)), by the boundary-MPS method of Fig. 1(d):
    rows are absorbed into a boundary MPS whose bond is truncated to Dc.
  * Delta_ij = B_ij / W (Eqs. (4)-(5)), B_ij = dW/dA_ij the four-index
    environment of site (i, j).
  * E(S) = sum_{S'} W(S')/W(S) <S'|H|S> for the J1-J2 model (Eq. (7)).

Readings where the paper is silent (each is listed in the design notes):
  R1  truncation = zip-up SVD.  Before a row is absorbed the boundary MPS is
      brought to right-canonical form by an exact LQ sweep; the row is then
      zipped in from the left and every two-column block X is cut by a thin
      SVD to chi = min(Dc, rows, cols) columns.  The paper says only that a
      boundary MPS with cut-off D_c1 is used (Fig. 1(d) and the text after
      Eq. (2)) and that a truncation is needed.
  R1b a truncation with relative gap (s[chi-1]-s[chi])/s[chi-1] <= 1e-8 is a
      near tie: the kept subspace is ill-defined; the sample is flagged.
  R2  each SVD step divides the carry by s[0] and adds log s[0] to a float64
      log-scale; the last column block is Frobenius-normalised the same way;
      row sandwiches and strips renormalise their running environments by their
      largest magnitude and keep the log.
  R3  the reported amplitude is psi = psi_{N-1} = <U_{N-2}| row N-1>, the pure
      top-down boundary contraction of Fig. 1(d).
  R4  Delta_ij = B_ij / psi_i with B_ij = d psi_i / dA_ij, psi_i the exact
      contraction <U_{i-1}| row i |Dn_{i+1}> (so <Delta_ij, A_ij> = 1).
  R5  W(S')/W(S) with shared environments: for a horizontal pair in row i the
      ratio of row-i sandwiches; for a vertical or diagonal pair in rows
      (i, i+1) the ratio of the exact two-row strips
      <U_{i-1}| row i, row i+1 |Dn_{i+2}>.
  R9  real tensors; sign in {-1, 0, +1}; W = 0 is flagged.

Environment conventions:
  top environment U_k: rows 0..k absorbed; tensors [a, p, a'] whose physical
      leg p is the down leg of row k.  U_{-1} is the trivial MPS.
  bottom environment Dn_k: rows k..N-1 absorbed; tensors [b, p, b'] whose
      physical leg p is the up leg of row k.  Dn_N is trivial.
"""
from __future__ import annotations

import math

import numpy as np

from . import hamiltonian

FLAG_ZERO_PSI = 1
FLAG_NONFINITE = 2
FLAG_NEAR_TIE = 4
NEAR_TIE_REL_GAP = 1e-8
# a kept singular value below this fraction of the largest one is numerically
# zero; no tie is reported for it
NEGLIGIBLE_REL_SV = 1e-13


def slices(T, S: np.ndarray):
    """A_ij = T_ij[s_ij], each [l, r, u, d] (Eq. (1))."""
    N, M = S.shape
    return [[T[i][j][int(S[i, j])] for j in range(M)] for i in range(N)]


# ---------------------------------------------------------------------------
# Boundary MPS (Fig. 1(d))
# ---------------------------------------------------------------------------

def row_as_mps(row, leg: str):
    """A single row read as an MPS: the open leg 'd' (top boundary) or 'u' (bottom)."""
    out = []
    for A in row:  # [l, r, u, d]
        if leg == "d":
            assert A.shape[2] == 1
            out.append(np.transpose(A[:, :, 0, :], (0, 2, 1)))  # [l, d, r]
        else:
            assert A.shape[3] == 1
            out.append(np.transpose(A[:, :, :, 0], (0, 2, 1)))  # [l, u, r]
    return out


def right_canonical(mps):
    """Exact LQ sweep from the right end down to site 1 (no truncation).

    Site j (j >= 1) becomes a matrix [a] x [(p, a')] with orthonormal rows; the
    bond becomes min(a, p*a') (the reduced factorisation).
    """
    mps = [t.copy() for t in mps]
    for j in range(len(mps) - 1, 0, -1):
        a, p, b = mps[j].shape
        q, r = np.linalg.qr(mps[j].reshape(a, p * b).T)  # mat^T = q r  =>  mat = r^T q^T
        k = q.shape[1]
        mps[j] = q.T.reshape(k, p, b)
        mps[j - 1] = np.tensordot(mps[j - 1], r.T, axes=([2], [0]))
    return mps


def thin_svd(X, driver: str = "gesdd"):
    """Thin SVD by LAPACK: divide and conquer (gesdd, numpy's default) or QR iteration (gesvd).

    The paper does not fix the SVD algorithm; both drivers are backward stable,
    and the spread of results between them measures how sensitive a truncated
    amplitude is to rounding.
    """
    if driver == "gesdd":
        return np.linalg.svd(X, full_matrices=False)
    import scipy.linalg as sl
    return sl.svd(X, full_matrices=False, lapack_driver=driver)


def zip_row(mps, log_scale: float, row, Dc: int, svd_driver: str = "gesdd", perturb=None):
    """Absorb ``row`` (slices [l, r, u, d]) into ``mps`` through the row's u legs.

    Returns (new_mps, new_log_scale, info) where the new MPS carries the row's
    d legs; info = dict(min_gap, zero, nonfinite, near_tie).  ``perturb``
    (used only to measure conditioning) maps every block X to the one that is
    cut.  A block with a NaN or an infinite entry stops the evaluation
    (flag NONFINITE).
    """
    M = len(row)
    mps = right_canonical(mps)
    C = np.ones((1, 1, 1))  # [k, a, l]
    out = []
    near_tie = False
    min_gap = math.inf
    for j in range(M):
        # X[k,d,b,r] = sum_{a,l,u} C[k,a,l] M_j[a,u,b] A_j[l,r,u,d]
        y = np.tensordot(C, mps[j], axes=([1], [0]))                  # [k,l,u,b]
        X4 = np.tensordot(y, row[j], axes=([1, 2], [0, 2]))          # [k,b,r,d]
        X4 = np.transpose(X4, (0, 3, 1, 2))                            # [k,d,b,r]
        k, d, b, r = X4.shape
        X = X4.reshape(k * d, b * r)
        if perturb is not None:
            X = perturb(X)
        if not np.all(np.isfinite(X)):
            return None, math.nan, dict(min_gap=min_gap, zero=False, nonfinite=True,
                                        near_tie=near_tie)
        if j < M - 1:
            U, s, Vt = thin_svd(X, svd_driver)
            chi = min(Dc, s.size)
            if s[0] == 0.0:
                return None, -math.inf, dict(min_gap=min_gap, zero=True, nonfinite=False,
                                             near_tie=near_tie)
            if chi < s.size and s[chi - 1] > NEGLIGIBLE_REL_SV * s[0]:
                gap = (s[chi - 1] - s[chi]) / s[chi - 1]
                min_gap = min(min_gap, gap)
                if gap <= NEAR_TIE_REL_GAP:
                    near_tie = True
            out.append(U[:, :chi].reshape(k, d, chi))
            C = (s[:chi, None] * Vt[:chi, :]).reshape(chi, b, r) / s[0]
            log_scale += math.log(s[0])
        else:
            nrm = np.linalg.norm(X)
            if nrm == 0.0:
                return None, -math.inf, dict(min_gap=min_gap, zero=True, nonfinite=False,
                                             near_tie=near_tie)
            out.append((X / nrm).reshape(k, d, b * r))
            log_scale += math.log(nrm)
    return out, log_scale, dict(min_gap=min_gap, zero=False, nonfinite=False, near_tie=near_tie)


def flip_row(row):
    """Exchange the u and d legs of every slice (used to absorb rows from below)."""
    return [np.transpose(A, (0, 1, 3, 2)) for A in row]


def trivial_mps(M: int):
    return [np.ones((1, 1, 1)) for _ in range(M)]


def environments(A, Dc: int, svd_driver: str = "gesdd", perturb=None):
    """Top environments U_{-1..N-2} and bottom environments Dn_{1..N} with log-scales."""
    N, M = len(A), len(A[0])
    info = dict(min_gap=math.inf, zero=False, nonfinite=False, near_tie=False)

    def merge(i2):
        info["min_gap"] = min(info["min_gap"], i2["min_gap"])
        info["zero"] |= i2["zero"]
        info["nonfinite"] |= i2["nonfinite"]
        info["near_tie"] |= i2["near_tie"]

    top = {-1: (trivial_mps(M), 0.0)}
    top[0] = (row_as_mps(A[0], "d"), 0.0)
    for k in range(1, N - 1):
        mps, ls = top[k - 1]
        if mps is None:
            top[k] = (None, -math.inf)
            continue
        new, ls2, i2 = zip_row(mps, ls, A[k], Dc, svd_driver, perturb)
        merge(i2)
        top[k] = (new, ls2)
    bot = {N: (trivial_mps(M), 0.0)}
    bot[N - 1] = (row_as_mps(A[N - 1], "u"), 0.0)
    for k in range(N - 2, 0, -1):
        mps, ls = bot[k + 1]
        if mps is None:
            bot[k] = (None, -math.inf)
            continue
        new, ls2, i2 = zip_row(mps, ls, flip_row(A[k]), Dc, svd_driver, perturb)
        merge(i2)
        bot[k] = (new, ls2)
    return top, bot, info


# ---------------------------------------------------------------------------
# Row sandwiches <U_{i-1}| row i |Dn_{i+1}>: amplitude, gradients, horizontal ratios
# ---------------------------------------------------------------------------

def _normalise(t, perturb=None):
    if perturb is not None and t.size:
        t = perturb(t)
    m = float(np.max(np.abs(t))) if t.size else 0.0
    if m == 0.0 or not np.isfinite(m):
        return t, m
    return t / m, m


def _col1(E, Ut, A, Dt):
    """Left environment [a, l, b] times one sandwich column -> [a', r, b']."""
    # E'[x,r,y] = sum E[a,l,b] U[a,u,x] A[l,r,u,d] Dn[b,d,y]
    t = np.tensordot(E, Ut, axes=([0], [0]))                  # [l,b,u,x]
    t = np.tensordot(t, A, axes=([0, 2], [0, 2]))             # [b,x,r,d]
    return np.tensordot(t, Dt, axes=([0, 3], [0, 1]))         # [x,r,y]


def _col1_right(E, Ut, A, Dt):
    """Column times right environment [a', r, b'] -> [a, l, b]."""
    # E'[a,l,b] = sum U[a,u,x] A[l,r,u,d] Dn[b,d,y] E[x,r,y]
    t = np.tensordot(Ut, E, axes=([2], [0]))                  # [a,u,r,y]
    t = np.tensordot(t, A, axes=([1, 2], [2, 1]))             # [a,y,l,d]
    return np.tensordot(t, Dt, axes=([1, 3], [2, 1]))         # [a,l,b]


def sandwich(Ut, Uls, row, Dt, Dls, J1=None, S_row=None, T_row=None, perturb=None):
    """Exact contraction of one row between its top and bottom environments.

    Returns dict with logabs/sign of psi_i, the list of Delta_ij = B_ij/psi_i,
    and the horizontal exchange ratios {j: psi_i(S_j<->j+1)/psi_i(S)} for every
    antiparallel pair in the row (needs S_row and T_row = full site tensors).
    """
    M = len(row)
    RE = [None] * (M + 1)
    RL = [0.0] * (M + 1)
    RE[M] = np.ones((1, 1, 1))
    for j in range(M - 1, -1, -1):
        t, m = _normalise(_col1_right(RE[j + 1], Ut[j], row[j], Dt[j]), perturb)
        if m == 0.0 or not np.isfinite(m):
            return dict(zero=True, nonfinite=not np.isfinite(m))
        RE[j], RL[j] = t, RL[j + 1] + math.log(m)
    psi_raw = float(RE[0].reshape(()))
    if psi_raw == 0.0 or not np.isfinite(psi_raw):
        return dict(zero=psi_raw == 0.0, nonfinite=not np.isfinite(psi_raw))
    logabs = RL[0] + math.log(abs(psi_raw)) + Uls + Dls
    sign = 1 if psi_raw > 0 else -1
    LE = [None] * (M + 1)
    LL = [0.0] * (M + 1)
    LE[0] = np.ones((1, 1, 1))
    grads = []
    for j in range(M):
        # B[l,r,u,d] = sum LE[a,l,b] U[a,u,x] Dn[b,d,y] RE[x,r,y]   (Eq. (5))
        t1 = np.tensordot(LE[j], Ut[j], axes=([0], [0]))          # [l,b,u,x]
        q = np.tensordot(Dt[j], RE[j + 1], axes=([2], [2]))       # [b,d,x,r]
        B = np.tensordot(t1, q, axes=([1, 3], [0, 2]))            # [l,u,d,r]
        B = np.transpose(B, (0, 3, 1, 2))
        grads.append(B / psi_raw * math.exp(LL[j] + RL[j + 1] - RL[0]))
        t, m = _normalise(_col1(LE[j], Ut[j], row[j], Dt[j]), perturb)
        LE[j + 1], LL[j + 1] = t, LL[j] + (math.log(m) if m > 0 else -math.inf)
    ratios = {}
    if S_row is not None:
        for j in range(M - 1):
            sa, sb = int(S_row[j]), int(S_row[j + 1])
            if sa == sb:
                continue
            Aa = T_row[j][sb]
            Ab = T_row[j + 1][sa]
            E1 = _col1(LE[j], Ut[j], Aa, Dt[j])
            val = np.einsum("xry,xry->", _col1(E1, Ut[j + 1], Ab, Dt[j + 1]), RE[j + 2])
            ratios[j] = float(val) / psi_raw * math.exp(LL[j] + RL[j + 2] - RL[0])
    return dict(zero=False, nonfinite=False, logabs=logabs, sign=sign, grads=grads,
                ratios=ratios)


# ---------------------------------------------------------------------------
# Two-row strips <U_{i-1}| row i, row i+1 |Dn_{i+2}>: vertical and diagonal ratios
# ---------------------------------------------------------------------------

def _col2(E, Ut, A1, A2, Dt):
    """Strip left environment [a, l1, l2, b] times one two-site column -> [a', r1, r2, b']."""
    # E'[x,r,s,y] = sum E[a,p,q,b] U[a,u,x] A1[p,r,u,m] A2[q,s,m,d] Dn[b,d,y]
    t = np.tensordot(E, Ut, axes=([0], [0]))                  # [p,q,b,u,x]
    t = np.tensordot(t, A1, axes=([0, 3], [0, 2]))            # [q,b,x,r,m]
    t = np.tensordot(t, A2, axes=([0, 4], [0, 2]))            # [b,x,r,s,d]
    return np.tensordot(t, Dt, axes=([0, 4], [0, 1]))         # [x,r,s,y]


def _col2_right(E, Ut, A1, A2, Dt):
    # E'[a,p,q,b] = sum U[a,u,x] A1[p,r,u,m] A2[q,s,m,d] Dn[b,d,y] E[x,r,s,y]
    t = np.tensordot(Ut, E, axes=([2], [0]))                  # [a,u,r,s,y]
    t = np.tensordot(t, A1, axes=([1, 2], [2, 1]))            # [a,s,y,p,m]
    t = np.tensordot(t, A2, axes=([1, 4], [1, 2]))            # [a,y,p,q,d]
    return np.tensordot(t, Dt, axes=([1, 4], [2, 1]))         # [a,p,q,b]


def strip(Ut, row1, row2, Dt, S1, S2, T1, T2, perturb=None):
    """Exchange ratios for vertical (i,j)-(i+1,j) and diagonal pairs of rows (i, i+1).

    Returns dict(zero, ratios) with ratios keyed by ('v', j), ('d1', j) for
    (i,j)-(i+1,j+1) and ('d2', j) for (i,j+1)-(i+1,j).
    """
    M = len(row1)
    RE = [None] * (M + 1)
    RL = [0.0] * (M + 1)
    RE[M] = np.ones((1, 1, 1, 1))
    for j in range(M - 1, -1, -1):
        t, m = _normalise(_col2_right(RE[j + 1], Ut[j], row1[j], row2[j], Dt[j]), perturb)
        if m == 0.0 or not np.isfinite(m):
            return dict(zero=True, nonfinite=not np.isfinite(m))
        RE[j], RL[j] = t, RL[j + 1] + math.log(m)
    val0 = float(RE[0].reshape(()))
    if val0 == 0.0 or not np.isfinite(val0):
        return dict(zero=val0 == 0.0, nonfinite=not np.isfinite(val0))
    LE = [None] * (M + 1)
    LL = [0.0] * (M + 1)
    LE[0] = np.ones((1, 1, 1, 1))
    ratios = {}
    for j in range(M):
        a, b = int(S1[j]), int(S2[j])
        if a != b:  # vertical exchange in column j
            E1 = _col2(LE[j], Ut[j], T1[j][b], T2[j][a], Dt[j])
            v = float(np.einsum("xrsy,xrsy->", E1, RE[j + 1]))
            ratios[("v", j)] = v / val0 * math.exp(LL[j] + RL[j + 1] - RL[0])
        if j < M - 1:
            c, e = int(S1[j + 1]), int(S2[j + 1])
            if a != e:  # (i,j) <-> (i+1,j+1)
                E1 = _col2(LE[j], Ut[j], T1[j][e], row2[j], Dt[j])
                E2 = _col2(E1, Ut[j + 1], row1[j + 1], T2[j + 1][a], Dt[j + 1])
                v = float(np.einsum("xrsy,xrsy->", E2, RE[j + 2]))
                ratios[("d1", j)] = v / val0 * math.exp(LL[j] + RL[j + 2] - RL[0])
            if c != b:  # (i,j+1) <-> (i+1,j)
                E1 = _col2(LE[j], Ut[j], row1[j], T2[j][c], Dt[j])
                E2 = _col2(E1, Ut[j + 1], T1[j + 1][b], row2[j + 1], Dt[j + 1])
                v = float(np.einsum("xrsy,xrsy->", E2, RE[j + 2]))
                ratios[("d2", j)] = v / val0 * math.exp(LL[j] + RL[j + 2] - RL[0])
        t, m = _normalise(_col2(LE[j], Ut[j], row1[j], row2[j], Dt[j]), perturb)
        LE[j + 1], LL[j + 1] = t, LL[j] + (math.log(m) if m > 0 else -math.inf)
    return dict(zero=False, nonfinite=False, ratios=ratios)


# ---------------------------------------------------------------------------
# Whole evaluation of one sample
# ---------------------------------------------------------------------------

def evaluate(T, S: np.ndarray, Dc: int, J1: float = 1.0, J2: float = 0.0,
             want_grad: bool = True, want_eloc: bool = True, svd_driver: str = "gesdd",
             perturb=None) -> dict:
    """Per-sample outputs: logabs, sign, eloc, grads (list over sites, row-major), flags.

    ``S`` is (N, M) or flat of length N*M.  ``T`` is the nested list of site
    tensors [s, l, r, u, d].  Also returns ``row_logabs`` (log|psi_i| per row)
    and ``min_gap`` (smallest relative gap at any truncation) as diagnostics.
    """
    N, M = len(T), len(T[0])
    S = np.asarray(S).reshape(N, M)
    A = slices(T, S)
    top, bot, info = environments(A, Dc, svd_driver, perturb)
    flags = FLAG_NEAR_TIE if info["near_tie"] else 0
    nan_out = dict(logabs=-math.inf, sign=0, eloc=math.nan,
                   grads=[np.full(A[i][j].shape, math.nan) for i in range(N) for j in range(M)]
                   if want_grad else None, flags=flags | FLAG_ZERO_PSI,
                   row_logabs=None, min_gap=info["min_gap"])
    if info["nonfinite"]:
        nan_out["flags"] = flags | FLAG_NONFINITE
        nan_out["logabs"] = math.nan
        return nan_out
    if info["zero"]:
        return nan_out
    grads = []
    row_logabs = []
    logabs = sign = None
    ratio = {}
    for i in range(N):
        Ut, Uls = top[i - 1]
        Dt, Dls = bot[i + 1]
        sw = sandwich(Ut, Uls, A[i], Dt, Dls, S_row=S[i], T_row=T[i], perturb=perturb)
        if sw.get("nonfinite"):
            nan_out["flags"] = flags | FLAG_NONFINITE
            nan_out["logabs"] = math.nan
            return nan_out
        if sw["zero"]:
            return nan_out
        row_logabs.append(sw["logabs"])
        grads.extend(sw["grads"])
        for j, r in sw["ratios"].items():
            ratio[("h", (i, j), (i, j + 1))] = r
        if i == N - 1:
            logabs, sign = sw["logabs"], sw["sign"]
    if want_eloc:
        for i in range(N - 1):
            Ut, _ = top[i - 1]
            Dt, _ = bot[i + 2]
            st = strip(Ut, A[i], A[i + 1], Dt, S[i], S[i + 1], T[i], T[i + 1], perturb=perturb)
            if st.get("nonfinite"):
                nan_out["flags"] = flags | FLAG_NONFINITE
                nan_out["logabs"] = math.nan
                return nan_out
            if st["zero"]:
                return nan_out
            for (kind, j), r in st["ratios"].items():
                if kind == "v":
                    ratio[("v", (i, j), (i + 1, j))] = r
                elif kind == "d1":
                    ratio[("d1", (i, j), (i + 1, j + 1))] = r
                else:
                    ratio[("d2", (i, j + 1), (i + 1, j))] = r
        eloc = hamiltonian.local_energy(S, J1, J2, lambda kind, a, b: ratio[(kind, a, b)])
    else:
        eloc = math.nan
    out_flags = flags
    if not (np.isfinite(logabs) and np.isfinite(eloc if want_eloc else 0.0)):
        out_flags |= FLAG_NONFINITE
    return dict(logabs=logabs, sign=sign, eloc=eloc, grads=grads if want_grad else None,
                flags=out_flags, row_logabs=row_logabs, min_gap=info["min_gap"], ratios=ratio)


def psi_only(T, S: np.ndarray, Dc: int):
    """(logabs, sign) of psi = <U_{N-2}| row N-1> without gradients or energies."""
    N, M = len(T), len(T[0])
    S = np.asarray(S).reshape(N, M)
    A = slices(T, S)
    top = (row_as_mps(A[0], "d"), 0.0)
    for k in range(1, N - 1):
        new, ls, info = zip_row(top[0], top[1], A[k], Dc)
        if new is None:
            return -math.inf, 0
        top = (new, ls)
    Dt = trivial_mps(M)
    sw = sandwich(top[0], top[1], A[N - 1], Dt, 0.0)
    if sw["zero"] or sw.get("nonfinite"):
        return -math.inf, 0
    return sw["logabs"], sw["sign"]
