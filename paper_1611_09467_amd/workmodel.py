"""Algorithmic work of one evaluation, per kernel class (host-side accounting).

Counts the floating-point operations (a multiply-add is 2) of the tensor
contractions each kernel performs, with the boundary-MPS bond dimensions that
the zip-up truncation produces (the same recurrence the library plans with),
and the antiparallel pairs of the actual configurations.  The truncation is
counted by the nominal thin-SVD convention 14 m n^2 + 8 n^3 (m >= n; 22 n^3
for a square block) and the LQ sweep by the Householder count
4 c r^2 - 4/3 r^3 for an r x c block (r <= c), whatever algorithm runs.
"""
from __future__ import annotations

import numpy as np

from .workloads import site_dims


def _row_bonds(M, D):
    return [1] + [D] * (M - 1) + [1]


def zip_shapes(N, M, D, Dc, chi_in, row, direction):
    pin, pout, dr, dl = [], [], [], []
    for j in range(M):
        l, r, u, d = site_dims(N, M, D, row, j)
        pin.append(u if direction == 0 else d)
        pout.append(d if direction == 0 else u)
        dr.append(r)
        dl.append(l)
    chic = [1] * (M + 1)
    for j in range(M - 1, 0, -1):
        chic[j] = min(chi_in[j], pin[j] * chic[j + 1])
    nb = [1] * (M + 1)
    for j in range(M - 1):
        nb[j + 1] = min(Dc, nb[j] * pout[j], chic[j + 1] * dr[j])
    return dict(pin=pin, pout=pout, dr=dr, dl=dl, chic=chic, nb=nb, chi_in=list(chi_in))


def envs(N, M, D, Dc):
    """Bond lists of every top (U_0..U_{N-2}) and bottom (Dn_1..Dn_{N-1}) environment."""
    top = {0: _row_bonds(M, D)}
    zt = {}
    for i in range(1, N - 1):
        zt[i] = zip_shapes(N, M, D, Dc, top[i - 1], i, 0)
        top[i] = zt[i]["nb"]
    bot = {N - 1: _row_bonds(M, D)}
    zb = {}
    for k in range(N - 2, 0, -1):
        zb[k] = zip_shapes(N, M, D, Dc, bot[k + 1], k, 1)
        bot[k] = zb[k]["nb"]
    return top, bot, zt, zb


def zip_flops(z):
    M = len(z["pin"])
    f_contract = f_trunc = f_lq = 0.0
    chi_in, chic, nb = z["chi_in"], z["chic"], z["nb"]
    for j in range(M - 1, 0, -1):
        r, c = chi_in[j], z["pin"][j] * chic[j + 1]
        if j < M - 1:
            f_contract += 2.0 * r * z["pin"][j] * chic[j + 1] * chi_in[j + 1]
        k = min(r, c)
        f_lq += 4.0 * max(r, c) * k * k - 4.0 / 3.0 * k ** 3
    f_contract += 2.0 * z["pin"][0] * chic[1] * chi_in[1]
    for j in range(M):
        Kd, Ad, Ld, Ud, Bd = nb[j], chic[j], z["dl"][j], z["pin"][j], chic[j + 1]
        Rd, Pd = z["dr"][j], z["pout"][j]
        f_contract += 2.0 * Kd * Ld * Ad * Ud * Bd + 2.0 * Kd * Bd * Ld * Ud * Rd * Pd
        rows, cols = Kd * Pd, Bd * Rd
        if j < M - 1:
            m, n = max(rows, cols), min(rows, cols)
            f_trunc += 14.0 * m * n * n + 8.0 * n ** 3
            f_contract += 2.0 * nb[j + 1] * rows * cols
    return f_contract, f_trunc, f_lq


def _upd1(Ad, Ld, Bd, Ud, Xd, Rd, Dd, Yd):
    return 2.0 * (Ld * Bd * Ad * Ud * Xd + Bd * Xd * Ud * Ld * Rd * Dd + Xd * Rd * Dd * Bd * Yd)


def _upd2(Ad, L1, L2, Bd, Ud, Xd, R1, Mm, R2, Dd, Yd):
    return 2.0 * Xd * (L1 * L2 * Bd * Ad * Ud + L2 * Bd * Ud * L1 * R1 * Mm
                       + Bd * R1 * L2 * Mm * R2 * Dd + R1 * R2 * Bd * Dd * Yd)


def evaluation_flops(N, M, D, Dc, configs, J2=0.5, want_grad=True, want_eloc=True):
    """Dict kernel_class -> total flops over the batch ``configs`` [B, N*M]."""
    S = np.asarray(configs).reshape(-1, N, M)
    B = S.shape[0]
    top, bot, zt, zb = envs(N, M, D, Dc)
    one = [1] * (M + 1)
    out = dict(zip=0.0, zip_truncation=0.0, zip_lq=0.0, sandwich=0.0, strip=0.0)
    for z in list(zt.values()) + list(zb.values()):
        c, t, q = zip_flops(z)
        out["zip"] += B * c
        out["zip_truncation"] += B * t
        out["zip_lq"] += B * q
    for i in range(N):
        ta = top[i - 1] if i >= 1 else one
        tb = bot[i + 1] if i + 1 <= N - 1 else one
        per_env = 0.0
        col = []
        for j in range(M):
            l, r, u, d = site_dims(N, M, D, i, j)
            c1 = _upd1(ta[j], l, tb[j], u, ta[j + 1], r, d, tb[j + 1])
            col.append(c1)
            per_env += c1  # right sweep
            if j < M - 1:
                per_env += c1  # left sweep
            if want_grad:
                per_env += 2.0 * tb[j] * d * tb[j + 1] * ta[j + 1] * r
                per_env += 2.0 * l * u * ta[j + 1] * tb[j] * r * d
        out["sandwich"] += B * per_env
        if want_eloc:
            anti = (S[:, i, :-1] != S[:, i, 1:])  # [B, M-1]
            # a ratio reuses T1 (first GEMM) for column j and does a full update for j+1
            for j in range(M - 1):
                l, r, u, d = site_dims(N, M, D, i, j)
                rest = col[j] - 2.0 * l * tb[j] * ta[j] * u * ta[j + 1]
                out["sandwich"] += anti[:, j].sum() * (rest + col[j + 1])
    if want_eloc:
        for i in range(N - 1):
            ta = top[i - 1] if i >= 1 else one
            tb = bot[i + 2] if i + 2 <= N - 1 else one
            col = []
            for j in range(M):
                l1, r1, u1, m1 = site_dims(N, M, D, i, j)
                l2, r2, m2, d2 = site_dims(N, M, D, i + 1, j)
                col.append(_upd2(ta[j], l1, l2, tb[j], u1, ta[j + 1], r1, m1, r2, d2, tb[j + 1]))
            env = sum(col) + sum(col[:-1])
            vert = (S[:, i, :] != S[:, i + 1, :]).astype(np.float64) @ np.asarray(col)
            f = B * env + vert.sum()
            if J2 != 0.0:
                d1 = (S[:, i, :-1] != S[:, i + 1, 1:]).astype(np.float64)
                d2 = (S[:, i, 1:] != S[:, i + 1, :-1]).astype(np.float64)
                pair = np.asarray([col[j] + col[j + 1] for j in range(M - 1)])
                f += (d1 @ pair).sum() + (d2 @ pair).sum()
            out["strip"] += f
    return out
