"""The gradient-optimisation step: the Monte Carlo energy gradient of Eq. (3)
and the sign update of Eq. (6).

Test infrastructure only: nothing in the GPU library calls this module.

Eq. (3): dE/dA = 2 <Delta E> - 2 <Delta><E>, averages over configurations drawn
with weight W(S)^2; Delta of sample S lives on the slice A_ij = T_ij[s_ij], so
it accumulates into that physical index of the site tensor.
Eq. (6): A <- A - p dt sign(dE/dA), with p uniform in [0, 1] drawn per tensor
element (passed in).
"""
from __future__ import annotations

import numpy as np

from . import peps as op


def accumulate(T, configs, Dc: int, J1: float, J2: float, weights=None):
    """Sums over samples: (sum_delta, sum_delta_e, n, sum_e, sum_e2).

    sum_delta / sum_delta_e are lists (row-major sites) of arrays shaped like the
    site tensors [s, l, r, u, d].  Samples the evaluation flags ZERO_PSI or
    NONFINITE are skipped.  ``weights`` (one per sample, default 1) turns the
    sums into weighted ones, e.g. W^2/Z for an exact average over all
    configurations.
    """
    N, M = len(T), len(T[0])
    sd = [np.zeros_like(T[i][j]) for i in range(N) for j in range(M)]
    sde = [np.zeros_like(T[i][j]) for i in range(N) for j in range(M)]
    n = se = se2 = 0.0
    for b, S in enumerate(configs):
        w = 1.0 if weights is None else float(weights[b])
        o = op.evaluate(T, S, Dc, J1, J2, want_grad=True)
        if o["flags"] & (op.FLAG_ZERO_PSI | op.FLAG_NONFINITE):
            continue
        s = np.asarray(S).reshape(-1)
        E = o["eloc"]
        for k, g in enumerate(o["grads"]):
            sd[k][s[k]] += w * g
            sde[k][s[k]] += w * g * E
        n += w
        se += w * E
        se2 += w * E * E
    return sd, sde, n, se, se2


def gradient(sd, sde, n: float, se: float):
    """Eq. (3) from the sums: 2 <Delta E> - 2 <Delta> <E>."""
    return [2.0 * a / n - 2.0 * (b / n) * (se / n) for b, a in zip(sd, sde)]


def sign_update(T, grad, dt: float, p):
    """Eq. (6): every element moves by p dt against the sign of its derivative.

    ``p`` is a list of arrays shaped like the site tensors (uniform in [0, 1])."""
    N, M = len(T), len(T[0])
    out = []
    for i in range(N):
        row = []
        for j in range(M):
            k = i * M + j
            row.append(T[i][j] - p[k] * dt * np.sign(grad[k]))
        out.append(row)
    return out
