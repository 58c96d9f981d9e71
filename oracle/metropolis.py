"""Metropolis chains over S^z-conserving nearest-neighbour exchanges.

Test and input-generation infrastructure only: nothing in the GPU library
calls this module.

The energy and the gradient are Monte Carlo averages over configurations
drawn with probability proportional to W(S)^2 (paper, Sec. II, the
definition of E and of its derivative as sampled averages).  The paper does
not state its proposal; the reading used here is the usual S^z-conserving
one: pick a nearest-neighbour bond uniformly, and when its two spins differ
propose their exchange S -> S' and accept with probability
min(1, W(S')^2 / W(S)^2), the amplitudes being this oracle's float64
boundary-MPS values at the workload's Dc.  The configuration is recorded
after every step, accepted or not.  All random numbers (start configuration,
bond picks, acceptance uniforms) come in as arrays.
"""
from __future__ import annotations

import math


import numpy as np

from . import peps as op


def run_chain(T, Dc: int, start: np.ndarray, picks: np.ndarray, uniforms: np.ndarray,
              bonds) -> np.ndarray:
    """Configurations [steps][N*M] of one chain."""
    s = np.array(start, dtype=np.uint8)
    la, sg = op.psi_only(T, s, Dc)
    out = np.empty((len(picks), s.size), dtype=np.uint8)
    for t, (p, u) in enumerate(zip(picks, uniforms)):
        a, b = bonds[int(p)]
        if s[a] != s[b]:
            s2 = s.copy()
            s2[a], s2[b] = s[b], s[a]
            la2, sg2 = op.psi_only(T, s2, Dc)
            if sg2 != 0:
                if sg == 0:
                    accept = True  # leave a zero-weight start at the first nonzero proposal
                else:
                    accept = u < math.exp(min(0.0, 2.0 * (la2 - la)))
                if accept:
                    s, la, sg = s2, la2, sg2
        out[t] = s
    return out


def shared_ratio_step(T, Dc: int, S: np.ndarray, bond, u: float, J1: float = 1.0,
                      J2: float = 0.0):
    """One Metropolis step that takes W(S')/W(S) from the evaluation of S itself.

    The evaluation of the current configuration already holds the exchange
    ratio of every antiparallel nearest-neighbour pair (the shared-environment
    ratios of the local energy, Eq. (7)), so a step proposing the exchange on
    ``bond`` = (a, b) (row-major site indices, a < b, horizontal or vertical)
    accepts it with probability min(1, R^2) from that ratio R, with no second
    contraction.  Returns (evaluation of S, new configuration, accepted, R).
    """
    N, M = len(T), len(T[0])
    S = np.asarray(S, dtype=np.uint8).reshape(-1)
    out = op.evaluate(T, S, Dc, J1, J2, want_grad=False)
    a, b = int(bond[0]), int(bond[1])
    if S[a] == S[b] or out["flags"] & (op.FLAG_ZERO_PSI | op.FLAG_NONFINITE):
        return out, S.copy(), False, math.nan
    ia, ja, ib, jb = a // M, a % M, b // M, b % M
    kind = "h" if ia == ib else "v"
    R = out["ratios"][(kind, (ia, ja), (ib, jb))]
    accept = u < min(1.0, R * R)
    S2 = S.copy()
    if accept:
        S2[a], S2[b] = S[b], S[a]
    return out, S2, accept, R
