"""How sensitive each output of the truncated evaluation is to rounding.

TEST INFRASTRUCTURE ONLY (see the package header).

Why this exists.  With truncation (the boundary MPS cut to Dc, Fig. 1(d) and
the text after Eq. (2)), psi(S), E(S) and Delta are functions of every
intermediate of the evaluation: the blocks X whose leading singular subspace
is kept, and the running sandwich and strip environments.  A backward-stable
float64 evaluation -- LAPACK's SVD drivers, or the GPU's bidiagonal route --
returns the exact result for intermediates that carry relative errors of
order n u at every step (n the largest inner dimension of a step, u the unit
roundoff).  Two such evaluations therefore differ by about n u times the
derivative of the output along those errors; on some samples of the 10x10
D=6 Dc=12 workload that exceeds 1e-10 in psi even between LAPACK's gesdd and
gesvd.  The parity tests hold each sample to max(fixed bound, BOUND_FACTOR
n u kappa), with kappa estimated here.

Estimator: small-sample statistical condition estimation (C. S. Kenney and
A. J. Laub, SIAM J. Sci. Comput. 15 (1994) 36-61).  Every intermediate is
perturbed at once, X -> X + h ||X||_F Z / ||Z||_F with Z iid standard normal;
the change of each output, in the parity measures below, divided by h is
recorded; kappa is the largest over q independent draws.  h = 1e-9 keeps the
change first order for kappa up to ~1e7 and far above the rounding noise.
"""
from __future__ import annotations

import math

import numpy as np

from . import correlations, peps

UNIT_ROUNDOFF = 2.0 ** -53
# allowed difference between two evaluations, in units of n u kappa
BOUND_FACTOR = 16.0


def inner_dim(D: int, Dc: int) -> int:
    """Largest inner dimension of a step: the side chi D of a truncated block."""
    return max(D, Dc) * D


def differences(a: dict, b: dict, want_grad: bool = True):
    """Parity measures between two evaluations of one sample.

    psi: |sign_a exp(logabs_a - logabs_b) - sign_b|; E: |E_a - E_b| / max(1, |E_b|);
    Delta: ||Delta_a - Delta_b||_F / ||Delta_b||_F (zero when not wanted).
    """
    d_psi = abs(a["sign"] * math.exp(a["logabs"] - b["logabs"]) - b["sign"])
    d_e = abs(a["eloc"] - b["eloc"]) / max(1.0, abs(b["eloc"]))
    d_g = 0.0
    if want_grad:
        ga = np.concatenate([g.ravel() for g in a["grads"]])
        gb = np.concatenate([g.ravel() for g in b["grads"]])
        d_g = float(np.linalg.norm(ga - gb) / np.linalg.norm(gb))
    return np.array([d_psi, d_e, d_g])


def perturbation(rng: np.random.Generator, h: float):
    """X -> X + h ||X||_F Z / ||Z||_F for every intermediate the evaluation hands over."""
    def perturb(X):
        Z = rng.standard_normal(X.shape)
        nz = np.linalg.norm(Z)
        if nz == 0.0:
            return X
        return X + (h * np.linalg.norm(X) / nz) * Z
    return perturb


def kappa(T, S, Dc: int, J1: float = 1.0, J2: float = 0.0, want_grad: bool = True,
          q: int = 4, h: float = 1e-9, seed: int = 0):
    """(base evaluation, kappa as an array [psi, E, Delta]) for one configuration."""
    base = peps.evaluate(T, S, Dc, J1, J2, want_grad=want_grad)
    rng = np.random.Generator(np.random.PCG64(seed))
    best = np.zeros(3)
    for _ in range(q):
        o = peps.evaluate(T, S, Dc, J1, J2, want_grad=want_grad, perturb=perturbation(rng, h))
        best = np.maximum(best, differences(o, base, want_grad) / h)
    return base, best


def bound(kap, D: int, Dc: int):
    """Allowed difference of two backward-stable evaluations: BOUND_FACTOR n u kappa."""
    return BOUND_FACTOR * inner_dim(D, Dc) * UNIT_ROUNDOFF * np.asarray(kap)


def kappa_ratios(T, S, Dc: int, window, q: int = 4, h: float = 1e-9, seed: int = 0):
    """(base (R, tie, flags) of correlations.ratio_matrix, kappa per pair [n, n]):
    the relative change |R' - R| / max(1, |R|) of each exchange ratio, divided by h."""
    base = correlations.ratio_matrix(T, S, Dc, window)
    R0 = base[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    best = np.zeros_like(R0)
    for _ in range(q):
        R1, _, _ = correlations.ratio_matrix(T, S, Dc, window, perturb=perturbation(rng, h))
        d = np.abs(R1 - R0) / np.maximum(1.0, np.abs(R0)) / h
        best = np.fmax(best, np.where(np.isnan(R0), 0.0, d))
    return base, best
