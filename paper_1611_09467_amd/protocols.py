"""The optimisation protocols of Sec. III, driven through the device entry points.

  go_schedule   step lengths dt(n) and sample counts M(n) of the gradient
                optimisation (Sec. III, Fig. 2): 50 steps at dt = 0.005 with M
                rising from 5e4 to 1e5; 50 steps with dt(n+1) = 0.968 dt(n)
                (0.005 down to about 0.001) with M rising to 5e5; 20 steps at
                dt = 0.001 and M = 5e5.
  su_converge   imaginary-time simple update until no tensor element changes
                by 1e-6 or more (relative) in one step of dtau, first with
                dtau = 0.01 and then with dtau = 0.001 (Sec. III).
  d_ramp        start from a random PEPS at a small D, converge it, pad it to
                the next D and converge again, up to the target (Sec. III).
  go_steps      gradient steps: Metropolis sweeps of resident chains, the
                Eq. (3) sums over M samples (REDUCED evaluations), the Eq. (6)
                sign update with p drawn uniformly in [0, 1] per element.
  exact_energy  <psi|H|psi>/<psi|psi> of a small lattice by enumerating every
                S^z = 0 configuration with weight W^2 (evaluations at a Dc that
                truncates nothing).

Readings where the paper leaves details open (listed in the design notes):
the growth of M inside a phase is linear in the step index; a schedule may be
scaled (fewer steps, smaller M) keeping its phases; the convergence test skips
elements below 1e-12 of the largest magnitude of their tensor (their relative
change is undefined) and checks one step of every ``check_every``.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import binding as bd


def go_schedule(first: int = 50, decay: int = 50, last: int = 20, dt0: float = 0.005,
                factor: float = 0.968, dt_last: float = 0.001, m0: int = 50000,
                m1: int = 100000, m_max: int = 500000):
    """[(dt, M)] per gradient step of the three phases of Sec. III."""
    out = []
    for n in range(first):
        m = m0 + (m1 - m0) * n / max(1, first - 1)
        out.append((dt0, int(round(m))))
    dt = dt0
    for n in range(decay):
        dt *= factor
        m = m1 + (m_max - m1) * (n + 1) / decay
        out.append((dt, int(round(m))))
    for n in range(last):
        out.append((dt_last, m_max))
    return out


def _represented(P):
    return P.read()


def su_converge(P, gamma, lambdas, J1: float = 1.0, dtaus=(0.01, 0.001), tol: float = 1e-6,
                check_every: int = 50, max_steps: int = 20000):
    """Simple update of (gamma, lambdas) in place until converged at each dtau in turn.

    Returns [(dtau, steps taken, converged, last max relative change)].
    Loads the represented PEPS into ``P`` (as pepsgo_su_to_peps does).
    """
    import torch
    log = []
    for dtau in dtaus:
        steps, change, done = 0, float("inf"), False
        while steps < max_steps:
            if check_every > 1:
                P.su_evolve(gamma, lambdas, J1, dtau, check_every - 1)
            P.su_to_peps(gamma, lambdas)
            before = _represented(P).clone()
            P.su_evolve(gamma, lambdas, J1, dtau, 1)
            P.su_to_peps(gamma, lambdas)
            after = _represented(P)
            steps += check_every
            change = _max_rel_change(P, before, after)
            if change < tol:
                done = True
                break
        torch.cuda.synchronize()
        log.append((dtau, steps, done, change))
    return log


def _max_rel_change(P, before, after) -> float:
    """Largest |after - before| / |before| over elements of non-negligible magnitude,
    site tensor by site tensor."""
    import torch
    worst = 0.0
    off = 0
    from .workloads import site_sizes
    for n in site_sizes(P.N, P.M, P.D):
        a, b = before[off:off + n], after[off:off + n]
        big = a.abs() > 1e-12 * a.abs().max()
        if bool(big.any()):
            worst = max(worst, float(((b - a).abs()[big] / a.abs()[big]).max()))
        off += n
    return worst


def d_ramp(ctx, N: int, M: int, Ds, seed: int = 0, J1: float = 1.0, **converge):
    """Random PEPS at Ds[0], converged by su_converge, padded to each next D and
    converged again.  Returns (Peps handle at Ds[-1], gamma, lambdas, logs)."""
    from . import workloads as wl
    P = bd.Peps(ctx, N, M, Ds[0], wl.pack_peps(wl.make_peps(N, M, Ds[0], seed=seed)))
    gam, lam = P.su_start()
    logs = [su_converge(P, gam, lam, J1, **converge)]
    for D in Ds[1:]:
        Q = bd.Peps(ctx, N, M, D, wl.pack_peps(wl.make_peps(N, M, D, seed=seed)))
        gam, lam = P.su_pad(gam, lam, Q)
        P.free()
        P = Q
        logs.append(su_converge(P, gam, lam, J1, **converge))
    return P, gam, lam, logs


def go_steps(P, cfg, schedule, Dc: int, J1: float = 1.0, J2: float = 0.0,
             sweeps: int = 1, precision: int = bd.PEPSGO_FP32, seed: int = 0):
    """Gradient steps over resident chains ``cfg`` (uint8 [B, N*M], updated in place).

    Per (dt, M) of ``schedule``: ceil(M / B) rounds of ``sweeps`` Metropolis sweeps
    followed by one REDUCED evaluation of every chain into the Eq. (3) sums, then the
    Eq. (6) update.  Returns [(dt, samples, <E>/site estimate)] per step.
    """
    import torch
    dev = cfg.device
    B = cfg.shape[0]
    gen = torch.Generator(dev).manual_seed(seed)
    hist = []
    for dt, m in schedule:
        sums = P.new_sums(dev)
        for _ in range(max(1, -(-m // B))):
            for _ in range(sweeps):
                u = torch.rand((B, P.nbonds), dtype=torch.float64, device=dev, generator=gen)
                P.metropolis_sweep(cfg, u, Dc)
            P.evaluate(cfg, Dc, J1, J2, precision=precision, sums=sums)
        p = torch.rand(P.nparams, dtype=torch.float64, device=dev, generator=gen)
        P.go_update(sums, dt, p)
        st = sums["stats"].cpu().numpy()
        hist.append((dt, int(st[0]), float(st[1] / st[0]) / (P.N * P.M) if st[0] else float("nan")))
    return hist


def sz0_configs(N: int, M: int) -> np.ndarray:
    """Every configuration with N M / 2 labels 1 (S^z = 0), uint8 [K, N*M]."""
    n = N * M
    out = []
    for ones in itertools.combinations(range(n), n // 2):
        c = np.zeros(n, dtype=np.uint8)
        c[list(ones)] = 1
        out.append(c)
    return np.array(out)


def exact_energy(P, J1: float = 1.0, J2: float = 0.0, Dc: int | None = None) -> float:
    """Energy per site of the loaded PEPS by exact enumeration of the S^z = 0 sector:
    sum_S W^2 E(S) / sum_S W^2 with W and E(S) from evaluations at a Dc that
    truncates nothing (D^ceil(M/2) by default)."""
    import torch
    Dc = Dc or P.D ** ((P.M + 1) // 2)
    S = torch.from_numpy(sz0_configs(P.N, P.M)).cuda()
    out = P.evaluate(S, Dc, J1, J2, precision=bd.PEPSGO_FP64, want_grad=False)
    la = out["logabs"].cpu().numpy()
    e = out["eloc"].cpu().numpy()
    keep = np.isfinite(la)
    w = np.exp(2.0 * (la[keep] - la[keep].max()))
    return float(np.sum(w * e[keep]) / np.sum(w)) / (P.N * P.M)
