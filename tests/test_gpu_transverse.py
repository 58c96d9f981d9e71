"""Transverse correlations on the device (pepsgo_transverse) against the oracle.

Per sample and window pair, the exchange ratio R_pq = W(S^{pq})/W(S) of the
GPU against oracle.correlations.ratio_matrix: relative error
|R_g - R_o| / max(1, |R_o|) within 1e-9 (a ratio of two amplitudes, each
held to 1e-10, passes through one more division), or, where a pair misses
it, within 16 n u kappa_pq of the oracle's estimate of that ratio's
sensitivity to rounding (the same reading as for psi).  Flags, the sums of
1/2 R_pq and the counted samples are compared too; exact-regime cases
against brute-force ratios.
"""
import math

import numpy as np
import pytest

from oracle import brute, conditioning as cond, correlations, observables
from oracle import peps as op
from paper_1611_09467_amd import binding as bd
from paper_1611_09467_amd import workloads as wl
from oracle_pool import OraclePool

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIXED = 1e-9


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    c = bd.Context(0)
    yield c
    c.close()


def run(P, S, window, Dc, max_ws=0, want_ratios=True):
    cfg = torch.from_numpy(np.ascontiguousarray(S)).cuda()
    acc, flags, rat = P.transverse(cfg, window, Dc, want_ratios=want_ratios,
                                   max_workspace_bytes=max_ws)
    torch.cuda.synchronize()
    return (acc["sums"].cpu().numpy(), int(acc["n"].cpu().item()),
            flags.cpu().numpy().astype(np.uint32), None if rat is None else rat.cpu().numpy())


def compare(T, S, D, Dc, window, flags, rat, idx):
    """Every sample in idx against the oracle; prints and returns the counts."""
    idx = list(idx)
    with OraclePool(T, Dc, want_grad=False) as pool:
        orc = pool.ratios([S[b] for b in idx], window)
        pairs = fine = ties = 0
        miss = []
        worst = 0.0
        for b, (R, tie, fl) in zip(idx, orc):
            fg = int(flags[b])
            if (fg | fl) & op.FLAG_NEAR_TIE:
                ties += 1
                continue
            assert (fg & 3) == (fl & 3), (b, fg, fl)
            if fl & 3:
                assert np.all(np.isnan(rat[b])), b
                continue
            m = ~np.isnan(R)
            assert np.array_equal(m, ~np.isnan(rat[b])), b
            d = np.abs(rat[b][m] - R[m]) / np.maximum(1.0, np.abs(R[m]))
            pairs += int(m.sum())
            worst = max(worst, float(d.max(initial=0.0)))
            fine += int(np.sum(d <= 1e-12))
            if np.any(d > FIXED):
                miss.append((b, R))
        kaps = pool.kappa_ratios([S[b] for b, _ in miss], window) if miss else []
    units = []
    nmiss = 0
    for (b, R), k in zip(miss, kaps):
        m = ~np.isnan(R)
        d = np.abs(rat[b] - R) / np.maximum(1.0, np.abs(R))
        over = m & (d > FIXED)
        lim = cond.bound(k, D, Dc)
        assert np.all(d[over] <= lim[over]), (b, d[over], lim[over])
        nmiss += int(over.sum())
        scale = lim[over] / cond.BOUND_FACTOR
        units.extend(list(d[over] / np.maximum(scale, 1e-300)))
    extra = ""
    if units:
        extra = f"; their errors {np.median(units):.2g} (median), {np.max(units):.2g} (max) n u kappa"
    print(f"  {len(idx) - ties} samples, {pairs} pairs: {fine} within 1e-12, {nmiss} pairs outside "
          f"{FIXED:g} and within their conditioning bound, {ties} samples with near ties "
          f"excluded; worst {worst:.3g}{extra}", flush=True)
    return dict(pairs=pairs, miss=nmiss, worst=worst)


@pytest.mark.parametrize("N,M,D,Dc,window", [
    (3, 4, 2, 3, (0, 0, 3, 4)),      # whole lattice, both edges
    (5, 4, 3, 4, (1, 1, 3, 2)),      # interior window
    (4, 6, 2, 3, (2, 0, 2, 6)),      # last rows, full width
    (6, 5, 3, 5, (0, 2, 6, 1)),      # one column, every row
    (2, 2, 1, 1, (0, 0, 2, 2)),      # D = 1
])
def test_ratios_match_oracle_small(ctx, N, M, D, Dc, window):
    T = wl.make_peps(N, M, D, seed=N * 13 + M, bias=0.1)
    S = wl.random_sz0_configs(N, M, 10, N + 5 * M)
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(T))
    print(f"[gpu] transverse {N}x{M} D={D} Dc={Dc} window {window}, 10 samples", flush=True)
    sums, n, flags, rat = run(P, S, window, Dc)
    compare(T, S, D, Dc, window, flags, rat, range(len(S)))
    want, n_o = correlations.transverse_sums(T, S, Dc, window)
    assert n == n_o
    assert np.allclose(sums, want, rtol=1e-9, atol=1e-9)
    P.free()


def test_exact_regime_against_brute_force(ctx):
    N, M, D = 3, 3, 2
    Dc = 16
    T = wl.make_peps(N, M, D, seed=91)
    S = wl.random_sz0_configs(N, M, 6, 92)
    window = (0, 0, 3, 3)
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(T))
    print(f"[gpu] transverse exact regime {N}x{M} D={D} Dc={Dc}", flush=True)
    _, _, flags, rat = run(P, S, window, Dc)
    assert np.all(flags == 0)
    sites = correlations.window_sites(N, M, window)
    for b, s in enumerate(S):
        w0 = brute.amplitude(T, s.reshape(N, M))
        for x, p in enumerate(sites):
            for y, q in enumerate(sites):
                if x == y or s[p] == s[q]:
                    assert math.isnan(rat[b, x, y])
                    continue
                t = s.copy()
                t[p], t[q] = s[q], s[p]
                want = brute.amplitude(T, t.reshape(N, M)) / w0
                assert abs(rat[b, x, y] - want) <= 1e-12 * max(1.0, abs(want)), (b, p, q)
    P.free()


def test_bulk_window_10x10_and_chunking(ctx):
    # the 10x10 D=6 Dc=12 chain states on the (L-2)^2 bulk window
    T, S = wl.workload_inputs("10x10_D6_Dc12")
    window = (1, 1, 8, 8)
    S = S[::512][:32].copy()
    P = bd.Peps(ctx, 10, 10, 6, wl.pack_peps(T))
    print(f"[gpu] transverse 10x10 D=6 Dc=12 window {window}, {len(S)} samples", flush=True)
    sums, n, flags, rat = run(P, S, window, 12)
    print("[gpu] transverse 10x10 in chunks of 5 samples", flush=True)
    per = bd.pepsgo_transverse_workspace_bytes(P.handle, bd.make_params(12), *window, 1)
    sums5, n5, flags5, _ = run(P, S, window, 12, max_ws=5 * per, want_ratios=False)
    assert n5 == n and np.array_equal(flags5, flags)
    assert np.array_equal(sums5, sums)          # pairs add their samples in order
    compare(T, S, 6, 12, window, flags, rat, range(8))
    P.free()


def test_flags_and_empty_batch(ctx):
    N, M, D, Dc = 4, 4, 2, 3
    window = (1, 1, 2, 2)
    # NaN in the other slice of one site: only exchanged configurations that
    # flip that site see it (those samples are flagged NONFINITE, not counted)
    T = wl.make_peps(N, M, D, seed=93)
    T[1][1][1][...] = np.nan
    S = wl.random_sz0_configs(N, M, 8, 94)
    S[:, 5] = 0
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(T))
    print("[gpu] transverse flags: NaN slice", flush=True)
    sums, n, flags, rat = run(P, S, window, Dc)
    want = [correlations.ratio_matrix(T, s, Dc, window) for s in S]
    for b, (R, tie, fl) in enumerate(want):
        assert (int(flags[b]) & 3) == (fl & 3), (b, flags[b], fl)
    assert n == sum(1 for R, _, fl in want if not fl & 3)
    assert n < len(S)
    P.free()
    # Neel product PEPS: only the Neel configuration has W != 0
    Tn = wl.neel_product_peps(N, M)
    neel = wl.neel_config(N, M)
    other = neel.copy()
    other[0], other[1] = neel[1], neel[0]
    P = bd.Peps(ctx, N, M, 1, wl.pack_peps(Tn))
    print("[gpu] transverse flags: Neel product state", flush=True)
    sums, n, flags, rat = run(P, np.stack([neel, other]), window, Dc)
    assert n == 1 and flags[1] & op.FLAG_ZERO_PSI and not flags[0] & 3
    off = sums - np.diag(np.diag(sums))
    assert np.all(off == 0.0) and np.allclose(np.diag(sums), 0.5)
    assert np.all(np.isnan(rat[1]))
    # an empty batch changes nothing
    cfg = torch.zeros((0, N * M), dtype=torch.uint8, device="cuda")
    acc, fl, _ = P.transverse(cfg, window, Dc)
    torch.cuda.synchronize()
    assert int(acc["n"].item()) == 0 and float(acc["sums"].abs().sum()) == 0.0
    P.free()


def test_spin_structure_factor(ctx):
    N, M, D, Dc = 5, 5, 2, 4
    T = wl.make_peps(N, M, D, seed=95, bias=0.1)
    S = wl.random_sz0_configs(N, M, 12, 96)
    window = (1, 1, 3, 3)
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(T))
    print("[gpu] spin structure factor 5x5 window (1,1,3,3)", flush=True)
    cfg = torch.from_numpy(S).cuda()
    trans, flags, _ = P.transverse(cfg, window, Dc)
    counts = bd.sz_correlations(cfg, N, M, window, flags=flags)
    ms = bd.spin_structure_factor(counts, trans, math.pi, math.pi)
    torch.cuda.synchronize()
    tot, n_t = correlations.transverse_sums(T, S, Dc, window)
    keep = np.array([not int(f) & 3 for f in flags.cpu().numpy()])
    same, n_z = observables.same_counts(S, N, M, *window, keep=keep)
    C = correlations.spin_correlations(same, n_z, tot, n_t)
    want = observables.structure_factor(C, 3, 3, math.pi, math.pi)
    assert float(ms.item()) == pytest.approx(want, rel=1e-12, abs=1e-14)
    P.free()


def test_window_errors(ctx):
    N, M, D = 4, 4, 2
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(wl.make_peps(N, M, D, seed=1)))
    cfg = torch.zeros((2, N * M), dtype=torch.uint8, device="cuda")
    for window in ((0, 0, 5, 1), (3, 0, 2, 1), (0, -1, 1, 1), (0, 0, 0, 2)):
        with pytest.raises(bd.PepsgoError):
            P.transverse(cfg, window, 2)
    P.free()
