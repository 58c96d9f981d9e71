"""Device Metropolis sweeps (pepsgo_metropolis_sweep) against oracle.sweep.

Each chain's sweep is replayed by the oracle from the configuration the GPU
started from, with the same uniforms: every decision, every ratio (to the
float64 parity bound) and the final configuration must agree.  A decision may
differ only where |u - min(1, R^2)| is within that bound (then the rest of
that chain's sweep is not compared, and the count is printed).
"""
import math

import numpy as np
import pytest

from oracle import sweep as osw
from paper_1611_09467_amd import binding as bd
from paper_1611_09467_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    c = bd.Context(0)
    yield c
    c.close()


def _compare(T, Dc, before, after, acc, rat, u, chains):
    order = osw.bond_order(len(T), len(T[0]))
    border = moves = 0
    for c in chains:
        new, oacc, orat = osw.sweep(T, Dc, before[c], u[c])
        for k in range(len(order)):
            if math.isnan(orat[k]):
                assert math.isnan(rat[c, k]) and acc[c, k] == 0, (c, k)
                continue
            R = orat[k]
            assert abs(rat[c, k] - R) <= 1e-9 * max(1.0, abs(R)), (c, k, rat[c, k], R)
            if bool(acc[c, k]) != bool(oacc[k]):
                assert abs(u[c, k] - min(1.0, R * R)) <= 1e-9, (c, k, u[c, k], R)
                border += 1
                break
            moves += int(oacc[k])
        else:
            assert np.array_equal(after[c], new), c
    print(f"  {len(chains)} chains compared, {moves} accepted moves, {border} borderline", flush=True)
    return moves


@pytest.mark.parametrize("N,M,D,Dc", [(6, 6, 3, 5), (5, 7, 2, 3), (3, 3, 2, 4), (2, 4, 2, 2)])
def test_sweeps_match_oracle_small(ctx, N, M, D, Dc):
    T = wl.make_peps(N, M, D, seed=N * 31 + M, bias=0.1)
    chains = 12
    S = wl.random_sz0_configs(N, M, chains, N * 7 + M)
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(T))
    cfg = torch.from_numpy(S.copy()).cuda()
    rng = np.random.default_rng(N + M)
    total = 0
    for t in range(2):
        before = cfg.cpu().numpy().copy()
        u = rng.random((chains, P.nbonds))
        print(f"[gpu] sweep {t}: {N}x{M} D={D} Dc={Dc}, {chains} chains", flush=True)
        acc, rat = P.metropolis_sweep(cfg, torch.from_numpy(u).cuda(), Dc, want_ratios=True)
        torch.cuda.synchronize()
        total += _compare(T, Dc, before, cfg.cpu().numpy(), acc.cpu().numpy(),
                          rat.cpu().numpy(), u, range(chains))
        assert np.all(cfg.cpu().numpy().sum(axis=1) == before.sum(axis=1))
    assert total > 0
    P.free()


def test_sweep_8x8_chains_and_full_10x10_batch(ctx):
    # 8x8 D=4 Dc=8: 64 chain states, all compared
    T, S = wl.workload_inputs("8x8_D4_Dc8")
    S = S[::64][:64].copy()
    P = bd.Peps(ctx, 8, 8, 4, wl.pack_peps(T))
    cfg = torch.from_numpy(S).cuda()
    u = np.random.default_rng(81).random((len(S), P.nbonds))
    print("[gpu] sweep 8x8 D=4 Dc=8, 64 chains", flush=True)
    acc, rat = P.metropolis_sweep(cfg, torch.from_numpy(u).cuda(), 8, want_ratios=True)
    torch.cuda.synchronize()
    _compare(T, 8, S, cfg.cpu().numpy(), acc.cpu().numpy(), rat.cpu().numpy(), u, range(64))
    P.free()
    # 10x10 D=6 Dc=12: the whole 16384-chain batch in one call, 16 chains compared
    T, S = wl.workload_inputs("10x10_D6_Dc12")
    P = bd.Peps(ctx, 10, 10, 6, wl.pack_peps(T))
    cfg = torch.from_numpy(S.copy()).cuda()
    u = np.random.default_rng(82).random((len(S), P.nbonds))
    print("[gpu] sweep 10x10 D=6 Dc=12, 16384 chains", flush=True)
    acc, rat = P.metropolis_sweep(cfg, torch.from_numpy(u).cuda(), 12, want_ratios=True)
    torch.cuda.synchronize()
    after = cfg.cpu().numpy()
    a = acc.cpu().numpy()
    assert 0.05 < a.sum() / (len(S) * P.nbonds) < 0.9
    idx = list(range(0, 16384, 1024))
    _compare(T, 12, S, after, a, rat.cpu().numpy(), u, idx)
    P.free()
