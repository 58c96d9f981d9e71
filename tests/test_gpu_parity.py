"""HIP path (through the C-ABI) against the FP64 CPU oracle, element by element.

Tolerances (float64 contractions, float64 truncation):
  psi       |sign_g exp(logabs_g - logabs_o) - sign_o| <= 1e-10 (the number of
            samples also within 1e-12 is printed)
  E(S)      |E_g - E_o| <= 1e-8 max(1, |E_o|)
  Delta     ||Delta_g - Delta_o||_F <= 1e-8 ||Delta_o||_F per sample
A sample that misses a bound is checked against the conditioning of its own
result: with truncation, the spread between the oracle run with two backward
stable LAPACK SVD drivers (gesdd and gesvd) -- the GPU must stay within 10x that
spread; without truncation, the rounding bound eps * W(|A|)/|W(A)| of any
summation order.  Counts of samples passing only the conditioning bound are
printed.  Samples flagged NEAR_TIE by either side (kept subspace ill-defined)
are excluded and counted.
"""
import math

import numpy as np
import pytest

from oracle import brute
from oracle import peps as op
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


def run_gpu(ctx, T, S, N, M, D, Dc, J1=1.0, J2=0.5, want_grad=True, want_eloc=True):
    print(f"[gpu] {N}x{M} D={D} Dc={Dc} batch={len(S)}", flush=True)
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(T))
    cfg = torch.from_numpy(np.ascontiguousarray(S, dtype=np.uint8)).cuda()
    out = P.evaluate(cfg, Dc, J1, J2, want_grad=want_grad, want_eloc=want_eloc)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["offsets"] = P.grad_offsets
    P.free()
    return res


def _diffs(res, b, o, want_grad):
    d_psi = abs(res["sign"][b] * math.exp(res["logabs"][b] - o["logabs"]) - o["sign"])
    d_e = abs(res["eloc"][b] - o["eloc"]) / max(1.0, abs(o["eloc"]))
    d_g = 0.0
    if want_grad:
        go = np.concatenate([g.ravel() for g in o["grads"]])
        d_g = np.linalg.norm(res["grad"][b] - go) / np.linalg.norm(go)
    return d_psi, d_e, d_g


def _spread(o, o2, want_grad):
    """Differences between two equally valid float64 oracle runs (same measures)."""
    s_psi = abs(o2["sign"] * math.exp(o2["logabs"] - o["logabs"]) - o["sign"])
    s_e = abs(o2["eloc"] - o["eloc"]) / max(1.0, abs(o["eloc"]))
    s_g = 0.0
    if want_grad:
        a = np.concatenate([g.ravel() for g in o["grads"]])
        c = np.concatenate([g.ravel() for g in o2["grads"]])
        s_g = np.linalg.norm(a - c) / np.linalg.norm(a)
    return s_psi, s_e, s_g


def compare(res, T, S, Dc, idx, J1=1.0, J2=0.5, psi_tol=1e-10, e_tol=1e-8, g_tol=1e-8,
            want_grad=True, exact=False):
    N, M = len(T), len(T[0])
    ties = conditioned = fine = 0
    worst = dict(psi=0.0, e=0.0, g=0.0)
    for b in idx:
        o = op.evaluate(T, S[b], Dc, J1, J2, want_grad=want_grad)
        fg = int(res["flags"][b])
        if (fg | o["flags"]) & op.FLAG_NEAR_TIE:
            ties += 1
            continue
        assert (fg & 3) == (o["flags"] & 3), (b, fg, o["flags"])
        if o["flags"] & op.FLAG_ZERO_PSI:
            assert res["sign"][b] == 0 and res["logabs"][b] == -math.inf
            continue
        d = _diffs(res, b, o, want_grad)
        for k, v in zip(("psi", "e", "g"), d):
            worst[k] = max(worst[k], v)
        fine += d[0] <= 1e-12
        if d[0] <= psi_tol and d[1] <= e_tol and d[2] <= g_tol:
            continue
        conditioned += 1
        if exact:
            # rounding bound of any evaluation order: eps * W(|A|) / |W(A)|
            s = S[b].reshape(N, M)
            Ta = [[np.abs(t) for t in row] for row in T]
            kappa = brute.amplitude(Ta, s) / abs(brute.amplitude(T, s))
            bound = 2.3e-16 * kappa
            assert d[0] <= max(psi_tol, bound), (b, d, kappa)
            assert d[1] <= max(e_tol, bound) and d[2] <= max(g_tol, bound), (b, d, kappa)
        else:
            o2 = op.evaluate(T, S[b], Dc, J1, J2, want_grad=want_grad, svd_driver="gesvd")
            sp = _spread(o, o2, want_grad)
            assert d[0] <= max(psi_tol, 10 * sp[0]), (b, d, sp)
            assert d[1] <= max(e_tol, 10 * sp[1]), (b, d, sp)
            assert d[2] <= max(g_tol, 10 * sp[2]), (b, d, sp)
    print(f"  compared {len(idx) - ties} samples ({conditioned} within their conditioning bound "
          f"only, {fine} with psi within 1e-12), {ties} near ties excluded; worst {worst}",
          flush=True)
    return ties


def test_exact_regime_4x4_D2_Dc4_1000_configs(ctx):
    # the 4x4 workload: nothing is truncated at Dc = 4 = D^2
    N = M = 4
    D, Dc = 2, 4
    T = wl.make_peps(N, M, D, seed=0)
    S = wl.random_sz0_configs(N, M, 1000, 1000)
    res = run_gpu(ctx, T, S, N, M, D, Dc)
    compare(res, T, S, Dc, range(1000), e_tol=1e-10, g_tol=1e-10, exact=True)


@pytest.mark.parametrize("N,M,D,Dc", [(2, 2, 1, 1), (2, 3, 2, 2), (3, 5, 3, 5), (5, 3, 3, 4),
                                      (4, 6, 2, 3), (6, 4, 3, 7), (7, 5, 2, 5), (3, 3, 4, 16)])
def test_ragged_small_lattices(ctx, N, M, D, Dc):
    T = wl.make_peps(N, M, D, seed=N * 100 + M * 10 + D, bias=0.1)
    S = wl.chain_configs(N, M, 3, 4, 17)
    res = run_gpu(ctx, T, S, N, M, D, Dc, J2=0.35)
    compare(res, T, S, Dc, range(len(S)), J2=0.35)


def test_8x8_D4_Dc8_chains(ctx):
    T, S = wl.workload_inputs("8x8_D4_Dc8", count=256)
    res = run_gpu(ctx, T, S, 8, 8, 4, 8)
    compare(res, T, S, 8, range(0, 256, 4))


def test_10x10_D6_Dc12_full_batch_sampled(ctx):
    # the full 16384-sample batch as the benchmark runs it; oracle on a spread subset
    T, S = wl.workload_inputs("10x10_D6_Dc12")
    assert S.shape == (16384, 100)
    res = run_gpu(ctx, T, S, 10, 10, 6, 12)
    idx = list(range(0, 16384, 16384 // 24))
    compare(res, T, S, 12, idx)
    assert np.all(np.isfinite(res["logabs"][(res["flags"] & 3) == 0]))


def test_row_decoupled_log_scale_16x16_D8(ctx):
    # |psi| ~ 10^500: only the log-scale bookkeeping keeps it finite; closed form per row
    N = M = 16
    D = 8
    T = wl.row_decoupled_peps(N, M, D, seed=32, scale=100.0)
    S = wl.random_sz0_configs(N, M, 4, 33)
    res = run_gpu(ctx, T, S, N, M, D, 16, want_grad=False, want_eloc=False)
    for b in range(4):
        s = S[b].reshape(N, M)
        logw, sgn = 0.0, 1
        for i in range(N):
            v = np.ones((1,))
            lv = 0.0
            for j in range(M):
                v = v @ T[i][j][s[i, j]][:, :, 0, 0]
                n = np.abs(v).max()
                v, lv = v / n, lv + math.log(n)
            logw += lv + math.log(abs(v.item()))
            sgn *= int(np.sign(v.item()))
        assert logw > 1000
        assert res["sign"][b] == sgn
        assert res["logabs"][b] == pytest.approx(logw, rel=1e-12)


def test_neel_product_state_flags_and_energy(ctx):
    N = M = 4
    T = wl.neel_product_peps(N, M)
    neel = wl.neel_config(N, M)
    other = neel.copy()
    other[0], other[1] = neel[1], neel[0]
    S = np.stack([neel, other, neel])
    res = run_gpu(ctx, T, S, N, M, 1, 2)
    assert res["eloc"][0] == pytest.approx(-3.75, abs=1e-14)
    assert res["logabs"][0] == 0.0 and res["sign"][0] == 1
    assert res["flags"][1] & bd.F_ZERO_PSI and res["sign"][1] == 0
    assert math.isnan(res["eloc"][1]) and np.all(np.isnan(res["grad"][1]))
    assert res["eloc"][2] == pytest.approx(-3.75, abs=1e-14)


def test_multilinearity_on_gpu_gradients(ctx):
    # <Delta_ij, A_ij> = 1 for every site, under truncation, straight from the GPU output
    N, M, D, Dc = 6, 6, 3, 5
    T = wl.make_peps(N, M, D, seed=50)
    S = wl.chain_configs(N, M, 2, 4, 51)
    res = run_gpu(ctx, T, S, N, M, D, Dc)
    offs = res["offsets"]
    for b in range(len(S)):
        s = S[b].reshape(N, M)
        for i in range(N):
            for j in range(M):
                k = i * M + j
                A = T[i][j][s[i, j]].ravel()
                assert np.dot(res["grad"][b][offs[k]:offs[k + 1]], A) == pytest.approx(1.0, abs=1e-10)


def test_empty_batch_and_bad_arguments(ctx):
    T = wl.make_peps(3, 3, 2, seed=1)
    P = bd.Peps(ctx, 3, 3, 2, wl.pack_peps(T))
    prm = bd.make_params(4, 1.0, 0.5)
    assert bd.pepsgo_evaluate(P.handle, prm, 0, 0, 0, 0, 0, 0, 0, 0, 0) == 0
    bad = bd.make_params(0, 1.0, 0.5)
    with pytest.raises(bd.PepsgoError) as e:
        bd.pepsgo_workspace_bytes(P.handle, bad, 4)
    assert e.value.code == bd.PEPSGO_EINVAL
    with pytest.raises(bd.PepsgoError) as e:
        bd.pepsgo_workspace_bytes(P.handle, bd.make_params(4, precision=7), 4)
    assert e.value.code == bd.PEPSGO_EUNSUPPORTED
    P.free()


def test_chunked_workspace_matches_single_pass(ctx):
    # a workspace for 3 samples forces 4 chunks over 10 samples: same results
    N, M, D, Dc = 5, 5, 3, 6
    T = wl.make_peps(N, M, D, seed=70)
    S = wl.chain_configs(N, M, 2, 5, 71)
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(T))
    cfg = torch.from_numpy(S).cuda()
    full = P.evaluate(cfg, Dc, 1.0, 0.5)
    prm = bd.make_params(Dc, 1.0, 0.5)
    small = torch.empty(P.workspace_bytes(prm, 3), dtype=torch.uint8, device="cuda")
    part = P.evaluate(cfg, Dc, 1.0, 0.5, workspace=small)
    torch.cuda.synchronize()
    for k in ("logabs", "sign", "eloc", "flags", "grad"):
        assert torch.equal(full[k], part[k]), k
    P.free()
