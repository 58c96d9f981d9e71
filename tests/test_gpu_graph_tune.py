"""Captured evaluations (pepsgo_graph_*) and the LDS-budget autotuner (pepsgo_autotune).

A graph replays exactly the launches of pepsgo_evaluate, so every replay must
equal an eager evaluation of the same buffer contents bit for bit, also after
the configuration buffer is rewritten in place and with eager work between
replays.  The autotuner only moves scratch buffers between LDS and the
workspace (and the eigensolver's batch width with it), so results after
tuning stay within the float64 parity bound of the untuned path.
"""

import numpy as np
import pytest

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


def _bits(t):
    return t.view(torch.uint8) if t.dtype == torch.float64 else t


@pytest.mark.parametrize("precision", [bd.PEPSGO_FP64, bd.PEPSGO_FP32])
def test_graph_replays_equal_eager(ctx, precision):
    N, M, D, Dc = 6, 6, 3, 6
    T = wl.make_peps(N, M, D, seed=91, bias=0.1)
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(T))
    batches = [wl.chain_configs(N, M, 8, 8, 92 + k) for k in range(3)]
    cfg = torch.from_numpy(batches[0]).cuda()
    print(f"[gpu] graph capture {N}x{M} D={D} Dc={Dc} precision={precision}", flush=True)
    G = P.capture(cfg, Dc, 1.0, 0.5, precision=precision)
    for k, S in enumerate(batches):
        cfg.copy_(torch.from_numpy(S))            # chain state rewritten in place
        eager = P.evaluate(cfg.clone(), Dc, 1.0, 0.5, precision=precision)
        torch.cuda.synchronize()
        out = G.launch()
        torch.cuda.synchronize()
        for key in ("logabs", "sign", "eloc", "flags", "grad"):
            assert torch.equal(_bits(out[key]), _bits(eager[key])), (k, key)
    G.free()
    P.free()


def test_autotune_choice_and_results(ctx, tmp_path):
    T, S = wl.workload_inputs("8x8_D4_Dc8", count=512)
    P = bd.Peps(ctx, 8, 8, 4, wl.pack_peps(T))
    cfg = torch.from_numpy(S).cuda()
    base = P.evaluate(cfg, 8, 1.0, 0.5)
    base = {k: v.cpu().numpy() for k, v in base.items()}
    print("[gpu] autotune 8x8 D=4 Dc=8", flush=True)
    t = P.autotune(cfg, 8, 1.0, 0.5)
    print(f"  chosen {t}", flush=True)
    lds = 160 * 1024
    assert t["zip_lds_bytes"] in (80 * 1024, lds)
    assert t["sandwich_lds_bytes"] in (32 * 1024, 40 * 1024, 53 * 1024, 80 * 1024, lds)
    assert t["strip_lds_bytes"] in (32 * 1024, 40 * 1024, 53 * 1024, 80 * 1024, lds)
    assert t["strip_xc"] in (1, 2, 3)
    got = bd.pepsgo_tune_get(ctx.handle, 4, 8, bd.PEPSGO_FP64).as_dict()
    assert got == t
    tuned = {k: v.cpu().numpy() for k, v in P.evaluate(cfg, 8, 1.0, 0.5).items()}
    assert np.array_equal(tuned["flags"], base["flags"])
    live = (base["flags"] & 3) == 0
    d_psi = np.abs(tuned["sign"][live] * np.exp(tuned["logabs"][live] - base["logabs"][live])
                   - base["sign"][live])
    assert d_psi.max() <= 1e-10
    e = np.abs(tuned["eloc"][live] - base["eloc"][live]) / np.maximum(1, np.abs(base["eloc"][live]))
    assert e.max() <= 1e-8
    # the table survives a save / load round trip
    path = str(tmp_path / "tune.txt")
    bd.pepsgo_tune_save(ctx.handle, path)
    bd.pepsgo_tune_set(ctx.handle, 4, 8, bd.PEPSGO_FP64, None)
    assert bd.pepsgo_tune_load(ctx.handle, path) >= 1
    assert bd.pepsgo_tune_get(ctx.handle, 4, 8, bd.PEPSGO_FP64).as_dict() == t
    assert open(path).readline().startswith("# pepsgo tuning v2 gfx")
    P.free()


def test_strip_budgets_agree(ctx):
    # every strip budget and stage width the tuner may pick gives identical strip arithmetic
    N, M, D, Dc = 6, 6, 4, 8
    T = wl.make_peps(N, M, D, seed=95, bias=0.1)
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(T))
    cfg = torch.from_numpy(wl.chain_configs(N, M, 4, 8, 96)).cuda()
    ref = None
    for prec in (bd.PEPSGO_FP64, bd.PEPSGO_FP32):
        ref = None
        for b, xc in ((40 * 1024, 1), (53 * 1024, 1), (80 * 1024, 1), (160 * 1024, 1),
                      (80 * 1024, 2), (160 * 1024, 3)):
            bd.pepsgo_tune_set(ctx.handle, D, Dc, prec, bd.Tuning(0, 0, b, xc))
            print(f"[gpu] strip budget {b} xc {xc} precision {prec}", flush=True)
            out = {k: v.cpu() for k, v in P.evaluate(cfg, Dc, 1.0, 0.5, precision=prec).items()}
            if ref is None:
                ref = out
            else:
                assert torch.equal(_bits(out["eloc"]), _bits(ref["eloc"])), (prec, b, xc)
        bd.pepsgo_tune_set(ctx.handle, D, Dc, prec, None)
    P.free()
