"""Reduced-precision modes against the float64 oracle and the float64 GPU path.

In every mode the boundary-MPS truncation, the row sandwiches (psi and every
Delta_ij) and all log-scales are float64; only the two-row strip contractions
that give the vertical and diagonal exchange ratios change precision.  A
strip is recomputed in float64 (flag REFINED) when its left/right environment
overlap strays from the strip value at some cut by more than 1e-3 (relative),
or when that largest deviation times the sum of |ratio terms| of the strip
exceeds its share (1 of N-1 strips) of 1e-4 per site; that product is an
estimate of the strip's energy error, not a bound, and the bound below is
what the tests hold.  So
psi and Delta must equal the float64 mode bit for bit, and the error sits in
E_loc.  Bound, for every mode and every sample, on the energy per site
|E_g - E_ref| / (N M) <= 1e-4, where E_ref is the oracle on a subset and the
float64 GPU path (itself held to 1e-8 relative against the oracle) on the
full batch.  The fraction of refined samples is printed.
"""
import numpy as np
import pytest

from oracle import peps as op
from paper_1611_09467_amd import binding as bd
from paper_1611_09467_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = [("fp32", bd.PEPSGO_FP32), ("bf16x6", bd.PEPSGO_BF16_MIXED), ("bf16", bd.PEPSGO_BF16)]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    c = bd.Context(0)
    yield c
    c.close()


def run_modes(ctx, T, S, N, M, D, Dc, J2=0.5):
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(T))
    cfg = torch.from_numpy(np.ascontiguousarray(S, dtype=np.uint8)).cuda()
    res = {}
    for name, prec in [("fp64", bd.PEPSGO_FP64)] + MODES:
        print(f"[gpu] {N}x{M} D={D} Dc={Dc} batch={len(S)} precision={name}", flush=True)
        out = P.evaluate(cfg, Dc, 1.0, J2, precision=prec)
        torch.cuda.synchronize()
        res[name] = {k: v.cpu().numpy() for k, v in out.items()}
    P.free()
    return res


def check_modes(res, nsites, e_ref, idx, label):
    base = res["fp64"]
    live = (base["flags"][idx] & 7) == 0
    sel = np.asarray(idx)[live]
    stats = {}
    for name, _ in MODES:
        r = res[name]
        # psi and Delta never pass through the reduced-precision contractions
        assert np.array_equal(r["logabs"][sel], base["logabs"][sel]), name
        assert np.array_equal(r["sign"][sel], base["sign"][sel]), name
        assert np.array_equal(r["grad"][sel], base["grad"][sel]), name
        assert np.all((r["flags"][sel] & 3) == 0), name
        err = np.abs(r["eloc"][sel] - e_ref[live]) / nsites
        mean_err = abs(r["eloc"][sel].mean() - e_ref[live].mean()) / nsites
        stats[name] = (float(err.max()), float(np.median(err)), float(mean_err))
        refined = int(((r["flags"][sel] & bd.F_REFINED) != 0).sum())
        print(f"  {label} {name}: E/site error max {err.max():.3e} median {np.median(err):.3e} "
              f"batch mean {mean_err:.3e} over {len(sel)} samples, {refined} refined in float64",
              flush=True)
    for name, _ in MODES:
        assert stats[name][0] <= 1e-4, (name, stats[name])
    return stats


def test_precision_modes_8x8_D4_Dc8(ctx):
    T, S = wl.workload_inputs("8x8_D4_Dc8", count=512)
    res = run_modes(ctx, T, S, 8, 8, 4, 8)
    sub = list(range(0, 512, 16))
    e_or = np.array([op.evaluate(T, S[b], 8, 1.0, 0.5, want_grad=False)["eloc"] for b in sub])
    check_modes(res, 64, e_or, sub, "vs oracle")
    check_modes(res, 64, res["fp64"]["eloc"], list(range(512)), "vs fp64 gpu")


def test_precision_modes_10x10_D6_Dc12_full_batch(ctx):
    T, S = wl.workload_inputs("10x10_D6_Dc12")
    res = run_modes(ctx, T, S, 10, 10, 6, 12)
    sub = list(range(0, 16384, 16384 // 12))
    e_or = np.array([op.evaluate(T, S[b], 12, 1.0, 0.5, want_grad=False)["eloc"] for b in sub])
    check_modes(res, 100, e_or, sub, "vs oracle")
    check_modes(res, 100, res["fp64"]["eloc"], list(range(len(S))), "vs fp64 gpu")


def test_precision_modes_16x16_D8_Dc16(ctx):
    T, S = wl.workload_inputs("16x16_D8_Dc16", count=256)
    res = run_modes(ctx, T, S, 16, 16, 8, 16)
    sub = [0, 97, 181]
    e_or = np.array([op.evaluate(T, S[b], 16, 1.0, 0.5, want_grad=False)["eloc"] for b in sub])
    check_modes(res, 256, e_or, sub, "vs oracle")
    check_modes(res, 256, res["fp64"]["eloc"], list(range(len(S))), "vs fp64 gpu")
