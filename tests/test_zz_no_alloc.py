"""pepsgo_evaluate_noalloc (the entry point that allocates nothing) against
pepsgo_evaluate, through the C-ABI.

Both run the same kernels with the same per-sample arithmetic; only the
workspace differs (the library's fixed device array, chunked, versus a caller
buffer holding the whole batch), so every output must be bitwise equal.  Two
calls in a row, the second on a smaller input, check that the array's left-over
contents do not leak into a later call.
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


def _outputs(P, B):
    dev = torch.device("cuda:0")
    return dict(logabs=torch.full((B,), 7.0, dtype=torch.float64, device=dev),
                sign=torch.full((B,), 9, dtype=torch.int8, device=dev),
                eloc=torch.full((B,), 7.0, dtype=torch.float64, device=dev),
                flags=torch.full((B,), 99, dtype=torch.int32, device=dev),
                grad=torch.full((B, P.grad_elems), 7.0, dtype=torch.float64, device=dev))


def _noalloc(P, cfg, Dc, J2, precision=bd.PEPSGO_FP64):
    B = cfg.shape[0]
    out = _outputs(P, B)
    prm = bd.make_params(Dc, 1.0, J2, precision)
    s = torch.cuda.current_stream()
    bd.pepsgo_evaluate_noalloc(P.handle, prm, B, cfg.data_ptr(), out["logabs"].data_ptr(),
                               out["sign"].data_ptr(), out["eloc"].data_ptr(),
                               out["flags"].data_ptr(), out["grad"].data_ptr(), s.cuda_stream)
    return out


def _check_equal(P, cfg, Dc, J2, precision=bd.PEPSGO_FP64):
    prm = bd.make_params(Dc, 1.0, J2, precision)
    per = P.workspace_bytes(prm, 1)
    print(f"[gpu] noalloc {P.N}x{P.M} D={P.D} Dc={Dc} batch={cfg.shape[0]}: {per} bytes per "
          f"sample, {bd.NOALLOC_SCRATCH_BYTES // per} samples per chunk", flush=True)
    ref = P.evaluate(cfg, Dc, 1.0, J2, precision=precision)
    got = _noalloc(P, cfg, Dc, J2, precision)
    torch.cuda.synchronize()
    for k in ("logabs", "sign", "eloc", "flags", "grad"):
        a, b = ref[k].cpu().numpy(), got[k].cpu().numpy()
        assert np.array_equal(a, b, equal_nan=a.dtype.kind == "f"), k
    return per


def test_noalloc_matches_evaluate_twice_then_smaller(ctx):
    # 1) 10x10 D=6 Dc=12: 200 samples need more than one chunk of the fixed array
    T, S = wl.workload_inputs("10x10_D6_Dc12", count=200)
    P = bd.Peps(ctx, 10, 10, 6, wl.pack_peps(T))
    cfg = torch.from_numpy(np.ascontiguousarray(S)).cuda()
    per = _check_equal(P, cfg, 12, 0.5, bd.PEPSGO_FP32)
    assert 200 * per > bd.NOALLOC_SCRATCH_BYTES
    P.free()
    # 2) right after, a smaller input on another lattice
    T2 = wl.make_peps(6, 6, 3, seed=81)
    S2 = wl.chain_configs(6, 6, 5, 7, 82)[:37]
    P2 = bd.Peps(ctx, 6, 6, 3, wl.pack_peps(T2))
    _check_equal(P2, torch.from_numpy(S2).cuda(), 5, 0.35)
    P2.free()


def test_noalloc_refuses_a_sample_larger_than_its_array(ctx):
    # 32x32 D=10 Dc=32 with in-call Eq. (3) sums (each sample keeps its Delta block
    # in the workspace): one sample's workspace exceeds the fixed array, so the
    # call is refused before anything is queued
    N = M = 32
    D, Dc = 10, 32
    flat = np.zeros(sum(wl.site_sizes(N, M, D)))
    P = bd.Peps(ctx, N, M, D, flat)
    prm = bd.make_params(Dc, 1.0, 0.5, grad_mode=bd.PEPSGO_GRAD_REDUCED)
    assert P.workspace_bytes(prm, 1) > bd.NOALLOC_SCRATCH_BYTES
    assert P.workspace_bytes(bd.make_params(Dc, 1.0, 0.5), 1) <= bd.NOALLOC_SCRATCH_BYTES
    B = 2
    cfg = torch.zeros((B, N * M), dtype=torch.uint8, device="cuda")
    out = _outputs(P, B)
    sums = P.new_sums()
    with pytest.raises(bd.PepsgoError) as e:
        bd.pepsgo_evaluate_noalloc(P.handle, prm, B, cfg.data_ptr(), out["logabs"].data_ptr(),
                                   out["sign"].data_ptr(), out["eloc"].data_ptr(),
                                   out["flags"].data_ptr(), sums["flat"].data_ptr(),
                                   torch.cuda.current_stream().cuda_stream)
    assert e.value.code == bd.PEPSGO_EUNSUPPORTED
    assert "fixed" in str(e.value)
    torch.cuda.synchronize()
    # nothing ran: the outputs keep their fill values
    assert torch.all(out["logabs"] == 7.0) and torch.all(sums["flat"] == 0.0)
    P.free()
