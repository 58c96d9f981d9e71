"""The throughput probes (pepsgo_peak_probe): flop counts as stated in the
header, launches that finish, and argument errors reported as codes."""
import pytest

from paper_1611_09467_amd import binding as bd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_probe_counts_and_errors():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    s = torch.cuda.current_stream()
    sink = torch.zeros(8, dtype=torch.float64, device="cuda")
    per_mfma = {1: 2 * 16 * 16 * 4, 2: 2 * 16 * 16 * 4, 3: 2 * 16 * 16 * 16}
    print("[gpu] peak probes, 8 workgroups x 10 rounds", flush=True)
    for name, kind in bd.PROBES.items():
        f = bd.pepsgo_peak_probe(kind, 8, 10, sink.data_ptr(), s.cuda_stream)
        if kind == 0:
            assert f == 2 * 8 * 10 * 8 * 256      # 8 chains per thread
        else:
            assert f == per_mfma[kind] * 8 * 10 * 8 * 4  # 8 chains per wave, 4 waves
    torch.cuda.synchronize()
    assert float(sink.abs().sum()) == 0.0         # the chains never hit the sentinel
    with pytest.raises(bd.PepsgoError) as e:
        bd.pepsgo_peak_probe(7, 8, 10, sink.data_ptr(), s.cuda_stream)
    assert e.value.code == bd.PEPSGO_EINVAL
    with pytest.raises(bd.PepsgoError):
        bd.pepsgo_peak_probe(0, 0, 10, sink.data_ptr(), s.cuda_stream)
