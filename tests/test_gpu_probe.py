"""The measurement probes behind the bench line's measured peaks: the FP64
matrix-core rate and the HBM copy bandwidth are positive and do not exceed
the published peaks (78.6 TFLOP/s, 8 TB/s) beyond timing noise; argument
checks."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda", 0)


@pytest.fixture(scope="module")
def h(torch_dev):
    from paper_1912_13403_amd import hsdm
    with hsdm.Handle(0) as handle:
        yield handle


def test_probe_rates_within_published_peaks(torch_dev, h):
    tf, ms, flops = h.hsdm_probe(0, 2000)
    assert ms > 0 and flops > 0
    assert 0.0 < tf <= 78.6 * 1.05
    gbs, ms, moved = h.hsdm_probe(1, float(256 << 20))
    assert ms > 0 and moved == 2.0 * (256 << 20)
    assert 0.0 < gbs <= 8000.0 * 1.05


def test_probe_argument_checks(torch_dev, h):
    import ctypes
    from paper_1912_13403_amd import hsdm
    lib = hsdm.load_library()
    out = (ctypes.c_double * 3)()
    assert lib.hsdm_probe(h._h, 2, 100.0, out, None) == -2
    assert lib.hsdm_probe(h._h, 0, 0.5, out, None) == -3
    assert lib.hsdm_probe(h._h, 1, 8.0, out, None) == -3
    assert lib.hsdm_probe(h._h, 0, 100.0, None, None) == -4
