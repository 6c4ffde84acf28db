"""The GEMM tile autotuner on the GPU: tuning solves and solves that use the
tuned table give the same D, E and eigenvalues as the built-in tile rule, in
the FP64 and the refined form; the table then holds the timed classes."""
import numpy as np
import pytest

from paper_1912_13403_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda", 0)


def _solve(h, torch_dev, H, S):
    torch, dev = torch_dev
    o = h.hsdm_solve_dm_real(torch.from_numpy(H).to(dev), torch.from_numpy(S).to(dev),
                             0.5 * H.shape[0], 0.01)
    return o["D"].cpu().numpy(), o["E"].cpu().numpy(), o["eval"].cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_tuned_tiles_same_results(torch_dev, tmp_path, prec):
    from paper_1912_13403_amd import hsdm
    lib = hsdm.load_library()
    n = 1100
    H, S = inputs.sized_problem(n, cfg=4321)
    lib.hsdm_tune_clear()
    try:
        with hsdm.Handle(0) as h:
            h.hsdm_set_int(hsdm.HSDM_KEY_PRECISION, prec)
            ref = _solve(h, torch_dev, H, S)
            h.hsdm_set_int(hsdm.HSDM_KEY_AUTOTUNE, 1)
            tuned = _solve(h, torch_dev, H, S)
            h.hsdm_set_int(hsdm.HSDM_KEY_AUTOTUNE, 0)
            k = lib.hsdm_tune_entries()
            print(f"[tune] precision {prec}: {k} classes timed", flush=True)
            assert k > 0
            after = _solve(h, torch_dev, H, S)
            path = str(tmp_path / "tiles.txt").encode()
            assert lib.hsdm_tune_save(path) == hsdm.HSDM_OK
            lib.hsdm_tune_clear()
            assert lib.hsdm_tune_load(path) == k
            again = _solve(h, torch_dev, H, S)
        for a, b, c, d in zip(ref, tuned, after, again):
            assert np.array_equal(a, b) and np.array_equal(a, c) and np.array_equal(a, d)
    finally:
        with hsdm.Handle(0) as h:
            h.hsdm_set_int(hsdm.HSDM_KEY_AUTOTUNE, 0)
        lib.hsdm_tune_clear()
