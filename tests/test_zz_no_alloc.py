"""hsdm_solve_dm_real_noalloc -- the variant of hsdm_solve_dm_real that
allocates no device memory, for callers that cannot allocate -- against
hsdm_solve_dm_real on the same inputs, through the C ABI: two calls in a
row, the second smaller than the first, every entry of D and E, the
eigenvalues, mu and the band energy at the parity tolerances; the first call
on a fresh handle leaves the device's free memory unchanged (its workspace
is the library's static scratch), and a size above the maximum is rejected
with an argument error."""
import ctypes

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


def test_noalloc_matches_the_allocating_solve(oracle, torch_dev):
    from paper_1912_13403_amd import hsdm
    torch, dev = torch_dev
    cases = [(512, 256.0, 0.0), (300, 150.0, 0.01)]
    probs = []
    for n, ne, kT in cases:
        H, S = inputs.sized_problem(n, cfg=2100 + n)
        Hd = torch.from_numpy(np.asfortranarray(H)).to(dev).t().contiguous().t()
        Sd = torch.from_numpy(np.asfortranarray(S)).to(dev).t().contiguous().t()
        out = (hsdm.empty_colmajor(n, n, dev), hsdm.empty_colmajor(n, n, dev),
               torch.empty(n, dtype=torch.float64, device=dev))
        probs.append((n, ne, kT, H, Hd, Sd, out))
    torch.cuda.synchronize()
    # the HIP runtime's own one-time set-up (first launches of the library's
    # kernels, cooperative launches, staging of host copies) is done by an
    # allocating solve on another handle first; its workspace is freed again
    with hsdm.Handle(0) as w:
        Hs, Ss = inputs.sized_problem(96, cfg=2099)
        w.hsdm_solve_dm_real(torch.from_numpy(Hs).to(dev), torch.from_numpy(Ss).to(dev), 48.0, 0.01)
        torch.cuda.synchronize()
    torch.cuda.synchronize()
    with hsdm.Handle(0) as h:
        for k, (n, ne, kT, H, Hd, Sd, out) in enumerate(probs):
            free0 = torch.cuda.mem_get_info(dev)[0]
            r = h.hsdm_solve_dm_real_noalloc(Hd, Sd, ne, kT, out=out)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info(dev)[0]
            print(f"[noalloc] call {k}: n={n}, device free memory {free0} -> {free1}", flush=True)
            assert free0 - free1 < (2 << 20)
            ref = h.hsdm_solve_dm_real(Hd, Sd, ne, kT)
            scale = oracle.norm1(H)
            D, E, w = (x.cpu().numpy() for x in out)
            assert np.max(np.abs(w - ref["eval"].cpu().numpy())) <= 1e-10 * scale
            assert np.max(np.abs(D - ref["D"].cpu().numpy())) <= 1e-9
            assert np.max(np.abs(E - ref["E"].cpu().numpy())) <= 1e-9 * max(1.0, scale)
            assert abs(r["band_energy"] - ref["band_energy"]) <= 1e-10 * scale * ne
            if kT > 0:
                assert abs(r["mu"] - ref["mu"]) <= 1e-10 * scale
        # above the maximum: argument 2, no launch
        lib = hsdm.load_library()
        n = hsdm.HSDM_NOALLOC_MAX_N + 1
        A = torch.zeros((n, n), dtype=torch.float64, device=dev)
        p = A.data_ptr()
        mu, eb = ctypes.c_double(), ctypes.c_double()
        st = lib.hsdm_solve_dm_real_noalloc(h._h, n, p, n, p, n, 1.0, 0.0, p, n, None, n, None,
                                            ctypes.byref(eb), ctypes.byref(mu), None)
        assert st == -2
        assert b"exceeds the maximum" in lib.hsdm_last_error(h._h)
