"""The serving loop on the GPU: a mixed stream of real and Hermitian requests
with SCF repeats, started on free slots while other requests run (single
solves, or groups through hsdm_solve_dm_group); every result in the mix
equals the same request solved alone (single-solve entry points) within the
parity tolerance, and the smaller ones equal the oracle."""
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


def _stream(count, seed, lo, hi):
    specs = inputs.request_specs(count, rate=2000.0, lo=lo, hi=hi, seed=seed)
    probs = {}
    reqs = []
    for s in specs:
        base = probs[s["base"]] if s["repeat"] else None
        probs[s["rid"]] = inputs.request_problem(s, base)
        H, S = probs[s["rid"]]
        reqs.append(dict(s, H=H, S=S))
    return reqs


def _alone(torch_dev, r):
    torch, dev = torch_dev
    from paper_1912_13403_amd import hsdm
    with hsdm.Handle(0) as h:
        h.hsdm_set_real(hsdm.HSDM_KEY_FMAX, r["f_max"])
        H = torch.from_numpy(np.asfortranarray(r["H"])).to(dev)
        S = torch.from_numpy(np.asfortranarray(r["S"])).to(dev)
        f = h.hsdm_solve_dm_complex if r["cplx"] else h.hsdm_solve_dm_real
        o = f(H, S, r["n_electrons"], r["kT"])
        return o["D"].cpu().numpy(), o["E"].cpu().numpy(), o["mu"], o["band_energy"]


@pytest.mark.parametrize("budget,group", [(200e9, 1), (0.0, 1), (200e9, 4)])
def test_each_result_same_alone_and_in_the_mix(oracle, torch_dev, budget, group):
    from paper_1912_13403_amd.serving import Server, host_maker
    reqs = _stream(12, seed=11, lo=40, hi=500)
    print(f"[serving] budget={budget:g} group={group} sizes={[r['n'] for r in reqs]}",
          flush=True)
    problems = {r["rid"]: (r["H"], r["S"]) for r in reqs}
    srv = Server(0, hbm_budget=budget, slots=2 if group > 1 else 4, max_group=group,
                 streams=3 if group > 1 else 0)
    try:
        recs = srv.run(reqs, host_maker(problems), keep=lambda rid: True)
    finally:
        srv.close()
    assert sorted(r["rid"] for r in recs) == list(range(len(reqs)))
    assert all(r["group"] <= group for r in recs)
    if group > 1:
        assert max(r["group"] for r in recs) > 1
    if budget == 0.0:
        assert all(r["concurrent"] == 0 for r in recs)  # one request at a time
    else:
        assert max(r["concurrent"] for r in recs) >= 1  # requests overlapped on the device
        # a slot was refilled while other requests were still on the device
        assert any(b["start"] < a["done"] and b["arrival"] > a["start"] and b["rid"] != a["rid"]
                   for a in recs for b in recs)
    by = {r["rid"]: r for r in recs}
    for q in reqs:
        rec = by[q["rid"]]
        D, E, mu, eb = _alone(torch_dev, q)
        scale = float(np.abs(q["H"]).sum(axis=0).max())
        assert np.max(np.abs(rec["D"].cpu().numpy() - D)) <= 1e-9
        assert np.max(np.abs(rec["E"].cpu().numpy() - E)) <= 1e-9 * max(1.0, scale)
        assert abs(rec["mu"] - mu) <= 1e-10 * scale
        assert abs(rec["band_energy"] - eb) <= 1e-10 * scale * q["n_electrons"]
        if q["n"] <= 200:
            if q["cplx"]:
                ref = oracle.solve_dm_complex(q["H"], q["S"], q["n_electrons"], q["kT"], f_max=1.0)
            else:
                ref = oracle.solve_dm(q["H"], q["S"], q["n_electrons"], q["kT"], f_max=2.0)
            assert np.max(np.abs(rec["D"].cpu().numpy() - ref["D"])) <= 1e-9


@pytest.mark.parametrize("group", [1, 4])
def test_device_drawn_requests_in_the_mix(torch_dev, group):
    """The benchmark's device-drawn request stream (per-request seeds, SCF
    repeats reusing the resident S on the slot that factored it): every
    result equals the same request solved alone."""
    from paper_1912_13403_amd import inputs
    from paper_1912_13403_amd.serving import Server
    torch, dev = torch_dev
    specs = inputs.request_specs(16, rate=1000.0, lo=64, hi=600, seed=21)
    make = lambda req, S: inputs.request_problem_device(req, specs[req["base"]], S, dev)
    srv = Server(0, hbm_budget=200e9, slots=3 if group == 1 else 2, max_group=group,
                 streams=3 if group > 1 else 0)
    try:
        recs = srv.run(specs, make, keep=lambda rid: True)
    finally:
        srv.close()
    assert max(r["concurrent"] for r in recs) >= 1
    from paper_1912_13403_amd import hsdm
    with hsdm.Handle(0) as h:
        for rec in recs:
            q = specs[rec["rid"]]
            H, S = inputs.request_problem_device(q, specs[q["base"]], None, dev)
            h.hsdm_set_real(hsdm.HSDM_KEY_FMAX, q["f_max"])
            f = h.hsdm_solve_dm_complex if q["cplx"] else h.hsdm_solve_dm_real
            o = f(H, S, q["n_electrons"], q["kT"])
            assert torch.max(torch.abs(o["D"] - rec["D"])).item() <= 1e-9
            assert abs(o["mu"] - rec["mu"]) <= 1e-10 * max(1.0, abs(o["mu"]))


def test_group_argument_errors(torch_dev):
    import ctypes
    from paper_1912_13403_amd import hsdm
    torch, dev = torch_dev
    lib = hsdm.load_library()
    n = 8
    A = torch.zeros((n, n), dtype=torch.float64, device=dev)
    I1, P1, F1 = ctypes.c_int * 1, ctypes.c_void_p * 1, ctypes.c_double * 1
    ptr = P1(A.data_ptr())
    with hsdm.Handle(0) as h:
        def call(nprob=1, cplx=0, nv=n, ne=1.0, kT=0.0, fm=2.0):
            return lib.hsdm_solve_dm_group(h._h, nprob, I1(cplx), I1(nv), ptr, I1(n), ptr, I1(n),
                                           F1(ne), F1(kT), F1(fm), ptr, I1(n), None, None, None,
                                           None, None)
        assert call(nprob=0) == -2
        assert call(cplx=3) == -3
        assert call(nv=0) == -4
        assert call(ne=17.0) == -9
        assert call(kT=-1.0) == -10
        assert call(fm=0.0) == -11


@pytest.mark.parametrize("n,cplx", [(700, False), (1100, False), (300, True)])
def test_concurrent_mode_same_bits(torch_dev, n, cplx):
    """A handle marked concurrent (HSDM_KEY_CONCURRENT: panel QR one launch
    per column, one stage-2 workgroup per strip, the bulge chasing alone on
    the device) gives the same bits as the default handle."""
    from paper_1912_13403_amd import hsdm
    torch, dev = torch_dev
    if cplx:
        H, _, S = inputs.kpoint_problem(5, n=n)
    else:
        H, S = inputs.sized_problem(n, cfg=2300 + n)
    outs = []
    for conc in (0, 1):
        with hsdm.Handle(0) as h:
            h.hsdm_set_int(hsdm.HSDM_KEY_CONCURRENT, conc)
            if cplx:
                h.hsdm_set_real(hsdm.HSDM_KEY_FMAX, 1.0)
            f = h.hsdm_solve_dm_complex if cplx else h.hsdm_solve_dm_real
            o = f(torch.from_numpy(H).to(dev), torch.from_numpy(S).to(dev),
                  (0.2 if cplx else 0.5) * n, 0.01)
            outs.append((o["D"].cpu().numpy(), o["E"].cpu().numpy(), o["eval"].cpu().numpy(),
                         o["mu"]))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_refined_slots_against_oracle(oracle, torch_dev):
    """Slots whose single solves run the refined form (precision = 1): each
    request of a mixed real / Hermitian stream meets the parity tolerances
    against the oracle while other requests share the device."""
    from paper_1912_13403_amd.serving import Server, host_maker
    reqs = _stream(8, seed=13, lo=40, hi=400)
    print(f"[serving refined] sizes={[r['n'] for r in reqs]}", flush=True)
    problems = {r["rid"]: (r["H"], r["S"]) for r in reqs}
    srv = Server(0, hbm_budget=200e9, slots=3, max_group=1, precision=1)
    try:
        recs = srv.run(reqs, host_maker(problems), keep=lambda rid: True)
    finally:
        srv.close()
    assert sorted(r["rid"] for r in recs) == list(range(len(reqs)))
    by = {r["rid"]: r for r in recs}
    for q in reqs:
        rec = by[q["rid"]]
        if q["cplx"]:
            ref = oracle.solve_dm_complex(q["H"], q["S"], q["n_electrons"], q["kT"], f_max=q["f_max"])
        else:
            ref = oracle.solve_dm(q["H"], q["S"], q["n_electrons"], q["kT"], f_max=q["f_max"])
        scale = float(np.abs(q["H"]).sum(axis=0).max())
        assert np.max(np.abs(rec["D"].cpu().numpy() - ref["D"])) <= 1e-9
        assert np.max(np.abs(rec["E"].cpu().numpy() - ref["E"])) <= 1e-9 * max(1.0, scale)
        assert abs(rec["mu"] - ref["mu"]) <= 1e-10 * scale
