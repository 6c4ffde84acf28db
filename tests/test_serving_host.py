"""Host logic of the serving loop (no GPU): admission by HBM budget and the
request stream recipe."""
import numpy as np

from paper_1912_13403_amd import inputs
from paper_1912_13403_amd.serving import admit, pick_slot, request_bytes, start_bytes


def _tb(n, cplx):
    return (2.0 if cplx else 1.0) * 10.0 * n * n * 8.0


def test_admission_prefix_fits_budget():
    q = [dict(n=1000, cplx=False), dict(n=2000, cplx=True), dict(n=500, cplx=False)]
    b = [request_bytes(r["n"], r["cplx"], _tb) for r in q]
    got, need = admit(q, budget=b[0] + b[1] + 1.0, resident=0.0, task_bytes=_tb)
    assert got == q[:2] and need == b[0] + b[1]
    # the first request is always admitted, even alone over the budget
    got, need = admit(q, budget=1.0, resident=0.0, task_bytes=_tb)
    assert got == q[:1]
    # resident bytes count against the budget
    got, _ = admit(q, budget=sum(b), resident=b[2] - 1.0, task_bytes=_tb)
    assert got == q[:2]
    # arrival order is kept: a later small request does not overtake
    got, _ = admit(q, budget=b[0] + b[2] + 1.0, resident=0.0, task_bytes=_tb)
    assert got == q[:1]


def test_request_stream_recipe():
    sp = inputs.request_specs(400, rate=40.0, seed=0)
    t = np.array([s["arrival"] for s in sp])
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 1.0 / 40.0) < 0.25 / 40.0
    ns = np.array([s["n"] for s in sp])
    assert ns.min() >= 256 and ns.max() <= 8192
    reps = [s for s in sp if s["repeat"]]
    assert 0.2 < len(reps) / len(sp) < 0.4
    for s in reps:
        b = sp[s["base"]]
        assert not b["repeat"] and b["n"] == s["n"] and b["cplx"] == s["cplx"]
        assert b["arrival"] < s["arrival"]
    frac_c = np.mean([s["cplx"] for s in sp if not s["repeat"]])
    assert 0.3 < frac_c < 0.5


def test_repeat_shares_s_and_perturbs_h():
    sp = inputs.request_specs(30, rate=40.0, lo=20, hi=40, seed=3)
    probs = {}
    for s in sp:
        base = probs.get(s["base"]) if s["repeat"] else None
        probs[s["rid"]] = inputs.request_problem(s, base)
        if s["repeat"]:
            H0, S0 = probs[s["base"]]
            H1, S1 = probs[s["rid"]]
            assert S1 is S0
            d = H1 - H0
            assert 1e-4 < np.abs(d).max() < 1e-2
            lo = np.tril(d)
            assert np.allclose(d, lo + np.tril(d, -1).conj().T)


def test_slot_choice_and_start_bytes():
    # a repeat goes to the slot that factored its S when that slot is free
    aff = {7: 2}
    assert pick_slot(dict(base=7), {0, 2, 3}, aff) == 2
    assert pick_slot(dict(base=7), {0, 3}, aff) == 0
    assert pick_slot(dict(base=9), {3, 1}, aff) == 1
    # bytes a request adds: H, D, E, S unless resident, workspace growth only
    r = dict(n=1000, cplx=False)
    m = 1000 * 1000 * 8.0
    assert start_bytes(r, 0.0, _tb, False) == 4 * m + _tb(1000, False)
    assert start_bytes(r, 0.0, _tb, True) == 3 * m + _tb(1000, False)
    assert start_bytes(r, 1e12, _tb, True) == 3 * m
