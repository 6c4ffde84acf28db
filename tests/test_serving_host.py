"""Host logic of the serving loop (no GPU): admission by HBM budget and the
request stream recipe."""
import numpy as np

from paper_1912_13403_amd import inputs
from paper_1912_13403_amd.serving import matrix_bytes, pick_slot, take_group


def _tb(n, cplx):
    return (2.0 if cplx else 1.0) * 10.0 * n * n * 8.0


def _req(n, cplx=False, base=None, rid=0):
    return dict(n=n, cplx=cplx, base=rid if base is None else base, rid=rid)


def _bytes(r, s_resident=False, held=0.0):
    m = matrix_bytes(r["n"], r["cplx"])
    return 3 * m + (0.0 if s_resident else m) + max(0.0, _tb(r["n"], r["cplx"]) - held)


def test_group_prefix_fits_budget():
    q = [_req(1000, rid=0), _req(2000, True, rid=1), _req(500, rid=2)]
    b = [_bytes(r) for r in q]
    got, need, _ = take_group(q, 8, b[0] + b[1] + 1.0, 0.0, 0.0, False, set(), _tb)
    assert got == q[:2] and need == b[0] + b[1]
    # the head starts alone over the budget when nothing else runs ...
    got, need, _ = take_group(q, 8, 1.0, 0.0, 0.0, False, set(), _tb)
    assert got == q[:1] and need == b[0]
    # ... and waits when something does
    got, _, _ = take_group(q, 8, 1.0, 0.0, 0.0, True, set(), _tb)
    assert got == []
    # bytes in use count against the budget
    got, _, _ = take_group(q, 8, sum(b), b[2] - 1.0, 0.0, False, set(), _tb)
    assert got == q[:2]
    # arrival order is kept: a later small request does not overtake
    got, _, _ = take_group(q, 8, b[0] + b[2] + 1.0, 0.0, 0.0, False, set(), _tb)
    assert got == q[:1]
    # the group size cap
    got, _, _ = take_group(q, 2, 1e15, 0.0, 0.0, False, set(), _tb)
    assert got == q[:2]


def test_group_bytes_resident_s_and_held_workspace():
    # a resident S, or one shared with an earlier member, is not counted again
    q = [_req(1000, rid=0), _req(1000, base=0, rid=1)]
    got, need, _ = take_group(q, 8, 1e15, 0.0, 0.0, False, set(), _tb)
    assert need == _bytes(q[0]) + _bytes(q[1], s_resident=True)
    got, need, _ = take_group(q, 8, 1e15, 0.0, 0.0, False, {0}, _tb)
    assert need == _bytes(q[0], True) + _bytes(q[1], True)
    # the slot's workspace covers the task contexts it already holds
    t = _tb(1000, False)
    got, need, room = take_group(q[:1], 8, 1e15, 5 * t, 5 * t, False, set(), _tb)
    assert need == 4 * matrix_bytes(1000, False)
    # room for the slot's workspace: the budget less everything else in use
    budget = 100 * t
    got, need, room = take_group(q[:1], 8, budget, 7 * t, 5 * t, False, set(), _tb)
    assert room == budget - 2 * t - 4 * matrix_bytes(1000, False)


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


def test_slot_choice():
    # a repeat goes to the slot that factored its S when that slot is free
    aff = {7: 2}
    assert pick_slot(dict(base=7), {0, 2, 3}, aff) == 2
    assert pick_slot(dict(base=7), {0, 3}, aff) == 0
    assert pick_slot(dict(base=9), {3, 1}, aff) == 1
