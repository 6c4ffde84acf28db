"""Serving loop for H,S -> D requests on one GPU: continuous batching over slots.

Requests (real or Hermitian, any size) arrive over time.  The server keeps a
few slots; each slot is a host thread with its own library handle (marked
concurrent, HSDM_KEY_CONCURRENT) and its own stream, so the work of
different slots overlaps on the device.  Whenever a slot is free, the
request at the head of the queue (arrival order, no overtaking) starts on it
if its device memory fits the HBM budget beside everything in use, together
with the requests queued behind it while they fit and the group size allows
(max_group): one request runs through the single-solve entry points, several
through hsdm_solve_dm_group, each with its own occupations.  With
precision = 1 the slots' solves, single and grouped, run the refined form
(HSDM_KEY_PRECISION).  A request that
arrives while others run is admitted as soon as a slot and memory free up.

A request that repeats an earlier request's S (the SCF steps of one
geometry, the re-initialization semantics of Sec. 2.7) finds that S still
resident on the device, and its group is sent to the slot whose handle
factored it when that slot is free: the library keeps the factor of S per
handle (per task context in a group), keyed by the content of S, so the
Cholesky factorization is skipped.

Latency is completion minus arrival on the host clock.  Inputs come from a
`make(spec, base, device)` callable run on the slot's stream (host arrays
copied in, or matrices drawn on the device).

Memory accounting (the budget covers the slots' library workspaces, the
resident overlap matrices and each running request's H, D and E): a slot's
handle keeps the workspace of its last solve, trimmed before a group to what
the budget leaves (hsdm_release_tasks); resident overlap matrices beyond half
the budget are dropped, oldest first, unless a running request uses them.
"""
from __future__ import annotations

import queue
import threading
import time
from collections import OrderedDict

import numpy as np
import torch

from . import hsdm


def matrix_bytes(n: int, cplx: bool) -> float:
    return float(n) * n * (16.0 if cplx else 8.0)


def take_group(waiting, max_group, budget, in_use, slot_held, busy, resident, task_bytes):
    """The requests that start together on a free slot whose handle holds
    slot_held bytes of workspace, with in_use bytes in use on the device
    (every slot's workspace, the resident overlap matrices, the running
    requests' matrices): the head of the queue (alone when nothing else runs,
    even over the budget) and the requests behind it, in arrival order,
    while their bytes fit and the group has fewer than max_group.  A request
    adds H, D, E, its S unless resident (`resident`: base ids on the
    device, or shared with an earlier member), and its task context beyond
    what the slot already holds.  Returns (requests, bytes they add, the
    room left for the slot's workspace)."""
    group, mats, tasks = [], 0.0, 0.0
    bases = set(resident)
    for r in waiting[:max_group]:
        m = 3.0 * matrix_bytes(r["n"], r["cplx"])
        if r["base"] not in bases:
            m += matrix_bytes(r["n"], r["cplx"])
        t = task_bytes(r["n"], r["cplx"])
        add = mats + m + max(0.0, tasks + t - slot_held)
        if (group or busy) and in_use + add > budget:
            break
        group.append(r)
        bases.add(r["base"])
        mats += m
        tasks += t
    need = mats + max(0.0, tasks - slot_held)
    room = max(tasks, budget - (in_use - slot_held) - mats)
    return group, need, room


def pick_slot(req, free_slots, affinity):
    """The free slot for a request: the one whose handle factored its S
    (affinity: base request id -> slot), else the lowest-numbered free slot."""
    k = affinity.get(req["base"])
    if k is not None and k in free_slots:
        return k
    return min(free_slots)


class _Slot:
    def __init__(self, idx, device, outbox, timing_level, streams, precision=0):
        self.idx = idx
        self.device = device
        self.outbox = outbox
        self.inbox = queue.Queue()
        self.h = hsdm.Handle(device)
        self.h.hsdm_set_int(hsdm.HSDM_KEY_CONCURRENT, 1)
        if precision:
            self.h.hsdm_set_int(hsdm.HSDM_KEY_PRECISION, precision)
        if streams:
            self.h.hsdm_set_int(hsdm.HSDM_KEY_STREAMS, streams)
        if timing_level:
            self.h.hsdm_set_int(hsdm.HSDM_KEY_TIMING, timing_level)
        self.held = 0.0  # workspace bytes the handle keeps after its last request
        self.thread = threading.Thread(target=self._loop, name=f"hsdm-slot-{idx}", daemon=True)
        self.thread.start()

    def _loop(self):
        torch.cuda.set_device(self.device)
        stream = torch.cuda.Stream(self.device)
        while True:
            job = self.inbox.get()
            if job is None:
                break
            reqs, S_in, make, keep_out, grouped, trim, t0, clock = job
            try:
                with torch.cuda.stream(stream):
                    start = clock() - t0
                    if trim is not None:
                        self.h.hsdm_release_tasks(trim)
                    mats = [make(r, S) for r, S in zip(reqs, S_in)]
                    # a fresh S is shared with later repeats on other slots
                    stream.synchronize()
                    if not grouped:
                        r, (H, S) = reqs[0], mats[0]
                        f = self.h.hsdm_solve_dm_complex if r["cplx"] else self.h.hsdm_solve_dm_real
                        self.h.hsdm_set_real(hsdm.HSDM_KEY_FMAX, r["f_max"])
                        outs = [f(H, S, r["n_electrons"], r["kT"])]
                    else:
                        outs = self.h.hsdm_solve_dm_group(
                            [dict(H=H, S=S, n_electrons=r["n_electrons"], kT=r["kT"],
                                  f_max=r["f_max"]) for r, (H, S) in zip(reqs, mats)])
                    stream.synchronize()
                    done = clock() - t0
                    held = self.h.hsdm_workspace_bytes()
                    res = []
                    for o, k in zip(outs, keep_out):
                        x = dict(mu=o["mu"], band_energy=o["band_energy"], start=start, done=done)
                        if k:
                            x["D"], x["E"] = o["D"], o["E"]
                        res.append(x)
                    Ss = [S for _, S in mats]
                    del mats, outs
                self.outbox.put((self.idx, reqs, Ss, res, held, None))
            except Exception as e:  # reported by the dispatcher
                self.outbox.put((self.idx, reqs, None, None, self.held, e))

    def close(self):
        self.inbox.put(None)
        self.thread.join()
        self.h.close()


class Server:
    def __init__(self, device=0, hbm_budget=200e9, slots=4, timing_level=0, max_group=1,
                 streams=0, precision=0):
        self.dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.budget = float(hbm_budget)
        self.max_group = int(max_group)
        self.outbox = queue.Queue()
        self.slots = [_Slot(k, self.dev, self.outbox, timing_level, streams, precision)
                      for k in range(slots)]
        self.s_dev = OrderedDict()  # base request id -> resident S on the device
        self.s_users = {}           # base request id -> running requests using it
        self.affinity = {}          # base request id -> slot whose handle factored its S

    def close(self):
        for s in self.slots:
            s.close()
        self.s_dev.clear()

    def _resident_bytes(self):
        return sum(matrix_bytes(x.shape[0], x.dtype == torch.complex128)
                   for x in self.s_dev.values())

    def run(self, requests, make, keep=None, clock=time.perf_counter, log=None):
        """Replay `requests` (dicts with rid, arrival, n, cplx, base, repeat,
        n_electrons, kT, f_max; sorted by arrival) against the clock;
        make(req, S or None) -> device (H, S) on the calling slot's stream.
        Returns one record per request: rid, arrival, start, done, latency,
        slot, group (requests solved with it), concurrent (requests on the
        device when it started, itself excluded), mu, band_energy, and D, E
        when keep(rid) is true."""
        pending = list(requests)
        waiting, records = [], []
        free = set(range(len(self.slots)))
        running = {}  # slot -> (requests, bytes they added)
        t0 = clock()
        while pending or waiting or running:
            now = clock() - t0
            while pending and pending[0]["arrival"] <= now:
                waiting.append(pending.pop(0))
            # start the head of the queue (and those behind it) while a slot
            # and memory are free
            while waiting and free:
                k = pick_slot(waiting[0], free, self.affinity)
                slot = self.slots[k]
                in_use = (sum(s.held for s in self.slots) + self._resident_bytes()
                          + sum(b for _, b in running.values()))
                group, need, room = take_group(waiting, self.max_group, self.budget, in_use,
                                               slot.held, bool(running), self.s_dev,
                                               hsdm.hsdm_task_bytes)
                if not group:
                    break
                del waiting[:len(group)]
                free.discard(k)
                running[k] = (group, need)
                S_in = []
                for r in group:
                    S = self.s_dev.get(r["base"])
                    if S is not None:
                        self.s_dev.move_to_end(r["base"])
                    S_in.append(S)
                    self.s_users[r["base"]] = self.s_users.get(r["base"], 0) + 1
                on_dev = sum(len(g) for g, _ in running.values())
                group = [dict(r, concurrent=on_dev - 1, group=len(group)) for r in group]
                keep_out = [keep is not None and keep(r["rid"]) for r in group]
                # the slot's task contexts are trimmed to the room the budget
                # leaves (that waits for the device) only when they exceed it
                trim = room if self.max_group > 1 and slot.held > room else None
                slot.inbox.put((group, S_in, make, keep_out, self.max_group > 1, trim, t0,
                                clock))
            # wait for a completion or the next arrival
            timeout = None
            if pending and (not waiting or free):
                timeout = max(0.0, pending[0]["arrival"] - (clock() - t0))
            if not running:
                if timeout is not None:
                    time.sleep(timeout)
                continue
            try:
                k, group, Ss, res, held, err = self.outbox.get(timeout=timeout)
            except queue.Empty:
                continue
            if err is not None:
                rids = [r["rid"] for r in group]
                raise RuntimeError(f"requests {rids} failed on slot {k}") from err
            running.pop(k)
            free.add(k)
            self.slots[k].held = held
            for r, S, x in zip(group, Ss, res):
                b = r["base"]
                self.affinity[b] = k
                self.s_users[b] -= 1
                if b not in self.s_dev:
                    self.s_dev[b] = S
                rec = dict(rid=r["rid"], arrival=r["arrival"], start=x["start"], done=x["done"],
                           latency=x["done"] - r["arrival"], slot=k, group=r["group"],
                           concurrent=r["concurrent"], mu=x["mu"], band_energy=x["band_energy"])
                if "D" in x:
                    rec["D"], rec["E"] = x["D"], x["E"]
                records.append(rec)
            # resident overlap matrices beyond half the budget go, oldest
            # first, unless a running request uses them
            for old in list(self.s_dev):
                if self._resident_bytes() <= 0.5 * self.budget:
                    break
                if self.s_users.get(old, 0) == 0:
                    self.s_dev.pop(old)
            if log and len(records) // 50 != (len(records) - len(group)) // 50:
                log(f"{len(records)} done, {len(waiting)} waiting, {len(pending)} to arrive, "
                    f"t = {clock() - t0:.1f} s")
        return records


def host_maker(problems):
    """make(req, S) for requests whose host matrices are in
    problems[rid] = (H, S): copies them in (S only when it is not resident)."""
    def make(req, S):
        H, Sh = problems[req["rid"]]
        dev = torch.cuda.current_device()
        Hd = torch.from_numpy(np.asfortranarray(H)).to(dev).t().contiguous().t()
        if S is None:
            S = torch.from_numpy(np.asfortranarray(Sh)).to(dev).t().contiguous().t()
        return Hd, S
    return make


def summarize(records):
    lat = np.array([r["latency"] for r in records])
    span = max(r["done"] for r in records) - min(r["arrival"] for r in records)
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "solves_per_s": len(records) / span,
            "requests": len(records),
            "max_concurrent": max(r["concurrent"] for r in records) + 1,
            "mean_group": float(np.mean([r["group"] for r in records]))}
