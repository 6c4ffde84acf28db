"""Serving loop for H,S -> D requests on one GPU: continuous batching over slots.

Requests (real or Hermitian, any size) arrive over time.  The server keeps a
few slots; each slot is a host thread with its own library handle (marked
concurrent, HSDM_KEY_CONCURRENT) and its own stream, so the solves of
different slots overlap on the device.  Whenever a slot is free, the request
at the head of the queue (arrival order, no overtaking) starts on it if its
device memory fits the HBM budget beside everything in use; a request that
arrives while others run is admitted as soon as a slot and memory free up.

A request that repeats an earlier request's S (the SCF steps of one
geometry, the re-initialization semantics of Sec. 2.7) finds that S still
resident on the device, and is sent to the slot whose handle factored it
when that slot is free: the library keeps the factor of S per handle, keyed
by the content of S, so the Cholesky factorization is skipped.

Latency is completion minus arrival on the host clock.  Inputs come from a
`make(spec, base, device)` callable run on the slot's stream (host arrays
copied in, or matrices drawn on the device).

Memory accounting (the budget covers the slots' library workspaces, the
resident overlap matrices and each running request's H, D and E): a slot's
handle keeps the workspace of its last request; resident overlap matrices
beyond half the budget are dropped, oldest first, unless a running request
uses them.
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


def request_bytes(n: int, cplx: bool, task_bytes) -> float:
    """Device bytes a request needs while it runs: its task context and H, D,
    E (S is accounted with the resident overlap matrices)."""
    return task_bytes(n, cplx) + 3.0 * matrix_bytes(n, cplx)


def admit(queue_, budget, resident, task_bytes):
    """Requests of `queue_` (arrival order) that fit together: the longest
    prefix whose needs plus the resident bytes fit the budget, and at least
    the first request.  Returns (admitted, their bytes)."""
    out, need = [], 0.0
    for r in queue_:
        b = request_bytes(r["n"], r["cplx"], task_bytes)
        if out and resident + need + b > budget:
            break
        out.append(r)
        need += b
    return out, need


def start_bytes(req, slot_held, task_bytes, s_resident):
    """Extra device bytes a request adds when it starts on a slot whose
    handle holds slot_held bytes of workspace: its matrices H, D, E, its S
    unless resident, and the growth of the slot's workspace."""
    n, cplx = req["n"], req["cplx"]
    extra = 3.0 * matrix_bytes(n, cplx) + (0.0 if s_resident else matrix_bytes(n, cplx))
    return extra + max(0.0, task_bytes(n, cplx) - slot_held)


def pick_slot(req, free_slots, affinity):
    """The free slot for a request: the one whose handle factored its S
    (affinity: base request id -> slot), else the lowest-numbered free slot."""
    k = affinity.get(req["base"])
    if k is not None and k in free_slots:
        return k
    return min(free_slots)


class _Slot:
    def __init__(self, idx, device, outbox, timing_level):
        self.idx = idx
        self.device = device
        self.outbox = outbox
        self.inbox = queue.Queue()
        self.h = hsdm.Handle(device)
        self.h.hsdm_set_int(hsdm.HSDM_KEY_CONCURRENT, 1)
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
            req, S_in, make, keep_out, t0, clock = job
            try:
                with torch.cuda.stream(stream):
                    start = clock() - t0
                    H, S = make(req, S_in)
                    if S_in is None:
                        stream.synchronize()  # S is shared with later repeats on other slots
                    f = self.h.hsdm_solve_dm_complex if req["cplx"] else self.h.hsdm_solve_dm_real
                    self.h.hsdm_set_real(hsdm.HSDM_KEY_FMAX, req["f_max"])
                    o = f(H, S, req["n_electrons"], req["kT"])
                    stream.synchronize()
                    done = clock() - t0
                    held = self.h.hsdm_workspace_bytes()
                    res = dict(mu=o["mu"], band_energy=o["band_energy"], start=start, done=done)
                    if keep_out:
                        res["D"], res["E"] = o["D"], o["E"]
                    del H, o
                self.outbox.put((self.idx, req, S, res, held, None))
            except Exception as e:  # reported by the dispatcher
                self.outbox.put((self.idx, req, None, None, self.held, e))

    def close(self):
        self.inbox.put(None)
        self.thread.join()
        self.h.close()


class Server:
    def __init__(self, device=0, hbm_budget=200e9, slots=4, timing_level=0):
        self.dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.budget = float(hbm_budget)
        self.outbox = queue.Queue()
        self.slots = [_Slot(k, self.dev, self.outbox, timing_level) for k in range(slots)]
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

    def run(self, requests, make, keep=None, clock=time.perf_counter, log=None, warm=False):
        """Replay `requests` (dicts with rid, arrival, n, cplx, base, repeat,
        n_electrons, kT, f_max; sorted by arrival) against the clock;
        make(req, S or None) -> device (H, S) on the calling slot's stream.
        Returns one record per request: rid, arrival, start, done, latency,
        slot, concurrent (requests running when it started), mu,
        band_energy, and D, E when keep(rid) is true."""
        pending = list(requests)
        waiting, records = [], []
        free = set(range(len(self.slots)))
        running = {}  # slot -> (request, matrix bytes)
        t0 = clock()
        task_bytes = hsdm.hsdm_task_bytes
        while pending or waiting or running:
            now = clock() - t0
            while pending and pending[0]["arrival"] <= now:
                waiting.append(pending.pop(0))
            # start the head of the queue while a slot and memory are free
            while waiting and free:
                req = waiting[0]
                k = pick_slot(req, free, self.affinity)
                res_s = req["base"] in self.s_dev
                in_use = (sum(s.held for s in self.slots) + self._resident_bytes()
                          + sum(b for _, b in running.values()))
                need = start_bytes(req, self.slots[k].held, task_bytes, res_s)
                if running and in_use + need > self.budget:
                    break
                waiting.pop(0)
                free.discard(k)
                mats = 3.0 * matrix_bytes(req["n"], req["cplx"])
                running[k] = (req, mats + max(0.0, task_bytes(req["n"], req["cplx"])
                                             - self.slots[k].held))
                S = self.s_dev.get(req["base"])
                if S is not None:
                    self.s_dev.move_to_end(req["base"])
                self.s_users[req["base"]] = self.s_users.get(req["base"], 0) + 1
                req = dict(req, concurrent=len(running) - 1)
                keep_out = keep is not None and keep(req["rid"])
                self.slots[k].inbox.put((req, S, make, keep_out, t0, clock))
            # wait for a completion or the next arrival
            timeout = None
            if pending and (not waiting or free):
                timeout = max(0.0, pending[0]["arrival"] - (clock() - t0))
            if not running:
                if timeout is not None:
                    time.sleep(timeout)
                continue
            try:
                k, req, S, res, held, err = self.outbox.get(timeout=timeout)
            except queue.Empty:
                continue
            if err is not None:
                raise RuntimeError(f"request {req['rid']} failed on slot {k}") from err
            running.pop(k)
            free.add(k)
            self.slots[k].held = held
            self.affinity[req["base"]] = k
            b = req["base"]
            self.s_users[b] -= 1
            if b not in self.s_dev:
                self.s_dev[b] = S
            # resident overlap matrices beyond half the budget go, oldest
            # first, unless a running request uses them
            for old in list(self.s_dev):
                if self._resident_bytes() <= 0.5 * self.budget:
                    break
                if self.s_users.get(old, 0) == 0:
                    self.s_dev.pop(old)
            rec = dict(rid=req["rid"], arrival=req["arrival"], start=res["start"],
                       done=res["done"], latency=res["done"] - req["arrival"], slot=k,
                       concurrent=req["concurrent"], mu=res["mu"],
                       band_energy=res["band_energy"])
            if "D" in res:
                rec["D"], rec["E"] = res["D"], res["E"]
            records.append(rec)
            if log and len(records) % 50 == 0:
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
            "max_concurrent": max(r["concurrent"] for r in records) + 1}
