"""Serving loop for H,S -> D requests on one GPU: continuous batching by rounds.

Requests (real or Hermitian, any size) arrive over time.  Whenever the device
finishes a round, every request that has arrived by then is admitted, in
arrival order, while the HBM budget allows, and the admitted requests run as
one hsdm_solve_dm_group call: each with its own occupations, their bands
chased in shared cooperative launches.  A request that repeats an earlier
request's S (the SCF steps of one geometry, the re-initialization semantics
of Sec. 2.7) finds that S still on the device and its factor in a library
task context, so its Cholesky factorization is skipped.  Latency is
completion minus arrival on the host clock; a request's host matrices are
copied to the device inside its round.

Memory accounting (the budget covers the library's task contexts, the
resident overlap matrices and the round's inputs and outputs): before a round
the library releases least recently used task contexts down to what the
budget leaves after the round's needs, and resident overlap matrices beyond
the budget are dropped, oldest first.
"""
from __future__ import annotations

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


def admit(queue, budget, resident, task_bytes):
    """Requests of `queue` (arrival order) admitted into the next round: the
    longest prefix whose needs plus the resident bytes fit the budget, and at
    least the first request.  Returns (admitted, their bytes)."""
    out, need = [], 0.0
    for r in queue:
        b = request_bytes(r["n"], r["cplx"], task_bytes)
        if out and resident + need + b > budget:
            break
        out.append(r)
        need += b
    return out, need


class Server:
    def __init__(self, device=0, hbm_budget=200e9, timing_level=0, streams=None):
        self.h = hsdm.Handle(device)
        self.dev = self.h.device
        self.budget = float(hbm_budget)
        self.s_dev = OrderedDict()  # base request id -> resident S on the device
        if timing_level:
            self.h.hsdm_set_int(hsdm.HSDM_KEY_TIMING, timing_level)
        if streams:
            self.h.hsdm_set_int(hsdm.HSDM_KEY_STREAMS, streams)

    def close(self):
        self.s_dev.clear()
        self.h.close()

    def _resident_bytes(self):
        return sum(matrix_bytes(x.shape[0], x.dtype == torch.complex128)
                   for x in self.s_dev.values())

    def _s_for(self, req):
        key = req["base"]
        if key in self.s_dev:
            self.s_dev.move_to_end(key)
            return self.s_dev[key]
        S = torch.from_numpy(np.asfortranarray(req["S"])).to(self.dev)
        S = S.t().contiguous().t()  # column-major, as the library reads it
        self.s_dev[key] = S
        return S

    def run_round(self, batch):
        """Solve the admitted requests in one group call; returns their results."""
        tasks = []
        for r in batch:
            H = torch.from_numpy(np.asfortranarray(r["H"])).to(self.dev)
            tasks.append(dict(H=H.t().contiguous().t(), S=self._s_for(r),
                              n_electrons=r["n_electrons"], kT=r["kT"], f_max=r["f_max"]))
        out = self.h.hsdm_solve_dm_group(tasks)
        torch.cuda.synchronize(self.dev)
        return out

    def run(self, requests, keep=None, clock=time.perf_counter, log=None):
        """Replay `requests` (dicts with rid, arrival, n, cplx, base, H, S,
        n_electrons, kT, f_max; sorted by arrival) against the clock.  Returns
        one record per request: rid, arrival, start, done, latency, round,
        round_size, mu, band_energy, and D, E when keep(rid) is true."""
        pending = list(requests)
        queue, records = [], []
        t0 = clock()
        rounds = 0
        task_bytes = hsdm.hsdm_task_bytes
        while pending or queue:
            now = clock() - t0
            while pending and pending[0]["arrival"] <= now:
                queue.append(pending.pop(0))
            if not queue:
                time.sleep(max(0.0, pending[0]["arrival"] - now))
                continue
            # overlap matrices beyond the budget are dropped, oldest first
            base_needed = {r["base"] for r in queue}
            while self.s_dev and self._resident_bytes() > 0.5 * self.budget:
                old = next(iter(self.s_dev))
                if old in base_needed and len(self.s_dev) == 1:
                    break
                self.s_dev.pop(old)
            resident = self._resident_bytes()
            batch, need = admit(queue, self.budget, resident, task_bytes)
            queue = queue[len(batch):]
            self.h.hsdm_release_tasks(max(0.0, self.budget - resident - need))
            start = clock() - t0
            out = self.run_round(batch)
            done = clock() - t0
            rounds += 1
            for r, o in zip(batch, out):
                rec = dict(rid=r["rid"], arrival=r["arrival"], start=start, done=done,
                           latency=done - r["arrival"], round=rounds, round_size=len(batch),
                           mu=o["mu"], band_energy=o["band_energy"])
                if keep is not None and keep(r["rid"]):
                    rec["D"], rec["E"] = o["D"], o["E"]
                records.append(rec)
            if log:
                log(f"round {rounds}: {len(batch)} requests, {done - start:.3f}s, "
                    f"queue {len(queue)}, pending {len(pending)}")
        return records


def summarize(records):
    lat = np.array([r["latency"] for r in records])
    span = max(r["done"] for r in records) - min(r["arrival"] for r in records)
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "solves_per_s": len(records) / span,
            "requests": len(records), "rounds": max(r["round"] for r in records)}
