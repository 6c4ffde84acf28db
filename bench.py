"""Benchmark of the dense H,S -> D solve on one MI355X.

One step = one hsdm_solve_dm_real call on the n=16384 problem (FP64, real
symmetric, decay length 128, S perturbation 0.05, N_e = 8192, kT = 0.005)
with a cold S factor: Cholesky + inverse, standard form, full-to-band,
band-to-tridiagonal, divide and conquer with the occupations, the three
back-transformations and D, E.  Inputs are resident in HBM before the timed
region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME]
                  [--no-cpu-baseline] [--copy-calibration]

With --config cfg3_batch one step is instead one hsdm_solve_dm_batch call on
the periodic spin-polarized system: 32 k-points x 2 spins = 64 Hermitian
FP64 tasks of sizes n_k ~ U{600..3000}, one chemical potential for all
(N_e = 0.4 sum_k n_k, kT = 0.01, f_max = 1), cold S factors; the metric is
tasks solved per second.

With --config cfg4_serving it replays a stream of --requests requests
(default 2000; Poisson arrivals at 40/s, sizes log-uniform on [256, 8192],
60 % real and 40 % Hermitian, 30 % SCF repeats sharing an earlier request's
S) through the serving loop (paper_1912_13403_amd/serving.py: --slots
requests on the device at once, each slot refilled as soon as it frees) and
reports the p50 latency, with p99 and solves/s beside it.  Request matrices
are drawn on the device when the request is dispatched (its latency
includes that).

The two multi-task configurations run their tasks' own phases on 6 worker
streams, with at least 8 hardware queues for the process (GPU_MAX_HW_QUEUES
is raised to 8 when lower; with the HIP runtime's default of 4 some of the
streams would run one after another).

The roofline entry is that of the kernel with the largest total time over the
timed steps, from HIP events recorded around each of its launches on the
solve's stream; its "traffic" comes from the committed counter summary
profiles/traffic_<config>.json while the kernel's source is unchanged.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# grouped multi-task kernels launched on the caller's stream while the worker
# streams are idle
ALONE_KERNELS = ("sb2st_group_kernel<32>", "bt2_group_kernel")
MT_QUEUES, MT_STREAMS = 8, 6  # hardware queues and worker streams of the multi-task configurations
FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix-core peak


def make_inputs(name, dev):
    import numpy as np
    import torch

    from paper_1912_13403_amd import inputs

    def gram(B):
        Bt = torch.from_numpy(B).to(dev)
        G = (Bt @ Bt.T).cpu().numpy()
        del Bt
        torch.cuda.empty_cache()
        return G

    H, S, p = inputs.config_problem(name, gram=gram)
    Hd = torch.from_numpy(np.asfortranarray(H)).to(dev)
    Sd = torch.from_numpy(np.asfortranarray(S)).to(dev)
    return H, S, Hd, Sd, p


def cpu_baseline(target_n: int):
    """Time the FP64 oracle on a bounded sample of the workload -- the n=4096
    problem drawn with the n=16384 recipe (decay 128, S perturbation 0.05,
    N_e = n/2, kT = 0.005), all host cores -- and project it by n^3 to the
    benchmarked size (the oracle at n = 16384 would take most of an hour)."""
    from oracle import oracle as O
    from paper_1912_13403_amd import inputs

    H, S, p = inputs.config_problem("cfg2sub_n4096")
    ns = p["n"]
    t0 = time.perf_counter()
    ref = O.solve_dm(H, S, p["n_electrons"], p["kT"], f_max=p["f_max"])
    dt = time.perf_counter() - t0
    scale = (target_n / ns) ** 3
    return ref, {
        "value": dt * scale,
        "unit": "s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "projection": True,
        "sample": (f"oracle solve_dm on the n={ns} problem of the n={target_n} recipe "
                   f"(decay 128, S perturbation 0.05, N_e={ns // 2}, kT=0.005) took "
                   f"{dt:.2f} s on {O.num_threads()} threads; value = that time x "
                   f"(n/{ns})^3, a projection"),
        "sample_seconds": dt,
    }


def oracle_timing():
    """The oracle on the small configurations, single-threaded and on all
    host cores (one subprocess per run, so that the thread count is fixed
    before OpenMP starts); one JSON line."""
    import platform
    import subprocess

    code = ("import sys, time, json; sys.path.insert(0, %r)\n"
            "from oracle import oracle as O\n"
            "from paper_1912_13403_amd import inputs\n"
            "H, S, p = inputs.config_problem(sys.argv[1])\n"
            "O.num_threads()\n"
            "t = time.perf_counter()\n"
            "O.solve_dm(H, S, p['n_electrons'], p['kT'], f_max=p['f_max'])\n"
            "print(json.dumps({'s': time.perf_counter() - t, 'threads': O.num_threads()}))\n"
            % ROOT)
    ncpu = os.cpu_count() or 1
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    runs = []
    for name in ("cfg0_n512", "cfg1_n4096", "cfg2sub_n4096"):
        for threads in (1, ncpu):
            env = dict(os.environ, OMP_NUM_THREADS=str(threads), ORC_PROGRESS="1")
            print(f"[oracle-timing] {name} threads={threads}: start", file=sys.stderr, flush=True)
            # the oracle's step reports go straight to this process's stderr
            r = subprocess.run([sys.executable, "-c", code, name], env=env,
                               stdout=subprocess.PIPE, text=True, check=True)
            rec = json.loads(r.stdout.strip().splitlines()[-1])
            runs.append({"config": name, "threads": rec["threads"], "seconds": rec["s"]})
            print(f"[oracle-timing] {name} threads={rec['threads']}: {rec['s']:.2f} s",
                  file=sys.stderr, flush=True)
    print(json.dumps({"oracle_timing": runs, "nproc": ncpu, "cpu_model": model,
                      "machine": platform.machine(),
                      "build": "gcc -O3 -march=x86-64-v3 -fopenmp -ffp-contract=off"}))


# source file of each timed kernel (a stored traffic measurement is only used
# while the kernel's source is unchanged)
KERNEL_SOURCES = {
    "gemm_kernel": ["gemm.hip", "hsdm_internal.h", "hsdm_util.h"],
    "gemm_batched_kernel": ["gemm.hip", "hsdm_internal.h", "hsdm_util.h"],
    "sb2st_kernel": ["sb2st.hip", "hsdm_internal.h"],
    "sb2st_group_kernel": ["sb2st.hip", "hsdm_internal.h"],
    "bt2_strip_kernel": ["bt.hip", "hsdm_internal.h"],
    "panel_qr_kernel": ["sy2sb.hip", "hsdm_internal.h"],
    "dm_kernel": ["dm.hip", "hsdm_internal.h", "hsdm_util.h"],
    "sym_pair_kernel": ["gemm.hip", "hsdm_internal.h", "hsdm_util.h"],
}


def kernel_source_sha(name: str):
    import hashlib
    base = name.split("<")[0]
    files = KERNEL_SOURCES.get(base)
    if not files:
        return None
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, "paper_1912_13403_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each divided by the copy-kernel calibration
    factor), or None if there is none for this kernel and source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("source_sha1") != kernel_source_sha(kernel):
        return None
    return (k["fetch_kib_per_dispatch"] / rec["copy_factor_fetch"]
            + k["write_kib_per_dispatch"] / rec["copy_factor_write"]) * 1024.0


FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
HBM_PEAK_GBS = 8000.0     # MI355X HBM3E


def roofline(stats, workload, steps, chain=None):
    """Roofline of the kernel with the largest total time in the timed steps:
    algorithmic flops (or bytes) per launch over the mean launch time from the
    HIP events recorded around every launch.  `chain`: task steps on the
    critical path of one bulge-chasing launch (its per-task period is
    reported beside the fractions)."""
    name = max(stats, key=lambda k: stats[k]["ms"])
    st = stats[name]
    per_launch_s = st["ms"] * 1e-3 / st["launches"]
    # the bulge chasing and the panel QR do vector work on data that one
    # launch must stream once (the band in and the reflectors out; the
    # panel): measured against HBM with those algorithmic bytes, their FP64
    # rate beside it; the GEMM-shaped kernels against the matrix cores
    by_bytes = name.startswith(("sb2st", "panel_qr")) or st["flops"] <= 0
    tflops = st["flops"] / st["launches"] / per_launch_s / 1e12
    algo_bytes = st["bytes"] / st["launches"]
    if by_bytes:
        achieved = algo_bytes / per_launch_s / 1e9
        peak, unit, bound = HBM_PEAK_GBS, "GB/s", "hbm"
    else:
        achieved = tflops
        peak, unit, bound = FP64_PEAK_TFLOPS, "TFLOP/s", "mfma"
    traffic = stored_traffic(workload, name)
    out = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
           "frac": achieved / peak, "traffic": traffic,
           "traffic_over_algorithmic": (traffic / algo_bytes) if traffic and algo_bytes > 0
           else None,
           "kernel": name, "launches_per_step": st["launches"] / steps,
           "mean_launch_ms": 1e3 * per_launch_s,
           "algorithmic_flops_per_launch": st["flops"] / st["launches"],
           "algorithmic_bytes_per_launch": algo_bytes,
           "fp64_tflops": tflops, "fp64_frac": tflops / FP64_PEAK_TFLOPS}
    if chain and name.startswith("sb2st"):
        out["chain_task_steps"] = chain
        out["task_period_us"] = 1e6 * per_launch_s / chain
    return out


def phase_table(phases_ms, phase_flops):
    """Per-phase algorithmic flops (the method's counts), rate and fraction of
    the FP64 matrix-core peak."""
    out = {}
    for k, ms in phases_ms.items():
        fl = phase_flops.get(k, 0.0)
        tf = fl / (ms * 1e-3) / 1e12 if ms > 0 and fl > 0 else None
        out[k] = {"ms": ms, "algorithmic_flops": fl, "tflops": tf,
                  "frac_fp64_peak": (tf / FP64_PEAK_TFLOPS) if tf is not None else None}
    return out


def batch_cpu_baseline(sizes):
    """The oracle on one task of the batch recipe at n = 1500, scaled by
    sum_p (n_p / 1500)^3 over the 64 tasks."""
    from oracle import oracle as O
    from paper_1912_13403_amd import inputs

    ns = 1500
    Hu, Hd, S = inputs.kpoint_problem(0, n=ns)
    t0 = time.perf_counter()
    O.solve_dm_complex(Hu, S, 0.2 * ns, 0.01, f_max=1.0)
    dt = time.perf_counter() - t0
    scale = sum((2 * (n / ns) ** 3) for n in sizes)
    return {
        "value": 2 * len(sizes) / (dt * scale),
        "unit": "solves/s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": (f"oracle solve_dm_complex on one n={ns} task of the k-point recipe took "
                   f"{dt:.2f} s; value = 64 / (that time x sum over the 64 tasks of (n_k/{ns})^3)"),
        "sample_seconds": dt,
    }


def batch_main(args):
    import numpy as np
    import torch

    from paper_1912_13403_amd import hsdm, inputs

    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    sizes = inputs.kpoint_sizes()
    Hs, Ss = [], []
    for k in range(len(sizes)):
        Hu, Hd, S = inputs.kpoint_problem(k)
        Sg = torch.from_numpy(S).to(dev)
        Hs += [torch.from_numpy(Hu).to(dev), torch.from_numpy(Hd).to(dev)]
        Ss += [Sg, Sg]
        del Hu, Hd, S
    ntask = len(Hs)
    ne, kT = 0.4 * sum(sizes), 0.01
    print(f"[bench] {ntask} tasks ready (sum n_k = {sum(sizes)}) in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    h = hsdm.Handle(0)
    h.hsdm_set_real(hsdm.HSDM_KEY_FMAX, 1.0)
    h.hsdm_set_int(hsdm.HSDM_KEY_TIMING, 2)
    h.hsdm_set_int(hsdm.HSDM_KEY_STREAMS, MT_STREAMS)
    refined = args.precision == "refined"
    if refined:
        h.hsdm_set_int(hsdm.HSDM_KEY_PRECISION, 1)

    def step():
        h.hsdm_reinit()
        return h.hsdm_solve_dm_batch(Hs, Ss, ne, kT)

    calib = None
    for i in range(max(1, args.warmup)):
        step()
        torch.cuda.synchronize()
        if i == 0:
            calib = h.kernel_stats()
            h.hsdm_set_int(hsdm.HSDM_KEY_TIMING, 3)
        print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)
    times, kstats = [], []
    t_all = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        r = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        kstats.append(h.kernel_stats())
        print(f"[bench] step {i}: {times[-1]:.3f}s", file=sys.stderr, flush=True)
    total = time.perf_counter() - t_all
    ts = time.perf_counter()
    h.hsdm_solve_dm_batch(Hs, Ss, ne, kT)
    torch.cuda.synchronize()
    warm = time.perf_counter() - ts
    vs_fp64 = None
    if refined:
        # the same batch in the FP64 form, for the differences of the results
        h.hsdm_set_int(hsdm.HSDM_KEY_PRECISION, 0)
        h.hsdm_reinit()
        f = h.hsdm_solve_dm_batch(Hs, Ss, ne, kT)
        torch.cuda.synchronize()
        vs_fp64 = {
            "max_abs_dD": max(torch.max(torch.abs(a - b)).item() for a, b in zip(r["D"], f["D"])),
            "max_abs_dE": max(torch.max(torch.abs(a - b)).item() for a, b in zip(r["E"], f["E"])),
            "abs_dmu": abs(r["mu"] - f["mu"]),
            "abs_dband_energy": abs(r["band_energy"] - f["band_energy"]),
        }
        del f
    agg = {}
    for ks in kstats:
        for k, v in ks.items():
            a = agg.setdefault(k, {"ms": 0.0, "flops": 0.0, "bytes": 0.0, "launches": 0})
            for f in a:
                a[f] += v[f]
    # In the timed steps the tasks' own phases overlap on the worker streams,
    # so a launch's event time there includes its neighbours'; the roofline
    # entry is that of the largest kernel that runs alone on the caller's
    # stream (the grouped bulge chasing or stage-2 back-transform), from the
    # timed steps.
    alone = {k: v for k, v in agg.items() if k in ALONE_KERNELS and v["ms"] > 0.0}
    if alone:
        roof = roofline(alone, args.config, args.steps)
        roof["timed_in"] = "timed steps (largest kernel running alone on the device)"
    else:
        roof = roofline(calib, args.config, 1)
        roof["timed_in"] = "warmup step with every launch timed"
    top = sorted(calib.items(), key=lambda kv: -kv[1]["ms"])[:8]
    kernels = {k: {"ms_per_step": v["ms"], "launches_per_step": v["launches"],
                   "tflops": (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 and v["flops"] > 0
                   else None} for k, v in top}
    step_s = float(np.mean(times))
    rec = {
        "metric": "batched solves/s",
        "value": ntask / step_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * step_s,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32+f64" if refined else "f64",
        "data": "synthetic",
        "config": {"workload": f"cfg3_batch: {ntask} Hermitian FP64 generalized tasks "
                               f"(32 k-points x 2 spins, n_k in [{min(sizes)}, {max(sizes)}]), "
                               f"one mu, N_e={ne:.1f}, kT={kT}, f_max=1, cold S factors"
                               + (", refined form" if refined else ""),
                   "precision": args.precision,
                   "tasks": ntask, "sum_n": sum(sizes), "n_electrons": ne, "kT": kT,
                   "worker_streams": MT_STREAMS,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "roofline": roof,
        "kernels": kernels,
        "warm_s_factor_solves_per_s": ntask / warm,
        "mu": r["mu"],
        "band_energy": r["band_energy"],
        "timed_total_s": total,
    }
    if vs_fp64 is not None:
        rec["refined_vs_fp64"] = vs_fp64
    h.close()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = batch_cpu_baseline(sizes)
    print(json.dumps(rec))


def serving_main(args):
    import numpy as np
    import torch

    from paper_1912_13403_amd import inputs, serving

    dev = torch.device("cuda", 0)
    specs = inputs.request_specs(args.requests, rate=40.0, lo=256, hi=8192, seed=0)
    make = lambda req, S: inputs.request_problem_device(req, specs[req["base"]], S, dev)
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    prec = 1 if args.precision == "refined" else 0
    srv = serving.Server(0, hbm_budget=200e9, slots=args.slots, max_group=args.group,
                         streams=MT_STREAMS if args.group > 1 else 0, precision=prec)
    # warmup: a short stream of small requests (kernels loaded, workspaces made)
    wspecs = inputs.request_specs(2 * args.slots, rate=1000.0, lo=256, hi=512, seed=99)
    wmake = lambda req, S: inputs.request_problem_device(req, wspecs[req["base"]], S, dev)
    srv.run(wspecs, wmake)  # (also sizes the refined form's workspaces)
    srv.s_dev.clear()
    srv.affinity.clear()
    torch.cuda.synchronize()
    log(f"replaying {len(specs)} requests on {args.slots} slots")
    try:
        ts = time.perf_counter()
        recs = srv.run(specs, make, log=log)
        wall = time.perf_counter() - ts
    finally:
        srv.close()
    summ = serving.summarize(recs)
    conc = np.array([r["concurrent"] + 1 for r in recs])
    rec = {
        "metric": "serving p50 latency",
        "value": summ["p50_s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": 1000.0 * wall,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64" if not prec else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"cfg4_serving: {len(specs)} requests, Poisson 40/s, n log-uniform "
                               "[256, 8192], 60% real / 40% Hermitian FP64, 30% SCF repeats, "
                               "HBM budget 200 GB, continuous batching over "
                               f"{args.slots} slots, up to {args.group} requests per start "
                               "(inputs drawn on the device at dispatch)"
                               + (", refined form" if prec else ""),
                   "requests": len(specs), "slots": args.slots, "max_group": args.group,
                   "precision": args.precision,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "p99_s": summ["p99_s"],
        "mean_latency_s": summ["mean_s"],
        "solves_per_s": summ["solves_per_s"],
        "offered_rate_per_s": 40.0,
        "mean_requests_on_device_at_start": float(conc.mean()),
        "mean_group": summ["mean_group"],
        "max_requests_on_device": int(conc.max()),
        "timed_total_s": wall,
        "roofline": None,
    }
    print(json.dumps(rec))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="cfg2_n16384")
    ap.add_argument("--requests", type=int, default=2000,
                    help="requests replayed by --config cfg4_serving")
    ap.add_argument("--group", type=int, default=16,
                    help="most requests started together on a slot by --config cfg4_serving "
                         "(1: single solves)")
    ap.add_argument("--slots", type=int, default=2,
                    help="concurrent request slots of --config cfg4_serving")
    ap.add_argument("--refine-steps", type=int, default=8,
                    help="most refinement steps of the refined form (HSDM_KEY_REFINE_STEPS)")
    ap.add_argument("--autotune", action="store_true",
                    help="run one untimed solve with the GEMM tile autotuner first "
                         "(HSDM_KEY_AUTOTUNE); the timed steps use its table")
    ap.add_argument("--precision", choices=["fp64", "refined"], default="fp64",
                    help="arithmetic of the solves of --config cfg3_batch and cfg4_serving "
                         "(refined: HSDM_KEY_PRECISION = 1)")
    ap.add_argument("--no-refined", action="store_true",
                    help="skip the refined form's steps (e.g. under a profiler)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-warm", action="store_true",
                    help="skip the extra solve with the S factor cached")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="time the CPU oracle on the small configurations, one thread and all "
                         "host cores, and print that record instead of a benchmark")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain device copy of 2 GiB (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters of a profiled run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    if args.oracle_timing:
        return oracle_timing()
    if args.config in ("cfg3_batch", "cfg4_serving"):
        # read by the HIP runtime when it starts (the first device call)
        if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < MT_QUEUES:
            os.environ["GPU_MAX_HW_QUEUES"] = str(MT_QUEUES)
    if args.config == "cfg3_batch":
        return batch_main(args)
    if args.config == "cfg4_serving":
        return serving_main(args)

    import numpy as np
    import torch

    from paper_1912_13403_amd import hsdm

    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {src.numel() * 8} bytes read, {dst.numel() * 8} written",
              file=sys.stderr, flush=True)
        del src, dst
        torch.cuda.empty_cache()
    t0 = time.perf_counter()
    H, S, Hd, Sd, p = make_inputs(args.config, dev)
    n = p["n"]
    print(f"[bench] inputs ready n={n} in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    h = hsdm.Handle(0)
    tile_classes = None
    if args.autotune:
        # one untimed solve with the tile autotuner on: each product class of
        # the solve times the candidate tiles once; the steps below use the table
        h.hsdm_set_int(hsdm.HSDM_KEY_AUTOTUNE, 1)
        h.hsdm_solve_dm_real(Hd, Sd, p["n_electrons"], p["kT"])
        h.hsdm_set_int(hsdm.HSDM_KEY_AUTOTUNE, 0)
        torch.cuda.synchronize()
        tile_classes = hsdm.load_library().hsdm_tune_entries()
        print(f"[bench] autotune: {tile_classes} product classes timed", file=sys.stderr,
              flush=True)
    # The first warmup step times every launch (timing level 2) to find the
    # dominant kernel; the timed steps then record events only around that
    # kernel's launches, so the other launches of a solve carry no event
    # overhead.
    h.hsdm_set_int(hsdm.HSDM_KEY_TIMING, 2)
    D = hsdm.empty_colmajor(n, n, dev)
    E = hsdm.empty_colmajor(n, n, dev)
    w = torch.empty(n, dtype=torch.float64, device=dev)
    out = (D, E, w)

    def step():
        h.hsdm_reinit()
        return h.hsdm_solve_dm_real(Hd, Sd, p["n_electrons"], p["kT"], out=out)

    calib = None
    for i in range(max(1, args.warmup)):
        step()
        torch.cuda.synchronize()
        if i == 0:
            calib = h.kernel_stats()
            dom = max(calib.items(), key=lambda kv: kv[1]["ms"]) if calib else None
            if dom is not None:
                # the timed steps record events only around the dominant
                # kernel's launches (and the nine phase boundaries)
                h.hsdm_timing_kernel(dom[0])
        print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times, phases, pflops, kstats = [], [], [], []
    t_all = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        r = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        phases.append(h.phase_times())
        pflops.append(h.phase_flops())
        kstats.append(h.kernel_stats())
        print(f"[bench] step {i}: {times[-1]:.3f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    # warm S factor (SCF repeat: the factor of S is reused), outside the timed steps
    warm = None
    if not args.skip_warm:
        ts = time.perf_counter()
        h.hsdm_solve_dm_real(Hd, Sd, p["n_electrons"], p["kT"], out=out)
        torch.cuda.synchronize()
        warm = time.perf_counter() - ts

    ph = {k: float(np.median([q[k] for q in phases])) for k in phases[0]}
    f_cut = 1e-16 * p["f_max"]
    # occupied-state count from the returned eigenvalues and mu
    ev = w.cpu().numpy()
    x = (ev - r["mu"]) / p["kT"]
    f = p["f_max"] / (1.0 + np.exp(np.clip(x, -700, 700)))
    m = int(np.sum(f > f_cut))
    # per-kernel totals summed over the timed steps
    agg = {}
    for ks in kstats:
        for k, v in ks.items():
            a = agg.setdefault(k, {"ms": 0.0, "flops": 0.0, "bytes": 0.0, "launches": 0})
            for f in a:
                a[f] += v[f]
    B = 32
    chain = 2 * max(n - 2, 0) + (n - 1 + B - 1) // B
    roof = roofline(agg, args.config, args.steps, chain=chain)
    # per-kernel table: every launch timed (the calibration step when there
    # is one, else the timed steps)
    table, tsteps = (calib, 1) if calib else (agg, args.steps)
    top = sorted(table.items(), key=lambda kv: -kv[1]["ms"])[:8]
    kernels = {k: {"ms_per_step": v["ms"] / tsteps, "launches_per_step": v["launches"] // tsteps,
                   "tflops": (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 and v["flops"] > 0
                   else None} for k, v in top}
    ms = 1000.0 * float(np.mean(times))
    rec = {
        "metric": "n=16384 H,S->D solve time",
        "value": ms / 1000.0,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: real symmetric FP64 generalized H,S->D, n={n}, "
                               f"N_e={p['n_electrons']:.0f}, kT={p['kT']}, cold S factor",
                   "n": n, "n_electrons": p["n_electrons"], "kT": p["kT"], "m_occupied": m},
        "roofline": roof,
        "phases_ms": ph,
        "phases": phase_table(ph, pflops[-1]),
        "dominant_phase": max(ph, key=lambda k: ph[k]),
        "kernels": kernels,
        "warm_s_factor_s": warm,
        "gemm_tiles": ({"autotuned_classes": tile_classes} if tile_classes is not None
                       else "built-in rule"),
        "mu": r["mu"],
        "band_energy": r["band_energy"],
        "timed_total_s": total,
    }
    # the device's own rates beside the published peaks the roofline uses
    mf = h.hsdm_probe(0, 20000)
    cp = h.hsdm_probe(1, float(1 << 30))
    rec["measured_peaks"] = {
        "fp64_mfma_tflops": mf[0], "hbm_copy_gbps": cp[0],
        "method": "hsdm_probe after the timed steps: FP64 16x16x4 MFMA chains on 2 workgroups "
                  "of 4 wavefronts per CU (8 independent accumulators per wavefront, 20000 "
                  "rounds); a 1 GiB device copy (bytes read + written), second launch timed"}
    h.close()
    if not args.no_refined:
        rec["refined_form"] = refined_form(args, Hd, Sd, p, D, E, w)
    if not args.no_cpu_baseline:
        ref, rec["cpu_baseline"] = cpu_baseline(n)
        rec["error_vs_oracle_n4096"] = forms_vs_oracle(ref, dev)
    print(json.dumps(rec))


def refined_form(args, Hd, Sd, p, D64, E64, w64):
    """The refined form (HSDM_KEY_PRECISION = 1) on the same inputs: one
    warmup and the same number of timed steps, its phases, refinement record
    and largest differences from the FP64 form's D, E and eigenvalues."""
    import numpy as np
    import torch

    from paper_1912_13403_amd import hsdm

    h = hsdm.Handle(0)
    try:
        h.hsdm_set_int(hsdm.HSDM_KEY_PRECISION, 1)
        h.hsdm_set_int(hsdm.HSDM_KEY_REFINE_STEPS, args.refine_steps)
        if args.autotune:
            h.hsdm_set_int(hsdm.HSDM_KEY_AUTOTUNE, 1)
            h.hsdm_solve_dm_real(Hd, Sd, p["n_electrons"], p["kT"])
            h.hsdm_set_int(hsdm.HSDM_KEY_AUTOTUNE, 0)
        h.hsdm_set_int(hsdm.HSDM_KEY_TIMING, 1)
        times, phases = [], []
        for i in range(1 + args.steps):
            h.hsdm_reinit()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            r = h.hsdm_solve_dm_real(Hd, Sd, p["n_electrons"], p["kT"])
            torch.cuda.synchronize()
            if i > 0:
                times.append(time.perf_counter() - ts)
                phases.append(h.phase_times())
            print(f"[bench] refined form step {i}: {time.perf_counter() - ts:.3f}s",
                  file=sys.stderr, flush=True)
        hist = h.refine_history()
        ph = {k: float(np.median([q[k] for q in phases])) for k in phases[0]}
        out = {
            "ms_per_step": 1000.0 * float(np.mean(times)),
            "steps": args.steps,
            "phases_ms": ph,
            "refinement_steps": [{"delta": a, "max_correction": b} for a, b in hist],
            "max_abs_dD_vs_fp64": float(torch.max(torch.abs(r["D"] - D64)).item()),
            "max_abs_dE_vs_fp64": float(torch.max(torch.abs(r["E"] - E64)).item()),
            "max_abs_deig_vs_fp64": float(torch.max(torch.abs(r["eval"] - w64)).item()),
            "mu": r["mu"],
            "band_energy": r["band_energy"],
        }
        del r
        return out
    finally:
        h.close()


def forms_vs_oracle(ref, dev):
    """Largest errors of both forms against the FP64 oracle on the n = 4096
    problem of the n = 16384 recipe (the oracle's solution from the CPU
    baseline run)."""
    import numpy as np
    import torch

    from paper_1912_13403_amd import hsdm, inputs

    H, S, p = inputs.config_problem("cfg2sub_n4096")
    Hd, Sd = torch.from_numpy(H).to(dev), torch.from_numpy(S).to(dev)
    scale = float(np.abs(H).sum(axis=0).max())
    res = {"norm1_H": scale}
    for name, prec in (("fp64", 0), ("refined", 1)):
        with hsdm.Handle(0) as h:
            h.hsdm_set_int(hsdm.HSDM_KEY_PRECISION, prec)
            o = h.hsdm_solve_dm_real(Hd, Sd, p["n_electrons"], p["kT"])
            res[name] = {
                "max_abs_dD": float(np.abs(o["D"].cpu().numpy() - ref["D"]).max()),
                "max_abs_dE": float(np.abs(o["E"].cpu().numpy() - ref["E"]).max()),
                "max_abs_deig": float(np.abs(o["eval"].cpu().numpy() - ref["eval"]).max()),
                "abs_dmu": abs(o["mu"] - ref["mu"]),
                "refinement_steps": len(h.refine_history()),
            }
    return res


if __name__ == "__main__":
    main()
