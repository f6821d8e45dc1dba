"""Benchmark of the race-check hot path on one MI355X.

A step is one pass of the whole path (interpretation, access logging, interval
checks, ordered race report) over one batch of synthetic instances, with inputs
seeded on the device.  Prints one JSON line.

    python bench.py [--config c2] [--steps K] [--warmup W] [--seeds N]

Configs: c1 (one random 20-statement kernel, 1 x 64, 1000 seeds),
c2 (six template kernels, 16 x 256, 10^4 seeds each; the default),
c3 (random kernels of widths 32..1024 in one batched call; --programs x --seeds),
c4 (large intervals, 64 x 1024 x 64 iterations, 16 seeds),
c5 (learned triage over the c3 generator: train, then sweep held-out
instances in learned and in plain order).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# algorithmic bytes per race-checked access: the simulated cell (4 B), the
# 12-byte access record written once (interpretation) and read once (check)
ALGO_BYTES = {"interpret": 16.0, "interval_check": 12.0}
KERNEL_OF_PHASE = {"interpret": "rc_interp_kernel", "log_sort": "rs_scatter_kernel/rs_hist_kernel",
                   "interval_check": "seg_check_kernel+seg_long_kernel",
                   "record_sort": "rs_scatter_kernel/rs_hist_kernel",
                   "output": "rec_gather_kernel", "setup": "fill kernels"}


def kernel_source_hash() -> str:
    """Hash of the HIP sources: counter-derived traffic is valid only for
    the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1308_3203_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload_name: str):
    """HBM bytes per launch of `kernel` on `workload_name` from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by the copy-kernel
    calibration), or None when absent or taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            table = json.load(fh)
    except (OSError, ValueError):
        return None
    e = table.get(f"{kernel}|{workload_name}")
    if not e or e.get("source_sha256_16") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def copy_probe(gib: float, reps: int = 3):
    """A plain device-to-device copy of known size, to calibrate the HBM
    byte counters (run under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)."""
    import torch
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "reps": reps,
                      "gbs": round(2 * n * 4 / dt / 1e9, 1)}), flush=True)


def workload(name: str, seeds: int | None):
    from paper_1308_3203_amd import workloads as WL
    if name == "c1":
        return [(WL.c1_kernel(1), seeds or 1000)], "c1: one random 20-statement kernel, G=1 x W=64"
    if name == "c2":
        return ([(w, seeds or 10000) for w in WL.c2_templates()],
                "c2: tree reduction, Hillis-Steele prefix sum, 32x32 tiled transpose (clean + injected), G=16 x W=256")
    if name == "c3":
        return None, "c3: random kernels, W in {32..1024}, 10-200 statements, 1-8 barriers, one batched call"
    if name == "c4":
        return [(WL.c4_kernel(), seeds or 16)], "c4: large intervals, G=64 x W=1024 x 64 iterations, 2^20 cells"
    if name == "c5":
        return None, "c5"
    raise SystemExit(f"unknown config {name}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--seeds", type=int, default=None, help="seeds per program (default: the config's)")
    ap.add_argument("--ws-gb", type=float, default=230.0, help="workspace budget over all programs (HBM is 288 GB)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample budget (0: skip)")
    ap.add_argument("--programs", type=int, default=10000, help="c3: number of random programs")
    ap.add_argument("--tune-cache", default=None, help="c3: autotuner cache file (default: a temp file)")
    ap.add_argument("--eval-programs", type=int, default=1000, help="c5: held-out programs")
    ap.add_argument("--epochs", type=int, default=5, help="c5: training epochs")
    ap.add_argument("--chunk", type=int, default=1000, help="c5: instances per sweep call")
    ap.add_argument("--copy-probe", type=float, default=0.0, help="only run a plain copy of this many GiB")
    ap.add_argument("--no-jit", action="store_true", help="c1/c2/c4: interpret instead of per-program kernels")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1308_3203_amd import binding as B

    if args.copy_probe > 0:
        return copy_probe(args.copy_probe)
    progs, desc = workload(args.config, args.seeds)
    ctx = B.Context(0)
    if args.config == "c3":
        return bench_c3(args, ctx, desc)
    if args.config == "c5":
        return bench_c5(args, ctx)
    runs = []
    per_ws = int(args.ws_gb * (1 << 30) / len(progs))
    for w, n in progs:
        p = B.Program(ctx, w.src)
        p.set_ndrange(w.G, w.W)
        p.bind(w.arrays, w.scalars)
        if not args.no_jit:
            p.jit(True)            # compiled here, outside the timed region
        # record capacity from a probe over the first seeds (every record of
        # the timed steps is written out)
        n_probe = min(n, 16)
        probe = B.Buffers(p, n_probe, cap=1 << 22, ws_limit=per_ws)
        p.check_async(0, n_probe, probe.ws, probe.records, probe.n_records, probe.summaries)
        try:
            ctx.sync()
        except B.RcError as err:        # the count is complete even when the list is cut
            if err.status != B.RC_E_OVERFLOW:
                raise
        per_inst = int(probe.n_records.item()) / n_probe
        del probe
        cap = int(per_inst * n * 1.25) + (1 << 16)
        buf = B.Buffers(p, n, cap=cap, ws_limit=per_ws)
        runs.append((w, n, p, buf))

    def step(seed0):
        for w, n, p, buf in runs:
            p.check_async(seed0, n, buf.ws, buf.records, buf.n_records, buf.summaries)

    # warmup (also the first-use clearing of each workspace); instances checked
    # per step are deterministic, so the access count is taken here
    for i in range(max(1, args.warmup)):
        step(0)
        ctx.sync()
    accesses = 0
    records = 0
    race_instances = 0
    for w, n, p, buf in runs:
        s = B.summaries_to_numpy(buf.summaries, n)
        accesses += int(s["n_accesses"].sum())
        records += int(buf.n_records.item())
        race_instances += int((s["n_race_cells"] > 0).sum())

    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(0)
        ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    elapsed = t1 - t0
    value = accesses * args.steps / elapsed

    # roofline of the dominant phase
    dom = max(prof, key=lambda k: prof[k][0])
    ms, launches = prof[dom]
    per_launch_ms = ms / max(1, launches)
    units_per_launch = accesses * args.steps / max(1, launches)
    algo = ALGO_BYTES.get(dom, 0.0) * units_per_launch
    achieved = algo / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
    kernel = KERNEL_OF_PHASE[dom]
    if dom == "interpret" and not args.no_jit:
        kernel = "rc_jit_kernel"       # the program's own kernel runs the interpret phase
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic(kernel, args.config),
                "kernel": kernel, "phase": dom,
                "algo_bytes_per_launch": round(algo),
                "avg_launch_ms": round(per_launch_ms, 4),
                "phases_ms": {k: round(v[0] / args.steps, 3) for k, v in prof.items()},
                "path_frac": round(28.0 * value / (HBM_PEAK_GBS * 1e9), 5)}
    if dom not in ALGO_BYTES:
        roofline["note"] = ("the dominant phase is a sort, whose passes carry no algorithmic bytes "
                            "(implementation cost); path_frac is the whole path against 28 B per access")

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline([(w, n) for w, n, _, _ in runs], args.cpu_seconds)

    line = {
        "metric": "race-checked accesses/s", "value": round(value, 1), "unit": "accesses/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": desc, "execution": "interpreter" if args.no_jit else "per-program kernels",
                   "programs": len(runs), "seeds_per_program": runs[0][1],
                   "instances_per_step": sum(n for _, n, _, _ in runs),
                   "accesses_per_step": accesses, "race_records_per_step": records,
                   "racy_instances_per_step": race_instances},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_c3(args, ctx, desc):
    """The batched sweep: every (program, seed) instance of the random-kernel
    generator in one rc_batch_check call per step."""
    import tempfile
    import numpy as np
    import torch
    from paper_1308_3203_amd import binding as B
    from paper_1308_3203_amd import workloads as WL
    seeds = args.seeds or 100
    t0 = time.perf_counter()
    works = [WL.c3_kernel(s) for s in range(args.programs)]
    progs = []
    for w in works:
        p = B.Program(ctx, w.src)
        p.set_ndrange(w.G, w.W)
        p.bind(w.arrays, w.scalars)
        progs.append(p)
    cache = args.tune_cache or os.path.join(tempfile.gettempdir(), f"rc_tune_{os.getpid()}.json")
    small = torch.empty(max(p.workspace_size(2) for p in progs[:64]) * 2, dtype=torch.uint8, device="cuda")
    tuned = {}
    for p in progs:
        need = p.workspace_size(2)
        if need > small.numel():
            small = torch.empty(need, dtype=torch.uint8, device="cuda")
        key = json.dumps(p.autotune(1 << 40, 2, small, cache), sort_keys=True)
        tuned[key] = tuned.get(key, 0) + 1
    del small
    setup_s = time.perf_counter() - t0
    handles = np.repeat(B.handles_of(progs), seeds)
    seed_arr = np.tile(np.arange(seeds, dtype=np.uint64), len(progs))
    n = int(handles.size)
    ws = torch.empty(int(args.ws_gb * (1 << 30)), dtype=torch.uint8, device="cuda")
    cap = 1 << 24
    rec = torch.empty(cap * B.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    summ = torch.empty(n * B.SUMMARY_BYTES, dtype=torch.uint8, device="cuda")

    def step():
        ctx.batch_check_async(handles, seed_arr, ws, rec, cnt, summ)
        ctx.sync()

    for _ in range(max(1, args.warmup)):
        step()
    s = B.summaries_to_numpy(summ, n)
    accesses = int(s["n_accesses"].sum())
    records = int(cnt.item())
    racy = int((s["n_race_cells"] > 0).sum())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # phase split from one more (profiled, eager) step
    ctx.profile(True)
    step()
    prof = ctx.profile_read()
    ctx.profile(False)
    value = accesses * args.steps / elapsed
    dom = max(prof, key=lambda k: prof[k][0])
    ms, launches = prof[dom]
    per_launch_ms = ms / max(1, launches)
    algo = ALGO_BYTES.get(dom, 0.0) * accesses / max(1, launches)
    achieved = algo / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic(KERNEL_OF_PHASE[dom], "c3"), "kernel": KERNEL_OF_PHASE[dom],
                "phase": dom, "avg_launch_ms": round(per_launch_ms, 4),
                "phases_ms": {k: round(v[0], 3) for k, v in prof.items()},
                "path_frac": round(28.0 * value / (HBM_PEAK_GBS * 1e9), 5)}
    if dom not in ALGO_BYTES:
        roofline["note"] = ("the dominant phase is a sort, whose passes carry no algorithmic bytes "
                            "(implementation cost); path_frac is the whole path against 28 B per access")
    cpu = cpu_baseline([(w, seeds) for w in works[: max(1, min(len(works), 50))]], args.cpu_seconds) \
        if args.cpu_seconds > 0 else None
    line = {
        "metric": "race-checked accesses/s", "value": round(value, 1), "unit": "accesses/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": desc, "programs": len(progs), "seeds_per_program": seeds, "instances_per_step": n,
                   "accesses_per_step": accesses, "race_records_per_step": records,
                   "racy_instances_per_step": racy, "setup_s": round(setup_s, 2), "tunings": tuned},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_c5(args, ctx):
    """Learned triage: label the training instances with the exact checker,
    train the network on the GPU, then sweep the held-out instances in plain
    and in learned order and compare what each finds within a quarter of the
    plain sweep's GPU time.  One step is the whole experiment."""
    import torch
    from paper_1308_3203_amd import triage as T
    from paper_1308_3203_amd import workloads as WL
    n_train, n_eval = args.programs, args.eval_programs
    seeds = args.seeds or 100
    t0 = time.perf_counter()
    r = T.run(ctx, [WL.c3_kernel(s) for s in range(n_train)], seeds,
              [WL.c3_kernel(10000 + s) for s in range(n_eval)], seeds,
              epochs=args.epochs, batch=4096, lr=1e-3, chunk=args.chunk, label_chunk=20000,
              ws_bytes=int(args.ws_gb * (1 << 30)),
              progress=lambda m: print(f"[c5 {time.perf_counter() - t0:.1f}s] {m}", file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rep = r.report
    line = {
        "metric": "RACE records found per GPU-second within 25% of the plain sweep's GPU time, learned order",
        "value": round(rep.races_per_gpu_s_learned, 1), "unit": "RACE records/GPU-s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(wall * 1e3, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 network, int32 checker", "data": "synthetic",
        "config": {"workload": "c5: learned triage over the c3 generator; train programs 0..%d x %d seeds, "
                               "held-out programs 10000..%d x %d seeds" % (n_train - 1, seeds, 10000 + n_eval - 1,
                                                                          seeds),
                   "train_instances": r.n_train, "eval_instances": r.n_eval,
                   "train_racy_frac": round(r.train_racy_frac, 4), "epochs": args.epochs,
                   "losses": [round(x, 5) for x in r.losses]},
        "triage": {"recall_racy_instances": round(rep.recall_instances, 4),
                   "recall_race_records": round(rep.recall_records, 4),
                   "plain_recall_racy_instances": round(rep.plain_recall_instances, 4),
                   "races_per_gpu_s_plain": round(rep.races_per_gpu_s_plain, 1),
                   "plain_sweep_gpu_ms": round(rep.plain_ms, 2), "budget_frac": rep.budget_frac,
                   "inference_gpu_ms": round(rep.inference_ms, 3), "label_sweep_gpu_ms": round(r.label_ms, 1),
                   "train_gpu_ms": round(r.train_ms, 1), "racy_instances": rep.n_racy,
                   "race_records": rep.n_race_records},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(programs, budget_s: float):
    """The oracle as it stands, single-threaded, on a bounded sample of the
    same instances (round-robin over the programs, seeds from 0)."""
    from oracle import oracle as O
    compiled = [(w, O.Program(w.src)) for w, _ in programs]
    t_total = 0.0
    acc = 0
    n_inst = 0
    seed = 0
    t_start = time.perf_counter()
    while time.perf_counter() - t_start < budget_s:
        for w, p in compiled:
            t = time.perf_counter()
            r = p.run(w.G, w.W, arrays=w.arrays, scalars=w.scalars, seed=seed, instance=seed)
            t_total += time.perf_counter() - t
            acc += int(r.summary["n_accesses"])
            n_inst += 1
            if time.perf_counter() - t_start >= budget_s:
                break
        seed += 1
    return {"value": round(acc / t_total, 1), "unit": "accesses/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_inst} instances (seeds from 0, round-robin over {len(compiled)} programs), "
                      f"{acc} accesses in {t_total:.1f} s"}


if __name__ == "__main__":
    main()
