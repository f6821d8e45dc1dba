"""Benchmark of the race-check hot path on one MI355X.

A step is one pass of the whole path (interpretation, access logging, interval
checks, ordered race report) over one batch of synthetic instances, with inputs
seeded on the device.  Prints one JSON line.

    python bench.py [--config c3] [--steps K] [--warmup W]

The headline is the batched random-kernel sweep (c3: 10^4 random kernels of
widths 32..1024 x 100 seeds, 10^6 instances, one rc_batch_check call per
step), the largest configuration.  The same line carries, as secondary
figures, the template kernels (c2: six programs, 16 x 256, 10^4 seeds each)
with the static proofs on and off, the large-interval kernel (c4: 64 x
1024 x 64 iterations, 16 seeds), and the learned triage (c5 over the c3
generator: 10^5 training programs x 10 seeds labelled by the checker, the
network trained, then 10^4 held-out programs x 10 seeds swept in learned,
plain, random and static-heuristic order; --no-c5 leaves it out).  Other
configurations: c1 (one random 20-statement kernel, 1 x 64, 1000 seeds),
and each of the secondaries alone (--config c2, c4, c5).

Roofline: a race-checked access costs 28 algorithmic bytes (4 for the
simulated cell, 12 to write its access record once, 12 to read it once).
Each kernel is credited the bytes of the work it does: the interpreting
kernel the cell and the record write of every access, and the record read
as well for every access whose check completes inside it (checked in LDS,
or exempt by a static proof); the checks after it (the global pass, or the
per-instance check of one-group programs' spilled intervals) the record
read of every access they check.  Sort passes are implementation
cost and are credited nothing.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_ACCESS = 28.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
PHASE_KERNELS = {"log_sort": "rs_hist_kernel/rs_scatter_lds_kernel", "interval_check": "sc_group_kernel/seg_check_kernel",
                 "record_sort": "rs_hist_kernel/rs_scatter_kernel", "output": "rec_place_out_kernel",
                 "setup": "fill kernels"}


def say(msg: str):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the library sources: counter-derived traffic is valid only for
    the kernels it was measured on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1308_3203_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")) and not f.startswith("_"):
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


def credited_bytes(phase: str, accesses: int, global_pass: int) -> float:
    """Algorithmic bytes a phase is credited for one step (module docstring):
    global_pass is the number of log entries the global pass checked."""
    if phase == "interpret":
        return 28.0 * (accesses - global_pass) + 16.0 * global_pass
    if phase == "interval_check":
        return 12.0 * global_pass
    return 0.0


# ---------------------------------------------------------------------------
# runners: one step = every instance of the workload checked once
# ---------------------------------------------------------------------------
class SingleRunner:
    """One rc_check call per program and step (c1, c2, c4)."""

    def __init__(self, ctx, works_seeds, ws_gb: float, jit: bool, proofs_off: bool = False):
        from paper_1308_3203_amd import binding as B
        self.B = B
        self.ctx = ctx
        self.jit = jit
        self.runs = []
        per_ws = int(ws_gb * (1 << 30) / len(works_seeds))
        for w, n in works_seeds:
            p = B.Program(ctx, w.src)
            p.set_ndrange(w.G, w.W)
            p.bind(w.arrays, w.scalars)
            if proofs_off:
                p.set_tuning(proofs_off=True)
            if jit:
                p.jit(True)            # compiled here, outside the timed region
            # record capacity from a probe over the first seeds (every record
            # of the timed steps is written out)
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
            self.runs.append((w, n, p, B.Buffers(p, n, cap=cap, ws_limit=per_ws)))
        self.n = sum(n for _, n, _, _ in self.runs)

    def step(self):
        for w, n, p, buf in self.runs:
            p.check_async(0, n, buf.ws, buf.records, buf.n_records, buf.summaries)

    def step_with_stats(self) -> dict:
        tot = {}
        for w, n, p, buf in self.runs:
            p.check_async(0, n, buf.ws, buf.records, buf.n_records, buf.summaries)
            self.ctx.sync()
            for k, v in self.ctx.call_stats().items():
                tot[k] = tot.get(k, 0) + v
        return tot

    def results(self):
        """Per program: (workload, numpy records, numpy summaries) of the last step."""
        B = self.B
        out = []
        for w, n, p, buf in self.runs:
            nr = int(buf.n_records.item())
            out.append((w, B.records_to_numpy(buf.records, min(nr, buf.cap)), B.summaries_to_numpy(buf.summaries, n)))
        return out

    def instance(self, i: int):
        """(workload, seed, index in its own call) of instance i of the step."""
        for w, n, _, _ in self.runs:
            if i < n:
                return w, i, i
            i -= n
        raise IndexError(i)

    def free(self):
        for _, _, p, _ in self.runs:
            p.close()
        self.runs = []


class BatchRunner:
    """The whole workload in one rc_batch_check call per step (c3)."""

    def __init__(self, ctx, n_programs: int, seeds: int, ws_gb: float, tune_cache: str | None):
        from paper_1308_3203_amd import batches
        self.ctx = ctx
        self.batch = batches.RandomKernelBatch(ctx, n_programs, seeds, ws_gb=ws_gb, tune_cache=tune_cache,
                                               progress=say)
        self.n = self.batch.n

    def step(self):
        self.batch.enqueue()

    def step_with_stats(self) -> dict:
        self.batch.step()
        return self.ctx.call_stats()

    def results(self):
        recs, summ = self.batch.results()
        return [(None, recs, summ)]

    def instance(self, i: int):
        w, seed = self.batch.instance(i)
        return w, seed, i

    def free(self):
        self.batch.free()


def measure(runner, ctx, steps: int, warmup: int, jit: bool, eager: bool = False) -> dict:
    """Warm up (the last warmup step also reads the log statistics), then
    time `steps` steps with the library's HIP events on its own stream.
    The timed steps launch every chunk eagerly (timing is on); eager: the
    warmup steps too, with no graph replay anywhere (rocprofv3 counter
    collection does not take graph-launched kernels)."""
    import torch
    if eager:
        ctx.profile(True)
    for _ in range(max(1, warmup) - 1):
        runner.step()
        ctx.sync()
    stats = runner.step_with_stats()
    accesses = 0
    records = 0
    racy = 0
    for _, recs, summ in runner.results():
        accesses += int(summ["n_accesses"].sum())
        records += len(recs)
        racy += int((summ["n_race_cells"] > 0).sum())
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        runner.step()
        ctx.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    value = accesses * steps / elapsed
    lg = int(stats.get("logged_global", 0))
    gp = int(stats.get("global_pass", 0))
    dom = max(prof, key=lambda k: prof[k][0])
    ms, launches = prof[dom]
    per_launch_ms = ms / max(1, launches)
    algo_step = credited_bytes(dom, accesses, gp)
    algo_launch = algo_step * steps / max(1, launches)
    achieved = algo_launch / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
    if dom == "interpret":
        kernel = "rc_jit_kernel" if jit else "rc_interp_kernel"
    else:
        kernel = PHASE_KERNELS[dom]
    return {
        "value": value, "ms_per_step": elapsed / steps * 1e3, "steps": steps, "accesses": accesses,
        "accesses_logged": int(stats.get("logged", 0)), "accesses_logged_global": lg,
        "accesses_global_pass": gp,
        "intervals": int(stats.get("intervals", 0)), "intervals_spilled": int(stats.get("intervals_spilled", 0)),
        "instructions": int(stats.get("instructions", 0)), "wave_instructions": int(stats.get("wave_instructions", 0)),
        "records": records, "racy_instances": racy,
        "dominant": {"phase": dom, "kernel": kernel, "launches_per_step": launches / steps,
                     "avg_launch_ms": per_launch_ms, "algo_bytes_per_launch": algo_launch,
                     "achieved_gbs": achieved, "frac": achieved / HBM_PEAK_GBS},
        "phases_ms": {k: round(v[0] / steps, 3) for k, v in prof.items()},
        "path_frac": BYTES_PER_ACCESS * value / (HBM_PEAK_GBS * 1e9),
    }


def summary_of(m: dict) -> dict:
    """The JSON fields of one measured configuration."""
    d = m["dominant"]
    out = {"value": round(m["value"], 1), "unit": "accesses/s", "ms_per_step": round(m["ms_per_step"], 3),
           "accesses_per_step": m["accesses"], "accesses_logged": m["accesses_logged"],
           "accesses_logged_global": m["accesses_logged_global"],
           "accesses_global_pass": m["accesses_global_pass"], "intervals": m["intervals"],
           "intervals_spilled": m["intervals_spilled"], "race_records_per_step": m["records"],
           "racy_instances_per_step": m["racy_instances"], "instructions": m["instructions"],
           "wave_instructions": m["wave_instructions"],
           "dominant_kernel": d["kernel"], "dominant_phase": d["phase"],
           "avg_launch_ms": round(d["avg_launch_ms"], 4), "frac": round(d["frac"], 5),
           "path_frac": round(m["path_frac"], 5), "phases_ms": m["phases_ms"]}
    return out


# ---------------------------------------------------------------------------
# the oracle beside the GPU: a bounded sample on the host's cores
# ---------------------------------------------------------------------------
def host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(runner, order, budget_s: float, threads: int):
    """The oracle as it stands (plain C, one instance per call) on `threads`
    host threads over instances taken in `order` until `budget_s` seconds of
    wall time have passed.  The ctypes calls release the interpreter lock, so
    the threads run the oracle in parallel.  Also returns SHA-256 hashes of
    the oracle's and the GPU's records and summaries over the same
    instances."""
    import concurrent.futures as cf
    import threading
    import numpy as np
    from oracle import oracle as O
    res = runner.results()
    # GPU output per instance: records are in instance order within each call
    gpu = []
    for w, recs, summ in res:
        counts = summ["n_race_cells"].astype(np.int64) + summ["n_benign_cells"].astype(np.int64)
        offs = np.concatenate([[0], np.cumsum(counts)])
        gpu.append((recs, summ, offs))
    call_of = []
    if len(res) == 1:
        call_of = None
    else:
        for k, (_, _, summ) in enumerate(res):
            call_of += [(k, j) for j in range(len(summ))]

    def gpu_bytes(i):
        k, j = (0, i) if call_of is None else call_of[i]
        recs, summ, offs = gpu[k]
        return recs[offs[j]:offs[j + 1]].tobytes() + summ[j:j + 1].tobytes()

    lock = threading.Lock()
    nxt = [0]
    done = {}
    deadline = time.perf_counter() + budget_s

    def worker():
        acc = 0
        while time.perf_counter() < deadline:
            with lock:
                if nxt[0] >= len(order):
                    break
                i = order[nxt[0]]
                nxt[0] += 1
            w, seed, local = runner.instance(i)
            r = O.Program(w.src).run(w.G, w.W, arrays=w.arrays, scalars=w.scalars, seed=seed, instance=local)
            out = r.records.tobytes() + np.array([r.summary], dtype=O.SUMMARY_DTYPE).tobytes()
            with lock:
                done[i] = out
            acc += int(r.summary["n_accesses"])
        return acc

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        accs = list(ex.map(lambda _: worker(), range(threads)))
    wall = time.perf_counter() - t0
    ids = sorted(done)
    h_o, h_g = hashlib.sha256(), hashlib.sha256()
    for i in ids:
        h_o.update(done[i])
        h_g.update(gpu_bytes(i))
    acc = sum(accs)
    return {"value": round(acc / wall, 1), "unit": "accesses/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(ids)} instances of the same step ({acc} accesses) in {wall:.1f} s of wall time "
                      f"on {threads} threads, one instance per oracle call",
            "parity_sha256_oracle": h_o.hexdigest(), "parity_sha256_gpu": h_g.hexdigest(),
            "parity_match": h_o.hexdigest() == h_g.hexdigest(), "parity_instances": len(ids)}


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------
C2_DESC = "c2: tree reduction, Hillis-Steele prefix sum, 32x32 tiled transpose (clean + injected), G=16 x W=256"
C3_DESC = ("c3: random kernels, W in {32..1024}, 10-200 statements, 1-8 barriers, loops to 16 iterations, "
           "arrays of 4096-262144 cells, one batched call")
C4_DESC = "c4: large intervals, G=64 x W=1024 x 64 iterations, 2^20 cells"


def single_works(name: str, seeds):
    from paper_1308_3203_amd import workloads as WL
    if name == "c1":
        return [(WL.c1_kernel(1), seeds or 1000)], "c1: one random 20-statement kernel, G=1 x W=64"
    if name == "c2":
        return [(w, seeds or 10000) for w in WL.c2_templates()], C2_DESC
    if name == "c4":
        return [(WL.c4_kernel(), seeds or 16)], C4_DESC
    raise SystemExit(f"unknown config {name}")


def run_secondary(ctx, name: str, args, proofs_off: bool = False) -> dict:
    import torch
    works, desc = single_works(name, None)
    say(f"secondary {name}{' (proofs off)' if proofs_off else ''}: set-up")
    r = SingleRunner(ctx, works, args.ws_gb, jit=True, proofs_off=proofs_off)
    try:
        m = measure(r, ctx, args.secondary_steps, 2, jit=True)
    finally:
        r.free()
        del r
        torch.cuda.empty_cache()
    out = summary_of(m)
    out["workload"] = desc + (", static proofs off (every access to a written array logged and checked)"
                              if proofs_off else "")
    out["execution"] = "per-program kernels"
    out["instances_per_step"] = sum(n for _, n in works)
    out["steps"] = m["steps"]
    # measured HBM bytes per launch (counters taken with the proofs on)
    t = None if proofs_off else measured_traffic(out["dominant_kernel"], name)
    out["traffic"] = t
    out["traffic_frac"] = (round(t / (out["avg_launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)
                           if t and out.get("avg_launch_ms") else None)
    say(f"secondary {name}: {out['value']:.3e} accesses/s, {out['ms_per_step']:.2f} ms per step")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", help="c3 (default), c1, c2, c4 or c5")
    ap.add_argument("--seeds", type=int, default=None, help="seeds per program (default: the config's)")
    ap.add_argument("--ws-gb", type=float, default=230.0, help="workspace budget over all programs (HBM is 288 GB)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="oracle sample budget in wall seconds (0: skip)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (default: the host's cores)")
    ap.add_argument("--programs", type=int, default=10000, help="c3: number of random programs")
    ap.add_argument("--tune-cache", default=None, help="c3: autotuner cache file (default: a temp file)")
    ap.add_argument("--no-secondary", action="store_true", help="only the headline configuration")
    ap.add_argument("--secondary-steps", type=int, default=10)
    ap.add_argument("--proofs-off", action="store_true", help="c1/c2/c4: no static proofs")
    ap.add_argument("--no-c5", action="store_true", help="c3: no learned-triage field in the line")
    ap.add_argument("--train-programs", type=int, default=100000, help="c5: training programs")
    ap.add_argument("--eval-programs", type=int, default=10000, help="c5: held-out programs")
    ap.add_argument("--epochs", type=int, default=5, help="c5: training epochs")
    ap.add_argument("--chunk", type=int, default=1000, help="c5: instances per sweep call")
    ap.add_argument("--weight-records", action="store_true",
                    help="c5: training rows repeated by their RACE record count (log2)")
    ap.add_argument("--copy-probe", type=float, default=0.0, help="only run a plain copy of this many GiB")
    ap.add_argument("--no-jit", action="store_true", help="c1/c2/c4: interpret instead of per-program kernels")
    ap.add_argument("--eager", action="store_true",
                    help="no graph replay, warmup included (for rocprofv3 --pmc runs)")
    ap.add_argument("--profile-summary", action="store_true",
                    help="summarize rocprofv3 output (no GPU): --kernel, --last, and the directories below")
    ap.add_argument("--kernel", default="rc_interp_kernel")
    ap.add_argument("--last", type=int, default=0, help="dispatches of the timed steps (the run's last ones)")
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--trace-dir", default=None)
    ap.add_argument("--counter-dir", default=None)
    ap.add_argument("--fetch-dir", default=None)
    ap.add_argument("--write-dir", default=None)
    ap.add_argument("--copy-fetch-dir", default=None)
    ap.add_argument("--copy-write-dir", default=None)
    ap.add_argument("--copy-gib", type=float, default=1.0)
    args = ap.parse_args()
    if args.profile_summary:
        return profile_main(args)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1308_3203_amd import binding as B

    if args.copy_probe > 0:
        return copy_probe(args.copy_probe)
    ctx = B.Context(0)
    if args.config == "c5":
        return bench_c5(args, ctx)
    jit = not args.no_jit and args.config != "c3"
    t_setup = time.perf_counter()
    if args.config == "c3":
        seeds = args.seeds or 100
        runner = BatchRunner(ctx, args.programs, seeds, args.ws_gb, args.tune_cache)
        desc = C3_DESC
        cfg_extra = {"programs": args.programs, "seeds_per_program": seeds, "execution": "interpreter",
                     "tunings": runner.batch.tunings}
        order = [p * seeds + s for s in range(seeds) for p in range(args.programs)]
    else:
        works, desc = single_works(args.config, args.seeds)
        runner = SingleRunner(ctx, works, args.ws_gb, jit=jit, proofs_off=args.proofs_off)
        cfg_extra = {"programs": len(works), "seeds_per_program": works[0][1],
                     "execution": "per-program kernels" if jit else "interpreter",
                     "static_proofs": not args.proofs_off}
        n_each = works[0][1]
        order = [k * n_each + s for s in range(n_each) for k in range(len(works))]
    setup_s = time.perf_counter() - t_setup
    say(f"{args.config}: set-up {setup_s:.1f} s, {runner.n} instances; warmup")
    m = measure(runner, ctx, args.steps, args.warmup, jit=jit, eager=args.eager)
    say(f"{args.config}: {m['value']:.3e} accesses/s, {m['ms_per_step']:.1f} ms per step")
    d = m["dominant"]
    roofline = {"bound": "hbm", "achieved": round(d["achieved_gbs"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(d["frac"], 5), "traffic": measured_traffic(d["kernel"], args.config),
                "kernel": d["kernel"], "phase": d["phase"],
                "launches_per_step": d["launches_per_step"],
                "algo_bytes_per_launch": round(d["algo_bytes_per_launch"]),
                "avg_launch_ms": round(d["avg_launch_ms"], 4),
                "phases_ms": m["phases_ms"], "path_frac": round(m["path_frac"], 5),
                "bytes_per_access": BYTES_PER_ACCESS}
    # the kernel's measured HBM bytes per launch (counters, when they were
    # taken on these sources) over its launch time, against the same peak
    t = roofline["traffic"]
    roofline["traffic_frac"] = (round(t / (d["avg_launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)
                                if t and d["avg_launch_ms"] > 0 else None)
    cpu = None
    if args.cpu_seconds > 0:
        threads = args.cpu_threads or host_cores()
        say(f"oracle sample on {threads} threads for {args.cpu_seconds:.0f} s")
        cpu = cpu_baseline(runner, order, args.cpu_seconds, threads)
        say(f"oracle: {cpu['value']:.3e} accesses/s, parity over {cpu['parity_instances']} instances: "
            f"{'match' if cpu['parity_match'] else 'MISMATCH'}")
    n_inst = runner.n
    runner.free()
    del runner
    torch.cuda.empty_cache()
    secondary = {}
    if not args.no_secondary and args.config == "c3":
        secondary["c2"] = run_secondary(ctx, "c2", args)
        secondary["c2_proofs_off"] = run_secondary(ctx, "c2", args, proofs_off=True)
        secondary["c4"] = run_secondary(ctx, "c4", args)
        if not args.no_c5:
            secondary["c5"] = c5_secondary(args, ctx)
    config = {"workload": desc, **cfg_extra, "instances_per_step": n_inst, "setup_s": round(setup_s, 2),
              "accesses_per_step": m["accesses"], "accesses_logged": m["accesses_logged"],
              "accesses_logged_global": m["accesses_logged_global"],
              "accesses_global_pass": m["accesses_global_pass"], "intervals": m["intervals"],
              "intervals_spilled": m["intervals_spilled"], "race_records_per_step": m["records"],
              "racy_instances_per_step": m["racy_instances"], "instructions": m["instructions"],
              "wave_instructions": m["wave_instructions"]}
    line = {
        "metric": "race-checked accesses/s", "value": round(m["value"], 1), "unit": "accesses/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": config, "roofline": roofline, "cpu_baseline": cpu, "secondary": secondary or None,
    }
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------------------
# rocprofv3 output -> the summaries kept under profiles/
# ---------------------------------------------------------------------------
def _csv_rows(directory: str, suffix: str):
    import csv
    rows = []
    for dp, _, files in os.walk(directory):
        for f in sorted(files):
            if f.endswith(suffix):
                with open(os.path.join(dp, f), newline="") as fh:
                    rows += list(csv.DictReader(fh))
    return rows


def _dispatch_key(r):
    return int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0)


def summarize_trace(directory: str, kernel: str, last: int) -> dict:
    """Kernel trace of one rocprofv3 run: the `last` dispatches of every
    kernel whose name contains `kernel` (the timed steps come last), and the
    whole run's per-kernel statistics."""
    rows = _csv_rows(directory, "kernel_trace.csv")
    mine = sorted((r for r in rows if kernel in r["Kernel_Name"]), key=_dispatch_key)
    sel = mine[-last:] if last else mine
    durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in sel]
    stats = _csv_rows(directory, "kernel_stats.csv")
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    return {"dispatches": len(mine), "selected": len(sel),
            "avg_ms": (sum(durs) / len(durs) / 1e6) if durs else None,
            "min_ms": min(durs) / 1e6 if durs else None, "max_ms": max(durs) / 1e6 if durs else None,
            "stats": [(r["Name"][:90], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
                       float(r["AverageNs"]) / 1e6, float(r["Percentage"])) for r in stats[:12]]}


def summarize_counters(directory: str, kernel: str, last: int) -> dict:
    """Per counter: its average per dispatch over the `last` dispatches of
    the kernel (all dispatches when last is 0)."""
    rows = _csv_rows(directory, "counter_collection.csv")
    per = {}
    for r in rows:
        if kernel in r["Kernel_Name"]:
            d = per.setdefault(_dispatch_key(r), {})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    keys = sorted(per)
    sel = keys[-last:] if last else keys
    out = {"dispatches": len(keys), "selected": len(sel)}
    names = sorted({c for k in sel for c in per[k]})
    for c in names:
        out[c] = sum(per[k].get(c, 0.0) for k in sel) / max(1, len(sel))
    return out


def profile_main(args):
    """--profile-summary: print a markdown summary of rocprofv3 output and,
    given the four FETCH_SIZE / WRITE_SIZE runs, record the kernel's HBM
    traffic per launch in profiles/traffic.json."""
    kernel, last = args.kernel, args.last
    lines = []
    if args.trace_dir:
        t = summarize_trace(args.trace_dir, kernel, last)
        if not t["selected"]:
            raise SystemExit(f"no dispatch of a kernel named like {kernel!r} under {args.trace_dir}")
        lines.append(f"## Kernel trace: `{kernel}`\n")
        lines.append(f"{t['selected']} of {t['dispatches']} dispatches (the last ones: the timed steps): "
                     f"average {t['avg_ms']:.4f} ms, min {t['min_ms']:.4f}, max {t['max_ms']:.4f}\n")
        lines.append("| kernel (whole run) | calls | total ms | avg ms | % |\n|---|---|---|---|---|")
        for name, calls, tot, avg, pct in t["stats"]:
            lines.append(f"| `{name}` | {calls} | {tot:.2f} | {avg:.4f} | {pct:.1f} |")
        lines.append("")
    if args.counter_dir:
        c = summarize_counters(args.counter_dir, kernel, last)
        lines.append(f"## Counters: `{kernel}`, average per dispatch over {c['selected']} of "
                     f"{c['dispatches']} dispatches\n")
        lines.append("| counter | per dispatch |\n|---|---|")
        for k, v in c.items():
            if k not in ("dispatches", "selected"):
                lines.append(f"| {k} | {v:.6g} |")
        if "SQ_LDS_BANK_CONFLICT" in c and "SQ_LDS_IDX_ACTIVE" in c:
            lines.append(f"| LdsBankConflict (conflict cycles per LDS access cycle) | "
                         f"{c['SQ_LDS_BANK_CONFLICT'] / max(1.0, c['SQ_LDS_IDX_ACTIVE'] - c['SQ_LDS_BANK_CONFLICT']):.4f} |")
        if "SQ_THREAD_CYCLES_VALU" in c and "SQ_ACTIVE_INST_VALU" in c:
            lines.append(f"| VALUUtilization (% active lanes per VALU instruction) | "
                         f"{100 * c['SQ_THREAD_CYCLES_VALU'] / max(1.0, 64 * c['SQ_ACTIVE_INST_VALU']):.2f} |")
        if "SQ_ACTIVE_INST_VALU" in c and "GRBM_GUI_ACTIVE" in c:
            # GRBM_GUI_ACTIVE comes summed over the 8 XCDs: the kernel's
            # cycles are an eighth of it; VALU busy = VALU issue cycles per
            # SIMD (4 per CU, 256 CUs) over those cycles
            cycles = c["GRBM_GUI_ACTIVE"] / 8.0
            lines.append(f"| GPU cycles per dispatch (GRBM_GUI_ACTIVE / 8 XCDs) | {cycles:.6g} |")
            lines.append(f"| VALUBusy (% of SIMD cycles issuing VALU) | "
                         f"{100 * c['SQ_ACTIVE_INST_VALU'] * 4 / 1024 / max(1.0, cycles):.2f} |")
        if "SQ_INSTS_SALU" in c and "SQ_WAVES" in c:
            lines.append(f"| SALU instructions per wave | {c['SQ_INSTS_SALU'] / max(1.0, c['SQ_WAVES']):.6g} |")
        if "SQ_INSTS_VALU" in c and "SQ_WAVES" in c:
            lines.append(f"| VALU instructions per wave | {c['SQ_INSTS_VALU'] / max(1.0, c['SQ_WAVES']):.6g} |")
        lines.append("")
    if args.fetch_dir and args.write_dir and args.copy_fetch_dir and args.copy_write_dir:
        cf = summarize_counters(args.copy_fetch_dir, "copyBuffer", 0)
        cw = summarize_counters(args.copy_write_dir, "copyBuffer", 0)
        f = summarize_counters(args.fetch_dir, kernel, last)
        w = summarize_counters(args.write_dir, kernel, last)
        copy_bytes = args.copy_gib * (1 << 30)
        ff = copy_bytes / (cf["FETCH_SIZE"] * 1024.0)
        wf = copy_bytes / (cw["WRITE_SIZE"] * 1024.0)
        per_launch = f["FETCH_SIZE"] * 1024.0 * ff + w["WRITE_SIZE"] * 1024.0 * wf
        lines.append(f"## HBM traffic: `{kernel}` on {args.workload}\n")
        lines.append("| counter | KiB per dispatch | copy calibration factor | bytes per launch |\n|---|---|---|---|")
        lines.append(f"| FETCH_SIZE | {f['FETCH_SIZE']:.1f} | {ff:.4f} | {f['FETCH_SIZE'] * 1024 * ff:.4e} |")
        lines.append(f"| WRITE_SIZE | {w['WRITE_SIZE']:.1f} | {wf:.4f} | {w['WRITE_SIZE'] * 1024 * wf:.4e} |")
        lines.append(f"| total | | | {per_launch:.4e} |\n")
        try:
            with open(TRAFFIC_FILE) as fh:
                table = json.load(fh)
        except (OSError, ValueError):
            table = {}
        table[f"{kernel}|{args.workload}"] = {
            "bytes_per_launch": int(per_launch), "fetch_kib_avg": round(f["FETCH_SIZE"], 1),
            "write_kib_avg": round(w["WRITE_SIZE"], 1), "fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
            "dispatches": f["selected"], "source_sha256_16": kernel_source_hash()}
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(table, fh, indent=1)
    print("\n".join(lines))


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


C5_HELD0 = 1000000   # first generator seed of the held-out programs


def c5_line(args, ctx) -> dict:
    """Learned triage: label the training instances with the exact checker,
    train the network on the GPU, then sweep the held-out instances in plain
    and in learned order and compare what each finds within a quarter of the
    plain sweep's GPU time.  One step is the whole experiment."""
    import torch
    from paper_1308_3203_amd import triage as T
    from paper_1308_3203_amd import workloads as WL
    # many programs, few seeds each: the network has to generalise across
    # programs (the seeds of one program differ only in their histograms);
    # held-out programs come from a disjoint range of generator seeds
    n_train, n_eval = args.train_programs, args.eval_programs
    seeds = args.seeds or 10
    t0 = time.perf_counter()
    r = T.run(ctx, [WL.c3_kernel(s) for s in range(n_train)], seeds,
              [WL.c3_kernel(C5_HELD0 + s) for s in range(n_eval)], seeds,
              epochs=args.epochs, batch=4096, lr=1e-3, chunk=args.chunk, label_chunk=20000,
              ws_bytes=int(args.ws_gb * (1 << 30)), weight_records=args.weight_records,
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
                               "held-out programs %d..%d x %d seeds" % (n_train - 1, seeds, C5_HELD0,
                                                                       C5_HELD0 + n_eval - 1, seeds),
                   "train_instances": r.n_train, "eval_instances": r.n_eval,
                   "train_racy_frac": round(r.train_racy_frac, 4), "epochs": args.epochs,
                   "weight_records": args.weight_records,
                   "losses": [round(x, 5) for x in r.losses]},
        "triage": {"recall_racy_instances": round(rep.recall_instances, 4),
                   "recall_race_records": round(rep.recall_records, 4),
                   "plain_recall_racy_instances": round(rep.plain_recall_instances, 4),
                   "races_per_gpu_s_plain": round(rep.races_per_gpu_s_plain, 1),
                   "plain_sweep_gpu_ms": round(rep.plain_ms, 2), "budget_frac": rep.budget_frac,
                   "inference_gpu_ms": round(rep.inference_ms, 3), "label_sweep_gpu_ms": round(r.label_ms, 1),
                   "train_gpu_ms": round(r.train_ms, 1), "racy_instances": rep.n_racy,
                   "race_records": rep.n_race_records,
                   "orders": {k: {"recall_racy_instances": round(o.recall_instances, 4),
                                  "recall_race_records": round(o.recall_records, 4),
                                  "races_per_gpu_s": round(o.races_per_gpu_s, 1),
                                  "curve_frac_time_instances_records": o.curve}
                              for k, o in rep.orders.items()}},
        "roofline": None, "cpu_baseline": None,
    }
    return line


def bench_c5(args, ctx):
    print(json.dumps(c5_line(args, ctx)), flush=True)


def c5_secondary(args, ctx) -> dict:
    """The learned-triage experiment as a field of the default line: its
    recalls, the baselines' and its own value."""
    line = c5_line(args, ctx)
    t = line["triage"]
    out = {"metric": line["metric"], "value": line["value"], "unit": line["unit"],
           "ms_per_step": line["ms_per_step"], "workload": line["config"]["workload"],
           "recall_racy_instances": t["recall_racy_instances"], "recall_race_records": t["recall_race_records"],
           "budget_frac": t["budget_frac"], "inference_gpu_ms": t["inference_gpu_ms"],
           "racy_instances": t["racy_instances"], "race_records": t["race_records"],
           "orders": {k: {"recall_racy_instances": o["recall_racy_instances"],
                          "recall_race_records": o["recall_race_records"]} for k, o in t["orders"].items()}}
    say(f"secondary c5: recall {out['recall_racy_instances']} of racy instances, "
        f"{out['recall_race_records']} of RACE records within {out['budget_frac']} of the plain sweep's GPU time")
    return out


if __name__ == "__main__":
    main()
