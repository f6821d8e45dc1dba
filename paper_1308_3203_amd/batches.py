"""Set-up of the batched random-kernel sweep, shared by the benchmark and its
full-size parity test: load the generator's programs, apply the autotuner's
choice per shape bucket, and allocate the call's buffers.  Nothing here
computes any part of the check; one step is one rc_batch_check call.
"""
from __future__ import annotations

import json
import os
import tempfile
import time

import numpy as np

from . import binding as B
from . import workloads as WL


class RandomKernelBatch:
    """Programs 0..n_programs-1 of the random-kernel generator, seeds
    0..seeds-1 each, as one list of instances: instance i is program
    i // seeds with seed i % seeds."""

    def __init__(self, ctx: B.Context, n_programs: int = 10000, seeds: int = 100, ws_gb: float = 230.0,
                 tune_cache: str | None = None, rec_cap: int = 1 << 24, proofs_off: bool = False,
                 program_seed0: int = 0, autotune: bool = True, progress=None):
        import torch
        say = progress or (lambda msg: None)
        t0 = time.perf_counter()
        self.ctx = ctx
        self.seeds = seeds
        self.works = [WL.c3_kernel(program_seed0 + s) for s in range(n_programs)]
        self.progs = []
        for w in self.works:
            p = B.Program(ctx, w.src)
            p.set_ndrange(w.G, w.W)
            p.bind(w.arrays, w.scalars)
            if proofs_off:
                p.set_tuning(proofs_off=True)
            self.progs.append(p)
        say(f"loaded {n_programs} programs in {time.perf_counter() - t0:.1f} s")
        self.tunings = {}
        self.tuning_of = []        # per program: its tuning (a JSON key)
        if autotune:
            cache = tune_cache or os.path.join(tempfile.gettempdir(), f"rc_tune_{os.getpid()}.json")
            small = torch.empty(max(p.workspace_size(2) for p in self.progs[:64]) * 2, dtype=torch.uint8,
                                device="cuda")
            for p in self.progs:
                need = p.workspace_size(2)
                if need > small.numel():
                    small = torch.empty(need, dtype=torch.uint8, device="cuda")
                key = json.dumps(p.autotune(1 << 40, 2, small, cache), sort_keys=True)
                self.tunings[key] = self.tunings.get(key, 0) + 1
                self.tuning_of.append(key)
            del small
            say(f"tuned in {time.perf_counter() - t0:.1f} s")
        self.setup_s = time.perf_counter() - t0
        self.handles = np.repeat(B.handles_of(self.progs), seeds)
        self.seed_arr = np.tile(np.arange(seeds, dtype=np.uint64), n_programs)
        self.n = int(self.handles.size)
        torch.cuda.empty_cache()
        self.ws = torch.empty(int(ws_gb * (1 << 30)), dtype=torch.uint8, device="cuda")
        self.rec_cap = rec_cap
        self.records = torch.empty(rec_cap * B.RECORD_BYTES, dtype=torch.uint8, device="cuda")
        self.n_records = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.summaries = torch.empty(self.n * B.SUMMARY_BYTES, dtype=torch.uint8, device="cuda")

    def enqueue(self):
        """One step: every instance in one rc_batch_check call (asynchronous)."""
        self.ctx.batch_check_async(self.handles, self.seed_arr, self.ws, self.records, self.n_records,
                                   self.summaries)

    def step(self):
        self.enqueue()
        self.ctx.sync()

    def instance(self, i: int):
        """(workload, seed) of instance i."""
        return self.works[i // self.seeds], i % self.seeds

    def results(self):
        """numpy (records, summaries) of the last step."""
        n = int(self.n_records.item())
        if n > self.rec_cap:
            raise RuntimeError(f"{n} records exceed the capacity {self.rec_cap}")
        return B.records_to_numpy(self.records, n), B.summaries_to_numpy(self.summaries, self.n)

    def free(self):
        for p in self.progs:
            p.close()
        self.progs = []
        self.ws = self.records = self.summaries = None
