"""Intervals of one-group programs that outgrow the LDS log, checked after
the interpreter by the group check kernel from the group's log region
(bucketed by cell window; each bucket sorted in LDS, or checked through a
per-cell table, or bucketed once more), against the oracle byte for byte,
and against the same programs sent to the global pass
(rc_tuning.global_spills = 1)."""
import numpy as np
import pytest
import torch

from paper_1308_3203_amd import binding as B
from paper_1308_3203_amd import workloads as WL
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _run(w, n, seed0=0, lds=0, global_spills=False, jit=False, cap=1 << 22):
    ctx = U.ctx()
    p = B.Program(ctx, w.src)
    p.set_ndrange(w.G, w.W)
    p.bind(w.arrays, w.scalars)
    p.set_tuning(lds_log_entries=lds, global_spills=global_spills)
    if jit:
        p.jit(True)
    buf = B.Buffers(p, n, cap=cap, ws_limit=16 << 30)
    ctx.profile(True)
    p.check_async(seed0, n, buf.ws, buf.records, buf.n_records, buf.summaries)
    ctx.sync()
    prof = ctx.profile_read()
    ctx.profile(False)
    stats = ctx.call_stats()
    # which path checked the spilled intervals: the global pass sorts the log
    stats["log_sort_launches"] = prof["log_sort"][1]
    k = int(buf.n_records.item())
    out = (B.records_to_numpy(buf.records, min(k, cap)), B.summaries_to_numpy(buf.summaries, n))
    p.close()
    return out, stats


# wide random kernels (W 672..1024) and injected races, at LDS log sizes
# from the smallest the check can work in to the largest
C3_WIDE = [0, 2, 7, 9, 15, 23, 53, 110, 131]


@pytest.mark.parametrize("lds", [1024, 4096, 16384])
@pytest.mark.parametrize("seed", C3_WIDE)
def test_random_kernels_spilled_in_group(seed, lds):
    w = WL.c3_kernel(seed)
    print(f"in-group spills: c3_{seed} (W={w.W}) lds_log_entries={lds}", flush=True)
    got, st = _run(w, 3, lds=lds)
    U.assert_same(got, U.oracle_run(w.src, w.G, w.W, w.arrays, w.scalars, n=3), f"c3_{seed} lds {lds}")
    assert st["log_sort_launches"] == 0
    assert st["global_pass"] == st["logged_global"]
    # the same through the global pass
    ref, st2 = _run(w, 3, lds=lds, global_spills=True)
    U.assert_same(got, ref, f"c3_{seed} lds {lds}, global pass")
    assert st2["global_pass"] == st2["logged_global"] == st["logged_global"]
    assert st2["intervals_spilled"] == st["intervals_spilled"]
    if st2["logged_global"]:
        assert st2["log_sort_launches"] > 0


def _three_paths_kernel():
    """One group of 1024 over two arrays of 2^18 cells: a loop of own-cell
    stores and strided reads spreads ~50K entries over the cell space, and a
    read of one cell by every work-item in every iteration makes one cell
    hold 16K of them (a bucket too large to sort, whose window is wider than
    the table: bucketed again, then checked through the table)."""
    src = """kernel three_paths(global int x[262144], global int y[262144]) {
  int v0, v1, i0;
  for i0 in 0..16 {
    v0 := x[(tid * 3 + i0 * 1024) mod 262144];
    x[(tid * 5 + 7) mod 262144] := tid & 3;
    v1 := y[7];
    y[(tid * 7 + i0) mod 262144] := v0 + v1;
  }
  barrier;
  y[(tid + 1) mod 1024] := tid;
  v0 := y[tid];
}
"""
    return WL.Workload("three_paths", src, 1, 1024, {"x": ("seeded", 0, 16), "y": ("seeded", 0, 16)})


@pytest.mark.parametrize("lds", [1024, 4096])
def test_sorted_table_and_second_level_buckets(lds):
    w = _three_paths_kernel()
    print(f"in-group spills: three_paths lds_log_entries={lds}", flush=True)
    got, st = _run(w, 2, lds=lds)
    assert st["intervals_spilled"] >= 2 and st["log_sort_launches"] == 0
    U.assert_same(got, U.oracle_run(w.src, w.G, w.W, w.arrays, w.scalars, n=2), f"three paths lds {lds}")
    assert len(got[0]) > 0


def test_fault_after_a_spill_checks_the_partial_interval():
    """A store out of bounds after the interval has spilled: the statement
    has no effect, the group stops, and its partial interval is checked."""
    src = """kernel spill_then_fault(global int x[4096], global int y[4096]) {
  int v0, i0;
  for i0 in 0..16 {
    x[(tid + i0 * 64) mod 4096] := i0;
    v0 := y[(tid * 3) mod 64];
  }
  y[tid + 3900] := 1;
  barrier;
  x[tid] := 2;
}
"""
    w = WL.Workload("spill_then_fault", src, 1, 512, {"x": ("seeded", 0, 16), "y": ("seeded", 0, 16)})
    got, st = _run(w, 2, lds=1024)
    assert st["intervals_spilled"] >= 1 and st["log_sort_launches"] == 0
    want = U.oracle_run(w.src, w.G, w.W, w.arrays, w.scalars, n=2)
    assert int(want[1]["status"][0]) == 1      # OOB
    U.assert_same(got, want, "spill then fault")


def test_program_not_proven_fault_free():
    """A data-dependent assert keeps the program off the elided-step path:
    the spilled interval goes through the interpreter's full group steps."""
    src = """kernel unproven(global int x[8192], global int y[8192]) {
  int v0, v1, i0;
  for i0 in 0..12 {
    v0 := x[(tid * 3 + i0) mod 8192];
    assert(v0 < 100);
    y[(tid + i0 * 7) mod 8192] := v0;
    v1 := y[(tid * 2) mod 8192];
  }
}
"""
    w = WL.Workload("unproven", src, 1, 768, {"x": ("seeded", 0, 16), "y": ("seeded", 0, 16)})
    owned, nf = B.owned_arrays(w.src, w.G, w.W, with_faults=True)
    assert not nf
    got, st = _run(w, 3, lds=1024)
    assert st["intervals_spilled"] >= 1 and st["log_sort_launches"] == 0
    U.assert_same(got, U.oracle_run(w.src, w.G, w.W, w.arrays, w.scalars, n=3), "unproven")


def test_per_program_kernel_spilled_in_group():
    w = WL.c3_kernel(7)
    got, st = _run(w, 2, lds=1024, jit=True)
    assert st["log_sort_launches"] == 0
    U.assert_same(got, U.oracle_run(w.src, w.G, w.W, w.arrays, w.scalars, n=2), "c3_7 per-program kernel")


def test_batch_mixing_in_group_and_global_pass():
    """A batch of one-group programs (spills checked in the group) and
    several-group templates (global pass): records placed by the full sort,
    the same as each program checked alone and as the oracle."""
    ctx = U.ctx()
    works = [WL.c3_kernel(s) for s in (0, 7, 53)] + [WL.tree_reduce(True), WL.transpose(True)]
    progs = []
    for w in works:
        p = B.Program(ctx, w.src)
        p.set_ndrange(w.G, w.W)
        p.bind(w.arrays, w.scalars)
        p.set_tuning(lds_log_entries=1024)
        progs.append(p)
    handles = np.repeat(B.handles_of(progs), 2)
    seeds = np.tile(np.arange(2, dtype=np.uint64), len(progs))
    n = len(handles)
    ws = torch.empty(8 << 30, dtype=torch.uint8, device="cuda")
    cap = 1 << 21
    rec = torch.empty(cap * B.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    summ = torch.empty(n * B.SUMMARY_BYTES, dtype=torch.uint8, device="cuda")
    ctx.batch_check_async(handles, seeds, ws, rec, cnt, summ)
    ctx.sync()
    recs = B.records_to_numpy(rec, int(cnt.item()))
    summs = B.summaries_to_numpy(summ, n)
    for i in range(n):
        w = works[i // 2]
        o_rec, o_sum = U.oracle_run(w.src, w.G, w.W, w.arrays, w.scalars, seed0=i % 2, n=1)
        o_rec = o_rec.copy()
        o_rec["instance"] = i
        U.assert_same((recs[recs["instance"] == i], summs[i:i + 1]), (o_rec, o_sum), f"batch instance {i} ({w.name})")
    for p in progs:
        p.close()
