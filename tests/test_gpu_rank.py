"""Record order without a record sort.  In a call with no global access log
every record comes from an interval closed in LDS, which emits its records
in cell-key order; a record's position then follows from the record counts
of the (instance, group, interval)s before it and its rank in its own.  The
same checks with the records radix-sorted by their full canonical key, and
the oracle, must agree byte for byte: on the per-cell table path, on the
sorted-log path (a local array too large for the table), with faults that
cut an interval short, and in batches of several programs."""
import pytest

from paper_1308_3203_amd import binding as B
from paper_1308_3203_amd import workloads as WL
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

TEMPLATES = {w.name: w for w in WL.c2_templates()}

LOCAL = [
    # (name, src, G, W)
    ("table", "kernel t(global int A[64]) {\n  local int L[64];\n  int v;\n  L[lid % 7] := lid;\n  barrier;\n"
              "  v := L[(lid + 1) % 7];\n  L[lid % 5] := v;\n  v := L[lid % 3];\n}\n", 4, 64),
    ("table_two_waves", "kernel t(global int A[64]) {\n  local int L[300];\n  int v, k;\n"
                        "  for k in 0..3 {\n    L[(lid * 7 + k) % 300] := lid + k;\n    v := L[(lid + k) % 300];\n"
                        "    barrier;\n  }\n}\n", 3, 130),
    # 5000 cells: beyond the per-cell table, the interval's log is sorted in LDS
    ("sorted_log", "kernel t(global int A[64]) {\n  local int L[5000];\n  int v;\n  L[(lid * 3) % 5000] := lid;\n"
                   "  L[(lid * 3 + 1) % 5000] := 1;\n  barrier;\n  v := L[lid % 97];\n  L[lid % 89] := v;\n}\n", 2, 256),
    # work-items 100 and up fail the assertion in the second interval
    ("fault", "kernel t(global int A[64]) {\n  local int L[64];\n  int v;\n  L[lid % 8] := lid;\n  barrier;\n"
              "  v := L[lid % 9];\n  L[lid % 6] := v;\n  assert(lid < 100);\n  barrier;\n  v := L[0];\n}\n", 2, 128),
]


def run(p, n, seed0, record_sort):
    p.set_tuning(record_sort=record_sort)
    buf = B.Buffers(p, n, 1 << 20)
    p.check_async(seed0, n, buf.ws, buf.records, buf.n_records, buf.summaries)
    U.ctx().sync()
    k = int(buf.n_records.item())
    return B.records_to_numpy(buf.records, k), B.summaries_to_numpy(buf.summaries, n), p.workspace_size(n)


def both_orders(src, G, W, arrays, scalars, n, seed0, jit):
    p = B.Program(U.ctx(), src)
    p.set_ndrange(G, W)
    p.bind(arrays, scalars)
    if jit:
        p.jit(True)
    rec_r, sum_r, ws_r = run(p, n, seed0, 0)
    rec_s, sum_s, ws_s = run(p, n, seed0, 1)
    orc = U.oracle_run(src, G, W, arrays, scalars, seed0, n)
    U.assert_same((rec_r, sum_r), orc, "rank order")
    U.assert_same((rec_s, sum_s), orc, "sorted order")
    # placing by rank drops the record sort's buffers
    assert ws_r < ws_s
    return len(rec_r)


@pytest.mark.parametrize("jit", [False, True])
@pytest.mark.parametrize("case", LOCAL, ids=lambda c: c[0])
def test_local_programs(case, jit):
    name, src, G, W = case
    assert both_orders(src, G, W, {"A": ("seeded", 0, 8)}, None, 5, 3, jit) > 0, name


@pytest.mark.parametrize("jit", [False, True])
@pytest.mark.parametrize("name", ["tree_reduce_race", "prefix_sum_race", "transpose_race", "transpose"])
def test_templates(name, jit):
    w = TEMPLATES[name]
    both_orders(w.src, 2, w.W, w.arrays, w.scalars, 3, 11, jit)


def test_batch_of_local_programs():
    """Several programs (two width classes) in one call, placed by rank."""
    import numpy as np
    import torch

    from oracle import oracle as O
    arrays = {"A": ("seeded", 0, 8)}
    progs = []
    for _, src, G, W in LOCAL:
        p = B.Program(U.ctx(), src)
        p.set_ndrange(G, W)
        p.bind(arrays)
        progs.append(p)
    order = [i % len(LOCAL) for i in range(7)]
    plist = [progs[k] for k in order]
    seeds = [50 + i for i in range(len(order))]
    recs, summs = [], []
    for i, (k, seed) in enumerate(zip(order, seeds)):
        _, src, G, W = LOCAL[k]
        r = O.Program(src).run(G, W, arrays=arrays, seed=seed, instance=i)
        recs.append(r.records)
        summs.append(r.summary)
    orc = (np.concatenate(recs), np.array(summs, dtype=O.SUMMARY_DTYPE))
    assert len(orc[0]) > 0
    n = len(plist)
    for rs in (0, 1):
        plist[0].set_tuning(record_sort=rs)   # a batch follows its first program
        ws = torch.empty(max(p.workspace_size(1) for p in progs) * 4, dtype=torch.uint8, device="cuda")
        rec = torch.empty((1 << 18) * B.RECORD_BYTES, dtype=torch.uint8, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        summ = torch.empty(n * B.SUMMARY_BYTES, dtype=torch.uint8, device="cuda")
        U.ctx().batch_check_async(plist, seeds, ws, rec, cnt, summ)
        U.ctx().sync()
        k = int(cnt.item())
        U.assert_same((B.records_to_numpy(rec, k), B.summaries_to_numpy(summ, n)), orc, f"batch record_sort={rs}")
