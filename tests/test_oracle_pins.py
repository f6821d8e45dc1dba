"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: the paper's
worked examples (Fig. 1, Fig. 3) with hand-derived expected records, closed
forms, library routines (numpy sums, cumulative sums, transposes), published
generator outputs, invariants from the race definition, and brute force over
every interleaving for tiny work-groups.
"""
import os
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_3203_amd import workloads as WL
from tests import interleave as IL

NONE = O.NONE
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def recs_as_tuples(recs):
    return [(int(r["gid"]), int(r["interval"]), int(r["array"]), int(r["cell"]), int(r["label"]),
             int(r["rw_a"]), int(r["rw_b"]), int(r["ww_a"]), int(r["ww_b"])) for r in recs]


def load_golden(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            out.append(tuple(NONE if x == "-" else int(x) for x in line.split()))
    return out


# ---------------------------------------------------------------------------
# Seeded inputs: SplitMix64 from its published definition
# ---------------------------------------------------------------------------
def test_splitmix64_published_sequence():
    # SplitMix64 started from state 0 yields 0xE220A8397B1DCDAF,
    # 0x6E789E6AA1B965F4, 0x06C45D188009454F (Steele, Lea, Flood 2014 reference
    # implementation); the generator keeps the top 32 bits of each output.
    expect = [0xE220A839, 0x6E789E6A, 0x06C45D18]
    got = [O.seeded_value(0, 0, i, 0, 2 ** 32) & 0xFFFFFFFF for i in range(3)]
    assert got == expect


def test_seeded_range_scaling_worked_by_hand():
    # value = lo + ((u * (hi - lo)) >> 32) with u the top 32 bits of the
    # output.  Worked from the three published outputs above:
    #   u = 0xE220A839 = 3793791033, 0x6E789E6A = 1853398634, 0x06C45D18 = 113532184
    #   U[0,16):   u >> 28                       -> 14, 6, 0
    #   U[0,100):  floor(u * 100 / 2^32)         -> 88 (88.33), 43 (43.15), 2 (2.64)
    #   U[-5,3):   -5 + (u >> 29)                -> -5 + 7, -5 + 3, -5 + 0 = 2, -2, -5
    # (a modulo reduction, u % 16, would give 9, 10, 8 instead)
    assert [O.seeded_value(0, 0, i, 0, 16) for i in range(3)] == [14, 6, 0]
    assert [O.seeded_value(0, 0, i, 0, 100) for i in range(3)] == [88, 43, 2]
    assert [O.seeded_value(0, 0, i, -5, 3) for i in range(3)] == [2, -2, -5]
    # full int32 range: -2^31 + u = -2147483648 + 3793791033
    assert O.seeded_value(0, 0, 0, -(2 ** 31), 2 ** 31) == 1646307385


def test_seeded_counter_form():
    # The seed is added to golden * counter: starting from seed = golden * k
    # the sequence is the published one shifted by k outputs.  Stream s,
    # index i is counter s * 2^32 + i + 1.
    golden = 0x9E3779B97F4A7C15
    assert O.seeded_value(golden % 2 ** 64, 0, 0, 0, 2 ** 32) & 0xFFFFFFFF == 0x6E789E6A
    assert O.seeded_value(2 * golden % 2 ** 64, 0, 0, 0, 2 ** 32) & 0xFFFFFFFF == 0x06C45D18
    for i in range(4):
        assert O.seeded_value(0, 1, i, 0, 2 ** 32) == O.seeded_value((golden << 32) % 2 ** 64, 0, i, 0, 2 ** 32)


def test_seeded_range_bounds():
    for lo, hi in [(0, 16), (-5, 3), (-(2 ** 31), 2 ** 31), (7, 8)]:
        vals = [O.seeded_value(123, 2, i, lo, hi) for i in range(2000)]
        assert min(vals) >= lo and max(vals) < hi
    vals = [O.seeded_value(9, 0, i, 0, 16) for i in range(16000)]
    counts = np.bincount(vals, minlength=16)
    assert counts.min() > 800   # roughly uniform


# ---------------------------------------------------------------------------
# The paper's worked examples
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [4, 64])
def test_fig1_literal_faults_out_of_bounds(n):
    # Fig. 1 with 0-based tid: thread 0's first load reads A[-1].  The
    # out-of-bounds access is a runtime error (Section 4, bottom state;
    # Table 1 bounds rule): statement 0, thread 0, nothing executed.
    w = WL.fig1(n, one_based=False)
    r = O.check(w.src, w.G, w.W, arrays=w.arrays, seed=3)
    assert r.status == "OOB"
    assert (int(r.summary["fault_pc"]), int(r.summary["fault_tid"]), int(r.summary["fault_gid"])) == (0, 0, 0)
    assert len(r.records) == 0
    assert int(r.summary["n_accesses"]) == 0 and int(r.summary["n_intervals"]) == 1


def fig1_expected(n):
    return [(0, 1, 2, c, 1, c - 2, c - 1, NONE, NONE) for c in range(2, n + 1)]


@pytest.mark.parametrize("n", [4, 5, 64, 200])
def test_fig1_one_based_closed_form(n):
    w = WL.fig1(n, one_based=True)
    for seed in (0, 7):
        r = O.check(w.src, w.G, w.W, arrays=w.arrays, seed=seed)
        assert r.status == "OK"
        assert recs_as_tuples(r.records) == fig1_expected(n)
        assert int(r.summary["n_intervals"]) == 2
        assert int(r.summary["n_accesses"]) == 5 * n
        assert int(r.summary["n_race_cells"]) == n - 1


def test_fig1_golden_fixture():
    w = WL.fig1(4, one_based=True)
    r = O.check(w.src, w.G, w.W, arrays=w.arrays, seed=0)
    assert recs_as_tuples(r.records) == load_golden("fig1_one_based_n4.txt")


def fig3_expected(n):
    out = [(0, 0, 1, 0, 4, NONE, NONE, 0, 1)]
    out += [(0, 1, 0, c, 1, c - 2, c - 1, NONE, NONE) for c in range(2, n + 1)]
    return out


@pytest.mark.parametrize("n", [2, 4, 33, 64])
def test_fig3_closed_form(n):
    w = WL.fig3(n)
    for last in (0, 5):     # A[n+1] decides whether thread n-1 writes g
        A = np.full(n + 2, 9, np.int32)
        A[n + 1] = last
        r = O.check(w.src, w.G, w.W, arrays={"A": A, "g": np.array([42], np.int32)}, seed=0, final="g")
        assert r.status == "OK"
        assert recs_as_tuples(r.records) == fig3_expected(n)
        assert int(r.summary["n_intervals"]) == 3
        assert int(r.summary["n_benign_cells"]) == 1
        # the lockstep run lets only thread n-1 reach g := 1, and only when the
        # cell past the end it reads still holds 0
        assert int(r.final[0]) == (1 if last == 0 else 0)


def test_fig3_golden_fixture():
    w = WL.fig3(4)
    r = O.check(w.src, w.G, w.W, arrays={"A": np.ones(6, np.int32), "g": np.zeros(1, np.int32)}, seed=0)
    assert recs_as_tuples(r.records) == load_golden("fig3_n4.txt")


# ---------------------------------------------------------------------------
# Invariants of the race definition
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("W", [2, 17, 64, 300])
def test_own_cell_writes_race_free(W):
    src = f"kernel k(global int A[{W}], global int B[{W}]) {{ int v; v := B[tid]; A[tid] := v * tid + 3; v := A[tid]; A[tid] := v + 1; }}"
    r = O.check(src, 1, W, seed=1)
    assert len(r.records) == 0


@pytest.mark.parametrize("W", [2, 64, 130])
def test_equal_value_writes_are_benign(W):
    # Section 1: several threads writing the same value is a benign race
    r = O.check("kernel k(global int A[8]) { A[3] := 7; }", 1, W)
    assert recs_as_tuples(r.records) == [(0, 0, 0, 3, 4, NONE, NONE, 0, 1)]
    assert int(r.summary["n_benign_cells"]) == 1 and int(r.summary["n_race_cells"]) == 0


@pytest.mark.parametrize("W", [2, 64, 130])
def test_different_value_writes_race(W):
    r = O.check("kernel k(global int A[8]) { A[3] := tid; }", 1, W)
    assert recs_as_tuples(r.records) == [(0, 0, 0, 3, 2, NONE, NONE, 0, 1)]


def test_barrier_separates_conflicts():
    racy = "kernel k(global int A[64]) { int v; A[tid] := tid; v := A[(tid + 1) mod 64]; }"
    fixed = "kernel k(global int A[64]) { int v; A[tid] := tid; barrier; v := A[(tid + 1) mod 64]; }"
    r1 = O.check(racy, 1, 64)
    r2 = O.check(fixed, 1, 64)
    assert len(r1.records) == 64 and all(r1.records["label"] == 1)
    assert len(r2.records) == 0


def test_same_thread_accesses_never_pair():
    r = O.check("kernel k(global int A[4]) { int v; A[0] := 1; v := A[0]; A[0] := 2; }", 1, 1)
    assert len(r.records) == 0


def test_reads_only_never_pair():
    r = O.check("kernel k(global int A[4]) { int v; v := A[0]; v := A[1]; }", 1, 256)
    assert len(r.records) == 0


def test_rw_with_same_value_is_still_a_race():
    # a write that re-stores the value another thread reads is still RW
    r = O.check("kernel k(global int A[4]) { int v; v := A[0]; A[0] := 0; }", 1, 2,
                arrays={"A": np.zeros(4, np.int32)})
    assert recs_as_tuples(r.records) == [(0, 0, 0, 0, 1, 0, 1, NONE, NONE)]


def test_mixed_labels_and_witnesses():
    # thread 0 reads cell 0, threads 1 and 2 write it with different values,
    # threads 3 write the same value as thread 1
    src = """kernel k(global int A[4]) { int v;
      if (tid == 0) { v := A[0]; }
      if (tid == 1) { A[0] := 5; }
      if (tid == 2) { A[0] := 6; }
      if (tid == 3) { A[0] := 5; } }"""
    r = O.check(src, 1, 4)
    assert recs_as_tuples(r.records) == [(0, 0, 0, 0, 3, 0, 1, 1, 2)]


# ---------------------------------------------------------------------------
# A single affine store, brute-forced independently in numpy
# ---------------------------------------------------------------------------
def _wrap32(x):
    return ((np.asarray(x, dtype=np.int64) + 2 ** 31) % 2 ** 32 - 2 ** 31).astype(np.int64)


@pytest.mark.parametrize("a,b,N,c,m,W", [(3, 5, 64, 1, 3, 64), (-4, 17, 32, 0, 7, 100),
                                         (2, 0, 256, 5, 1, 200), (0, 9, 16, 1, 0, 10),
                                         (7, 1, 128, 3, 15, 1024)])
def test_affine_store_brute_force(a, b, N, c, m, W):
    src = f"kernel k(global int A[{N}]) {{ A[({a} * tid + {b}) mod {N}] := (tid * {c}) & {m}; }}"
    r = O.check(src, 1, W)
    tids = np.arange(W, dtype=np.int64)
    cells = np.mod(a * tids + b, N)
    vals = _wrap32(tids * c) & m
    exp = []
    for cell in range(N):
        ts = tids[cells == cell]
        if len(ts) < 2:
            continue
        vs = vals[cells == cell]
        diff = [(int(ts[i]), int(ts[j])) for i in range(len(ts)) for j in range(i + 1, len(ts)) if vs[i] != vs[j]]
        if diff:
            exp.append((0, 0, 0, cell, 2, NONE, NONE) + min(diff))
        else:
            exp.append((0, 0, 0, cell, 4, NONE, NONE, int(ts[0]), int(ts[1])))
    assert recs_as_tuples(r.records) == exp


# ---------------------------------------------------------------------------
# int32 semantics: hard-coded values from the operator definitions
# ---------------------------------------------------------------------------
def test_int32_arithmetic_corners():
    src = """kernel ar(global int out[24], int m) {
      out[0] := 0 - 7 / 2;
      out[1] := (0 - 7) / 2;
      out[2] := (0 - 7) % 2;
      out[3] := (0 - 7) mod 2;
      out[4] := 7 mod (0 - 2);
      out[5] := m / (0 - 1);
      out[6] := m % (0 - 1);
      out[7] := 1 << 33;
      out[8] := (0 - 8) >> 1;
      out[9] := (0 - 1) >> 40;
      out[10] := m - 1;
      out[11] := 2147483647 + 1;
      out[12] := 65536 * 65536;
      out[13] := 0 - m;
      out[14] := m mod 3;
      out[15] := (0 - 7) mod (0 - 2);
      out[16] := (3 < 4) + (4 <= 4) * 2 + (5 == 5) * 4 + !0 * 8 + (0 && 1) * 16 + (0 || 2) * 32;
      out[17] := ~5;
      out[18] := min(0 - 3, 2) * 10 + max(0 - 3, 2);
      out[19] := (12 ^ 10) + (12 | 3) * 100;
      out[20] := 4294967295;
      out[21] := (0 - 9) >> 2;
      out[22] := m >> 31;
      out[23] := 7 % (0 - 3);
    }"""
    r = O.check(src, 1, 1, arrays={"out": np.zeros(24, np.int32)}, scalars={"m": -(2 ** 31)}, final="out")
    assert r.status == "OK"
    imin, imax = -(2 ** 31), 2 ** 31 - 1
    expect = [-3, -3, -1, 1, 1, imin, 0, 2, -4, -1, imax, imin, 0, imin, 1, 1, 47, -6, -28, 6 + 1500,
              -1, -3, -1, 1]
    assert [int(x) for x in r.final] == expect


@pytest.mark.parametrize("op", ["/", "%", "mod"])
def test_division_by_zero_faults(op):
    src = f"kernel k(global int A[8]) {{ int v; A[tid] := 1; v := 5 {op} (tid - 3); A[tid] := v; }}"
    r = O.check(src, 1, 8)
    assert r.status == "DIV_ZERO"
    assert (int(r.summary["fault_pc"]), int(r.summary["fault_tid"])) == (1, 3)
    # the faulting statement has no effect; the partial interval is checked
    assert int(r.summary["n_accesses"]) == 8 and len(r.records) == 0


# ---------------------------------------------------------------------------
# Faults (runtime errors and blocked paths) and their reporting
# ---------------------------------------------------------------------------
def test_assert_assume_divergence_oob():
    r = O.check("kernel k(global int A[8]) { assert(tid < 5); }", 1, 8)
    assert (r.status, int(r.summary["fault_tid"])) == ("ASSERT", 5)
    r = O.check("kernel k(global int A[8]) { A[0] := 1; assume(tid != 2); }", 1, 8)
    assert (r.status, int(r.summary["fault_pc"]), int(r.summary["fault_tid"])) == ("ASSUME", 1, 2)
    r = O.check("kernel k(global int A[8]) { if (tid < 2) { barrier; } }", 1, 8)
    assert (r.status, int(r.summary["fault_pc"]), int(r.summary["fault_tid"])) == ("BARRIER_DIVERGENCE", 1, 2)
    r = O.check("kernel k(global int A[8]) { A[tid + 6] := 1; }", 1, 4)
    assert (r.status, int(r.summary["fault_tid"])) == ("OOB", 2)
    assert int(r.summary["n_accesses"]) == 0


def test_barrier_in_uniform_branch_is_fine():
    r = O.check("kernel k(global int A[8]) { int v; v := 1; if (v == 1) { barrier; } }", 1, 8)
    assert r.status == "OK" and int(r.summary["n_intervals"]) == 2
    r = O.check("kernel k(global int A[8]) { int v; if (v == 1) { barrier; } }", 1, 8)
    assert r.status == "OK" and int(r.summary["n_intervals"]) == 1


def test_partial_interval_checked_on_fault():
    r = O.check("kernel k(global int A[8]) { int v; A[0] := tid; v := 1 / (tid - 3); }", 1, 8)
    assert r.status == "DIV_ZERO"
    assert recs_as_tuples(r.records) == [(0, 0, 0, 0, 2, NONE, NONE, 0, 1)]


def test_lowest_faulting_group_sets_status():
    src = "kernel k(global int A[64]) { int v; A[tid] := tid; v := 1 / (gid - 1); v := 2 / (gid - 2); }"
    r = O.check(src, 4, 8)
    assert (r.status, int(r.summary["fault_gid"]), int(r.summary["fault_tid"]), int(r.summary["fault_pc"])) == \
        ("DIV_ZERO", 1, 8, 1)
    # every group ran: 4 groups x 8 stores
    assert int(r.summary["n_accesses"]) == 32 and int(r.summary["n_intervals"]) == 4


def test_first_fault_in_time_wins_over_lower_pc():
    # pc 2 faults in iteration 0; pc 1 would fault only in iteration 1
    src = """kernel k(global int A[8]) { int i, v;
      for i in 0..3 {
        v := 1 / (i - 1 + 100 * tid);
        v := 1 / (tid - 3);
      } }"""
    r = O.check(src, 1, 8)
    assert (r.status, int(r.summary["fault_pc"]), int(r.summary["fault_tid"])) == ("DIV_ZERO", 2, 3)


# ---------------------------------------------------------------------------
# Work-groups, scopes and the merge rule
# ---------------------------------------------------------------------------
def test_groups_run_on_isolated_views_and_inter_scope():
    # every group writes cell 0 (value gid) and reads cell 1, which group 0 writes
    src = """kernel k(global int A[4]) { int v;
      if (lid == 0) { A[0] := gid; }
      if (gid == 0) { if (lid == 1) { A[1] := 9; } }
      barrier;
      v := A[1];
      if (lid == 0) { A[2] := v; } }"""
    r = O.check(src, 3, 2, arrays={"A": np.array([1, 2, 3, 4], np.int32)}, final="A")
    recs = recs_as_tuples(r.records)
    inter = [x for x in recs if x[0] == NONE]
    intra = [x for x in recs if x[0] != NONE]
    # INTER: cell 0 written by tids 0, 2, 4 with values 0, 1, 2 -> WW_DIFF (0, 2);
    # cell 1: group 0 writes (tid 1), groups 1 and 2 read -> RW (1, 2);
    # cell 2: each group writes its own view of A[1]: 9, 2, 2 -> WW_DIFF (0, 2)
    assert inter == [(NONE, 0, 0, 0, 2, NONE, NONE, 0, 2), (NONE, 0, 0, 1, 1, 1, 2, NONE, NONE),
                     (NONE, 0, 0, 2, 2, NONE, NONE, 0, 2)]
    assert intra == []
    # final memory: highest writing gid wins per cell
    assert [int(x) for x in r.final] == [2, 9, 2, 4]


# ---------------------------------------------------------------------------
# c2 templates: library routines and hand-derived closed forms
# ---------------------------------------------------------------------------
def _template_inputs(seed):
    rng = np.random.default_rng(seed)
    return rng.integers(-(2 ** 31), 2 ** 31, size=65536, dtype=np.int64).astype(np.int32)


def test_tree_reduce_sums():
    w = WL.tree_reduce(False)
    x = _template_inputs(1)
    out0 = _template_inputs(2)
    r = O.check(w.src, w.G, w.W, arrays={"inp": x, "out": out0}, final="out")
    assert len(r.records) == 0 and r.status == "OK"
    sums = _wrap32(x.astype(np.int64).reshape(16, 4096).sum(axis=1))
    exp = out0.copy()
    exp[:16] = sums
    assert np.array_equal(r.final, exp)


def test_prefix_sum_cumsum():
    w = WL.prefix_sum(False)
    x = _template_inputs(3)
    r = O.check(w.src, w.G, w.W, arrays={"inp": x, "out": _template_inputs(4)}, final="out")
    assert len(r.records) == 0
    exp = _wrap32(np.cumsum(x.astype(np.int64).reshape(16, 4096), axis=1)).reshape(-1)
    assert np.array_equal(r.final, exp)


def test_transpose_matches_numpy():
    w = WL.transpose(False)
    x = _template_inputs(5)
    r = O.check(w.src, w.G, w.W, arrays={"inp": x, "out": _template_inputs(6)}, final="out")
    assert len(r.records) == 0
    assert np.array_equal(r.final, x.reshape(256, 256).T.reshape(-1))


def test_tree_reduce_off_by_one_closed_form():
    # loc[lid + s - 1] makes thread 0 read loc[s-1], which thread s-1 writes:
    # one RW record per level with s >= 2, in the interval after j barriers
    w = WL.tree_reduce(True)
    r = O.check(w.src, w.G, w.W, arrays=w.arrays, seed=11)
    exp = []
    for g in range(16):
        for j in range(7):
            s = 128 >> j
            exp.append((g, j + 1, 2, s - 1, 1, 256 * g, 256 * g + s - 1, NONE, NONE))
    assert recs_as_tuples(r.records) == exp


def test_prefix_sum_off_by_one_closed_form():
    # the wrapped write index lets thread 255 write the first cell of the read
    # half, which threads 0 and 'off' read: one RW record per level
    w = WL.prefix_sum(True)
    r = O.check(w.src, w.G, w.W, arrays=w.arrays, seed=12)
    exp = []
    for g in range(16):
        for d in range(8):
            rd = (d & 1) * 256
            exp.append((g, d + 1, 2, rd, 1, 256 * g, 256 * g + 255, NONE, NONE))
    assert recs_as_tuples(r.records) == exp


def test_transpose_off_by_one_closed_form():
    # tile 2's read-out and tile 3's fill share interval 5: cell i*33+j is read
    # by lid (j%8)*32+i and written by lid (i%8)*32+j
    w = WL.transpose(True)
    r = O.check(w.src, w.G, w.W, arrays=w.arrays, seed=13)
    exp = []
    for g in range(16):
        for i in range(32):
            for j in range(32):
                if i == j:
                    continue
                rl, wl = (j % 8) * 32 + i, (i % 8) * 32 + j
                exp.append((g, 5, 2, i * 33 + j, 1, 256 * g + min(rl, wl), 256 * g + max(rl, wl), NONE, NONE))
    exp.sort(key=lambda t: (t[0], t[1], t[2], t[3]))
    assert recs_as_tuples(r.records) == exp
    assert int(r.summary["n_intervals"]) == 16 * 7


# ---------------------------------------------------------------------------
# Bucketed pairs equal literal all-pairs; brute force over interleavings
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(12))
def test_bucketed_equals_literal(seed):
    r = random.Random(seed)
    prog, arrays, vars_ = IL.random_program(r, r.randint(3, 9), r.choice([2, 4, 8]), r.randint(0, 2))
    src = IL.render(prog, arrays, vars_)
    W = r.choice([2, 3, 5, 9])
    G = r.choice([1, 2, 3])
    a = O.check(src, G, W, seed=seed)
    b = O.check(src, G, W, seed=seed, literal=True)
    assert recs_as_tuples(a.records) == recs_as_tuples(b.records)
    assert a.summary.tobytes() == b.summary.tobytes()


@pytest.mark.parametrize("seed", range(40))
def test_soundness_against_every_interleaving(seed):
    """If lockstep reports no race, every schedule ends in the same state
    (shared and private); in every case the lockstep state is reachable."""
    r = random.Random(1000 + seed)
    W = r.choice([2, 2, 3])
    N = r.choice([2, 3, 4])
    n = r.randint(2, 5 if W == 3 else 7)
    prog, arrays, vars_ = IL.random_program(r, n, N, r.randint(0, 1))
    init = {a: [r.randint(0, 3) for _ in range(sz)] for a, sz in arrays.items()}
    src = IL.render(prog, arrays, vars_)
    res = O.check(src, 1, W, arrays={a: np.array(v, np.int32) for a, v in init.items()})
    finals = IL.final_states(prog, W, init, vars_)
    lock = IL.lockstep_state(prog, W, init, vars_)
    assert lock in finals
    # the oracle's final memory is the lockstep schedule's
    for a in arrays:
        fin = O.check(src, 1, W, arrays={k: np.array(v, np.int32) for k, v in init.items()}, final=a).final
        assert tuple(int(x) for x in fin) == dict(lock[0])[a]
    racy = bool(res.summary["n_race_cells"])
    if not racy:
        assert finals == {lock}


def test_soundness_detects_schedule_dependence():
    # a racy program whose outcome differs between schedules is flagged
    prog = [("store", "A", 0, "tid"), ("load", "p", "A", 0)]
    finals = IL.final_states(prog, 2, {"A": [5, 5]}, ["p", "q"])
    assert len(finals) > 1
    res = O.check(IL.render(prog, {"A": 2}, ["p", "q"]), 1, 2)
    assert int(res.summary["n_race_cells"]) == 1


# ---------------------------------------------------------------------------
# Parser rejections
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("src", [
    "kernel k(global int A[4]) { v := 1; }",                                  # unknown name
    "kernel k(global int A[4], int s) { s := 1; }",                           # scalar is read-only
    "kernel k(global int A[4]) { int i; for i in 0..3 { i := 2; } }",         # loop var assigned
    "kernel k(global int A[4]) { int v; v := A[0] + 1; }",                    # load inside an expression
    "kernel k(global int A[0]) { }",                                          # empty array
    "kernel k(global int A[4]) { int v; v := 1 }",                            # missing ';'
    "kernel k(global int A[4]) { int v; v := 1 @ 2; }",                       # bad character
    "kernel k(global int A[4]) { int A; }",                                   # duplicate name
    "kernel k(global int A[4]) { int i, j; for i in 0..2 { for i in 0..2 { } } }",
])
def test_parse_errors(src):
    with pytest.raises(O.OracleError):
        O.Program(src)


# ---------------------------------------------------------------------------
# The loop-iteration limit (reading R13's safety net): a work-group that would
# start more loop iterations than its limit stops at that for statement.
# ---------------------------------------------------------------------------
STEP_SRC = """kernel s(global int x[64]) {
  int v, i, j;
  x[5] := tid;
  for i in 0..100 {
    for j in 0..100 {
      v := v + 1;
    }
  }
  x[7] := tid;
}
"""


@pytest.mark.parametrize("limit,G", [(5000, 1), (5000, 3), (10099, 1), (10100, 2)])
def test_step_limit_closed_form(limit, G):
    # Iteration starts run 1 (outer), 2..101 (inner), 102 (outer), ...: the
    # outer loop's k-th start is number 1 + 101 (k - 1), every other number
    # is an inner start, 10100 in all.  Past the limit the group stops at
    # the statement that would start one more: the inner for (pc 2) for
    # limits 5000 and 10099 (5001 and 10100 are inner starts).  Interval 0
    # then holds only the store to x[5], whose writes all differ.
    r = O.check(STEP_SRC, G, 64, arrays={"x": ("seeded", 0, 4)}, step_limit=limit)
    recs = recs_as_tuples(r.records)
    if limit >= 10100:
        assert r.status == "OK"
        expect = [(g, 0, 0, c, 2, NONE, NONE, g * 64, g * 64 + 1) for g in range(G) for c in (5, 7)]
        inter = [(NONE, 0, 0, c, 2, NONE, NONE, 0, 64) for c in (5, 7)] if G > 1 else []
        assert recs == expect + inter
    else:
        assert r.status == "STEP_LIMIT"
        assert (int(r.summary["fault_gid"]), int(r.summary["fault_pc"]), int(r.summary["fault_tid"])) == (0, 2, 0)
        expect = [(g, 0, 0, 5, 2, NONE, NONE, g * 64, g * 64 + 1) for g in range(G)]
        inter = [(NONE, 0, 0, 5, 2, NONE, NONE, 0, 64)] if G > 1 else []
        assert recs == expect + inter
        assert int(r.summary["n_accesses"]) == 64 * G


def test_step_limit_default():
    # 4200 outer x 4000 inner iterations: 4200 + 4200 * 4000 = 16 804 200
    # starts, above 2^24.  Start 2^24 + 1 = 16 777 217 falls after the
    # 4194-th outer start (number 1 + 4001 * 4193 = 16 776 194): an inner start.
    src = STEP_SRC.replace("0..100 {\n    for j in 0..100", "0..4200 {\n    for j in 0..4000")
    r = O.check(src, 1, 1, arrays={"x": ("seeded", 0, 4)})
    assert r.status == "STEP_LIMIT" and int(r.summary["fault_pc"]) == 2
    r = O.check(src, 1, 1, arrays={"x": ("seeded", 0, 4)}, step_limit=16804200)
    assert r.status == "OK"
