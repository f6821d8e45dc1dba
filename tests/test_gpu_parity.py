"""GPU parity: the HIP library (through the C ABI) against the CPU oracle,
record for record and summary for summary, on the same seeded instances."""
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_3203_amd import binding as B
from paper_1308_3203_amd import workloads as WL
from tests import gpu_util as U
from tests import interleave as IL

pytestmark = pytest.mark.gpu


def both(src, G, W, arrays=None, scalars=None, seed0=0, n=1, **kw):
    dev_arrays = U.host_arrays_to_device(arrays)
    g = U.gpu_run(src, G, W, dev_arrays, scalars, seed0, n, **kw)
    o = U.oracle_run(src, G, W, arrays, scalars, seed0, n)
    return g, o


# ---------------------------------------------------------------------------
# the paper's examples
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("one_based", [False, True])
@pytest.mark.parametrize("n", [4, 64, 65, 200])
def test_fig1(n, one_based):
    w = WL.fig1(n, one_based)
    g, o = both(w.src, w.G, w.W, w.arrays, n=3)
    U.assert_same(g, o, w.name)


@pytest.mark.parametrize("n", [2, 64, 100])
def test_fig3(n):
    w = WL.fig3(n)
    g, o = both(w.src, w.G, w.W, w.arrays, seed0=5, n=8)
    U.assert_same(g, o, w.name)


# ---------------------------------------------------------------------------
# c1: one random kernel, 1000 seeds
# ---------------------------------------------------------------------------
def test_c1_all_seeds():
    w = WL.c1_kernel(1)
    g, o = both(w.src, w.G, w.W, w.arrays, seed0=0, n=1000)
    U.assert_same(g, o, "c1")


@pytest.mark.parametrize("pseed", [2, 3, 4, 5])
def test_c1_other_programs(pseed):
    w = WL.c1_kernel(pseed)
    g, o = both(w.src, w.G, w.W, w.arrays, seed0=100, n=50)
    U.assert_same(g, o, w.name)


# ---------------------------------------------------------------------------
# random small kernels across launch shapes (single and multi-wave groups,
# ragged last waves, several groups)
# ---------------------------------------------------------------------------
SHAPES = [(1, 1), (1, 7), (1, 64), (1, 65), (2, 33), (3, 130), (1, 256), (2, 300), (1, 1000), (4, 1024),
          # one group, widths whose last waves leave part of the workgroup idle
          (1, 130), (1, 200), (1, 352), (1, 600), (1, 900)]


@pytest.mark.parametrize("G,W", SHAPES)
@pytest.mark.parametrize("pseed", range(3))
def test_random_shapes(G, W, pseed):
    r = random.Random(pseed * 101 + W)
    prog, arrays, vars_ = IL.random_program(r, r.randint(4, 12), r.choice([4, 16, 64]), r.randint(0, 3))
    src = IL.render(prog, arrays, vars_)
    g, o = both(src, G, W, {a: ("seeded", 0, 4) for a in arrays}, seed0=pseed, n=4)
    U.assert_same(g, o, f"random G={G} W={W}\n{src}")


# ---------------------------------------------------------------------------
# control flow, faults, int32 semantics
# ---------------------------------------------------------------------------
FAULTS = [
    "kernel k(global int A[8]) { int v; A[tid % 8] := 1; v := 5 / (tid - 3); A[tid % 8] := v; }",
    "kernel k(global int A[8]) { int v; A[0] := tid; v := 1 mod (tid - 70); }",
    "kernel k(global int A[8]) { assert(tid < 5); }",
    "kernel k(global int A[8]) { A[0] := 1; assume(tid != 100); }",
    "kernel k(global int A[8]) { if (tid < 2) { barrier; } }",
    "kernel k(global int A[8]) { if (lid < 70) { barrier; } }",
    "kernel k(global int A[8]) { A[tid + 6] := 1; }",
    "kernel k(global int A[8]) { int v; v := A[(tid * 7) mod 9]; }",
    """kernel k(global int A[8]) { int i, v;
       for i in 0..3 { v := 1 / (i - 1 + 100 * tid); v := 1 / (tid - 67); } }""",
    """kernel k(global int A[64]) { int v; A[lid % 64] := tid; v := 1 / (gid - 1); v := 2 / (gid - 2); }""",
    """kernel k(global int A[8]) { int v; A[9] := 5 / (tid - 3); }""",
]


@pytest.mark.parametrize("src", FAULTS)
@pytest.mark.parametrize("G,W", [(1, 8), (1, 100), (4, 130)])
def test_faults(src, G, W):
    g, o = both(src, G, W, {"A": ("seeded", 0, 16)}, n=2)
    U.assert_same(g, o, src)


CONTROL = [
    """kernel k(global int A[256], global int B[256]) { int i, j, v, w;
       for i in 0..5 { for j in 2..4 { v := A[(tid + i * j) mod 256]; if (v < 8) { B[tid mod 256] := v + i; } else { w := v * j; } } barrier; }
       if ((tid & 3) == 1) { B[(tid * 3) mod 256] := w; } else { if (tid > 100) { v := B[5]; } } }""",
    """kernel k(global int A[64]) { int i, v; for i in 0..0 { A[0] := 1; } for i in 5..2 { A[1] := 2; } v := i; A[tid mod 64] := v; }""",
    """kernel k(global int A[64], int s, int t) { int v; v := s * tid + t; A[(v mod 64)] := v; barrier; v := A[(tid + 1) mod 64]; }""",
    """kernel k(global int A[32]) { local int L[32]; int v; L[lid mod 32] := tid; barrier; v := L[(lid + 1) mod 32]; A[lid mod 32] := v; L[0] := v; }""",
    """kernel k(global int A[16]) { int v; if (tid == 0) { v := A[3]; } if (tid == 1) { A[3] := 5; } if (tid == 2) { A[3] := 6; } if (tid == 3) { A[3] := 5; } }""",
]


@pytest.mark.parametrize("src", CONTROL)
@pytest.mark.parametrize("G,W", [(1, 4), (1, 64), (2, 100), (3, 257)])
def test_control_flow(src, G, W):
    scal = {"s": ("seeded", -1000, 1000), "t": 7} if "int s" in src else None
    g, o = both(src, G, W, {"A": ("seeded", 0, 16)} | ({"B": ("seeded", 0, 16)} if "B[" in src else {}),
                scal, seed0=9, n=3)
    U.assert_same(g, o, src)


def test_int32_corners_final_memory():
    src = """kernel ar(global int out[24], int m) {
      out[0] := 0 - 7 / 2; out[1] := (0 - 7) / 2; out[2] := (0 - 7) % 2; out[3] := (0 - 7) mod 2;
      out[4] := 7 mod (0 - 2); out[5] := m / (0 - 1); out[6] := m % (0 - 1); out[7] := 1 << 33;
      out[8] := (0 - 8) >> 1; out[9] := (0 - 1) >> 40; out[10] := m - 1; out[11] := 2147483647 + 1;
      out[12] := 65536 * 65536; out[13] := 0 - m; out[14] := m mod 3; out[15] := (0 - 7) mod (0 - 2);
      out[16] := (3 < 4) + (4 <= 4) * 2 + (5 == 5) * 4 + !0 * 8 + (0 && 1) * 16 + (0 || 2) * 32;
      out[17] := ~5; out[18] := min(0 - 3, 2) * 10 + max(0 - 3, 2); out[19] := (12 ^ 10) + (12 | 3) * 100;
      out[20] := 4294967295; out[21] := (0 - 9) >> 2; out[22] := m >> 31; out[23] := 7 % (0 - 3); }"""
    import torch
    prog = B.Program(U.ctx(), src)
    prog.set_ndrange(1, 1)
    prog.bind({"out": torch.zeros(24, dtype=torch.int32, device="cuda")}, {"m": -(2 ** 31)})
    ws = torch.empty(prog.workspace_size(1), dtype=torch.uint8, device="cuda")
    fin = prog.read_final(0, "out", ws)
    U.ctx().sync()
    orc = O.check(src, 1, 1, arrays={"out": np.zeros(24, np.int32)}, scalars={"m": -(2 ** 31)}, final="out")
    assert np.array_equal(fin.cpu().numpy(), orc.final)


@pytest.mark.parametrize("jit", [False, True])
def test_mod_by_powers_of_two_final_memory(jit):
    """mod by a positive power of two takes the low bits; other divisors,
    negative ones and zero's neighbours take the division path.  Lanes mix
    both (divisor tid + 1), with negative dividends, and the corners of
    int32 (m = -2^31)."""
    src = """kernel md(global int out[72], int m, int s) {
      out[tid] := (s * tid - 77) mod (tid + 1);
      out[64] := m mod 65536; out[65] := m mod 1; out[66] := (0 - 1) mod 4096; out[67] := m mod 1073741824;
      out[68] := (m + 5) mod (0 - 4); out[69] := (0 - 4097) mod 4096; out[70] := 2147483647 mod 2;
      out[71] := (0 - 1) mod (m + 2147483647 + 1 + 8); }"""
    import torch
    prog = B.Program(U.ctx(), src)
    prog.set_ndrange(1, 64)
    prog.bind({"out": torch.zeros(72, dtype=torch.int32, device="cuda")}, {"m": -(2 ** 31), "s": -12345})
    if jit:
        prog.jit(True)
    ws = torch.empty(prog.workspace_size(1), dtype=torch.uint8, device="cuda")
    fin = prog.read_final(0, "out", ws)
    U.ctx().sync()
    orc = O.check(src, 1, 64, arrays={"out": np.zeros(72, np.int32)}, scalars={"m": -(2 ** 31), "s": -12345},
                  final="out")
    assert np.array_equal(fin.cpu().numpy(), orc.final)


# ---------------------------------------------------------------------------
# c2 templates
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("w", WL.c2_templates(), ids=lambda w: w.name)
def test_c2_templates(w):
    g, o = both(w.src, w.G, w.W, w.arrays, seed0=0, n=4)
    U.assert_same(g, o, w.name)


@pytest.mark.parametrize("tmpl", ["tree_reduce", "prefix_sum", "transpose"])
def test_c2_final_memory(tmpl):
    import torch
    w = getattr(WL, tmpl)(False)
    prog = B.Program(U.ctx(), w.src)
    prog.set_ndrange(w.G, w.W)
    x = np.random.default_rng(1).integers(-(2 ** 31), 2 ** 31, 65536, dtype=np.int64).astype(np.int32)
    out0 = np.random.default_rng(2).integers(-(2 ** 31), 2 ** 31, 65536, dtype=np.int64).astype(np.int32)
    prog.bind({"inp": torch.from_numpy(x).cuda(), "out": torch.from_numpy(out0).cuda()})
    ws = torch.empty(prog.workspace_size(1), dtype=torch.uint8, device="cuda")
    fin = prog.read_final(0, "out", ws).cpu().numpy()
    U.ctx().sync()
    orc = O.check(w.src, w.G, w.W, arrays={"inp": x, "out": out0}, final="out")
    assert np.array_equal(fin, orc.final)


# ---------------------------------------------------------------------------
# c3 random kernels and c4 large intervals
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pseed", list(range(0, 24)) + [100, 101, 137, 250])
def test_c3_kernels(pseed):
    w = WL.c3_kernel(pseed)
    g, o = both(w.src, w.G, w.W, w.arrays, seed0=1 << 40, n=2)
    U.assert_same(g, o, w.name)


@pytest.mark.parametrize("groups,wg,iters", [(4, 64, 8), (8, 256, 16), (3, 1000, 4)])
def test_c4_scaled(groups, wg, iters):
    w = WL.c4_kernel(groups, wg, iters, log2_cells=14)
    g, o = both(w.src, w.G, w.W, w.arrays, w.scalars, seed0=3, n=3)
    U.assert_same(g, o, f"c4 {groups}x{wg}x{iters}")


def test_c4_full_size_one_seed():
    w = WL.c4_kernel()
    g, o = both(w.src, w.G, w.W, w.arrays, w.scalars, seed0=0, n=1, cap=1 << 21)
    U.assert_same(g, o, "c4 full")


# ---------------------------------------------------------------------------
# library mechanics
# ---------------------------------------------------------------------------
def test_determinism_and_passes():
    w = WL.c1_kernel(7)
    a = U.gpu_run(w.src, w.G, w.W, w.arrays, None, 0, 300)
    b = U.gpu_run(w.src, w.G, w.W, w.arrays, None, 0, 300)
    assert a[0].tobytes() == b[0].tobytes() and a[1].tobytes() == b[1].tobytes()
    # a workspace that fits only a few instances per pass gives the same bytes
    prog = B.Program(U.ctx(), w.src)
    prog.set_ndrange(w.G, w.W)
    small = prog.workspace_size(7)
    c = U.gpu_run(w.src, w.G, w.W, w.arrays, None, 0, 300, ws_limit=small)
    assert a[0].tobytes() == c[0].tobytes() and a[1].tobytes() == c[1].tobytes()


def test_record_overflow():
    w = WL.fig1(64, True)
    with pytest.raises(B.RcError) as ei:
        U.gpu_run(w.src, w.G, w.W, w.arrays, None, 0, 4, cap=100)
    assert ei.value.status == B.RC_E_OVERFLOW


def test_record_overflow_global_path():
    """More records than the capacity on the path of the log sort, the
    segmented check and the record gather (a program of several groups):
    the first cap records are the canonical ones, exactly the instances that
    lost records have flags bit 0 (the rest of every summary unchanged), the
    counter holds the full count, and the call reports the overflow."""
    # (seeds 0..2 have 198, 147 and 137 records by the oracle: a capacity of
    # half the total keeps instance 0 whole, cuts instance 1 and drops 2)
    w = WL.c4_kernel(8, 64, 8, log2_cells=12)
    full_recs, full_sums = U.gpu_run(w.src, w.G, w.W, w.arrays, w.scalars, 0, 3)
    n = len(full_recs)
    assert n >= 4 and len(set(full_recs["instance"].tolist())) == 3
    cap = n // 2
    ctx = U.ctx()
    p = B.Program(ctx, w.src)
    p.set_ndrange(w.G, w.W)
    p.bind(w.arrays, w.scalars)
    buf = B.Buffers(p, 3, cap=cap, ws_limit=4 << 30)
    p.check_async(0, 3, buf.ws, buf.records, buf.n_records, buf.summaries)
    with pytest.raises(B.RcError) as ei:
        ctx.sync()
    assert ei.value.status == B.RC_E_OVERFLOW
    assert int(buf.n_records.item()) == n
    recs = B.records_to_numpy(buf.records, cap)
    sums = B.summaries_to_numpy(buf.summaries, 3)
    p.close()
    assert recs.tobytes() == full_recs[:cap].tobytes()
    lost = set(full_recs["instance"][cap:].tolist())
    assert lost == {1, 2}
    for j in range(3):
        assert (int(sums[j]["flags"]) & 1) == (1 if j in lost else 0), j
        a, b = sums[j].copy(), full_sums[j].copy()
        a["flags"] = b["flags"] = 0
        assert a.tobytes() == b.tobytes(), j


def test_api_errors():
    ctx = U.ctx()
    with pytest.raises(B.RcError) as ei:
        B.Program(ctx, "kernel k(global int A[4]) { v := 1; }")
    assert ei.value.status == B.RC_E_PARSE
    p = B.Program(ctx, "kernel k(global int A[4]) { A[0] := 1; }")
    with pytest.raises(B.RcError) as ei:
        p.set_ndrange(1, 2000)
    assert ei.value.status == B.RC_E_LIMIT
    with pytest.raises(B.RcError) as ei:
        p.workspace_size(1)
    assert ei.value.status == B.RC_E_STATE
    p.set_ndrange(1, 4)
    import torch
    ws = torch.empty(p.workspace_size(1), dtype=torch.uint8, device="cuda")
    rec = torch.empty(400, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    summ = torch.empty(40, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.RcError) as ei:
        p.check_async(0, 1, ws, rec, cnt, summ)     # A is unbound
    assert ei.value.status == B.RC_E_STATE


# ---------------------------------------------------------------------------
# the LDS interval log: results do not depend on its size (small logs spill
# intervals to the global pass)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("entries", [2, 64, 1024])
@pytest.mark.parametrize("case", ["c1", "fig3", "tree", "transpose_race", "c3_1", "c3_5"])
def test_lds_log_size_invariance(case, entries):
    w = {"c1": lambda: WL.c1_kernel(1), "fig3": lambda: WL.fig3(64), "tree": lambda: WL.tree_reduce(True),
         "transpose_race": lambda: WL.transpose(True), "c3_1": lambda: WL.c3_kernel(1),
         "c3_5": lambda: WL.c3_kernel(5)}[case]()
    g = U.gpu_run(w.src, w.G, w.W, w.arrays, w.scalars, 0, 3, lds_log_entries=entries)
    o = U.oracle_run(w.src, w.G, w.W, w.arrays, w.scalars, 0, 3)
    U.assert_same(g, o, f"{case} lds_log_entries={entries}")


# ---------------------------------------------------------------------------
# batches of different programs in one call; chunked calls replay a graph
# ---------------------------------------------------------------------------
def _batch(programs_and_seeds, ws_bytes=None, profile=False):
    import torch
    ctx = U.ctx()
    progs = {}
    plist, seeds = [], []
    for w, seed in programs_and_seeds:
        if w.name not in progs:
            p = B.Program(ctx, w.src)
            p.set_ndrange(w.G, w.W)
            p.bind(w.arrays, w.scalars)
            progs[w.name] = p
        plist.append(progs[w.name])
        seeds.append(seed)
    n = len(plist)
    need = max(p.workspace_size(1) for p in progs.values()) * 2 if ws_bytes is None else ws_bytes
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    cap = 1 << 20
    rec = torch.empty(cap * B.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    summ = torch.empty(n * B.SUMMARY_BYTES, dtype=torch.uint8, device="cuda")
    if profile:
        ctx.profile(True)
    ctx.batch_check_async(plist, seeds, ws, rec, cnt, summ)
    ctx.sync()
    if profile:
        ctx.profile_read()
        ctx.profile(False)
    k = int(cnt.item())
    return B.records_to_numpy(rec, k), B.summaries_to_numpy(summ, n)


def _oracle_batch(programs_and_seeds):
    recs, summs = [], []
    cache = {}
    for i, (w, seed) in enumerate(programs_and_seeds):
        if w.name not in cache:
            cache[w.name] = O.Program(w.src)
        r = cache[w.name].run(w.G, w.W, arrays=w.arrays, scalars=w.scalars, seed=seed, instance=i)
        recs.append(r.records)
        summs.append(r.summary)
    return np.concatenate(recs), np.array(summs, dtype=O.SUMMARY_DTYPE)


def test_batch_of_different_programs():
    ws = [WL.c3_kernel(s) for s in range(6)] + [WL.fig3(40), WL.c1_kernel(3), WL.tree_reduce(True)]
    items = [(ws[(i * 7) % len(ws)], 1000 + i) for i in range(27)]
    g = _batch(items)
    o = _oracle_batch(items)
    U.assert_same(g, o, "batch")


def test_chunked_batch_graph_replay_matches_eager():
    items = [(WL.c3_kernel(s % 4), s) for s in range(40)]
    import torch  # noqa: F401
    progs_ws = None
    # a small workspace forces many chunks: the graph is replayed once per chunk
    small = max(B.Program(U.ctx(), w.src).workspace_size(1) if False else 0 for w, _ in items[:1])
    g1 = _batch(items, ws_bytes=None)
    ctx = U.ctx()
    p = B.Program(ctx, items[0][0].src)
    p.set_ndrange(items[0][0].G, items[0][0].W)
    one = p.workspace_size(3)
    g2 = _batch(items, ws_bytes=one * 3)            # graphs (several chunks)
    g3 = _batch(items, ws_bytes=one * 3, profile=True)  # eager launches
    o = _oracle_batch(items)
    U.assert_same(g1, o, "one chunk")
    U.assert_same(g2, o, "graph replay")
    U.assert_same(g3, o, "eager chunks")
    del progs_ws, small


def test_workspace_overwritten_between_calls():
    """A workspace whose bytes changed since the last call (new buffer at a
    reused address, or scribbled on) is detected and its overlay pool cleared."""
    import torch
    w = WL.tree_reduce(True)
    ctx = U.ctx()
    p = B.Program(ctx, w.src)
    p.set_ndrange(w.G, w.W)
    p.bind(w.arrays, w.scalars)
    buf = B.Buffers(p, 3, cap=1 << 16)
    o = U.oracle_run(w.src, w.G, w.W, w.arrays, w.scalars, 0, 3)
    for trial in range(3):
        if trial:
            buf.ws.random_(0, 255)   # every byte, header included
        p.check_async(0, 3, buf.ws, buf.records, buf.n_records, buf.summaries)
        ctx.sync()
        n = int(buf.n_records.item())
        g = (B.records_to_numpy(buf.records, n), B.summaries_to_numpy(buf.summaries, 3))
        U.assert_same(g, o, f"trial {trial}")
    del torch


# ---------------------------------------------------------------------------
# autotuner: every candidate must give the same report; the cache is reused
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["c3_2", "tree_race", "c4_small"])
def test_autotune_invariance_and_cache(case, tmp_path):
    import json
    import torch
    w = {"c3_2": lambda: WL.c3_kernel(2), "tree_race": lambda: WL.tree_reduce(True),
         "c4_small": lambda: WL.c4_kernel(4, 256, 8, 14)}[case]()
    ctx = U.ctx()
    p = B.Program(ctx, w.src)
    p.set_ndrange(w.G, w.W)
    p.bind(w.arrays, w.scalars)
    ws = torch.empty(p.workspace_size(4), dtype=torch.uint8, device="cuda")
    cache = str(tmp_path / "tune.json")
    chosen = p.autotune(0, 4, ws, cache)
    entries = json.load(open(cache))
    assert len(entries) == 1 and list(entries.values())[0]["radix_bits"] == chosen["radix_bits"]
    again = p.autotune(0, 4, ws, cache)          # from the cache
    assert again == chosen
    buf = B.Buffers(p, 4, cap=1 << 20)
    p.check_async(0, 4, buf.ws, buf.records, buf.n_records, buf.summaries)
    ctx.sync()
    n = int(buf.n_records.item())
    g = (B.records_to_numpy(buf.records, n), B.summaries_to_numpy(buf.summaries, 4))
    U.assert_same(g, U.oracle_run(w.src, w.G, w.W, w.arrays, w.scalars, 0, 4), f"{case} tuned {chosen}")


def test_many_registers_interpreted_from_lds():
    """A program with more private variables than the VGPR register file
    holds runs on the interpreter that keeps them in LDS."""
    names = [f"r{i}" for i in range(20)]
    body = "\n".join(f"  {n} := tid * {i + 1} + {i};" for i, n in enumerate(names))
    body += "\n  " + "\n  ".join(f"x[({n}) mod 512] := {n};" for n in names[::3])
    body += "\n  barrier;\n  r0 := x[(tid + 1) mod 512];\n  y[tid mod 64] := r0 + r19;"
    src = f"kernel many(global int x[512], global int y[64]) {{\n  int {', '.join(names)};\n{body}\n}}\n"
    for G, W in [(1, 64), (2, 100), (3, 256)]:
        g, o = both(src, G, W, {"x": ("seeded", 0, 16), "y": ("seeded", 0, 16)}, seed0=3, n=3)
        U.assert_same(g, o, f"many registers G={G} W={W}")


@pytest.mark.parametrize("jit", [False, True])
@pytest.mark.parametrize("limit,G,W", [(5000, 1, 64), (5000, 3, 130), (10099, 2, 64), (10100, 2, 64)])
def test_step_limit(limit, G, W, jit):
    """A work-group that would start more loop iterations than the limit
    stops there with STEP_LIMIT (reading R13); interpreter and per-program
    kernel against the oracle, with the limit set through the tuning."""
    from tests.test_oracle_pins import STEP_SRC
    src = STEP_SRC.replace("x[64]", "x[512]")
    arrays = {"x": ("seeded", 0, 4)}
    p = B.Program(U.ctx(), src)
    p.set_ndrange(G, W)
    p.bind(arrays, None)
    p.set_tuning(step_limit=limit)
    if jit:
        p.jit(True)
    buf = B.Buffers(p, 3, 1 << 16)
    p.check_async(4, 3, buf.ws, buf.records, buf.n_records, buf.summaries)
    U.ctx().sync()
    n = int(buf.n_records.item())
    g = (B.records_to_numpy(buf.records, n), B.summaries_to_numpy(buf.summaries, 3))
    o = [O.Program(src).run(G, W, arrays=arrays, seed=4 + j, instance=j, step_limit=limit) for j in range(3)]
    orc = (np.concatenate([x.records for x in o]), np.array([x.summary for x in o], dtype=O.SUMMARY_DTYPE))
    U.assert_same(g, orc, f"limit={limit} G={G} W={W} jit={jit}")
    assert (g[1]["status"] == (6 if limit < 10100 else 0)).all()
