"""GPU parity of the per-program kernels (rc_prog_jit): the same oracle
comparisons as the interpreter's, with each program translated to its own
kernel.  Every program is compiled once per work-group width class."""
import random

import numpy as np
import pytest

from paper_1308_3203_amd import binding as B
from paper_1308_3203_amd import workloads as WL
from tests import gpu_util as U
from tests import interleave as IL
from tests.test_gpu_parity import CONTROL, FAULTS

pytestmark = pytest.mark.gpu


def both(src, G, W, arrays=None, scalars=None, seed0=0, n=1, **kw):
    dev_arrays = U.host_arrays_to_device(arrays)
    g = U.gpu_run(src, G, W, dev_arrays, scalars, seed0, n, jit=True, **kw)
    o = U.oracle_run(src, G, W, arrays, scalars, seed0, n)
    return g, o


@pytest.mark.parametrize("n,one_based", [(64, True), (65, True), (200, False)])
def test_fig1(n, one_based):
    w = WL.fig1(n, one_based)
    U.assert_same(*both(w.src, w.G, w.W, w.arrays, n=3), w.name)


def test_fig3():
    w = WL.fig3(100)
    U.assert_same(*both(w.src, w.G, w.W, w.arrays, seed0=5, n=8), w.name)


def test_c1_all_seeds():
    w = WL.c1_kernel(1)
    U.assert_same(*both(w.src, w.G, w.W, w.arrays, seed0=0, n=1000), "c1")


@pytest.mark.parametrize("G,W", [(1, 7), (1, 65), (3, 130), (2, 300), (1, 900), (4, 1024)])
def test_random_shapes(G, W):
    r = random.Random(7 * W + G)
    prog, arrays, vars_ = IL.random_program(r, r.randint(6, 12), r.choice([4, 16, 64]), r.randint(1, 3))
    src = IL.render(prog, arrays, vars_)
    U.assert_same(*both(src, G, W, {a: ("seeded", 0, 4) for a in arrays}, seed0=3, n=4), f"G={G} W={W}\n{src}")


@pytest.mark.parametrize("src", FAULTS)
def test_faults(src):
    for G, W in [(1, 8), (4, 130)]:
        U.assert_same(*both(src, G, W, {"A": ("seeded", 0, 16)}, n=2), f"{src} G={G} W={W}")


@pytest.mark.parametrize("src", CONTROL)
def test_control_flow(src):
    scal = {"s": ("seeded", -1000, 1000), "t": 7} if "int s" in src else None
    arrays = {"A": ("seeded", 0, 16)} | ({"B": ("seeded", 0, 16)} if "B[" in src else {})
    for G, W in [(1, 64), (3, 257)]:
        U.assert_same(*both(src, G, W, arrays, scal, seed0=9, n=3), f"{src} G={G} W={W}")


@pytest.mark.parametrize("w", WL.c2_templates(), ids=lambda w: w.name)
def test_c2_templates(w):
    U.assert_same(*both(w.src, w.G, w.W, w.arrays, w.scalars, seed0=11, n=3), w.name)


def test_c4_scaled():
    w = WL.c4_kernel(groups=4, wgsize=256, iters=8, log2_cells=12)
    U.assert_same(*both(w.src, w.G, w.W, w.arrays, w.scalars, seed0=2, n=2), w.name)


def test_jit_and_interpreter_agree_across_width_change():
    """A program re-shaped into another width class is recompiled; results
    match the interpreter's byte for byte."""
    w = WL.c1_kernel(3)
    p = B.Program(U.ctx(), w.src)
    p.bind(w.arrays, w.scalars)
    for W in (64, 200):
        p.set_ndrange(1, W)
        outs = []
        for jit in (False, True):
            p.jit(jit)
            buf = B.Buffers(p, 16, 1 << 16)
            p.check_async(0, 16, buf.ws, buf.records, buf.n_records, buf.summaries)
            U.ctx().sync()
            n = int(buf.n_records.item())
            outs.append((B.records_to_numpy(buf.records, n).tobytes(), B.summaries_to_numpy(buf.summaries, 16).tobytes()))
        assert outs[0] == outs[1], W


def test_jit_follows_shape_and_tuning():
    """The per-program kernel is specialised for the launch shape: a new
    number of groups or LDS log size compiles another kernel (or takes the
    one compiled for that shape before), and every result stays the
    oracle's."""
    w = [x for x in WL.c2_templates() if x.name == "tree_reduce_race"][0]
    p = B.Program(U.ctx(), w.src)
    p.bind(w.arrays, w.scalars)
    p.set_ndrange(2, w.W)
    p.jit(True)
    for G, T in [(2, 0), (5, 0), (5, 64), (2, 0)]:
        p.set_ndrange(G, w.W)
        p.set_tuning(lds_log_entries=T)
        buf = B.Buffers(p, 3, 1 << 16)
        p.check_async(7, 3, buf.ws, buf.records, buf.n_records, buf.summaries)
        U.ctx().sync()
        n = int(buf.n_records.item())
        g = (B.records_to_numpy(buf.records, n), B.summaries_to_numpy(buf.summaries, 3))
        U.assert_same(g, U.oracle_run(w.src, G, w.W, w.arrays, w.scalars, 7, 3), f"G={G} T={T}")


ELIDE = [
    # a load at the loop's start after a store at its end (the back edge)
    "  L[lid] := lid;\n  barrier;\n  for k in 0..4 {\n    v := L[(lid + 64) % 256];\n    L[lid] := v + k;\n  }\n",
    # a store after a load of the same array, in straight-line code
    "  L[lid] := lid;\n  barrier;\n  v := L[(lid + 64) % 256];\n  L[lid] := v;\n  v := L[(lid + 128) % 256];\n"
    "  L[lid] := v + 1;\n",
    # the same across a branch (its vote synchronises the group)
    "  L[lid] := lid;\n  barrier;\n  for k in 0..3 {\n    if (lid < 128) {\n      v := L[lid + 128];\n    }\n"
    "    L[lid] := v + 1;\n  }\n",
    # stores only between synchronisations, then loads only
    "  for k in 0..4 {\n    L[(lid * 3 + k) % 256] := lid + k;\n  }\n  barrier;\n  for k in 0..4 {\n"
    "    v := L[(lid + k * 64) % 256];\n    A[lid] := v;\n  }\n",
]


@pytest.mark.parametrize("body", ELIDE)
def test_elided_group_steps(body):
    """Never-faulting programs whose intervals fit LDS run with most group
    steps elided; the steps kept for conflicting accesses (including across
    a loop's back edge) keep the results the oracle's, over four waves."""
    src = f"kernel t(global int A[256]) {{\n  local int L[256];\n  int v, k;\n{body}}}\n"
    assert B.owned_arrays(src, 1, 256, with_faults=True)[1]
    U.assert_same(*both(src, 1, 256, {"A": ("seeded", 0, 8)}, n=20), src)
    U.assert_same(*both(src, 2, 256, {"A": ("seeded", 0, 8)}, seed0=40, n=8), src)


def quiet_step_src(W):
    """A global array shared between work-items (not owned) next to a local
    array that is race-free in interval 0 and racy in interval 1: the load of
    L in interval 0 keeps its group step only in logged intervals, so it must
    not stand in for the synchronisation the following load of A needs."""
    return (f"kernel q(global int A[{W}], global int Bo[{W}]) {{\n  local int L[{W}];\n  int x, y;\n"
            f"  A[(lid + 1) % {W}] := lid;\n  L[lid] := lid;\n  x := L[lid];\n  y := A[lid];\n"
            f"  Bo[lid] := y + x;\n  barrier;\n  L[(lid + 1) % {W}] := x;\n  x := L[lid];\n}}\n")


@pytest.mark.parametrize("W", [128, 256])
def test_elided_step_after_quiet_local_access(W):
    """Regression: a shared global array logged in LDS, read after a group
    step on a local array that the runtime skips in a quiet interval.  The
    per-program kernel must read the other wave's store (final memory and
    records equal the oracle's)."""
    import torch
    from oracle import oracle as O
    src = quiet_step_src(W)
    owned, nofault = B.owned_arrays(src, 1, W, with_faults=True)
    assert nofault and owned == [False, True, False]
    assert B.log_intervals(src, 1, W) == (0b10, False)
    arrays = {"A": ("seeded", 0, 1000), "Bo": ("seeded", 0, 8)}
    U.assert_same(*both(src, 1, W, arrays, seed0=1, n=6), src)
    p = B.Program(U.ctx(), src)
    p.set_ndrange(1, W)
    p.bind(arrays, None)
    p.jit(True)
    ws = torch.empty(p.workspace_size(1), dtype=torch.uint8, device="cuda")
    for seed in (0, 3):
        for name in ("A", "Bo"):
            fin = p.read_final(seed, name, ws).cpu().numpy()
            U.ctx().sync()
            orc = O.check(src, 1, W, arrays=arrays, seed=seed, final=name)
            assert np.array_equal(fin, orc.final), (W, seed, name)


@pytest.mark.parametrize("G,W", [(2, 128), (4, 256)])
@pytest.mark.parametrize("jit", [True, False])
def test_elided_step_after_quiet_local_access_groups(G, W, jit):
    """The same program with several groups: the shared global array is
    logged globally.  The per-program kernel keeps every step on it; the
    interpreter's elided steps do not, so the skipped local step must not
    settle it there either.  Records and summaries equal the oracle's."""
    src = quiet_step_src(W)
    owned, nofault = B.owned_arrays(src, G, W, with_faults=True)
    assert nofault and owned == [False, False, False]
    assert B.log_intervals(src, G, W) == (0b10, False)
    arrays = {"A": ("seeded", 0, 1000), "Bo": ("seeded", 0, 8)}
    g = U.gpu_run(src, G, W, arrays, None, 1, 6, jit=jit)
    U.assert_same(g, U.oracle_run(src, G, W, arrays, None, 1, 6), f"{src} G={G} jit={jit}")


@pytest.mark.parametrize("w", WL.c2_templates(), ids=lambda w: w.name)
def test_proofs_off_same_reports(w):
    """With the static proofs turned off every written array is logged and
    every memory statement takes its group step; the reports stay the
    oracle's, for the per-program kernel and the interpreter."""
    o = U.oracle_run(w.src, w.G, w.W, w.arrays, w.scalars, 21, 3)
    for jit in (True, False):
        p = B.Program(U.ctx(), w.src)
        p.set_ndrange(w.G, w.W)
        p.bind(w.arrays, w.scalars)
        p.set_tuning(proofs_off=True)
        assert not any(p.owned(a[0]) for a in p.arrays)
        if jit:
            p.jit(True)
        buf = B.Buffers(p, 3, 1 << 18)
        p.check_async(21, 3, buf.ws, buf.records, buf.n_records, buf.summaries)
        U.ctx().sync()
        n = int(buf.n_records.item())
        U.assert_same((B.records_to_numpy(buf.records, n), B.summaries_to_numpy(buf.summaries, 3)), o,
                      f"{w.name} jit={jit}")
