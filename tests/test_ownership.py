"""The owned-array proofs (host logic of the library, no device).

An array is owned when no two work-items can touch a common cell of it; the
library then skips logging its accesses.  Two proofs: affine index forms
(which also give the lane-major overlay placement), and, when no index or
branch depends on loaded values or scalars, enumeration of every work-item's
cells.  Hand cases pin what they accept and reject, including int32
wrap-around, loop-carried variables and branch joins; a randomised check
against the oracle (which logs every access) confirms that no owned array
ever carries a record."""
import random

import pytest

from oracle import oracle as O
from paper_1308_3203_amd import binding as B
from paper_1308_3203_amd import workloads as WL


def owned(body, G, W, decl="global int x[4096], global int y[4096]", vars_="int v, w, k, j"):
    src = f"kernel t({decl}) {{\n  {vars_};\n{body}\n}}\n"
    return B.owned_arrays(src, G, W)


CASES = [
    # (body, G, W, expected ownership of x, y)
    ("  x[tid] := 1;", 4, 64, [True, True]),
    ("  x[tid] := 1;\n  v := x[tid + 1];", 4, 64, [False, True]),
    ("  x[2 * tid] := 1;\n  x[2 * tid + 1] := 2;", 4, 64, [True, True]),
    ("  x[2 * tid] := 1;\n  x[2 * tid + 2] := 2;", 4, 64, [False, True]),
    ("  x[lid] := 1;", 2, 64, [False, True]),
    ("  x[lid] := 1;", 1, 64, [True, True]),
    ("  x[gid] := 1;", 8, 1, [True, True]),
    ("  x[gid * wgsize + lid] := 1;", 8, 32, [True, True]),
    ("  x[gid * 64 + lid] := 1;", 8, 32, [True, True]),      # not affine in tid; enumerated
    ("  x[gid * 16 + lid] := 1;", 8, 32, [False, True]),
    ("  x[1000 - tid] := 1;", 4, 64, [True, True]),
    ("  x[tid << 2] := 1;\n  x[(tid << 2) + 3] := 1;", 4, 64, [True, True]),
    ("  for k in 0..4 {\n    x[tid * 4 + k] := k;\n  }", 4, 64, [True, True]),
    ("  for k in 0..5 {\n    x[tid * 4 + k] := k;\n  }", 4, 64, [False, True]),
    ("  for k in 0..4 {\n    for j in 0..4 {\n      x[tid * 16 + k * 4 + j] := 1;\n    }\n  }", 2, 32,
     [True, True]),
    ("  for k in 0..4 {\n    for j in 0..4 {\n      x[tid * 16 + k * 4 + j * 2] := 1;\n    }\n  }", 2, 32,
     [False, True]),
    ("  v := tid * 4;\n  for k in 0..4 {\n    x[v + k] := 1;\n  }", 4, 64, [True, True]),
    # a loop-carried index: tid, tid + 1, tid + 2 overlap between work-items
    ("  v := tid;\n  for k in 0..3 {\n    x[v] := 1;\n    v := v + 1;\n  }", 4, 64, [False, True]),
    # branches that assign different forms join to unknown
    ("  if (tid < 5) {\n    v := tid;\n  } else {\n    v := tid - 1;\n  }\n  x[v] := 1;", 4, 64,
     [False, True]),
    ("  if (tid < 5) {\n    v := tid * 2;\n  } else {\n    v := tid * 2;\n  }\n  x[v] := 1;", 4, 64,
     [True, True]),
    # 4 * 2^30 wraps to 0 in int32: work-items 0 and 4 share cell 0
    ("  x[tid * 1073741824] := 1;", 1, 8, [False, True]),
    ("  x[tid mod 64] := 1;", 1, 64, [True, True]),
    ("  x[tid mod 32] := 1;", 1, 64, [False, True]),
    ("  if (lid == 0) {\n    x[gid] := 1;\n  }", 8, 64, [True, True]),
    ("  if (lid < 2) {\n    x[gid] := 1;\n  }", 8, 64, [False, True]),
    ("  x[(lid / 8) * 64 + (lid % 8) + gid * 8] := 1;", 8, 64, [True, True]),
    ("  v := y[tid];\n  x[v] := 1;", 4, 64, [False, True]),
    ("  v := x[0];\n  x[tid] := v;", 4, 64, [False, True]),
    ("  x[tid] := 1;\n  barrier;\n  v := x[tid];\n  y[tid] := v;", 4, 64, [True, True]),
]


@pytest.mark.parametrize("body,G,W,expect", CASES)
def test_owned_cases(body, G, W, expect):
    assert owned(body, G, W) == expect


def test_data_dependent_paths_are_not_enumerated():
    # a branch on a loaded value: the accessed cells depend on the inputs
    body = "  v := y[tid];\n  if (v < 3) {\n    x[tid] := 1;\n  } else {\n    x[tid + 1] := 1;\n  }"
    assert owned(body, 2, 32) == [False, True]
    # the affine proof is path-insensitive and still owns x when both paths agree
    body = "  v := y[tid];\n  if (v < 3) {\n    x[tid] := 1;\n  } else {\n    x[tid] := 2;\n  }"
    assert owned(body, 2, 32) == [True, True]


def test_scalar_in_index_is_unknown():
    src = "kernel t(global int x[4096], int s) {\n  x[tid + s] := 1;\n}\n"
    assert B.owned_arrays(src, 4, 64) == [False]
    src = "kernel t(global int x[4096], int s) {\n  x[tid] := s;\n}\n"
    assert B.owned_arrays(src, 4, 64) == [True]


def test_one_work_item_owns_everything():
    assert owned("  v := x[7];\n  x[v] := 1;\n  y[0] := 2;", 1, 1) == [True, True]


def test_local_arrays():
    src = ("kernel t(global int x[4096]) {\n  local int l[256];\n  int v;\n  l[lid] := 1;\n  barrier;\n"
           "  v := l[lid];\n  x[tid] := v;\n}\n")
    assert B.owned_arrays(src, 1, 64) == [True, True]
    # each group has its own copy of a local array
    assert B.owned_arrays(src, 4, 64) == [True, True]
    src2 = src.replace("v := l[lid];", "v := l[lid + 1];")
    assert B.owned_arrays(src2, 1, 64) == [True, False]


def test_c2_templates():
    got = {w.name: B.owned_arrays(w.src, w.G, w.W) for w in WL.c2_templates()}
    # prefix sum: each work-item scans its own 16 cells of inp and out
    assert got["prefix_sum"] == [True, True, False]
    assert got["prefix_sum_race"] == [True, True, False]
    # out[gid] written by lid 0 only, and the transpose's div / mod index:
    # neither is affine in tid; both are enumerated
    assert got["tree_reduce"][1:] == [True, False]
    assert got["transpose"][1:] == [True, False]
    assert got["transpose_race"][1:] == [True, False]


def test_errors():
    with pytest.raises(B.RcError):
        B.owned_arrays("kernel t(global int x[4]) { x[tid] := ; }", 1, 4)
    with pytest.raises(B.RcError):
        B.owned_arrays("kernel t(global int x[4]) { x[tid] := 1; }", 1, 2000)


def _random_affine_program(r: random.Random):
    """Affine indices over tid, lid, gid, loop counters and variables, with
    branches and loop-carried updates; cells stay small so collisions are
    common when the proof does not hold."""
    def atom(loops):
        k = r.random()
        if k < 0.3:
            return r.choice(["tid", "lid", "gid"])
        if k < 0.5 and loops:
            return r.choice(loops)
        if k < 0.75:
            return r.choice(["v", "w"])
        return str(r.randint(0, 8))

    def expr(loops, d=0):
        if d >= 2 or r.random() < 0.4:
            return atom(loops)
        op = r.choice(["+", "-", "*", "<<"])
        if op == "*":
            return f"({expr(loops, d + 1)} * {r.randint(-3, 4)})"
        if op == "<<":
            return f"({expr(loops, d + 1)} << {r.randint(0, 3)})"
        return f"({expr(loops, d + 1)} {op} {expr(loops, d + 1)})"

    def stmts(n, loops, depth):
        out = []
        for _ in range(n):
            k = r.random()
            if k < 0.3:
                out.append(f"{r.choice(['v', 'w'])} := {expr(loops)};")
            elif k < 0.6:
                out.append(f"x[{expr(loops)}] := {expr(loops)};")
            elif k < 0.75:
                out.append(f"{r.choice(['v', 'w'])} := x[{expr(loops)}];")
            elif k < 0.85 and depth < 2:
                body = " ".join(stmts(r.randint(1, 3), loops, depth + 1))
                els = " ".join(stmts(r.randint(0, 2), loops, depth + 1))
                out.append(f"if (tid < {r.randint(0, 40)}) {{ {body} }} else {{ {els} }}")
            elif depth < 2:
                lv = ["k", "j"][len(loops)] if len(loops) < 2 else None
                if lv is None:
                    continue
                body = " ".join(stmts(r.randint(1, 3), loops + [lv], depth + 1))
                out.append(f"for {lv} in 0..{r.randint(1, 4)} {{ {body} }}")
        return out

    # a few templates that the proof accepts, mixed with random statements
    stride = r.choice([1, 2, 3, 4])
    own = [f"x[tid * {stride} + {o}] := {expr([])};" for o in range(r.randint(1, stride))]
    body = own + stmts(r.randint(1, 6), [], 0) if r.random() < 0.5 else own
    return ("kernel t(global int x[256]) {\n  int v, w, k, j;\n  " + "\n  ".join(body) + "\n}\n")


def test_owned_arrays_never_carry_records():
    r = random.Random(20240611)
    n_owned = 0
    for case in range(300):
        src = _random_affine_program(r)
        G, W = r.choice([(1, 8), (2, 8), (4, 4), (3, 16)])
        own = B.owned_arrays(src, G, W)
        res = O.Program(src).run(G, W, arrays={"x": ("seeded", 0, 4)}, seed=case)
        if own[0]:
            n_owned += 1
            assert not any(int(rec["array"]) == 0 for rec in res.records), (src, G, W)
    assert n_owned >= 50


FAULT_CASES = [
    # (body, G, W, never faults)
    ("  x[tid] := 1;", 4, 64, True),
    ("  x[tid + 4000] := 1;", 4, 64, False),                  # tid >= 96 is out of bounds
    ("  v := tid / 3;\n  x[v] := 1;", 4, 64, True),
    ("  v := 100 / lid;\n  x[tid] := v;", 4, 64, False),        # lid 0 divides by zero
    ("  v := y[tid];\n  w := 7 mod v;\n  x[tid] := w;", 4, 64, False),   # divisor from the inputs
    ("  assert(tid >= 0);\n  x[tid] := 1;", 4, 64, True),
    ("  assert(lid < 10);\n  x[tid] := 1;", 4, 64, False),
    ("  if (lid < 5) {\n    barrier;\n  }\n  x[tid] := 1;", 4, 64, False),   # part of a group at a barrier
    ("  if (gid < 1) {\n    barrier;\n  }\n  x[tid] := 1;", 4, 64, True),    # whole groups agree
    # a data-dependent path whose accesses are all in bounds (value ranges)
    ("  v := y[tid];\n  if (v < 3) {\n    x[tid] := 1;\n  }", 4, 64, True),
    ("  v := y[tid];\n  x[v mod 4096] := 1;", 4, 64, True),           # Euclidean mod: in [0, 4096)
    ("  v := y[tid];\n  x[v & 4095] := 1;", 4, 64, True),
    ("  v := y[tid];\n  x[v % 4096] := 1;", 4, 64, False),           # C99 remainder can be negative
    ("  v := y[tid];\n  x[v] := 1;", 4, 64, False),                  # a loaded index
    ("  v := y[tid];\n  x[(v mod 64) + tid] := 1;", 4, 64, True),     # at most 63 + 255
    ("  v := y[tid];\n  x[(v mod 64) * 64 + 4032] := 1;", 4, 64, False),   # up to 8064
    ("  v := y[tid];\n  if (v < 3) {\n    barrier;\n  }", 4, 64, False),   # a data-dependent barrier
    ("  v := y[tid];\n  w := 100 / (v mod 7 + 1);\n  x[tid] := w;", 4, 64, True),   # divisor in [1, 7]
    ("  v := y[tid];\n  w := 100 / (v mod 7);\n  x[tid] := w;", 4, 64, False),      # divisor may be 0
    ("  v := y[tid];\n  assert(v mod 5 < 5);\n  x[tid] := 1;", 4, 64, False),  # a condition is 0 or 1
    ("  for k in 0..16 {\n    v := y[(v + k) mod 4096];\n    x[v mod 4096] := k;\n  }", 1, 256, True),
    ("  for k in 0..4 {\n    barrier;\n    x[tid * 4 + k] := k;\n  }", 4, 64, True),
]


@pytest.mark.parametrize("body,G,W,expect", FAULT_CASES)
def test_never_faults(body, G, W, expect):
    src = f"kernel t(global int x[4096], global int y[4096]) {{\n  int v, w, k, j;\n{body}\n}}\n"
    assert B.owned_arrays(src, G, W, with_faults=True)[1] == expect


def test_never_faults_agrees_with_the_oracle():
    """Where the proof says a program cannot fault, the oracle's runs on
    several inputs end without a fault."""
    r = random.Random(99)
    proven = 0
    for case in range(200):
        src = _random_affine_program(r)
        G, W = r.choice([(1, 8), (2, 8), (4, 4)])
        _, nf = B.owned_arrays(src, G, W, with_faults=True)
        if not nf:
            continue
        proven += 1
        prog = O.Program(src)
        for seed in range(3):
            res = prog.run(G, W, arrays={"x": ("seeded", 0, 4)}, seed=seed)
            assert res.status == "OK", (src, G, W, res.status)
    assert proven >= 20


def race_free(body, G, W, decl="global int x[4096]", locs="local int l[512]"):
    src = f"kernel t({decl}) {{\n  {locs};\n  int v, w, k, j;\n{body}\n}}\n"
    return B.owned_arrays(src, G, W, race_free=True)


RACE_FREE_CASES = [
    # (body, G, W, local array race-free within every interval)
    ("  l[lid] := 1;\n  barrier;\n  v := l[lid + 1];\n  x[tid] := v;", 2, 64, True),
    ("  l[lid] := 1;\n  v := l[lid + 1];\n  x[tid] := v;", 2, 64, False),     # same interval
    ("  l[lid % 32] := lid;", 1, 64, False),                                     # two writers
    ("  l[lid] := 1;\n  barrier;\n  v := l[0];\n  x[tid] := v;", 1, 64, True),   # readers only
    ("  l[lid] := 1;\n  v := l[lid];\n  l[lid] := v + 1;", 1, 64, False),        # owned, not race-free
    ("  for k in 0..4 {\n    l[lid + 64 * (k % 2)] := k;\n    barrier;\n    v := l[(lid + 1) % 64 + 64 * (k % 2)];\n"
     "    barrier;\n  }", 1, 64, True),
    ("  for k in 0..4 {\n    l[lid + 64 * (k % 2)] := k;\n    v := l[(lid + 1) % 64 + 64 * ((k + 1) % 2)];\n"
     "    barrier;\n  }", 1, 64, True),                                          # double buffering
    ("  for k in 0..4 {\n    l[lid] := k;\n    v := l[(lid + 1) % 64];\n    barrier;\n  }", 1, 64, False),
    ("  assert(lid < 10);\n  l[lid] := 1;\n  barrier;\n  v := l[lid + 1];", 1, 64, False),   # may fault
    ("  v := x[tid];\n  l[v % 64] := 1;", 1, 64, False),                         # data-dependent index
]


@pytest.mark.parametrize("body,G,W,expect", RACE_FREE_CASES)
def test_race_free_locals(body, G, W, expect):
    assert race_free(body, G, W)[1] == expect


def test_c2_templates_race_free():
    got = {w.name: B.owned_arrays(w.src, w.G, w.W, race_free=True)[-1] for w in WL.c2_templates()}
    assert got == {"tree_reduce": True, "tree_reduce_race": False, "prefix_sum": True, "prefix_sum_race": False,
                   "transpose": True, "transpose_race": False}


def _random_local_program(r: random.Random):
    """Loads and stores of one local array with indices over lid, loop
    counters and constants, barriers, loops and branches on lid; small
    arrays, so conflicts are common when the proof does not hold."""
    def idx(loops):
        t = r.choice(["lid", f"(lid + {r.randint(1, 5)})", f"(lid * {r.randint(1, 3)})", f"{r.randint(0, 7)}",
                      f"(lid / {r.randint(2, 4)})"])
        if loops and r.random() < 0.4:
            t = f"({t} + {r.choice(loops)} * {r.randint(0, 16)})"
        return f"({t}) % 64"

    def stmts(n, loops, depth):
        out = []
        for _ in range(n):
            k = r.random()
            if k < 0.3:   # stores mostly to the work-item's own cell, so the proof often holds
                out.append(f"l[{idx(loops) if r.random() < 0.3 else 'lid % 64'}] := lid;")
            elif k < 0.6:
                out.append(f"v := l[{idx(loops)}];")
            elif k < 0.8:
                out.append("barrier;")
            elif k < 0.87 and depth < 2:
                out.append(f"if (lid < {r.randint(0, 40)}) {{ " + " ".join(
                    s for s in stmts(r.randint(1, 2), loops, depth + 1) if s != "barrier;") + " }")
            elif depth < 2 and len(loops) < 2:
                lv = ["k", "j"][len(loops)]
                out.append(f"for {lv} in 0..{r.randint(1, 3)} {{ " + " ".join(
                    stmts(r.randint(1, 3), loops + [lv], depth + 1)) + " }")
        return out

    body = stmts(r.randint(2, 7), [], 0)
    return ("kernel t(global int x[64]) {\n  local int l[64];\n  int v, w, k, j;\n  " + "\n  ".join(body) +
            "\n  x[lid] := v;\n}\n")


def test_race_free_locals_never_carry_records():
    """Where the proof says a local array is race-free in every interval,
    the oracle (which logs every access) reports no record on it."""
    r = random.Random(31337)
    n_rf = 0
    for case in range(1500):
        src = _random_local_program(r)
        G, W = r.choice([(1, 8), (2, 16), (1, 32), (3, 8)])
        try:
            rf = B.owned_arrays(src, G, W, race_free=True)
        except B.RcError:
            continue
        if not rf[1]:
            continue
        n_rf += 1
        res = O.Program(src).run(G, W, arrays={"x": ("seeded", 0, 4)}, seed=case)
        assert res.status == "OK", (src, G, W)
        assert not any(int(rec["array"]) == 1 for rec in res.records), (src, G, W)
    assert n_rf >= 60


def test_logged_intervals_of_the_racy_templates():
    """Only the intervals with a conflicting local-array cell keep their log
    (worked out by hand from the template texts): the transpose with the
    injected race lacks the barrier between reading tile 2 and writing tile
    3, so interval 5 holds both; the racy prefix sum writes one cell past its
    half into the cell work-item 0 reads, at every level (intervals 1-8); the
    racy tree reduction reads loc[s - 1] written by work-item s - 1 at the
    levels with s >= 2 (intervals 1-7)."""
    T = {w.name: w for w in WL.c2_templates()}
    got = {n: B.log_intervals(T[n].src, T[n].G, T[n].W) for n in ("transpose_race", "prefix_sum_race",
                                                                   "tree_reduce_race")}
    assert got == {"transpose_race": (1 << 5, False), "prefix_sum_race": (0x1FE, False),
                   "tree_reduce_race": (0xFE, False)}
    # not proven (a data-dependent index, a possible fault): every interval
    src = "kernel t(global int x[64]) {\n  local int l[64];\n  int v;\n  v := x[lid];\n  l[v % 64] := 1;\n}\n"
    assert B.log_intervals(src, 1, 64) == ((1 << 64) - 1, True)


def test_records_only_in_logged_intervals():
    """The oracle's records on the local array fall in intervals the proof
    keeps logged."""
    r = random.Random(4242)
    n_partial = 0
    for case in range(800):
        src = _random_local_program(r)
        G, W = r.choice([(1, 8), (2, 16), (1, 32), (3, 8)])
        try:
            mask, later = B.log_intervals(src, G, W)
        except B.RcError:
            continue
        if mask == (1 << 64) - 1 and later:
            continue
        n_partial += mask != 0
        res = O.Program(src).run(G, W, arrays={"x": ("seeded", 0, 4)}, seed=case)
        for rec in res.records:
            if int(rec["array"]) == 1:
                k = int(rec["interval"])
                assert (k < 64 and (mask >> k) & 1) or (k >= 64 and later), (src, G, W, k, hex(mask))
    assert n_partial >= 50


def test_quiet_interval_proof_of_shared_global_next_to_local():
    """The proof the per-program kernels' step elision relies on, for a
    shared global array beside a local array race-free in interval 0 only:
    A is not owned (work-item l writes A[l+1], l+1 reads it), Bo is owned,
    L is logged in interval 1 only, and the program cannot fault."""
    for W in (128, 256):
        src = (f"kernel q(global int A[{W}], global int Bo[{W}]) {{\n  local int L[{W}];\n  int x, y;\n"
               f"  A[(lid + 1) % {W}] := lid;\n  L[lid] := lid;\n  x := L[lid];\n  y := A[lid];\n"
               f"  Bo[lid] := y + x;\n  barrier;\n  L[(lid + 1) % {W}] := x;\n  x := L[lid];\n}}\n")
        owned, nofault = B.owned_arrays(src, 1, W, with_faults=True)
        assert nofault and owned == [False, True, False]
        assert B.log_intervals(src, 1, W) == (0b10, False)
        # the oracle: records on A in interval 0, on L in interval 1 only
        r = O.check(src, 1, W, arrays={"A": ("seeded", 0, 1000), "Bo": ("seeded", 0, 8)}, seed=1)
        got = {(int(x["interval"]), int(x["array"])) for x in r.records}
        assert got == {(0, 0), (1, 2)}


def test_never_faults_on_random_kernels_agrees_with_the_oracle():
    """The batched random kernels (indices of loaded values reduced mod the
    array size) are proven fault-free by their value ranges; the oracle's
    runs confirm it on every sampled input."""
    for pseed in range(0, 400, 20):
        w = WL.c3_kernel(pseed)
        assert B.owned_arrays(w.src, w.G, w.W, with_faults=True)[1], w.name
        prog = O.Program(w.src)
        for seed in (0, 7):
            r = prog.run(w.G, w.W, arrays=w.arrays, scalars=w.scalars, seed=seed)
            assert r.status == "OK", (w.name, seed)


def _random_fault_program(r: random.Random) -> str:
    """Random statements over every operator, loaded values, scalars,
    asserts, loops and barriers (some under branches)."""
    ops = ["+", "-", "*", "/", "%", "mod", "&", "|", "^", "<<", ">>", "<", "==", "&&"]

    def e(d=0):
        k = r.random()
        if d >= 2 or k < 0.3:
            return r.choice(["v", "w", "tid", "lid", "gid", "s", str(r.randint(-9, 300)), "k", "j"])
        if k < 0.4:
            return f"min({e(d + 1)}, {e(d + 1)})"
        if k < 0.5:
            return f"max({e(d + 1)}, {e(d + 1)})"
        return f"({e(d + 1)} {r.choice(ops)} {e(d + 1)})"

    def idx():
        k = r.random()
        if k < 0.4:
            return f"({e()}) mod {r.choice([64, 256, 300])}"
        if k < 0.6:
            return f"({e()}) & {r.choice([63, 255, 511])}"
        if k < 0.8:
            return f"tid + {r.randint(-2, 40)}"
        return e()

    def stmts(n, depth):
        out = []
        for _ in range(n):
            k = r.random()
            if k < 0.3:
                out.append(f"{r.choice(['v', 'w'])} := {e()};")
            elif k < 0.5:
                out.append(f"{r.choice(['v', 'w'])} := {r.choice(['x', 'y'])}[{idx()}];")
            elif k < 0.65:
                out.append(f"x[{idx()}] := {e()};")
            elif k < 0.7:
                out.append(f"assert({e()});")
            elif k < 0.78:
                out.append("barrier;")
            elif k < 0.9 and depth < 2:
                out.append(f"if ({e()} < {r.randint(0, 50)}) {{ " + " ".join(stmts(r.randint(1, 3), depth + 1)) + " }")
            elif depth < 2:
                lv = "kj"[depth]
                out.append(f"for {lv} in 0..{r.randint(1, 5)} {{ " + " ".join(stmts(r.randint(1, 3), depth + 1)) + " }")
        return out
    return ("kernel f(global int x[300], global int y[300], int s) {\n  int v, w, k, j;\n  "
            + "\n  ".join(stmts(r.randint(3, 8), 0)) + "\n}\n")


def test_range_proof_never_contradicts_the_oracle():
    """Fuzz: wherever the proofs say a program cannot fault, the oracle runs
    it without a fault on several inputs and launch shapes."""
    r = random.Random(4242)
    proven = 0
    for case in range(600):
        src = _random_fault_program(r)
        G, W = r.choice([(1, 64), (2, 32), (3, 7), (1, 100)])
        if not B.owned_arrays(src, G, W, with_faults=True)[1]:
            continue
        proven += 1
        prog = O.Program(src)
        for seed in range(3):
            res = prog.run(G, W, arrays={"x": ("seeded", -50, 400), "y": ("seeded", -(2 ** 31), 2 ** 31)},
                           scalars={"s": ("seeded", -(2 ** 31), 2 ** 31)}, seed=seed)
            assert res.status == "OK", (src, G, W, seed, res.status)
    assert proven >= 60


def test_never_faults_needs_the_iteration_limit():
    """A program that can start more loop iterations than the default limit
    (2^24) can stop with STEP_LIMIT, so it is not proven fault-free."""
    body = "  for k in 0..{} {{\n    for j in 0..4000 {{\n      v := v + 1;\n    }}\n  }}\n  x[tid] := v;"
    assert B.owned_arrays(f"kernel t(global int x[64]) {{\n  int v, k, j;\n{body.format(4000)}\n}}\n", 1, 64,
                          with_faults=True)[1]
    assert not B.owned_arrays(f"kernel t(global int x[64]) {{\n  int v, k, j;\n{body.format(4200)}\n}}\n", 1, 64,
                              with_faults=True)[1]
