"""Seeded synthetic workloads: kernel programs in the minimal kernel language
plus their launch shapes and input bindings.

This module only writes program text and picks launch shapes and binding
ranges; it holds none of the race semantics.  Both the GPU path and the CPU
oracle consume what it produces.

Workloads:
  * ``fig1`` / ``fig3``        -- the paper's example kernel (Fig. 1) and its
                                  counterexample (Fig. 3), Sections 2 and 6.
  * ``c1_kernel(seed)``        -- a random 20-statement kernel: int32 assigns,
                                  loads/stores indexed by (a*tid+b) mod 256, an
                                  if on tid parity, two barriers; G=1, W=64.
  * ``c2_templates()``         -- tree reduction, Hillis-Steele prefix sum and
                                  a 32x32 LDS-tiled transpose, each clean and
                                  with one injected off-by-one race; G=16, W=256.
  * ``c3_kernel(seed)``        -- random kernels for the batched sweep: W in
                                  {32..1024}, 10-200 statements, 1-8 barriers,
                                  loops of 1-16 iterations (nesting <= 2), two
                                  global arrays of 2^12..2^18 cells, with a
                                  race-injection knob.
  * ``c4_kernel()``            -- large intervals: 64 x 1024 work-items, a
                                  64-iteration loop over a 2^20-cell array.
"""
from __future__ import annotations

import random
from dataclasses import dataclass, field

INT32_LO, INT32_HI = -(2 ** 31), 2 ** 31


@dataclass
class Workload:
    name: str
    src: str
    G: int
    W: int
    arrays: dict = field(default_factory=dict)    # name -> ("seeded", lo, hi)
    scalars: dict = field(default_factory=dict)   # name -> ("seeded", lo, hi) | int
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# The paper's two example kernels
# --------------------------------------------------------------------------
def fig1(n: int = 64, one_based: bool = True) -> Workload:
    """Fig. 1, with its compound statements split into single-access ones.

    ``one_based=False`` keeps the paper's indices with a 0-based tid, so the
    first load reads A[-1]; ``one_based=True`` runs thread t as t+1 over arrays
    of n+2 cells, which keeps every access in bounds.
    """
    if not one_based:
        src = f"""kernel fig1(global int A[{n}], global int B[{n}], global int R[{n}]) {{
  int t1, t2, t3;
  t1 := A[tid - 1];
  t2 := B[tid + 1];
  R[tid] := t1 + t2;
  barrier;
  t3 := R[tid + 1];
  R[tid] := 2 * t3;
}}
"""
    else:
        src = f"""kernel fig1(global int A[{n + 2}], global int B[{n + 2}], global int R[{n + 2}]) {{
  int u, t1, t2, t3;
  u := tid + 1;
  t1 := A[u - 1];
  t2 := B[u + 1];
  R[u] := t1 + t2;
  barrier;
  t3 := R[u + 1];
  R[u] := 2 * t3;
}}
"""
    arr = {k: ("seeded", 0, 16) for k in "ABR"}
    return Workload("fig1" + ("_1based" if one_based else "_literal"), src, 1, n, arr)


def fig3(n: int = 64) -> Workload:
    """Fig. 3: the shared scalar g becomes a one-cell global array."""
    src = f"""kernel fig3(global int A[{n + 2}], global int g[1]) {{
  int u, x;
  u := tid + 1;
  g[0] := 0;
  A[u] := 0;
  barrier;
  A[u] := 1;
  x := A[u + 1];
  if (x == 0) {{ g[0] := 1; }}
  barrier;
}}
"""
    return Workload("fig3", src, 1, n, {"A": ("seeded", 0, 16), "g": ("seeded", 0, 16)})


# --------------------------------------------------------------------------
# c1: one random 20-statement kernel, one work-group of 64
# --------------------------------------------------------------------------
def _affine_index(r: random.Random, N: int) -> str:
    a = r.randint(-8, 8)
    b = r.randrange(0, N)
    return f"({a} * tid + {b}) mod {N}"


def _rand_expr(r: random.Random, vars_: list, depth: int = 0) -> str:
    choice = r.random()
    if depth >= 2 or choice < 0.3:
        pick = r.random()
        if pick < 0.5:
            return r.choice(vars_)
        if pick < 0.7:
            return "tid"
        return str(r.randint(0, 15))
    op = r.choice(["+", "-", "*", "&", "^", "|"])
    return f"({_rand_expr(r, vars_, depth + 1)} {op} {_rand_expr(r, vars_, depth + 1)})"


def c1_kernel(seed: int = 1, n_stmts: int = 20) -> Workload:
    r = random.Random(seed)
    vars_ = ["r0", "r1", "r2", "r3"]
    arrays = ["x", "y"]
    N = 256

    def simple() -> str:
        k = r.random()
        if k < 0.3:
            return f"{r.choice(vars_)} := {_rand_expr(r, vars_)};"
        if k < 0.65:
            return f"{r.choice(vars_)} := {r.choice(arrays)}[{_affine_index(r, N)}];"
        return f"{r.choice(arrays)}[{_affine_index(r, N)}] := {_rand_expr(r, vars_)};"

    n_then = r.randint(2, 4)
    n_else = r.randint(2, 4)
    n_top = n_stmts - 1 - n_then - n_else           # includes the two barriers
    top = [simple() for _ in range(n_top - 2)]
    # two barriers at distinct top-level positions (never first)
    for _ in range(2):
        top.insert(r.randint(1, len(top)), "barrier;")
    if_stmt = ("if ((tid & 1) == 0) {\n    " + "\n    ".join(simple() for _ in range(n_then)) +
               "\n  } else {\n    " + "\n    ".join(simple() for _ in range(n_else)) + "\n  }")
    top.insert(r.randint(0, len(top)), if_stmt)
    body = "\n  ".join(top)
    src = (f"kernel c1_{seed}(global int x[{N}], global int y[{N}]) {{\n"
           f"  int {', '.join(vars_)};\n  {body}\n}}\n")
    return Workload(f"c1_{seed}", src, 1, 64, {"x": ("seeded", 0, 16), "y": ("seeded", 0, 16)},
                    meta={"n_stmts": n_stmts})


# --------------------------------------------------------------------------
# c2: template kernels, 16 work-groups of 256, arrays of 65536 cells
# --------------------------------------------------------------------------
def tree_reduce(inject: bool = False) -> Workload:
    """Per-group sum of 4096 inputs; the injected variant reads loc[lid+s-1]."""
    q = "lid + s - 1" if inject else "lid + s"
    src = f"""kernel tree_reduce{'_race' if inject else ''}(global int inp[65536], global int out[65536]) {{
  local int loc[256];
  int acc, j, k, s, p, q;
  acc := 0;
  for k in 0..16 {{
    p := inp[gid * 4096 + k * 256 + lid];
    acc := acc + p;
  }}
  loc[lid] := acc;
  barrier;
  for j in 0..8 {{
    s := 128 >> j;
    if (lid < s) {{
      p := loc[lid];
      q := loc[{q}];
      loc[lid] := p + q;
    }}
    barrier;
  }}
  if (lid == 0) {{
    p := loc[0];
    out[gid] := p;
  }}
}}
"""
    return Workload("tree_reduce" + ("_race" if inject else ""), src, 16, 256,
                    {"inp": ("seeded", INT32_LO, INT32_HI), "out": ("seeded", INT32_LO, INT32_HI)},
                    meta={"template": "tree_reduce", "inject": inject})


def prefix_sum(inject: bool = False) -> Workload:
    """Per-group inclusive prefix sum of 4096 inputs: a 16-cell sequential scan
    per work-item, then a 256-wide Hillis-Steele scan in a double buffer.  The
    injected variant writes the double buffer one cell too far (wrapping)."""
    widx = "(wr + lid + 1) mod 512" if inject else "wr + lid"
    src = f"""kernel prefix_sum{'_race' if inject else ''}(global int inp[65536], global int out[65536]) {{
  local int buf[512];
  int k, d, acc, p, q, base, off, rd, wr;
  base := gid * 4096 + lid * 16;
  acc := 0;
  for k in 0..16 {{
    p := inp[base + k];
    acc := acc + p;
    out[base + k] := acc;
  }}
  buf[lid] := acc;
  barrier;
  for d in 0..8 {{
    off := 1 << d;
    rd := (d & 1) * 256;
    wr := 256 - rd;
    p := buf[rd + lid];
    if (lid >= off) {{
      q := buf[rd + lid - off];
      p := p + q;
    }}
    buf[{widx}] := p;
    barrier;
  }}
  p := 0;
  if (lid > 0) {{
    p := buf[lid - 1];
  }}
  for k in 0..16 {{
    q := out[base + k];
    out[base + k] := q + p;
  }}
}}
"""
    return Workload("prefix_sum" + ("_race" if inject else ""), src, 16, 256,
                    {"inp": ("seeded", INT32_LO, INT32_HI), "out": ("seeded", INT32_LO, INT32_HI)},
                    meta={"template": "prefix_sum", "inject": inject})


def transpose(inject: bool = False) -> Workload:
    """Transpose of the 256x256 view through a padded 32x33 local tile, four
    tiles per work-group.  The last barrier of the tile loop is skipped as
    unnecessary; the injected variant's bound is off by one, so tile 2's
    read-out and tile 3's fill share an interval."""
    bound = 2 if inject else 3
    src = f"""kernel transpose{'_race' if inject else ''}(global int inp[65536], global int out[65536]) {{
  local int tile[1056];
  int t, r, T, tr, tc, tx, ty, row, v;
  tx := lid % 32;
  ty := lid / 32;
  for t in 0..4 {{
    T := gid * 4 + t;
    tr := T / 8;
    tc := T % 8;
    for r in 0..4 {{
      row := ty + 8 * r;
      v := inp[(tr * 32 + row) * 256 + tc * 32 + tx];
      tile[row * 33 + tx] := v;
    }}
    barrier;
    for r in 0..4 {{
      row := ty + 8 * r;
      v := tile[tx * 33 + row];
      out[(tc * 32 + row) * 256 + tr * 32 + tx] := v;
    }}
    if (t < {bound}) {{
      barrier;
    }}
  }}
}}
"""
    return Workload("transpose" + ("_race" if inject else ""), src, 16, 256,
                    {"inp": ("seeded", INT32_LO, INT32_HI), "out": ("seeded", INT32_LO, INT32_HI)},
                    meta={"template": "transpose", "inject": inject})


def c2_templates() -> list:
    out = []
    for fn in (tree_reduce, prefix_sum, transpose):
        out.append(fn(False))
        out.append(fn(True))
    return out


# --------------------------------------------------------------------------
# c3: random kernels for the batched sweep
# --------------------------------------------------------------------------
class _C3Gen:
    def __init__(self, seed: int, race_rate: float):
        self.r = random.Random(0x5EED0000 + seed)
        self.seed = seed
        r = self.r
        self.W = 32 * r.randint(1, 32)
        self.sizes = {"x": 2 ** r.randint(12, 18), "y": 2 ** r.randint(12, 18)}
        self.target = r.randint(10, 200)
        self.n_barriers = r.randint(1, 8)
        self.vars = [f"v{i}" for i in range(6)]
        self.loopvars = ["i0", "i1"]
        self.count = 0
        self.racy = r.random() < race_rate
        self.injected = False

    def odd(self) -> int:
        return 2 * self.r.randint(0, 40) + 1

    def expr(self, depth=0, allow_loop=()) -> str:
        r = self.r
        if depth >= 2 or r.random() < 0.35:
            k = r.random()
            if k < 0.45:
                return r.choice(self.vars)
            if k < 0.6 and allow_loop:
                return r.choice(allow_loop)
            if k < 0.75:
                return "tid"
            return str(r.randint(0, 31))
        op = r.choice(["+", "-", "*", "&", "^", "|", ">>", "min", "max"])
        a, b = self.expr(depth + 1, allow_loop), self.expr(depth + 1, allow_loop)
        if op in ("min", "max"):
            return f"{op}({a}, {b})"
        if op == ">>":
            return f"({a} >> {r.randint(0, 4)})"
        return f"({a} {op} {b})"

    def phase_roles(self):
        # each array is either written at own cells (stride s odd, offset o)
        # or only read in a phase
        roles = {}
        for a in ("x", "y"):
            if self.r.random() < 0.5:
                roles[a] = ("own", self.odd(), self.r.randrange(self.sizes[a]))
            else:
                roles[a] = ("read",)
        return roles

    def own_index(self, a, role, loopvar=None) -> str:
        _, s, o = role
        N = self.sizes[a]
        return f"(tid * {s} + {o}) mod {N}"

    def read_index(self, a, loops) -> str:
        N = self.sizes[a]
        r = self.r
        k = r.random()
        if k < 0.4:
            return f"({r.randint(-8, 8)} * tid + {r.randrange(N)}) mod {N}"
        if k < 0.7 and loops:
            return f"(tid * {self.odd()} + {r.choice(loops)} * {r.randint(1, 64)} + {r.randrange(N)}) mod {N}"
        return f"({self.expr(1, tuple(loops))}) mod {N}"

    def simple(self, roles, loops, in_if) -> str:
        r = self.r
        self.count += 1
        k = r.random()
        if k < 0.35:
            return f"{r.choice(self.vars)} := {self.expr(0, tuple(loops))};"
        a = r.choice(["x", "y"])
        role = roles[a]
        if k < 0.7:
            if role[0] == "own":
                return f"{r.choice(self.vars)} := {a}[{self.own_index(a, role)}];"
            return f"{r.choice(self.vars)} := {a}[{self.read_index(a, loops)}];"
        if role[0] == "own":
            return f"{a}[{self.own_index(a, role)}] := {self.expr(0, tuple(loops))};"
        # a read-only array in this phase: turn the store into a read
        return f"{r.choice(self.vars)} := {a}[{self.read_index(a, loops)}];"

    def injection(self, roles) -> str:
        """One racy statement: a shared-cell store of a tid-dependent value,
        a read of a neighbour's own cell, or a data-guarded shared store."""
        r = self.r
        self.injected = True
        self.count += 1
        owned = [a for a in ("x", "y") if roles[a][0] == "own"]
        kind = r.randrange(3)
        if kind == 0 or not owned:
            a = r.choice(["x", "y"])
            c = r.randrange(self.sizes[a])
            roles[a] = ("shared",)
            return f"{a}[{c}] := tid & {r.choice([1, 3, 7, 15])};"
        a = r.choice(owned)
        _, s, o = roles[a]
        N = self.sizes[a]
        if kind == 1:
            return f"{r.choice(self.vars)} := {a}[((tid + 1) * {s} + {o}) mod {N}];"
        self.count += 1
        v = r.choice(self.vars)
        return (f"if ({v} < {r.randint(1, 15)}) {{\n    {a}[{r.randrange(N)}] := tid;\n  }}")

    def block(self, n, roles, loops, depth, in_if) -> list:
        out = []
        r = self.r
        while len(out) < n and self.count < self.target:
            k = r.random()
            if k < 0.15 and depth < 2:
                self.count += 1
                lv = self.loopvars[len(loops)]
                bound = r.randint(1, 16)
                inner = self.block(r.randint(1, 3), roles, loops + [lv], depth + 1, in_if)
                out.append(f"for {lv} in 0..{bound} {{\n    " + "\n    ".join(inner) + "\n  }")
            elif k < 0.3 and depth < 3:
                self.count += 1
                cond = (f"(tid & {r.choice([1, 3, 7])}) == {r.randint(0, 1)}" if r.random() < 0.5
                        else f"{r.choice(self.vars)} < {r.randint(0, 16)}")
                then = self.block(r.randint(1, 3), roles, loops, depth + 1, True)
                s = f"if ({cond}) {{\n    " + "\n    ".join(then) + "\n  }"
                if r.random() < 0.4:
                    els = self.block(r.randint(1, 2), roles, loops, depth + 1, True)
                    s += " else {\n    " + "\n    ".join(els) + "\n  }"
                out.append(s)
            else:
                out.append(self.simple(roles, loops, in_if))
        return out

    def build(self) -> Workload:
        r = self.r
        phases = self.n_barriers + 1
        per_phase = max(1, (self.target - self.n_barriers) // phases)
        inj_phase = r.randrange(phases) if self.racy else -1
        lines = []
        for ph in range(phases):
            roles = self.phase_roles()
            body = self.block(per_phase, roles, [], 0, False)
            if ph == inj_phase:
                body.insert(r.randint(0, len(body)), self.injection(roles))
            lines.extend(body)
            if ph < phases - 1:
                lines.append("barrier;")
                self.count += 1
        src = (f"kernel c3_{self.seed}(global int x[{self.sizes['x']}], global int y[{self.sizes['y']}]) {{\n"
               f"  int {', '.join(self.vars + self.loopvars)};\n  " + "\n  ".join(lines) + "\n}\n")
        return Workload(f"c3_{self.seed}", src, 1, self.W,
                        {"x": ("seeded", 0, 16), "y": ("seeded", 0, 16)},
                        meta={"injected": self.injected, "n_barriers": self.n_barriers})


def c3_kernel(seed: int, race_rate: float = 0.10) -> Workload:
    return _C3Gen(seed, race_rate).build()


# --------------------------------------------------------------------------
# c4: large intervals
# --------------------------------------------------------------------------
def c4_kernel(groups: int = 64, wgsize: int = 1024, iters: int = 64, log2_cells: int = 20) -> Workload:
    """Each work-item visits a[(tid*(s|1) + i*k) mod 2^20] for 64 iterations.
    A cell's class u = cls[A] in [0,100) decides the access: u < 68 reads a,
    68 <= u < 98 writes cval[A] (equal values: benign), u >= 98 writes
    cval[A] + tid (different values: a race)."""
    N = 2 ** log2_cells
    src = f"""kernel large_intervals(global int a[{N}], global int cls[{N}], global int cval[{N}], int s, int k) {{
  int i, A, u, t, v, w;
  for i in 0..{iters} {{
    A := (tid * (s | 1) + i * k) & {N - 1};
    u := cls[A];
    if (u < 68) {{
      t := a[A];
    }} else {{
      v := cval[A];
      w := 0;
      if (98 <= u) {{
        w := tid;
      }}
      a[A] := v + w;
    }}
  }}
}}
"""
    return Workload("large_intervals", src, groups, wgsize,
                    {"a": ("seeded", INT32_LO, INT32_HI), "cls": ("seeded", 0, 100),
                     "cval": ("seeded", INT32_LO, INT32_HI)},
                    {"s": ("seeded", INT32_LO, INT32_HI), "k": ("seeded", INT32_LO, INT32_HI)})
