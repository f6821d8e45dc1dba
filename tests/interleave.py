"""Brute-force enumerator of every interleaving of a tiny kernel (test helper).

It is a third, independent reading of the paper's Section 4 semantics: the
global rules let any thread take the next atomic step ("these rules describe
any scheduling"), and a barrier releases only when every thread waits at it.
It runs straight-line programs (no if/for) of one work-group over global
arrays, enumerating all schedules by depth-first search over states.

Programs are lists of tuples:
  ("assign", v, e) | ("load", v, A, e) | ("store", A, e, e2) | ("barrier",)
expressions: int | "tid" | var-name | (op, e1, e2) with op in + - * & mod
"""
from __future__ import annotations

import random

M32 = 0xFFFFFFFF


def _w(x: int) -> int:
    x &= M32
    return x - (1 << 32) if x & 0x80000000 else x


def ev(e, tid: int, env: dict) -> int:
    if isinstance(e, int):
        return _w(e)
    if e == "tid":
        return tid
    if isinstance(e, str):
        return env[e]
    op, a, b = e
    x, y = ev(a, tid, env), ev(b, tid, env)
    if op == "+":
        return _w(x + y)
    if op == "-":
        return _w(x - y)
    if op == "*":
        return _w(x * y)
    if op == "&":
        return _w(x & y)
    if op == "mod":          # y is always a positive constant here
        return x % y
    raise ValueError(op)


def render_expr(e) -> str:
    if isinstance(e, int):
        return str(e) if e >= 0 else f"(0 - {-e})"
    if isinstance(e, str):
        return e
    op, a, b = e
    return f"({render_expr(a)} {op} {render_expr(b)})"


def render(prog, arrays: dict, vars_: list) -> str:
    lines = []
    for s in prog:
        if s[0] == "assign":
            lines.append(f"{s[1]} := {render_expr(s[2])};")
        elif s[0] == "load":
            lines.append(f"{s[1]} := {s[2]}[{render_expr(s[3])}];")
        elif s[0] == "store":
            lines.append(f"{s[1]}[{render_expr(s[2])}] := {render_expr(s[3])};")
        else:
            lines.append("barrier;")
    params = ", ".join(f"global int {a}[{n}]" for a, n in arrays.items())
    return (f"kernel tiny({params}) {{\n  int {', '.join(vars_)};\n  " +
            "\n  ".join(lines) + "\n}\n")


def final_states(prog, W: int, init: dict, vars_: list):
    """Every (shared memory, private vars) state reachable at kernel exit."""
    n = len(prog)
    results = set()
    seen = set()

    def freeze(mem, envs):
        return (tuple((a, tuple(v)) for a, v in sorted(mem.items())),
                tuple(tuple(env[v] for v in vars_) for env in envs))

    def dfs(pcs, mem, envs):
        key = (pcs, freeze(mem, envs))
        if key in seen:
            return
        seen.add(key)
        if all(pc == n for pc in pcs):
            results.add(freeze(mem, envs))
            return
        # barrier release: every thread waits at the same barrier
        if all(pc < n and prog[pc][0] == "barrier" for pc in pcs):
            if len(set(pcs)) != 1:
                raise AssertionError("threads wait at different barriers")
            dfs(tuple(pc + 1 for pc in pcs), mem, envs)
            return
        for t in range(W):
            pc = pcs[t]
            if pc == n or prog[pc][0] == "barrier":
                continue
            s = prog[pc]
            mem2 = {a: list(v) for a, v in mem.items()}
            envs2 = [dict(e) for e in envs]
            env = envs2[t]
            if s[0] == "assign":
                env[s[1]] = ev(s[2], t, env)
            elif s[0] == "load":
                env[s[1]] = mem2[s[2]][ev(s[3], t, env)]
            else:
                mem2[s[1]][ev(s[2], t, env)] = ev(s[3], t, env)
            dfs(tuple(p + 1 if i == t else p for i, p in enumerate(pcs)), mem2, envs2)

    dfs(tuple([0] * W), {a: list(v) for a, v in init.items()}, [dict.fromkeys(vars_, 0) for _ in range(W)])
    return results


def lockstep_state(prog, W: int, init: dict, vars_: list):
    """The schedule the checker fixes: statement by statement, ascending tid."""
    mem = {a: list(v) for a, v in init.items()}
    envs = [dict.fromkeys(vars_, 0) for _ in range(W)]
    for s in prog:
        if s[0] == "barrier":
            continue
        for t in range(W):
            env = envs[t]
            if s[0] == "assign":
                env[s[1]] = ev(s[2], t, env)
            elif s[0] == "load":
                env[s[1]] = mem[s[2]][ev(s[3], t, env)]
            else:
                mem[s[1]][ev(s[2], t, env)] = ev(s[3], t, env)
    return (tuple((a, tuple(v)) for a, v in sorted(mem.items())),
            tuple(tuple(env[v] for v in vars_) for env in envs))


def random_program(r: random.Random, n_stmts: int, N: int, n_barriers: int):
    vars_ = ["p", "q"]
    arrays = ["A", "B"]

    def idx():
        k = r.random()
        if k < 0.35:
            return ("mod", ("+", "tid", r.randint(0, N - 1)), N)
        if k < 0.55:
            return r.randint(0, N - 1)
        if k < 0.75:
            return ("mod", ("*", "tid", r.randint(1, 3)), N)
        return ("mod", ("&", ("+", r.choice(vars_), "tid"), 1023), N)

    def val():
        k = r.random()
        if k < 0.3:
            return r.randint(0, 3)
        if k < 0.6:
            return r.choice(vars_)
        return ("+", r.choice(vars_ + ["tid"]), r.randint(0, 2))

    prog = []
    for _ in range(n_stmts):
        k = r.random()
        if k < 0.2:
            prog.append(("assign", r.choice(vars_), val()))
        elif k < 0.6:
            prog.append(("load", r.choice(vars_), r.choice(arrays), idx()))
        else:
            prog.append(("store", r.choice(arrays), idx(), val()))
    for _ in range(n_barriers):
        prog.insert(r.randint(1, len(prog)), ("barrier",))
    return prog, {a: N for a in arrays}, vars_
