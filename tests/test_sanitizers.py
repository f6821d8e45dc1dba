"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle (plain C) and the library's host C++ front end and static proofs
are built with -fsanitize=address,undefined by gcc / g++ into two small
drivers (tests/sanitize/), run over the workload programs, reduced shapes of
the large ones, and malformed texts.  A sanitizer report fails the test;
the sanitized oracle must also give the same results as the regular build,
and the sanitized proofs the same flags as the library."""
import os
import random
import shutil
import subprocess

import pytest

from oracle import oracle as O
from paper_1308_3203_amd import binding as B
from paper_1308_3203_amd import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")


def _build(tmp, compiler, out, sources, lang_flags):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    exe = os.path.join(tmp, out)
    cmd = [compiler, *SAN, *lang_flags, "-o", exe, *sources]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        if "asan" in res.stderr.lower() or "sanitize" in res.stderr.lower():
            pytest.skip(f"sanitizer runtime not available: {res.stderr[-300:]}")
        raise AssertionError(res.stderr)
    return exe


def _cases(tmp):
    """(path, workload-or-None, G, W, lo, hi, seed0, n) case files."""
    r = random.Random(11)
    cases = []

    def add(name, src, G, W, lo, hi, n, w=None):
        path = os.path.join(tmp, f"{name}.case")
        with open(path, "w") as fh:
            fh.write(f"{G} {W} {lo} {hi} 0 {n}\n{src}")
        cases.append((path, src, G, W, lo, hi, n))

    add("fig1_literal", WL.fig1(16, one_based=False).src, 1, 16, 0, 16, 2)
    add("fig1", WL.fig1(16).src, 1, 16, 0, 16, 2)
    add("fig3", WL.fig3(16).src, 1, 16, 0, 16, 2)
    add("c1", WL.c1_kernel(1).src, 1, 64, 0, 16, 3)
    for w in WL.c2_templates():
        add(w.name, w.src, 2, w.W, -2 ** 31, 2 ** 31, 1)
    c4 = WL.c4_kernel(groups=2, wgsize=64, iters=8, log2_cells=12)
    add("c4_small", c4.src, c4.G, c4.W, -2 ** 31, 2 ** 31, 2)
    for s in range(24):
        w = WL.c3_kernel(s)
        if w.W <= 512:
            add(f"c3_{s}", w.src, 1, w.W, 0, 16, 1)
        # malformed: the same text cut short, or with a character replaced
        cut = r.randrange(10, len(w.src) - 2)
        add(f"bad_cut_{s}", w.src[:cut], 1, 64, 0, 16, 1)
        k = r.randrange(len(w.src))
        add(f"bad_chr_{s}", w.src[:k] + r.choice("@#${}[];:=") + w.src[k + 1:], 1, 64, 0, 16, 1)
    # faults of every kind
    add("oob", "kernel f(global int A[4]) { int x; x := A[tid]; }", 1, 8, 0, 16, 1)
    add("div0", "kernel f(global int A[8]) { int x; x := 5 / (tid - 3); A[tid] := x; }", 1, 8, 0, 16, 1)
    add("bardiv", "kernel f(global int A[8]) { if (tid < 3) { barrier; } }", 1, 8, 0, 16, 1)
    add("intmin", "kernel f(global int A[8]) { int x; x := (0 - 2147483647 - 1) / (0 - 1); "
        "A[tid] := (0 - 2147483647 - 1) % (0 - 1) + x; }", 1, 8, 0, 16, 1)
    return cases


@pytest.fixture(scope="module")
def cases(tmp_path_factory):
    tmp = str(tmp_path_factory.mktemp("san"))
    return tmp, _cases(tmp)


def _run(exe, paths):
    res = subprocess.run([exe, *paths], capture_output=True, text=True, env=ENV, timeout=600)
    assert "runtime error" not in res.stderr and "Sanitizer" not in res.stderr, res.stderr[-4000:]
    assert res.returncode == 0, res.stderr[-4000:]
    return res.stdout.splitlines()


def test_oracle_under_sanitizers(cases):
    tmp, cs = cases
    exe = _build(tmp, "gcc", "oracle_san", [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                                            os.path.join(ROOT, "oracle", "oracle.c")], ["-std=c99"])
    lines = _run(exe, [c[0] for c in cs])
    got = {}
    for ln in lines:
        f = ln.split()
        got.setdefault(f[0], []).append(f[1:])
    for path, src, G, W, lo, hi, n in cs:
        try:
            prog = O.Program(src)
        except Exception:
            assert got[path] == [["parse-error"]], path
            continue
        arrays = {a: ("seeded", lo, hi) for a, _ in prog.arrays}
        scalars = {s: ("seeded", lo, hi) for s in prog.scalars}
        for j in range(n):
            r = prog.run(G, W, arrays=arrays, scalars=scalars, seed=j, instance=j)
            s = r.summary
            want = [str(j), str(int(s["status"])), str(len(r.records)), str(int(s["n_race_cells"])),
                    str(int(s["n_benign_cells"])), str(int(s["n_accesses"]))]
            assert got[path][j] == want, (path, j, got[path][j], want)


def test_host_front_end_and_proofs_under_sanitizers(cases):
    tmp, cs = cases
    csrc = os.path.join(ROOT, "paper_1308_3203_amd", "csrc")
    exe = _build(tmp, "g++", "host_san", [os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                                          os.path.join(csrc, "frontend.cpp"), os.path.join(csrc, "ownership.cpp")],
                 ["-std=c++17"])
    lines = _run(exe, [c[0] for c in cs])
    by = {ln.split()[0]: ln.split()[1:] for ln in lines}
    n_ok = 0
    for path, src, G, W, lo, hi, n in cs:
        try:
            owned, nofault = B.owned_arrays(src, G, W, with_faults=True)
        except B.RcError:
            assert by[path] == ["compile-error"], path
            continue
        n_ok += 1
        f = by[path]
        assert f[2] == str(int(nofault)), (path, f)
        assert [c == "o" for c in f[3]] == [bool(x) for x in owned], (path, f, owned)
    assert n_ok >= 25
