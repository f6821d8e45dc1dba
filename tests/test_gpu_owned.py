"""GPU parity on arrays the ownership proof accepts (not logged, overlay words
placed lane by lane): records, summaries and final memory against the
oracle, which logs every access and keeps one word per cell."""
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_3203_amd import binding as B
from tests import gpu_util as U
from tests.test_ownership import _random_affine_program

pytestmark = pytest.mark.gpu


def parity_and_final(src, G, W, arrays, n=3, seed0=0, jit=False, final=("x",)):
    import torch
    dev = U.host_arrays_to_device(arrays)
    g = U.gpu_run(src, G, W, dev, None, seed0, n, jit=jit)
    o = U.oracle_run(src, G, W, arrays, None, seed0, n)
    U.assert_same(g, o, src)
    prog = B.Program(U.ctx(), src)
    prog.set_ndrange(G, W)
    prog.bind(dev)
    if jit:
        prog.jit(True)
    ws = torch.empty(prog.workspace_size(1), dtype=torch.uint8, device="cuda")
    for name in final:
        fin = prog.read_final(seed0, name, ws).cpu().numpy()
        U.ctx().sync()
        orc = O.Program(src).run(G, W, arrays=arrays, seed=seed0, final=name)
        assert np.array_equal(fin, orc.final), (src, name)
    return prog


HAND = [
    # (body, G, W, owned x)
    ("x[tid] := tid * 3;\n  v := x[tid];\n  x[tid] := v + 1;", 4, 64, True),
    ("x[1000 - tid] := tid;\n  v := x[1000 - tid];\n  x[1000 - tid] := v * 2;", 3, 96, True),
    ("x[3 * tid + 1] := 5;\n  x[3 * tid + 2] := 6;\n  v := x[3 * tid + 1];\n  x[3 * tid + 2] := v + tid;", 2, 80,
     True),
    ("for k in 0..4 {\n    x[tid * 4 + k] := k + tid;\n  }\n  v := x[tid * 4 + 2];\n  y[tid] := v;", 4, 32, True),
    ("x[gid * 7 + 3] := gid;\n  v := x[gid * 7 + 3];\n  y[gid] := v;", 16, 1, True),
    ("x[lid * 2] := lid;\n  barrier;\n  v := x[lid * 2 + 2];\n  y[lid] := v;", 1, 64, False),
    ("x[lid * 2] := lid;\n  v := x[lid * 2];\n  y[lid] := v;", 1, 64, True),
    # an owned array beside a racy one
    ("x[tid] := tid;\n  y[0] := tid;\n  v := x[tid];\n  w := y[1];", 2, 64, True),
]


@pytest.mark.parametrize("case", range(len(HAND)))
@pytest.mark.parametrize("jit", [False, True])
def test_owned_hand_cases(case, jit):
    body, G, W, expect = HAND[case]
    src = f"kernel t(global int x[4096], global int y[4096]) {{\n  int v, w, k;\n  {body}\n}}\n"
    assert B.owned_arrays(src, G, W)[0] == expect
    prog = parity_and_final(src, G, W, {"x": ("seeded", -100, 100), "y": ("seeded", 0, 8)}, jit=jit,
                            final=("x", "y"))
    assert prog.owned("x") == expect


def test_owned_random_programs():
    r = random.Random(7)
    n_owned = 0
    for case in range(60):
        src = _random_affine_program(r)
        G, W = r.choice([(1, 8), (2, 8), (4, 4), (3, 16), (2, 64)])
        own = B.owned_arrays(src, G, W)
        n_owned += own[0]
        parity_and_final(src, G, W, {"x": ("seeded", 0, 4)}, n=2, seed0=case, final=("x",))
    assert n_owned >= 20
