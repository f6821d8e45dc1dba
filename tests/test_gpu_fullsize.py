"""Parity at the full size of the template workload, in the launch
configuration bench.py times: 10^4 seeds of one template in one call, with
the per-program workspace bench.py gives it (230 GB over six programs: the
tree-reduction and transpose calls run as several chunked launches, the
prefix sum in one), per-program kernels, records placed by rank.  The
oracle cannot check 10^4 instances in a test, so sampled instances (the
first and last, and both sides of the chunk boundaries) are compared one by
one, and every instance's record counts are checked against the length of
the record list."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_3203_amd import binding as B
from paper_1308_3203_amd import workloads as WL
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

N_SEEDS = 10000
WS_BYTES = int(230 * (1 << 30) / 6)
SAMPLES = [0, 1, 2499, 2500, 3333, 3334, 5000, 6667, 6668, 9998, 9999]


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("name", [w.name for w in WL.c2_templates()])
def test_c2_full_size_sampled(name, jit):
    if not jit and name not in ("transpose_race", "prefix_sum"):
        pytest.skip("the interpreter is sampled on two templates")
    w = [x for x in WL.c2_templates() if x.name == name][0]
    p = B.Program(U.ctx(), w.src)
    p.set_ndrange(w.G, w.W)
    p.bind(w.arrays, w.scalars)
    p.jit(jit)
    probe = B.Buffers(p, 16, cap=1 << 22, ws_limit=WS_BYTES)
    p.check_async(0, 16, probe.ws, probe.records, probe.n_records, probe.summaries)
    U.ctx().sync()
    cap = int(int(probe.n_records.item()) / 16 * N_SEEDS * 1.25) + (1 << 16)
    del probe
    buf = B.Buffers(p, N_SEEDS, cap=cap, ws_limit=WS_BYTES)
    p.check_async(0, N_SEEDS, buf.ws, buf.records, buf.n_records, buf.summaries)
    U.ctx().sync()
    summ = B.summaries_to_numpy(buf.summaries, N_SEEDS)
    counts = summ["n_race_cells"].astype(np.int64) + summ["n_benign_cells"].astype(np.int64)
    total = int(buf.n_records.item())
    assert total == int(counts.sum()) and total <= cap
    offs = np.concatenate([[0], np.cumsum(counts)])
    prog = O.Program(w.src)
    for j in SAMPLES:
        a, b = int(offs[j]), int(offs[j + 1])
        raw = buf.records[a * B.RECORD_BYTES:b * B.RECORD_BYTES].cpu().numpy()
        got = raw.view(B.RECORD_DTYPE)
        o = prog.run(w.G, w.W, arrays=w.arrays, scalars=w.scalars, seed=j, instance=j)
        U.assert_same((got, summ[j:j + 1]), (o.records, np.array([o.summary], dtype=O.SUMMARY_DTYPE)),
                      f"{name} instance {j}")
