"""rc_check_static (the entry point for callers that cannot allocate) against
rc_check with a caller-owned workspace: byte-identical records and
summaries, on two calls in a row of one program, the second with fewer
seeds, through the C ABI."""
import numpy as np
import pytest
import torch

from paper_1308_3203_amd import binding as B
from paper_1308_3203_amd import workloads as WL
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _out(n, cap):
    rec = torch.empty(cap * B.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    summ = torch.empty(n * B.SUMMARY_BYTES, dtype=torch.uint8, device="cuda")
    return rec, cnt, summ


def _host(rec, cnt, summ, n):
    k = int(cnt.item())
    return B.records_to_numpy(rec, k), B.summaries_to_numpy(summ, n)


CASES = [("fig3", lambda: WL.fig3(64), False), ("c1_1", lambda: WL.c1_kernel(1), False),
         ("tree_reduce_race", lambda: WL.tree_reduce(True), False),
         ("tree_reduce_race", lambda: WL.tree_reduce(True), True),
         ("transpose_race", lambda: WL.transpose(True), True),
         ("c3_7", lambda: WL.c3_kernel(7), False)]


@pytest.mark.parametrize("name,make,jit", CASES, ids=[f"{c[0]}-{'jit' if c[2] else 'interp'}" for c in CASES])
def test_static_workspace_matches_caller_workspace(name, make, jit):
    w = make()
    ctx = U.ctx()
    p = B.Program(ctx, w.src)
    p.set_ndrange(w.G, w.W)
    p.bind(w.arrays, w.scalars)
    if jit:
        p.jit(True)
    cap = 1 << 20
    # two calls in a row on the static workspace, the second smaller; each
    # against a call of its own with a caller-owned workspace
    for seed0, n in ((0, 48), (1000, 5)):
        print(f"static workspace: {name} jit={jit} seeds {seed0}..{seed0 + n - 1}", flush=True)
        rec, cnt, summ = _out(n, cap)
        p.check_static_async(seed0, n, rec, cnt, summ)
        ctx.sync()
        got = _host(rec, cnt, summ, n)
        buf = B.Buffers(p, n, cap=cap, ws_limit=4 << 30)
        p.check_async(seed0, n, buf.ws, buf.records, buf.n_records, buf.summaries)
        ctx.sync()
        want = _host(buf.records, buf.n_records, buf.summaries, n)
        assert int(cnt.item()) == int(buf.n_records.item())
        U.assert_same(got, want, f"{name} seeds {seed0}+{n}")
        assert len(got[0]) > 0 or name == "c3_7"
    p.close()


def test_static_workspace_rejects_a_large_instance():
    """The large-interval kernel needs far more than the static workspace for
    one instance: a clear error, nothing enqueued."""
    w = WL.c4_kernel()
    ctx = U.ctx()
    p = B.Program(ctx, w.src)
    p.set_ndrange(w.G, w.W)
    p.bind(w.arrays, w.scalars)
    assert p.workspace_size(1) > (256 << 20)
    rec, cnt, summ = _out(1, 16)
    with pytest.raises(B.RcError) as e:
        p.check_static_async(0, 1, rec, cnt, summ)
    assert e.value.status == B.RC_E_INVAL
    assert "static workspace" in str(e.value)
    ctx.sync()
    p.close()


def test_static_workspace_many_seeds_in_passes():
    """More seeds than the static workspace holds at once: several passes,
    the same report as one call with a workspace that holds them all."""
    w = WL.prefix_sum(True)
    ctx = U.ctx()
    p = B.Program(ctx, w.src)
    p.set_ndrange(w.G, w.W)
    p.bind(w.arrays, w.scalars)
    one = p.workspace_size(1)
    n = min(4000, int(3 * (256 << 20) // one) + 2)
    assert p.workspace_size(n) > (256 << 20)
    cap = 1 << 22
    rec, cnt, summ = _out(n, cap)
    print(f"static workspace: prefix_sum_race, {n} seeds ({one} bytes each)", flush=True)
    p.check_static_async(0, n, rec, cnt, summ)
    ctx.sync()
    got = _host(rec, cnt, summ, n)
    buf = B.Buffers(p, n, cap=cap, ws_limit=64 << 30)
    p.check_async(0, n, buf.ws, buf.records, buf.n_records, buf.summaries)
    ctx.sync()
    U.assert_same(got, _host(buf.records, buf.n_records, buf.summaries, n), "prefix_sum_race in passes")
    assert np.all(got[1]["n_race_cells"] > 0)
    p.close()
