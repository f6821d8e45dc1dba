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


# ---------------------------------------------------------------------------
# the batched random kernels exactly as bench.py runs them: 10^4 programs x
# 100 seeds in one rc_batch_check over the 230 GB workspace, with the
# autotuner's per-bucket choices
# ---------------------------------------------------------------------------
def _batch_samples(batch, summ):
    """~300 instances: the first and last, an even stride over the whole
    list, the first instance of every width class and of every tuning
    bucket, and the racy instances of the first programs."""
    n = batch.n
    ids = {0, 1, n - 2, n - 1}
    ids.update(range(0, n, n // 200))
    seen_w = {}
    for i in range(0, n, batch.seeds):
        w, _ = batch.instance(i)
        seen_w.setdefault(w.W, i)
    ids.update(seen_w.values())
    seen_t = {}
    for k, key in enumerate(batch.tuning_of):
        seen_t.setdefault(key, k * batch.seeds + batch.seeds - 1)
    ids.update(seen_t.values())
    racy = np.nonzero(summ["n_race_cells"][: 50 * batch.seeds] > 0)[0]
    ids.update(int(x) for x in racy[:40])
    return sorted(ids)


@pytest.mark.timeout(900)
def test_c3_bench_batch_sampled():
    import concurrent.futures as cf
    import torch
    from paper_1308_3203_amd import batches
    torch.cuda.empty_cache()
    batch = batches.RandomKernelBatch(U.ctx(), 10000, 100, ws_gb=230.0,
                                      progress=lambda m: print(f"batched random kernels: {m}", flush=True))
    try:
        batch.step()
        recs, summ = batch.results()
        print(f"batched random kernels: checked {batch.n} instances, {len(recs)} records", flush=True)
        # every instance's record counts against the record list
        counts = summ["n_race_cells"].astype(np.int64) + summ["n_benign_cells"].astype(np.int64)
        per_inst = np.bincount(recs["instance"].astype(np.int64), minlength=batch.n)
        assert len(recs) == int(counts.sum())
        assert np.array_equal(per_inst, counts)
        assert np.all(np.diff(recs["instance"].astype(np.int64)) >= 0)
        assert not np.any(summ["flags"])
        offs = np.concatenate([[0], np.cumsum(counts)])
        ids = _batch_samples(batch, summ)

        def one(i):
            w, seed = batch.instance(i)
            o = O.Program(w.src).run(w.G, w.W, arrays=w.arrays, scalars=w.scalars, seed=seed, instance=i)
            return i, o

        with cf.ThreadPoolExecutor(max_workers=8) as ex:
            for k, (i, o) in enumerate(ex.map(one, ids)):
                if k % 50 == 0:
                    print(f"batched random kernels: oracle comparison {k} of {len(ids)}", flush=True)
                got = recs[offs[i]:offs[i + 1]]
                U.assert_same((got, summ[i:i + 1]), (o.records, np.array([o.summary], dtype=O.SUMMARY_DTYPE)),
                              f"batched random kernels, instance {i} ({batch.instance(i)[0].name}, "
                              f"seed {batch.instance(i)[1]})")
    finally:
        batch.free()
        torch.cuda.empty_cache()


@pytest.mark.timeout(300)
def test_c4_all_seeds_full_size():
    """The large-interval kernel at its full size, all 16 seeds of bench.py's
    step in one call (per-program kernel), against the oracle instance by
    instance."""
    import concurrent.futures as cf
    w = WL.c4_kernel()
    p = B.Program(U.ctx(), w.src)
    p.set_ndrange(w.G, w.W)
    p.bind(w.arrays, w.scalars)
    p.jit(True)
    n = 16
    buf = B.Buffers(p, n, cap=1 << 23, ws_limit=int(230 * (1 << 30)))
    p.check_async(0, n, buf.ws, buf.records, buf.n_records, buf.summaries)
    U.ctx().sync()
    summ = B.summaries_to_numpy(buf.summaries, n)
    counts = summ["n_race_cells"].astype(np.int64) + summ["n_benign_cells"].astype(np.int64)
    total = int(buf.n_records.item())
    assert total == int(counts.sum())
    recs = B.records_to_numpy(buf.records, total)
    offs = np.concatenate([[0], np.cumsum(counts)])

    def one(j):
        return j, O.Program(w.src).run(w.G, w.W, arrays=w.arrays, scalars=w.scalars, seed=j, instance=j)

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        for j, o in ex.map(one, range(n)):
            U.assert_same((recs[offs[j]:offs[j + 1]], summ[j:j + 1]),
                          (o.records, np.array([o.summary], dtype=O.SUMMARY_DTYPE)), f"c4 seed {j}")
    p.close()
