"""Helpers shared by the GPU tests: run the HIP library and the oracle on the
same seeded instances and compare the results byte for byte."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_1308_3203_amd import binding as B

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = B.Context(0)
    return _CTX


def gpu_run(src, G, W, arrays=None, scalars=None, seed0=0, n=1, cap=1 << 20, ws_limit=4 << 30,
            lds_log_entries=0, jit=False):
    return B.check(src, G, W, arrays=arrays, scalars=scalars, seed0=seed0, n_seeds=n, cap=cap,
                   ctx=ctx(), ws_limit=ws_limit, lds_log_entries=lds_log_entries, jit=jit)


def oracle_run(src, G, W, arrays=None, scalars=None, seed0=0, n=1):
    prog = O.Program(src)
    recs, summs = [], []
    for j in range(n):
        r = prog.run(G, W, arrays=arrays, scalars=scalars, seed=seed0 + j, instance=j)
        recs.append(r.records)
        summs.append(r.summary)
    recs = np.concatenate(recs) if recs else np.zeros(0, O.RECORD_DTYPE)
    return recs, np.array(summs, dtype=O.SUMMARY_DTYPE)


def assert_same(gpu, orc, what=""):
    g_rec, g_sum = gpu
    o_rec, o_sum = orc
    if g_sum.tobytes() != o_sum.tobytes():
        for j in range(len(o_sum)):
            if g_sum[j].tobytes() != o_sum[j].tobytes():
                raise AssertionError(f"{what}: summary {j} differs:\n gpu    {g_sum[j]}\n oracle {o_sum[j]}")
    if g_rec.tobytes() != o_rec.tobytes():
        n = min(len(g_rec), len(o_rec))
        for i in range(n):
            if g_rec[i].tobytes() != o_rec[i].tobytes():
                raise AssertionError(f"{what}: record {i} of {len(o_rec)} differs:\n gpu    {g_rec[i]}\n"
                                     f" oracle {o_rec[i]}")
        raise AssertionError(f"{what}: {len(g_rec)} records on the GPU, {len(o_rec)} from the oracle")


def host_arrays_to_device(arrays):
    """numpy int32 bindings -> cuda tensors for the library; tuples pass through."""
    import torch
    out = {}
    for k, v in (arrays or {}).items():
        out[k] = v if isinstance(v, tuple) else torch.from_numpy(np.ascontiguousarray(v, np.int32)).cuda()
    return out
