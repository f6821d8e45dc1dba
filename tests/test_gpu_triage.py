"""GPU tests of the triage rows: features (bit-exact against the oracle's
orc_features) and the network's forward, gradient and Adam kernels (fp32
against the float64 numpy oracle)."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from oracle import oracle as O
from paper_1308_3203_amd import binding as B
from paper_1308_3203_amd import workloads as WL

from .gpu_util import ctx, host_arrays_to_device
from .test_features_oracle import SRC1, SRC2, SRC3

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------
def _gpu_features(items):
    """items: list of (Program, seed) -> float32 [n, 128] from the library."""
    torch = _torch()
    progs = [p for p, _ in items]
    seeds = [s for _, s in items]
    n = len(items)
    n_progs = len({id(p) for p in progs})
    ws = torch.empty(max(1, B.Context.features_workspace_size(n, n_progs)), dtype=torch.uint8, device="cuda")
    feat = torch.empty(n * B.N_FEATURES, dtype=torch.float32, device="cuda")
    c = ctx()
    c.features_async(progs, seeds, feat, ws)
    c.sync()
    return feat.cpu().numpy().reshape(n, B.N_FEATURES)


def _load(w, device_arrays=None):
    p = B.Program(ctx(), w.src)
    p.set_ndrange(w.G, w.W)
    p.bind(device_arrays if device_arrays is not None else w.arrays, w.scalars)
    return p


def _check_rows(got, want, what):
    for i in range(len(want)):
        if got[i].tobytes() != want[i].tobytes():
            bad = np.nonzero(got[i] != want[i])[0]
            raise AssertionError(f"{what}: row {i} differs at {bad[:8]}: gpu {got[i][bad[:8]]} oracle {want[i][bad[:8]]}")


def test_features_match_oracle_on_every_workload_family():
    ws = [WL.fig1(64), WL.fig3(64), WL.c1_kernel(1), WL.c1_kernel(7), WL.c4_kernel(groups=4, wgsize=128, iters=4,
                                                                                log2_cells=12)]
    ws += WL.c2_templates()
    ws += [WL.c3_kernel(s) for s in range(60)]
    items, want = [], []
    for w in ws:
        p = _load(w)
        op = O.Program(w.src)
        for seed in (0, 1, 12345, 2**40 + 3):
            items.append((p, seed))
            want.append(op.features(w.G, w.W, w.arrays, seed=seed))
    got = _gpu_features(items)
    _check_rows(got, np.array(want), "workloads")


def test_features_hand_programs_with_bound_buffers():
    torch = _torch()
    Bdata = np.array([-2**31, -1, 0, 2**31 - 1, 536870911, 536870912, -536870913, 100], dtype=np.int32)
    A64 = np.arange(-32, 32, dtype=np.int32) * 40000000
    cases = [
        (SRC1, 3, 40, {"A": ("seeded", 0, 16), "B": Bdata}),
        (SRC1, 1, 64, {"A": A64, "B": ("seeded", -2**31, 2**31)}),
        (SRC1, 2, 8, {"A": ("seeded", -2**31, 2**31), "B": ("seeded", -7, 2**31)}),
        (SRC2, 1, 16, {"A": ("seeded", -5, 300)}),
        (SRC3, 2, 8, {"A": ("seeded", 0, 16)}),
    ]
    items, want, keep = [], [], []
    for src, G, W, arrays in cases:
        dev = host_arrays_to_device(arrays)
        keep.append(dev)
        p = B.Program(ctx(), src)
        p.set_ndrange(G, W)
        p.bind(dev, {"s": 3} if "int s" in src else None)
        op = O.Program(src)
        for seed in (0, 5, 99):
            items.append((p, seed))
            want.append(op.features(G, W, arrays, seed=seed))
    got = _gpu_features(items)
    torch.cuda.synchronize()
    _check_rows(got, np.array(want), "hand programs")


def test_features_ragged_batch_and_errors():
    torch = _torch()
    w = WL.c3_kernel(3)
    p = _load(w)
    op = O.Program(w.src)
    n = 4 * 37 + 3      # not a multiple of the four instances per block
    got = _gpu_features([(p, s) for s in range(n)])
    want = np.array([op.features(w.G, w.W, w.arrays, seed=s) for s in range(n)])
    _check_rows(got, want, "ragged")
    # workspace below the documented size
    feat = torch.empty(2 * 128, dtype=torch.float32, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.RcError):
        ctx().features_async([p, p], [0, 1], feat, small)
    # a program with no launch shape
    q = B.Program(ctx(), w.src)
    ws = torch.empty(B.Context.features_workspace_size(1, 1), dtype=torch.uint8, device="cuda")
    with pytest.raises(B.RcError):
        ctx().features_async([q], [0], feat[:128], ws)


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def _init(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = {
        "W1": rng.normal(0, scale / math.sqrt(M.D_IN), (M.D_H, M.D_IN)),
        "b1": rng.normal(0, 0.1, M.D_H),
        "W2": rng.normal(0, scale / math.sqrt(M.D_H), (M.D_H, M.D_H)),
        "b2": rng.normal(0, 0.1, M.D_H),
        "w3": rng.normal(0, 1 / math.sqrt(M.D_H), M.D_H),
        "b3": rng.normal(0, 0.1, 1),
    }
    return M.pack(parts).astype(np.float32).astype(np.float64)


def _data(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (n, M.D_IN)).astype(np.float32).astype(np.float64)
    y = (rng.random(n) < 0.3).astype(np.float64)
    return X, y


def _clear_data(theta, seed, n, margin=1e-4):
    """n rows whose every pre-activation is at least `margin` away from the
    ReLU kink (judged by the float64 oracle), so that fp32 and fp64 take the
    same branch everywhere and only arithmetic error remains."""
    X, y = _data(seed, 2 * n + 64)
    _, (_, a1, _, a2, _) = M.forward(theta, X)
    ok = (np.abs(a1).min(axis=1) > margin) & (np.abs(a2).min(axis=1) > margin)
    keep = np.nonzero(ok)[0][:n]
    assert keep.size == n
    return X[keep], y[keep]


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).reshape(-1)).cuda()


def _ws(n):
    torch = _torch()
    return torch.empty(B.Context.mlp_workspace_size(n), dtype=torch.uint8, device="cuda")


def _blocks(v):
    out, at = {}, 0
    for name, shape in M.SHAPES:
        k = int(np.prod(shape))
        out[name] = v[at:at + k]
        at += k
    return out


@pytest.mark.parametrize("n", [1, 63, 1000, 4099])
def test_forward_matches_oracle(n):
    torch = _torch()
    theta = _init(n)
    X, _ = _data(n + 1, n)
    logits = torch.empty(n, dtype=torch.float32, device="cuda")
    ctx().mlp_forward_async(_dev(theta), _dev(X), logits, _ws(n))
    ctx().sync()
    z, _ = M.forward(theta, X)
    got = logits.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - z)) <= 1e-5, np.max(np.abs(got - z))


@pytest.mark.parametrize("n", [5, 777, 4096])
def test_gradient_matches_oracle(n):
    torch = _torch()
    theta = _init(10 + n, scale=1.5)
    X, y = _clear_data(theta, 20 + n, n)
    grad = torch.empty(B.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ctx().mlp_grad_async(_dev(theta), _dev(X), _dev(y), grad, loss, _ws(n))
    ctx().sync()
    g, l = M.grad(theta, X, y)
    assert abs(loss.item() - l) <= 1e-5 * max(1.0, abs(l))
    _assert_grad_close(grad.cpu().numpy().astype(np.float64), g)


def _assert_grad_close(got, want):
    """Block-wise relative L2 error <= 1e-4, and no element off by more than
    1e-4 of its block's largest entry (inputs from _clear_data: no ReLU
    decision is within rounding of its kink)."""
    gg, go = _blocks(got), _blocks(want)
    for name in go:
        d = gg[name] - go[name]
        rel = np.linalg.norm(d) / max(np.linalg.norm(go[name]), 1e-30)
        assert rel <= 1e-4, (name, rel)
        assert np.max(np.abs(d)) <= 1e-4 * np.max(np.abs(go[name])) + 1e-12, name


def test_adam_step_matches_oracle():
    torch = _torch()
    n, lr = 512, 1e-3
    theta = _init(3)
    X, y = _clear_data(theta, 4, n)
    p = _dev(theta)
    m = torch.zeros(B.MLP_PARAMS, dtype=torch.float32, device="cuda")
    v = torch.zeros(B.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ctx().mlp_train_step_async(p, m, v, 1, _dev(X), _dev(y), lr, loss, _ws(n))
    ctx().sync()
    g, l = M.grad(theta, X, y)
    t1, m1, v1 = M.adam_step(theta, np.zeros_like(theta), np.zeros_like(theta), g, 1, lr)
    assert abs(loss.item() - l) <= 1e-5 * max(1.0, abs(l))
    gm = m.cpu().numpy().astype(np.float64)
    gv = v.cpu().numpy().astype(np.float64)
    gt = p.cpu().numpy().astype(np.float64)
    _assert_grad_close(gm / 0.1, m1 / 0.1)                      # m = (1 - beta1) g
    for blk, (ga, ob) in enumerate(zip(_blocks(gv).values(), _blocks(v1).values())):
        assert np.linalg.norm(ga - ob) <= 2e-4 * np.linalg.norm(ob) + 1e-30, blk   # v = (1 - beta2) g^2
    # the update is lr g / (|g| + eps): exact where |g| is clearly above the
    # fp32 gradient error, and never longer than lr anywhere
    d_gpu = gt - theta
    d_orc = t1 - theta
    for name in go_names():
        gb = _blocks(g)[name]
        sel = np.abs(gb) > 1e-3 * np.max(np.abs(gb))
        assert np.max(np.abs(_blocks(d_gpu)[name][sel] - _blocks(d_orc)[name][sel])) <= 1e-4 * lr, name
    assert np.max(np.abs(d_gpu)) <= lr * (1 + 1e-3)


def go_names():
    return [name for name, _ in M.SHAPES]


def test_output_bias_only_closed_form_on_gpu():
    torch = _torch()
    theta = _init(5)
    blk = _blocks(theta)
    blk["w3"][:] = 0.0
    blk["b3"][0] = 0.75
    n = 300
    X, y = _data(6, n)
    logits = torch.empty(n, dtype=torch.float32, device="cuda")
    ctx().mlp_forward_async(_dev(theta), _dev(X), logits, _ws(n))
    grad = torch.empty(B.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ctx().mlp_grad_async(_dev(theta), _dev(X), _dev(y), grad, loss, _ws(n))
    ctx().sync()
    assert np.all(logits.cpu().numpy() == np.float32(0.75))
    g = grad.cpu().numpy()
    assert abs(g[-1] - (1 / (1 + math.exp(-0.75)) - y.mean())) <= 1e-6
    gb = _blocks(g)
    for name in ("W1", "b1", "W2", "b2"):
        assert np.all(gb[name] == 0.0), name


def test_training_on_gpu_tracks_oracle_and_reduces_loss():
    torch = _torch()
    n, lr, steps = 1024, 2e-3, 30
    theta = _init(8)
    rng = np.random.default_rng(9)
    X = rng.normal(size=(n, M.D_IN)).astype(np.float32).astype(np.float64)
    y = ((X[:, 0] - 0.7 * X[:, 3] + 0.2 * X[:, 5]) > 0.3).astype(np.float64)
    p = _dev(theta)
    m = torch.zeros(B.MLP_PARAMS, dtype=torch.float32, device="cuda")
    v = torch.zeros(B.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    Xd, yd, ws = _dev(X), _dev(y), _ws(n)
    gl = []
    for t in range(1, steps + 1):
        ctx().mlp_train_step_async(p, m, v, t, Xd, yd, lr, loss, ws)
        gl.append(loss.item())
    ot, om, ov = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    ol = []
    for t in range(1, steps + 1):
        g, l = M.grad(ot, X, y)
        ol.append(l)
        ot, om, ov = M.adam_step(ot, om, ov, g, t, lr)
    assert gl[-1] < 0.5 * gl[0]
    assert np.max(np.abs(np.array(gl) - np.array(ol))) <= 1e-3 * max(ol)


def test_network_argument_errors():
    torch = _torch()
    p = torch.zeros(B.MLP_PARAMS, dtype=torch.float32, device="cuda")
    X = torch.zeros(4 * 128, dtype=torch.float32, device="cuda")
    y = torch.zeros(4, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    with pytest.raises(B.RcError):       # workspace too small
        ctx().mlp_forward_async(p, X, y, torch.empty(64, dtype=torch.uint8, device="cuda"))
    with pytest.raises(B.RcError):       # Adam steps count from 1
        ctx().mlp_train_step_async(p, p.clone(), p.clone(), 0, X, y, 1e-3, loss, _ws(4))
    with pytest.raises(ValueError):      # wrong parameter count
        ctx().mlp_forward_async(p[:10], X, y, _ws(4))


def test_gradient_over_a_row_list_matches_oracle_on_those_rows():
    torch = _torch()
    total, n = 900, 300
    theta = _init(21)
    X, y = _clear_data(theta, 22, total)
    rows = np.random.default_rng(23).permutation(total)[:n].astype(np.int32)
    grad = torch.empty(B.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ctx().mlp_grad_async(_dev(theta), _dev(X), _dev(y), grad, loss, _ws(n), rows=torch.from_numpy(rows).cuda())
    ctx().sync()
    g, l = M.grad(theta, X[rows], y[rows])
    assert abs(loss.item() - l) <= 1e-5 * max(1.0, abs(l))
    _assert_grad_close(grad.cpu().numpy().astype(np.float64), g)


# ---------------------------------------------------------------------------
# ranking
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 7, 1000, 70001])
def test_rank_orders_by_score_then_index(n):
    torch = _torch()
    rng = np.random.default_rng(n)
    s = rng.normal(size=n).astype(np.float32)
    if n > 10:
        s[rng.integers(0, n, n // 5)] = 0.5          # ties
        s[rng.integers(0, n, 3)] = -0.0
        s[rng.integers(0, n, 3)] = np.inf
        s[rng.integers(0, n, 3)] = -np.inf
        s[rng.integers(0, n, 2)] = np.nan
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = torch.empty(B.Context.rank_workspace_size(n), dtype=torch.uint8, device="cuda")
    ctx().rank_async(torch.from_numpy(s).cuda(), order, ws)
    ctx().sync()
    got = order.cpu().numpy()
    key = np.where(np.isnan(s), -np.inf, s).astype(np.float64)
    nan_last = np.isnan(s).astype(np.int64)
    # -0.0 and +0.0 are different keys on the GPU (bit order): +0.0 ranks first
    negzero = ((s == 0) & np.signbit(s)).astype(np.int64)
    want = np.lexsort((np.arange(n), negzero, -key, nan_last))
    assert np.array_equal(got, want)


# ---------------------------------------------------------------------------
# the learned order against the plain one
# ---------------------------------------------------------------------------
def test_learned_order_finds_races_sooner_than_plain_order():
    from paper_1308_3203_amd import triage as T
    # many programs with few seeds each, as the benchmark runs it (the
    # network has to generalise across programs); held-out programs from a
    # disjoint range of generator seeds
    train = [WL.c3_kernel(s) for s in range(12000)]
    held = [WL.c3_kernel(1000000 + s) for s in range(1500)]
    r = T.run(ctx(), train, 2, held, 2, epochs=10, batch=1024, lr=2e-3, chunk=100, label_chunk=4000,
              ws_bytes=8 << 30)
    rep = r.report
    print("triage:", rep, "losses", r.losses[0], r.losses[-1], "train racy", r.train_racy_frac, flush=True)
    assert rep.n_racy > 0
    # within a quarter of the plain sweep's GPU time the learned order reaches
    # most racy instances and nearly every RACE record, far more than the
    # plain order does
    assert rep.recall_instances >= 0.9
    assert rep.recall_records >= 0.95
    assert rep.recall_instances >= rep.plain_recall_instances + 0.3
    # (records per GPU-second over the same budget: with the records spread
    # over many programs the plain order finds about the budget's fraction
    # of them, so the ratio cannot pass about 1 / budget_frac = 4)
    assert rep.races_per_gpu_s_learned >= 3 * rep.races_per_gpu_s_plain
    # and more than the orders without the network: a random permutation
    # and the static count of candidate conflicting pairs
    assert set(rep.orders) == {"learned", "plain", "random", "static_heuristic"}
    for base in ("random", "static_heuristic"):
        assert rep.recall_records >= rep.orders[base].recall_records, base
    # every curve ends with the plain sweep's GPU time spent and is monotone
    for o in rep.orders.values():
        inst = [c[1] for c in o.curve]
        assert inst == sorted(inst)
