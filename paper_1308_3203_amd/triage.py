"""Learned triage of a race-check sweep.

A small network scores every (program, seed) instance for how likely the
exact check is to report a race in it; the sweep then checks instances in
descending score order, so racy instances are found early.  Every instance
the sweep reaches is still checked exactly by the library, and the plain
sweep (instances in index order) is the reference the learned order is
measured against.  Labels come from the exact checker itself.

Every computation runs in the HIP library: features (rc_features), the
network's forward, gradient and Adam steps (rc_mlp_*), the ranking (rc_rank)
and the checks (rc_batch_check).  This module only moves buffers and loops
over minibatches and chunks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import binding as B


def _torch():
    import torch
    return torch


# ---------------------------------------------------------------------------
# instance sets
# ---------------------------------------------------------------------------
@dataclass
class Instances:
    """Instances (programs[prog[i]], seed[i]) of a set of loaded programs."""
    programs: list                 # binding.Program, shaped and bound
    prog: np.ndarray               # int64 [n] program index per instance
    seed: np.ndarray               # uint64 [n]
    handles: np.ndarray = field(init=False)

    def __post_init__(self):
        self.handles = B.handles_of(self.programs)

    def __len__(self):
        return int(self.prog.size)

    @staticmethod
    def grid(programs, seeds_per_program: int, seed0: int = 0) -> "Instances":
        n_p = len(programs)
        prog = np.repeat(np.arange(n_p, dtype=np.int64), seeds_per_program)
        seed = np.tile(np.arange(seed0, seed0 + seeds_per_program, dtype=np.uint64), n_p)
        return Instances(list(programs), prog, seed)


def load_programs(ctx: B.Context, workloads) -> list:
    out = []
    for w in workloads:
        p = B.Program(ctx, w.src)
        p.set_ndrange(w.G, w.W)
        p.bind(w.arrays, w.scalars)
        out.append(p)
    return out


def features(ctx: B.Context, inst: Instances, batch: int = 1 << 18):
    """float32 device tensor [n, 128] of triage features."""
    torch = _torch()
    n = len(inst)
    feat = torch.empty((max(n, 1), B.N_FEATURES), dtype=torch.float32, device="cuda")
    n_progs = len(inst.programs)
    ws = torch.empty(B.Context.features_workspace_size(min(batch, max(n, 1)), n_progs), dtype=torch.uint8,
                     device="cuda")
    for a in range(0, n, batch):
        b = min(n, a + batch)
        ctx.features_async(inst.handles[inst.prog[a:b]], inst.seed[a:b], feat[a:b].reshape(-1), ws)
    return feat[:n]


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------
def init_params(seed: int = 7) -> np.ndarray:
    """He-normal hidden layers, small output layer, zero biases (float32)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, math.sqrt(2 / 128), (256, 128))
    W2 = rng.normal(0, math.sqrt(2 / 256), (256, 256))
    w3 = rng.normal(0, 1 / 16, 256)
    return np.concatenate([W1.ravel(), np.zeros(256), W2.ravel(), np.zeros(256), w3, np.zeros(1)]).astype(np.float32)


class TriageNet:
    def __init__(self, ctx: B.Context, seed: int = 7):
        torch = _torch()
        self.ctx = ctx
        self.params = torch.from_numpy(init_params(seed)).cuda()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._ws = None

    def _workspace(self, n: int):
        torch = _torch()
        need = B.Context.mlp_workspace_size(n)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        return self._ws

    def train(self, feat, labels, epochs: int = 5, batch: int = 4096, lr: float = 1e-3, shuffle_seed: int = 7,
              copies=None):
        """Adam on minibatches of a seeded permutation each epoch; returns the
        loss of each epoch's last minibatch (read back once per epoch).
        copies (int array, one per row, or None): how many times each row
        appears in an epoch; a row seen k times weighs k times in the loss."""
        torch = _torch()
        n = feat.shape[0]
        rows_all = np.arange(n, dtype=np.int32) if copies is None else np.repeat(
            np.arange(n, dtype=np.int32), np.asarray(copies, dtype=np.int64))
        total = rows_all.size
        batch = min(batch, total)
        rng = np.random.default_rng(shuffle_seed)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        ws = self._workspace(batch)
        flat = feat.reshape(-1)
        history = []
        for _ in range(epochs):
            # the kernels read each minibatch's rows through the index list
            perm = torch.from_numpy(rows_all[rng.permutation(total)]).cuda()
            for a in range(0, total - batch + 1, batch):      # full batches only
                self.step += 1
                self.ctx.mlp_train_step_async(self.params, self.m, self.v, self.step, flat, labels, lr, loss, ws,
                                              rows=perm[a:a + batch])
            history.append(float(loss.item()))            # loss of the epoch's last minibatch
        return history

    def scores(self, feat, batch: int = 1 << 16):
        torch = _torch()
        n = feat.shape[0]
        out = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        ws = self._workspace(min(batch, max(n, 1)))
        for a in range(0, n, batch):
            b = min(n, a + batch)
            self.ctx.mlp_forward_async(self.params, feat[a:b].reshape(-1), out[a:b], ws)
        return out[:n]


def rank(ctx: B.Context, scores):
    """Device int32 tensor: instance indices by descending score, ties by index."""
    torch = _torch()
    n = scores.numel()
    order = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    ws = torch.empty(B.Context.rank_workspace_size(max(n, 1)), dtype=torch.uint8, device="cuda")
    if n:
        ctx.rank_async(scores, order[:n], ws)
    return order[:n]


# ---------------------------------------------------------------------------
# sweeps
# ---------------------------------------------------------------------------
@dataclass
class SweepResult:
    order: np.ndarray          # instance indices in visiting order
    chunk_end: np.ndarray      # index into order where each chunk ends
    chunk_ms: np.ndarray       # GPU time of each chunk's check
    racy: np.ndarray           # bool per instance (original index): any RACE record
    race_cells: np.ndarray     # RACE records per instance (original index)

    def cumulative(self, start_ms: float = 0.0):
        """(cumulative GPU ms, racy instances, race records) after each chunk."""
        t = start_ms + np.cumsum(self.chunk_ms)
        racy_o = self.racy[self.order].astype(np.int64)
        cells_o = self.race_cells[self.order]
        c_racy = np.cumsum(racy_o)[self.chunk_end - 1]
        c_cells = np.cumsum(cells_o)[self.chunk_end - 1]
        return t, c_racy, c_cells


def sweep(ctx: B.Context, inst: Instances, order=None, chunk: int = 2000, ws_bytes: int = 16 << 30,
          rec_cap: int = 1 << 22, ws=None) -> SweepResult:
    """Check every instance, in `order` (default: index order), `chunk`
    instances per rc_batch_check call, timing each call by the library's HIP
    event spans around its kernels.  Records are counted per instance; record
    buffers that overflow only truncate the written list, not the counts.
    `ws`: a workspace to use (else one of ws_bytes is allocated)."""
    torch = _torch()
    n = len(inst)
    order = np.arange(n, dtype=np.int64) if order is None else np.asarray(order, dtype=np.int64)
    if ws is None:
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    records = torch.empty(rec_cap * B.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    n_rec = torch.zeros(1, dtype=torch.int64, device="cuda")
    summ = torch.empty(chunk * B.SUMMARY_BYTES, dtype=torch.uint8, device="cuda")
    racy = np.zeros(n, dtype=bool)
    cells = np.zeros(n, dtype=np.int64)
    ends, times = [], []
    ctx.profile(True)
    try:
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            ids = order[a:b]
            ctx.batch_check_async(inst.handles[inst.prog[ids]], inst.seed[ids], ws, records, n_rec, summ)
            try:
                ctx.sync()
            except B.RcError as err:
                if err.status != B.RC_E_OVERFLOW:
                    raise
            # GPU time of the call: its kernels' event spans, without host gaps
            times.append(sum(ms for ms, _ in ctx.profile_read().values()))
            s = B.summaries_to_numpy(summ, b - a)
            if np.any(s["flags"] & 2):
                raise RuntimeError("staging overflow in the sweep: counts would be incomplete")
            racy[ids] = s["n_race_cells"] > 0
            cells[ids] = s["n_race_cells"]
            ends.append(b)
    finally:
        ctx.profile(False)
    return SweepResult(order, np.array(ends, dtype=np.int64), np.array(times), racy, cells)


@dataclass
class OrderResult:
    """What one visiting order finds within the budget."""
    recall_instances: float      # racy instances found within budget / all racy instances
    recall_records: float        # RACE records found within budget / all RACE records
    races_per_gpu_s: float       # RACE records found per GPU-second of the budget
    curve: list                  # (fraction of the plain sweep's GPU time, instance recall, record recall)


@dataclass
class TriageReport:
    plain_ms: float
    budget_frac: float
    inference_ms: float
    recall_instances: float      # learned order (inference counted)
    recall_records: float
    plain_recall_instances: float
    races_per_gpu_s_learned: float
    races_per_gpu_s_plain: float
    n_racy: int
    n_race_records: int
    orders: dict = field(default_factory=dict)   # name -> OrderResult: learned, plain and the baselines


def order_result(res: SweepResult, start_ms: float, plain_ms: float, budget_frac: float, n_racy: int,
                 n_cells: int, points: int = 24) -> OrderResult:
    t, c_racy, c_cells = res.cumulative(start_ms)
    budget = budget_frac * plain_ms
    k = np.searchsorted(t, budget, side="right")
    got_i = int(c_racy[k - 1]) if k > 0 else 0
    got_c = int(c_cells[k - 1]) if k > 0 else 0
    curve = []
    for f in np.linspace(0.0, 1.0, points + 1)[1:]:
        j = np.searchsorted(t, f * plain_ms, side="right")
        curve.append((round(float(f), 4), round((int(c_racy[j - 1]) if j > 0 else 0) / max(1, n_racy), 4),
                      round((int(c_cells[j - 1]) if j > 0 else 0) / max(1, n_cells), 4)))
    return OrderResult(got_i / max(1, n_racy), got_c / max(1, n_cells),
                       got_c / (budget * 1e-3) if budget > 0 else 0.0, curve)


def evaluate(plain: SweepResult, learned: SweepResult, inference_ms: float, budget_frac: float = 0.25,
             baselines: dict | None = None) -> TriageReport:
    """Recall of the learned order within budget_frac of the plain sweep's GPU
    time (inference counted), against everything the plain sweep found; the
    same for the plain order and for baseline orders (name -> (sweep, GPU
    time spent before it starts))."""
    T = float(plain.chunk_ms.sum())
    n_racy = int(plain.racy.sum())
    n_cells = int(plain.race_cells.sum())
    orders = {"learned": order_result(learned, inference_ms, T, budget_frac, n_racy, n_cells),
              "plain": order_result(plain, 0.0, T, budget_frac, n_racy, n_cells)}
    for name, (res, start) in (baselines or {}).items():
        orders[name] = order_result(res, start, T, budget_frac, n_racy, n_cells)
    L, P = orders["learned"], orders["plain"]
    return TriageReport(
        plain_ms=T, budget_frac=budget_frac, inference_ms=inference_ms,
        recall_instances=L.recall_instances, recall_records=L.recall_records,
        plain_recall_instances=P.recall_instances,
        races_per_gpu_s_learned=L.races_per_gpu_s, races_per_gpu_s_plain=P.races_per_gpu_s,
        n_racy=n_racy, n_race_records=n_cells, orders=orders)


def static_heuristic(feat_host: np.ndarray) -> np.ndarray:
    """The baseline without a network: the number of candidate conflicting
    access pairs the affine index analysis finds (features 16..23: stores
    every work-item aims at one cell, non-affine stores, overlapping affine
    pairs, pairs across loops holding a barrier), higher first, ties by
    index."""
    score = feat_host[:, 16:24].astype(np.float64).sum(axis=1)
    return np.lexsort((np.arange(score.size), -score))


def timed(fn):
    """Run fn() between two events on the current stream; (result, GPU ms)."""
    torch = _torch()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    out = fn()
    e1.record(s)
    e1.synchronize()
    return out, e0.elapsed_time(e1)


# ---------------------------------------------------------------------------
# the whole experiment: label, train, score, sweep in both orders
# ---------------------------------------------------------------------------
@dataclass
class TriageRun:
    report: TriageReport
    losses: list
    label_ms: float            # GPU time of the labelling sweep
    train_ms: float            # GPU time of training (features + Adam steps)
    n_train: int
    n_eval: int
    train_racy_frac: float


def record_copies(race_cells: np.ndarray) -> np.ndarray:
    """Rows per training instance: 1, plus floor(log2(1 + RACE records)) for a
    racy instance, so that instances with many records weigh more and the
    order finds records, not only racy instances, early."""
    return 1 + np.floor(np.log2(1.0 + race_cells.astype(np.float64))).astype(np.int64)


def run(ctx: B.Context, train_workloads, train_seeds: int, eval_workloads, eval_seeds: int, epochs: int = 5,
        batch: int = 4096, lr: float = 1e-3, chunk: int = 2000, label_chunk: int = 20000, init_seed: int = 7,
        ws_bytes: int = 16 << 30, budget_frac: float = 0.25, progress=None, weight_records: bool = False,
        baselines: bool = True) -> TriageRun:
    torch = _torch()
    say = progress or (lambda msg: None)
    train = Instances.grid(load_programs(ctx, train_workloads), train_seeds)
    held = Instances.grid(load_programs(ctx, eval_workloads), eval_seeds)
    say(f"loaded {len(train_workloads)} + {len(eval_workloads)} programs")
    # one workspace for every sweep (a large one freed and asked for again
    # may not fit beside what the caching allocator keeps)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    # labels from the exact checker
    lab = sweep(ctx, train, chunk=label_chunk, ws=ws)
    say(f"labelled {len(train)} instances ({int(lab.racy.sum())} racy)")
    labels = torch.from_numpy(lab.racy.astype(np.float32)).cuda()
    net = TriageNet(ctx, seed=init_seed)

    copies = record_copies(lab.race_cells) if weight_records else None

    def fit():
        f = features(ctx, train)
        return net.train(f, labels, epochs=epochs, batch=batch, lr=lr, copies=copies)
    losses, train_ms = timed(fit)
    say(f"trained: losses {losses}")
    # warm the held-out programs' tables, then the plain sweep
    sweep(ctx, Instances(held.programs, held.prog[:64], held.seed[:64]), chunk=chunk, ws=ws)
    plain = sweep(ctx, held, chunk=chunk, ws=ws)
    say("plain sweep done")

    def infer():
        return rank(ctx, net.scores(features(ctx, held)))
    order_dev, infer_ms = timed(infer)
    order = order_dev.cpu().numpy().astype(np.int64)
    learned = sweep(ctx, held, order=order, chunk=chunk, ws=ws)
    if not np.array_equal(learned.racy, plain.racy) or not np.array_equal(learned.race_cells, plain.race_cells):
        raise RuntimeError("the two sweeps disagree on an instance: the exact check must not depend on the order")
    base = {}
    if baselines:
        # a seeded random order, and the static heuristic (its features are
        # computed on the GPU like the network's; the ordering is counted as
        # the same feature time)
        rnd = np.random.default_rng(12345).permutation(len(held)).astype(np.int64)
        base["random"] = (sweep(ctx, held, order=rnd, chunk=chunk, ws=ws), 0.0)
        fh, feat_ms = timed(lambda: features(ctx, held))
        heur = static_heuristic(fh.cpu().numpy())
        base["static_heuristic"] = (sweep(ctx, held, order=heur, chunk=chunk, ws=ws), feat_ms)
        say("baseline sweeps done")
    rep = evaluate(plain, learned, infer_ms, budget_frac, base)
    return TriageRun(rep, losses, float(lab.chunk_ms.sum()), train_ms, len(train), len(held),
                     float(lab.racy.mean()) if len(train) else 0.0)
