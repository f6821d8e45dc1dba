"""Thin Python binding of the race-checker C ABI (include/rc.h).

Argument marshalling only: every step of the check runs in the HIP library
``librc.so``.  torch supplies device memory (workspace, record and summary
buffers) and the stream.  There is no CPU fallback: without the built library
every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librc.so")

RC_OK, RC_E_INVAL, RC_E_PARSE, RC_E_LIMIT, RC_E_STATE, RC_E_OVERFLOW, RC_E_HIP = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", 1: "OOB", 2: "DIV_ZERO", 3: "ASSERT", 4: "ASSUME", 5: "BARRIER_DIVERGENCE",
                6: "STEP_LIMIT"}
NONE = 0xFFFFFFFF

RECORD_DTYPE = np.dtype([
    ("instance", "<u4"), ("gid", "<u4"), ("interval", "<u4"),
    ("array", "<u2"), ("label", "<u2"), ("cell", "<u4"),
    ("rw_a", "<u4"), ("rw_b", "<u4"), ("ww_a", "<u4"), ("ww_b", "<u4"), ("pad", "<u4"),
])
SUMMARY_DTYPE = np.dtype([
    ("n_accesses", "<u8"), ("n_race_cells", "<u4"), ("n_benign_cells", "<u4"),
    ("n_intervals", "<u4"), ("status", "<i4"), ("fault_gid", "<u4"),
    ("fault_pc", "<u4"), ("fault_tid", "<u4"), ("flags", "<u4"),
])
RECORD_BYTES = 40
SUMMARY_BYTES = 40

EXPORTS = [
    "rc_last_error", "rc_ctx_create", "rc_ctx_destroy", "rc_ctx_set_stream", "rc_prog_load",
    "rc_prog_free", "rc_prog_get_info", "rc_prog_array", "rc_prog_scalar", "rc_set_ndrange",
    "rc_bind_seeded", "rc_bind_device", "rc_bind_scalar_seeded", "rc_bind_scalar",
    "rc_workspace_size", "rc_check", "rc_sync", "rc_read_final", "rc_ctx_profile",
    "rc_ctx_profile_read", "rc_prog_set_tuning", "rc_batch_check", "rc_autotune",
    "rc_features_workspace_size", "rc_features", "rc_mlp_workspace_size", "rc_mlp_forward", "rc_mlp_grad",
    "rc_mlp_train_step", "rc_rank_workspace_size", "rc_rank", "rc_prog_jit", "rc_prog_owned",
    "rc_owned_arrays",
    "rc_log_intervals", "rc_call_stats", "rc_check_static",
]
N_FEATURES = 128
MLP_PARAMS = 99073
PHASES = ["interpret", "log_sort", "interval_check", "record_sort", "output", "setup"]


class RcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rc status {status}: {msg}")
        self.status = status


class _Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("launches", ctypes.c_uint32 * 8)]


class _Stats(ctypes.Structure):
    _fields_ = [("logged", ctypes.c_uint64), ("logged_global", ctypes.c_uint64),
                ("intervals_spilled", ctypes.c_uint64), ("intervals", ctypes.c_uint64),
                ("instructions", ctypes.c_uint64), ("wave_instructions", ctypes.c_uint64),
                ("global_pass", ctypes.c_uint64)]


class _Tuning(ctypes.Structure):
    _fields_ = [("lds_log_entries", ctypes.c_uint32), ("radix_bits", ctypes.c_uint32),
                ("record_sort", ctypes.c_uint32), ("proofs_off", ctypes.c_uint32),
                ("step_limit", ctypes.c_uint32), ("global_spills", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 2)]


class _ProgInfo(ctypes.Structure):
    _fields_ = [("n_global_arrays", ctypes.c_uint32), ("n_local_arrays", ctypes.c_uint32),
                ("n_scalars", ctypes.c_uint32), ("n_vars", ctypes.c_uint32), ("n_stmts", ctypes.c_uint32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1308_3203_amd/build.py "
                           "(there is no CPU fallback)")
    # torch ships its own HIP runtime; it has to be in the process before the
    # library pulls in a runtime of its own, or the two do not share devices
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, u32, u64, i32, i64, sz = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                                  ctypes.c_int64, ctypes.c_size_t)
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "rc_last_error": ([], ctypes.c_char_p),
        "rc_ctx_create": ([ctypes.c_int, vp, pp], ctypes.c_int),
        "rc_ctx_destroy": ([vp], ctypes.c_int),
        "rc_ctx_set_stream": ([vp, vp], ctypes.c_int),
        "rc_prog_load": ([vp, ctypes.c_char_p, sz, pp], ctypes.c_int),
        "rc_prog_free": ([vp], ctypes.c_int),
        "rc_prog_get_info": ([vp, ctypes.POINTER(_ProgInfo)], ctypes.c_int),
        "rc_prog_array": ([vp, u32, ctypes.c_char_p, sz, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_int)],
                          ctypes.c_int),
        "rc_prog_scalar": ([vp, u32, ctypes.c_char_p, sz], ctypes.c_int),
        "rc_set_ndrange": ([vp, u32, u32], ctypes.c_int),
        "rc_prog_owned": ([vp, u32, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "rc_owned_arrays": ([ctypes.c_char_p, sz, u32, u32, ctypes.POINTER(ctypes.c_uint8), u32,
                             ctypes.POINTER(u32), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "rc_log_intervals": ([ctypes.c_char_p, sz, u32, u32, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_int)],
                             ctypes.c_int),
        "rc_bind_seeded": ([vp, u32, i64, i64], ctypes.c_int),
        "rc_bind_device": ([vp, u32, vp], ctypes.c_int),
        "rc_bind_scalar_seeded": ([vp, u32, i64, i64], ctypes.c_int),
        "rc_bind_scalar": ([vp, u32, i32], ctypes.c_int),
        "rc_workspace_size": ([vp, u32, ctypes.POINTER(sz)], ctypes.c_int),
        "rc_check": ([vp, u64, u32, vp, sz, vp, u64, vp, vp], ctypes.c_int),
        "rc_check_static": ([vp, u64, u32, vp, u64, vp, vp], ctypes.c_int),
        "rc_sync": ([vp], ctypes.c_int),
        "rc_read_final": ([vp, u64, u32, vp, vp, sz], ctypes.c_int),
        "rc_ctx_profile": ([vp, ctypes.c_int], ctypes.c_int),
        "rc_ctx_profile_read": ([vp, ctypes.POINTER(_Profile)], ctypes.c_int),
        "rc_call_stats": ([vp, ctypes.POINTER(_Stats)], ctypes.c_int),
        "rc_prog_set_tuning": ([vp, ctypes.POINTER(_Tuning)], ctypes.c_int),
        "rc_autotune": ([vp, u64, u32, vp, sz, ctypes.c_char_p, ctypes.POINTER(_Tuning)], ctypes.c_int),
        "rc_batch_check": ([vp, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_uint64), u32, vp, sz,
                            vp, u64, vp, vp], ctypes.c_int),
        "rc_features_workspace_size": ([u32, u32, ctypes.POINTER(sz)], ctypes.c_int),
        "rc_features": ([vp, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_uint64), u32, vp, vp, sz],
                        ctypes.c_int),
        "rc_mlp_workspace_size": ([u32, ctypes.POINTER(sz)], ctypes.c_int),
        "rc_rank_workspace_size": ([u32, ctypes.POINTER(sz)], ctypes.c_int),
        "rc_rank": ([vp, vp, u32, vp, vp, sz], ctypes.c_int),
        "rc_prog_jit": ([vp, ctypes.c_int], ctypes.c_int),
        "rc_mlp_forward": ([vp, vp, vp, u32, vp, vp, sz], ctypes.c_int),
        "rc_mlp_grad": ([vp, vp, vp, vp, vp, u32, vp, vp, vp, sz], ctypes.c_int),
        "rc_mlp_train_step": ([vp, vp, vp, vp, u32, vp, vp, vp, u32, ctypes.c_float, vp, vp, sz], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _call(fn, *args):
    st = fn(*args)
    if st != RC_OK:
        raise RcError(st, _lib.rc_last_error().decode())
    return st


def owned_arrays(src: str, groups: int, group_size: int, with_faults: bool = False, race_free: bool = False):
    """Per array (global arrays first, then local ones): True when no two
    work-items of the shape can touch a common cell of it (host only).
    race_free: instead, True for the local arrays that are not owned but
    race-free within every barrier interval (never logged either).
    with_faults: also return whether the program is proven never to fault."""
    lib = load_library()
    b = src.encode()
    n = ctypes.c_uint32(0)
    nf = ctypes.c_int(0)
    _call(lib.rc_owned_arrays, b, len(b), groups, group_size, None, 0, ctypes.byref(n), None)
    out = (ctypes.c_uint8 * max(1, n.value))()
    _call(lib.rc_owned_arrays, b, len(b), groups, group_size, out, n.value, ctypes.byref(n), ctypes.byref(nf))
    owned = [out[i] == (2 if race_free else 1) for i in range(n.value)]
    return (owned, bool(nf.value)) if with_faults else owned


def log_intervals(src: str, groups: int, group_size: int):
    """(mask, later): the barrier intervals whose local-array accesses are
    logged under the shape (bit k: interval k < 64; later: every interval
    from 64 on), host only."""
    lib = load_library()
    b = src.encode()
    m = ctypes.c_uint64(0)
    later = ctypes.c_int(0)
    _call(lib.rc_log_intervals, b, len(b), groups, group_size, ctypes.byref(m), ctypes.byref(later))
    return int(m.value), bool(later.value)


class Context:
    """A library context on one device, bound to a torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        lib = load_library()
        self.device = device
        self._torch_stream = stream if stream is not None else torch.cuda.current_stream(device)
        out = ctypes.c_void_p()
        _call(lib.rc_ctx_create, device, ctypes.c_void_p(self._torch_stream.cuda_stream), ctypes.byref(out))
        self._h = out

    def sync(self):
        _call(_lib.rc_sync, self._h)

    def batch_check_async(self, programs, seeds, ws, records, n_records, summaries):
        """Enqueue a check of instances (programs[i], seeds[i]) into caller-owned
        buffers.  `programs` is a list of Program or a numpy uint64 array of
        handles (see handles()); `seeds` any integer sequence."""
        if isinstance(programs, np.ndarray):
            handles = np.ascontiguousarray(programs, dtype=np.uint64)
        else:
            handles = handles_of(programs)
        sarr = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
        n = int(handles.size)
        cap = records.numel() // RECORD_BYTES
        _call(_lib.rc_batch_check, self._h, handles.ctypes.data_as(ctypes.POINTER(ctypes.c_void_p)),
              sarr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n, ctypes.c_void_p(ws.data_ptr()),
              ws.numel(), ctypes.c_void_p(records.data_ptr() if cap else 0), cap,
              ctypes.c_void_p(n_records.data_ptr()), ctypes.c_void_p(summaries.data_ptr()))

    def profile(self, enable: bool = True):
        _call(_lib.rc_ctx_profile, self._h, 1 if enable else 0)

    # ---- triage -------------------------------------------------------------
    @staticmethod
    def features_workspace_size(n: int, n_programs: int) -> int:
        out = ctypes.c_size_t()
        _call(load_library().rc_features_workspace_size, n, n_programs, ctypes.byref(out))
        return out.value

    def features_async(self, programs, seeds, feat, ws):
        """Triage features of instances (programs[i], seeds[i]) into the float32
        device tensor feat [n, 128]."""
        handles = (np.ascontiguousarray(programs, dtype=np.uint64) if isinstance(programs, np.ndarray)
                   else handles_of(programs))
        sarr = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
        n = int(handles.size)
        _check_f32(feat, n * N_FEATURES, "feat")
        _call(_lib.rc_features, self._h, handles.ctypes.data_as(ctypes.POINTER(ctypes.c_void_p)),
              sarr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n, ctypes.c_void_p(feat.data_ptr()),
              ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size())

    @staticmethod
    def rank_workspace_size(n: int) -> int:
        out = ctypes.c_size_t()
        _call(load_library().rc_rank_workspace_size, n, ctypes.byref(out))
        return out.value

    def rank_async(self, scores, order, ws):
        """order (int32/uint32 device tensor of n) = indices by descending score."""
        import torch
        n = scores.numel()
        _check_f32(scores, n, "scores")
        if order.numel() != n or order.dtype not in (torch.int32,) or not order.is_cuda:
            raise ValueError("order: expected an int32 device tensor of n elements")
        _call(_lib.rc_rank, self._h, _p(scores), n, _p(order), _p(ws), ws.numel() * ws.element_size())

    @staticmethod
    def mlp_workspace_size(n: int) -> int:
        out = ctypes.c_size_t()
        _call(load_library().rc_mlp_workspace_size, n, ctypes.byref(out))
        return out.value

    def mlp_forward_async(self, params, feat, logits, ws):
        n = logits.numel()
        _check_f32(params, MLP_PARAMS, "params")
        _check_f32(feat, n * N_FEATURES, "feat")
        _call(_lib.rc_mlp_forward, self._h, _p(params), _p(feat), n, _p(logits), _p(ws),
              ws.numel() * ws.element_size())

    @staticmethod
    def _batch(feat, labels, rows):
        """(n, rows pointer) of a minibatch: all rows, or the int32 row list."""
        import torch
        total = labels.numel()
        _check_f32(labels, total, "labels")
        _check_f32(feat, total * N_FEATURES, "feat")
        if rows is None:
            return total, ctypes.c_void_p(0)
        if rows.dtype != torch.int32 or not rows.is_cuda or not rows.is_contiguous():
            raise ValueError("rows: expected a contiguous int32 device tensor")
        return rows.numel(), _p(rows)

    def mlp_grad_async(self, params, feat, labels, grad, loss, ws, rows=None):
        n, rp = self._batch(feat, labels, rows)
        for t, k, name in ((params, MLP_PARAMS, "params"), (grad, MLP_PARAMS, "grad"), (loss, 1, "loss")):
            _check_f32(t, k, name)
        _call(_lib.rc_mlp_grad, self._h, _p(params), _p(feat), _p(labels), rp, n, _p(grad), _p(loss), _p(ws),
              ws.numel() * ws.element_size())

    def mlp_train_step_async(self, params, m, v, step: int, feat, labels, lr: float, loss, ws, rows=None):
        """One Adam step on rows `rows` (int32 device tensor, row indices into
        feat / labels; None: every row)."""
        n, rp = self._batch(feat, labels, rows)
        for t, k, name in ((params, MLP_PARAMS, "params"), (m, MLP_PARAMS, "m"), (v, MLP_PARAMS, "v"),
                           (loss, 1, "loss")):
            _check_f32(t, k, name)
        _call(_lib.rc_mlp_train_step, self._h, _p(params), _p(m), _p(v), step, _p(feat), _p(labels), rp, n,
              ctypes.c_float(lr), _p(loss), _p(ws), ws.numel() * ws.element_size())

    def profile_read(self) -> dict:
        """Per-phase {name: (total ms, spans)} since profiling started."""
        out = _Profile()
        _call(_lib.rc_ctx_profile_read, self._h, ctypes.byref(out))
        return {PHASES[i]: (float(out.ms[i]), int(out.launches[i])) for i in range(len(PHASES))}

    def call_stats(self) -> dict:
        """Log statistics of the last check call (waits for the stream)."""
        out = _Stats()
        _call(_lib.rc_call_stats, self._h, ctypes.byref(out))
        return {k: int(getattr(out, k)) for k, _ in _Stats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib.rc_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_f32(t, numel: int, name: str):
    import torch
    if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != numel or not t.is_cuda:
        raise ValueError(f"{name}: expected a contiguous float32 device tensor of {numel} elements")


def handles_of(programs) -> np.ndarray:
    """Library handles of Program objects, for batch_check_async."""
    return np.array([p._h.value for p in programs], dtype=np.uint64)


class Program:
    """A compiled kernel program with its launch shape and input bindings."""

    def __init__(self, ctx: Context, src: str):
        lib = load_library()
        self.ctx = ctx
        self.src = src
        raw = src.encode()
        out = ctypes.c_void_p()
        _call(lib.rc_prog_load, ctx._h, raw, len(raw), ctypes.byref(out))
        self._h = out
        info = _ProgInfo()
        _call(lib.rc_prog_get_info, self._h, ctypes.byref(info))
        self.info = info
        self.arrays = []
        name = ctypes.create_string_buffer(64)
        cells = ctypes.c_uint64()
        glob = ctypes.c_int()
        for i in range(info.n_global_arrays + info.n_local_arrays):
            _call(lib.rc_prog_array, self._h, i, name, 64, ctypes.byref(cells), ctypes.byref(glob))
            self.arrays.append((name.value.decode(), int(cells.value), bool(glob.value)))
        self.scalars = []
        for j in range(info.n_scalars):
            _call(lib.rc_prog_scalar, self._h, j, name, 64)
            self.scalars.append(name.value.decode())
        self._keep = {}
        self.G = self.W = None

    def close(self):
        if getattr(self, "_h", None):
            _lib.rc_prog_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def array_id(self, name: str) -> int:
        for i, (n, _, _) in enumerate(self.arrays):
            if n == name:
                return i
        raise KeyError(name)

    def set_ndrange(self, groups: int, group_size: int):
        _call(_lib.rc_set_ndrange, self._h, groups, group_size)
        self.G, self.W = groups, group_size

    def owned(self, name: str) -> bool:
        """True when the array can carry no record under the current shape,
        so its accesses are not logged: no two work-items can touch a common
        cell of it, or (a local array of a program that cannot fault) no cell
        is written by one work-item and touched by another within an
        interval."""
        v = ctypes.c_int(0)
        _call(_lib.rc_prog_owned, self._h, self.array_id(name), ctypes.byref(v))
        return bool(v.value)

    def bind(self, arrays: dict | None = None, scalars: dict | None = None):
        """arrays: name -> ("seeded", lo, hi) or an int32 cuda tensor;
        scalars: name -> ("seeded", lo, hi) or an int."""
        for name, b in (arrays or {}).items():
            aid = self.array_id(name)
            if isinstance(b, tuple):
                _call(_lib.rc_bind_seeded, self._h, aid, int(b[1]), int(b[2]))
            else:
                t = b.contiguous()
                self._keep[name] = t
                _call(_lib.rc_bind_device, self._h, aid, ctypes.c_void_p(t.data_ptr()))
        for name, b in (scalars or {}).items():
            sid = self.scalars.index(name)
            if isinstance(b, tuple):
                _call(_lib.rc_bind_scalar_seeded, self._h, sid, int(b[1]), int(b[2]))
            else:
                _call(_lib.rc_bind_scalar, self._h, sid, ((int(b) + 2 ** 31) % 2 ** 32) - 2 ** 31)

    def jit(self, enable: bool = True):
        """Compile this program's own kernel (needs the NDRange); single-program
        checks then run it instead of the interpreter."""
        _call(_lib.rc_prog_jit, self._h, 1 if enable else 0)

    def set_tuning(self, lds_log_entries: int = 0, radix_bits: int = 0, record_sort: int = 0,
                   proofs_off: bool = False, step_limit: int = 0, global_spills: bool = False):
        t = _Tuning()
        t.lds_log_entries = lds_log_entries
        t.radix_bits = radix_bits
        t.record_sort = record_sort
        t.proofs_off = 1 if proofs_off else 0
        t.step_limit = step_limit
        t.global_spills = 1 if global_spills else 0
        _call(_lib.rc_prog_set_tuning, self._h, ctypes.byref(t))

    def autotune(self, seed0: int, n_seeds: int, ws, cache_path: str | None = None) -> dict:
        """Pick (and apply) the fastest tuning on a calibration slice."""
        t = _Tuning()
        _call(_lib.rc_autotune, self._h, ctypes.c_uint64(seed0), n_seeds, ctypes.c_void_p(ws.data_ptr()),
              ws.numel(), cache_path.encode() if cache_path else None, ctypes.byref(t))
        return {"lds_log_entries": int(t.lds_log_entries), "radix_bits": int(t.radix_bits)}

    def workspace_size(self, n_seeds: int) -> int:
        out = ctypes.c_size_t()
        _call(_lib.rc_workspace_size, self._h, n_seeds, ctypes.byref(out))
        return int(out.value)

    def check_async(self, seed0: int, n_seeds: int, ws, records, n_records, summaries):
        """Enqueue a check into caller-owned torch buffers (uint8 workspace,
        uint8 records of 40*cap bytes, one int64 counter, uint8 summaries)."""
        cap = records.numel() // RECORD_BYTES
        _call(_lib.rc_check, self._h, ctypes.c_uint64(seed0 & (2 ** 64 - 1)), n_seeds,
              ctypes.c_void_p(ws.data_ptr()), ws.numel(),
              ctypes.c_void_p(records.data_ptr() if cap else 0), cap,
              ctypes.c_void_p(n_records.data_ptr()), ctypes.c_void_p(summaries.data_ptr()))

    def check_static_async(self, seed0: int, n_seeds: int, records, n_records, summaries):
        """check_async with the library's static workspace (rc_check_static):
        no workspace argument, no device allocation."""
        cap = records.numel() // RECORD_BYTES
        _call(_lib.rc_check_static, self._h, ctypes.c_uint64(seed0 & (2 ** 64 - 1)), n_seeds,
              ctypes.c_void_p(records.data_ptr() if cap else 0), cap,
              ctypes.c_void_p(n_records.data_ptr()), ctypes.c_void_p(summaries.data_ptr()))

    def read_final(self, seed: int, name: str, ws):
        import torch
        aid = self.array_id(name)
        out = torch.empty(self.arrays[aid][1], dtype=torch.int32, device=ws.device)
        _call(_lib.rc_read_final, self._h, ctypes.c_uint64(seed & (2 ** 64 - 1)), aid,
              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel())
        return out


class Buffers:
    """Device buffers for checks of up to n_seeds instances."""

    def __init__(self, prog: Program, n_seeds: int, cap: int, ws_limit: int = 8 << 30, device=None):
        import torch
        dev = device or torch.device("cuda", prog.ctx.device)
        need = prog.workspace_size(n_seeds)
        if need > ws_limit:
            need = max(prog.workspace_size(1), ws_limit)
        self.ws = torch.empty(need, dtype=torch.uint8, device=dev)
        self.records = torch.empty(max(cap, 1) * RECORD_BYTES, dtype=torch.uint8, device=dev)
        self.cap = cap
        self.n_records = torch.zeros(1, dtype=torch.int64, device=dev)
        self.summaries = torch.empty(max(n_seeds, 1) * SUMMARY_BYTES, dtype=torch.uint8, device=dev)
        self.n_seeds = n_seeds


def records_to_numpy(records_u8, n: int) -> np.ndarray:
    raw = records_u8[: n * RECORD_BYTES].cpu().numpy()
    return raw.view(RECORD_DTYPE).copy()


def summaries_to_numpy(summ_u8, n: int) -> np.ndarray:
    raw = summ_u8[: n * SUMMARY_BYTES].cpu().numpy()
    return raw.view(SUMMARY_DTYPE).copy()


def check(src: str, G: int, W: int, arrays: dict | None = None, scalars: dict | None = None,
          seed0: int = 0, n_seeds: int = 1, cap: int | None = None, ctx: Context | None = None,
          ws_limit: int = 8 << 30, lds_log_entries: int = 0, jit: bool = False):
    """Compile, bind and check n_seeds instances; returns numpy (records, summaries)."""
    ctx = ctx or Context()
    prog = Program(ctx, src)
    prog.set_ndrange(G, W)
    if jit:
        prog.jit(True)
    if lds_log_entries:
        prog.set_tuning(lds_log_entries)
    prog.bind(arrays, scalars)
    if cap is None:
        cap = 1 << 20
    buf = Buffers(prog, n_seeds, cap, ws_limit)
    prog.check_async(seed0, n_seeds, buf.ws, buf.records, buf.n_records, buf.summaries)
    ctx.sync()
    n = int(buf.n_records.item())
    recs = records_to_numpy(buf.records, min(n, cap))
    summ = summaries_to_numpy(buf.summaries, n_seeds)
    prog.close()
    return recs, summ
