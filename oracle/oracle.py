"""Python handle on the CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  The tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg are the only users.  It never touches the GPU
library and the GPU library never touches it.

``check(src, G, W, arrays=..., scalars=..., seed=...)`` runs one instance of the
concrete SIMD semantics (paper Section 4) and returns its race records, in the
canonical order, plus the per-instance summary.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

RECORD_DTYPE = np.dtype([
    ("instance", "<u4"), ("gid", "<u4"), ("interval", "<u4"),
    ("array", "<u2"), ("label", "<u2"), ("cell", "<u4"),
    ("rw_a", "<u4"), ("rw_b", "<u4"), ("ww_a", "<u4"), ("ww_b", "<u4"), ("pad", "<u4"),
])
assert RECORD_DTYPE.itemsize == 40

SUMMARY_DTYPE = np.dtype([
    ("n_accesses", "<u8"), ("n_race_cells", "<u4"), ("n_benign_cells", "<u4"),
    ("n_intervals", "<u4"), ("status", "<i4"), ("fault_gid", "<u4"),
    ("fault_pc", "<u4"), ("fault_tid", "<u4"), ("flags", "<u4"),
])
assert SUMMARY_DTYPE.itemsize == 40

LABEL_RW, LABEL_WW_DIFF, LABEL_BENIGN = 1, 2, 4
STATUS = {0: "OK", 1: "OOB", 2: "DIV_ZERO", 3: "ASSERT", 4: "ASSUME", 5: "BARRIER_DIVERGENCE", 6: "STEP_LIMIT"}
STEP_LIMIT = 1 << 24   # loop iterations a work-group may start (reading R13's safety net)
NONE = 0xFFFFFFFF


class _Bind(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("lo", ctypes.c_int64), ("hi", ctypes.c_int64),
                ("data", ctypes.POINTER(ctypes.c_int32))]


class _Summary(ctypes.Structure):
    _fields_ = [("n_accesses", ctypes.c_uint64), ("n_race_cells", ctypes.c_uint32),
                ("n_benign_cells", ctypes.c_uint32), ("n_intervals", ctypes.c_uint32),
                ("status", ctypes.c_int32), ("fault_gid", ctypes.c_uint32),
                ("fault_pc", ctypes.c_uint32), ("fault_tid", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class _Result(ctypes.Structure):
    _fields_ = [("records", ctypes.c_void_p), ("n_records", ctypes.c_uint64),
                ("summary", _Summary), ("final_mem", ctypes.POINTER(ctypes.c_int32)),
                ("final_cells", ctypes.c_uint64)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C99, -O2)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_parse.restype = ctypes.c_void_p
        lib.orc_parse.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int]
        lib.orc_prog_free.argtypes = [ctypes.c_void_p]
        for fn in ("orc_n_global_arrays", "orc_n_scalars", "orc_n_local_arrays"):
            getattr(lib, fn).argtypes = [ctypes.c_void_p]
            getattr(lib, fn).restype = ctypes.c_int
        lib.orc_global_array.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p, ctypes.c_int]
        lib.orc_global_array.restype = ctypes.c_int64
        lib.orc_scalar.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p, ctypes.c_int]
        lib.orc_scalar.restype = ctypes.c_int
        lib.orc_run.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.POINTER(_Bind), ctypes.c_int,
                                ctypes.POINTER(_Bind), ctypes.c_int,
                                ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(_Result), ctypes.c_char_p, ctypes.c_int]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_run_limit.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.POINTER(_Bind), ctypes.c_int,
                                      ctypes.POINTER(_Bind), ctypes.c_int,
                                      ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                      ctypes.POINTER(_Result), ctypes.c_char_p, ctypes.c_int]
        lib.orc_run_limit.restype = ctypes.c_int
        lib.orc_result_free.argtypes = [ctypes.POINTER(_Result)]
        lib.orc_seeded_value.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_int64, ctypes.c_int64]
        lib.orc_seeded_value.restype = ctypes.c_int32
        lib.orc_features.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(_Bind),
                                     ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float),
                                     ctypes.c_char_p, ctypes.c_int]
        lib.orc_features.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


@dataclass
class OracleResult:
    records: np.ndarray     # RECORD_DTYPE, canonical order
    summary: np.ndarray     # SUMMARY_DTYPE scalar record
    final: np.ndarray | None = None

    @property
    def status(self) -> str:
        return STATUS[int(self.summary["status"])]


class Program:
    """A parsed program (names and sizes of its parameters)."""

    def __init__(self, src: str):
        lib = _load()
        err = ctypes.create_string_buffer(512)
        self.src = src
        self._p = lib.orc_parse(src.encode(), err, 512)
        if not self._p:
            raise OracleError("parse error: " + err.value.decode())
        self.arrays = []
        name = ctypes.create_string_buffer(64)
        for i in range(lib.orc_n_global_arrays(self._p)):
            size = lib.orc_global_array(self._p, i, name, 64)
            self.arrays.append((name.value.decode(), int(size)))
        self.scalars = []
        for j in range(lib.orc_n_scalars(self._p)):
            lib.orc_scalar(self._p, j, name, 64)
            self.scalars.append(name.value.decode())

    def __del__(self):
        p = getattr(self, "_p", None)
        if p and _lib is not None:
            _lib.orc_prog_free(p)
            self._p = None

    def _array_binds(self, arrays, keep):
        abind = (_Bind * max(1, len(self.arrays)))()
        for i, (name, size) in enumerate(self.arrays):
            b = arrays.get(name, ("seeded", 0, 16))
            if isinstance(b, tuple):
                abind[i].kind, abind[i].lo, abind[i].hi = 0, int(b[1]), int(b[2])
            else:
                data = np.ascontiguousarray(b, dtype=np.int32)
                if data.size != size:
                    raise OracleError(f"array {name}: {data.size} cells bound, {size} declared")
                keep.append(data)
                abind[i].kind = 1
                abind[i].data = data.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        return abind

    def features(self, G: int, W: int, arrays: dict | None = None, seed: int = 0) -> np.ndarray:
        """The 128 float32 triage features of one instance."""
        lib = _load()
        keep = []
        abind = self._array_binds(arrays or {}, keep)
        out = np.zeros(128, dtype=np.float32)
        err = ctypes.create_string_buffer(256)
        rc = lib.orc_features(self._p, G, W, abind, len(self.arrays), ctypes.c_uint64(seed & (2**64 - 1)),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), err, 256)
        if rc != 0:
            raise OracleError(err.value.decode())
        return out

    def run(self, G: int, W: int, arrays: dict | None = None, scalars: dict | None = None,
            seed: int = 0, instance: int = 0, literal: bool = False,
            final: str | None = None, step_limit: int = STEP_LIMIT) -> OracleResult:
        lib = _load()
        arrays = arrays or {}
        scalars = scalars or {}
        keep = []
        abind = self._array_binds(arrays, keep)
        sbind = (_Bind * max(1, len(self.scalars)))()
        for j, name in enumerate(self.scalars):
            b = scalars.get(name, ("seeded", 0, 16))
            if isinstance(b, tuple):
                sbind[j].kind, sbind[j].lo, sbind[j].hi = 0, int(b[1]), int(b[2])
            else:
                v = np.array([int(b)], dtype=np.int64).astype(np.int32)
                keep.append(v)
                sbind[j].kind = 1
                sbind[j].data = v.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        final_idx = -1
        if final is not None:
            final_idx = [n for n, _ in self.arrays].index(final)
        res = _Result()
        err = ctypes.create_string_buffer(512)
        rc = lib.orc_run_limit(self._p, G, W, abind, len(self.arrays), sbind, len(self.scalars),
                               ctypes.c_uint64(seed & (2**64 - 1)), instance,
                               1 if literal else 0, final_idx, ctypes.c_uint64(step_limit), ctypes.byref(res), err, 512)
        if rc != 0:
            raise OracleError(err.value.decode())
        try:
            n = int(res.n_records)
            if n:
                buf = (ctypes.c_char * (n * 40)).from_address(res.records)
                recs = np.frombuffer(bytes(buf), dtype=RECORD_DTYPE).copy()
            else:
                recs = np.zeros(0, dtype=RECORD_DTYPE)
            summ = np.frombuffer(bytes(res.summary), dtype=SUMMARY_DTYPE)[0].copy()
            fin = None
            if final_idx >= 0:
                fin = np.ctypeslib.as_array(res.final_mem, shape=(int(res.final_cells),)).copy()
        finally:
            lib.orc_result_free(ctypes.byref(res))
        return OracleResult(recs, summ, fin)


def check(src: str, G: int, W: int, **kw) -> OracleResult:
    return Program(src).run(G, W, **kw)


def seeded_value(seed: int, stream: int, idx: int, lo: int, hi: int) -> int:
    return int(_load().orc_seeded_value(seed & (2**64 - 1), stream, idx, lo, hi))
