"""Host-CPU baseline of the event generator, organised as the paper's CPU code
(Algorithm 3: chunks of 64 particles, vector loops over the particles still in
flight, OpenMP threads over chunks; Algorithm 2 for the generations).

A measurement baseline beside the GPU library -- it is not on the library's
path and shares no code with it.  Its tables are node values that the caller
supplies (the benchmark and the tests take them from the FP64 oracle).
Built three times (x86-64-v4 with AVX-512, x86-64-v3 with AVX2/FMA, baseline
x86-64); ``lib()`` loads the best one the host supports.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_DIR = Path(__file__).resolve().parent
_SRC = _DIR / "host_simd.cpp"
VARIANTS = {
    "x86-64-v4": ["-march=x86-64-v4", "-mtune=icelake-server", "-mprefer-vector-width=512"],
    "x86-64-v3": ["-march=x86-64-v3", "-mtune=skylake"],
    "x86-64": ["-march=x86-64"],
}


def _path(isa: str) -> Path:
    return _DIR / f"libhost_simd_{isa.replace('-', '_')}.so"


def build() -> None:
    for isa, fl in VARIANTS.items():
        out = _path(isa)
        tmp = out.with_suffix(".so.tmp")
        obj = out.with_suffix(".o")
        # fast-math for the compile only: linked with it, the library would set
        # flush-to-zero for every thread of the process that loads it
        subprocess.run(["g++", "-O3", "-ffast-math", "-fopenmp", "-fPIC", "-std=c++17", *fl, f'-DHS_ISA="{isa}"',
                        "-c", str(_SRC), "-o", str(obj)], check=True)
        subprocess.run(["g++", "-shared", "-fopenmp", str(obj), "-o", str(tmp)], check=True)
        obj.unlink()
        os.replace(tmp, out)


def host_isa() -> str:
    flags = set()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("flags"):
                flags = set(line.split(":", 1)[1].split())
                break
    except OSError:
        pass
    if {"avx512f", "avx512dq", "avx512bw", "avx512vl"} <= flags:
        return "x86-64-v4"
    if {"avx2", "fma", "bmi2"} <= flags:
        return "x86-64-v3"
    return "x86-64"


class Species(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("px", "py", "pz", "x", "y", "z")] + \
               [("w", C.c_void_p), ("tau", C.c_void_p), ("id", C.c_void_p), ("alive", C.c_void_p),
                ("nev", C.c_void_p), ("t_birth", C.c_void_p), ("root", C.c_void_p),
                ("count", C.c_int64), ("capacity", C.c_int64)]


class FieldsC(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ex", "ey", "ez", "bx", "by", "bz")] + [("stride", C.c_int64)]


class Cfg(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("emission", C.c_int32), ("pair", C.c_int32), ("push", C.c_int32),
                ("positions", C.c_int32), ("gamma_min", C.c_double), ("max_events", C.c_int64),
                ("threads", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_emit", C.c_int64), ("n_pair", C.c_int64), ("n_new", C.c_int64 * 3), ("n_rounds", C.c_int64),
                ("overflow", C.c_int64)]


class TablesIn(C.Structure):
    _fields_ = [("nr", C.c_int32), ("s0", C.c_double), ("hs", C.c_double), ("lnr", C.c_void_p * 2),
                ("rows", C.c_int32 * 2), ("cols", C.c_int32 * 2), ("qs0", C.c_double * 2), ("qhs", C.c_double * 2),
                ("qx0", C.c_double * 2), ("qhx", C.c_double * 2), ("q", C.c_void_p * 2)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _path(host_isa())
        if not path.exists():
            build()
        L = C.CDLL(str(path))
        v, p, i64 = C.c_void_p, C.c_void_p, C.c_int64
        for name, res, args in [
            ("hs_tables_create", v, [C.POINTER(TablesIn), C.c_int32]),
            ("hs_tables_free", None, [v, C.c_int32]),
            ("hs_step", C.c_int, [v, C.POINTER(Cfg), C.POINTER(Species), C.POINTER(FieldsC), C.POINTER(Species),
                                  C.c_double, C.c_uint64, C.c_uint32, C.POINTER(Stats)]),
            ("hs_eval_rate", None, [v, C.c_int32, C.c_int32, p, i64, p]),
            ("hs_sample", None, [v, C.c_int32, C.c_int32, p, p, i64, p]),
            ("hs_max_threads", C.c_int32, []),
            ("hs_isa", C.c_char_p, []),
        ]:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


class Tables:
    """Node values (a dict: nr, s0, hs, lnr [2, nr], and per process rows,
    cols, qs0, qhs, qx0, qhx, q [rows, cols]) in the baseline's layout."""

    def __init__(self, nodes: dict, dtype=np.float32):
        self.dtype = np.dtype(dtype)
        self.code = 0 if self.dtype == np.float32 else 1
        self._keep = [np.ascontiguousarray(nodes["lnr"][k], dtype=np.float64) for k in range(2)] + \
                     [np.ascontiguousarray(nodes["q"][k], dtype=np.float64) for k in range(2)]
        t = TablesIn()
        t.nr, t.s0, t.hs = int(nodes["nr"]), float(nodes["s0"]), float(nodes["hs"])
        for k in range(2):
            t.lnr[k] = self._keep[k].ctypes.data
            t.q[k] = self._keep[2 + k].ctypes.data
            t.rows[k], t.cols[k] = self._keep[2 + k].shape
            t.qs0[k], t.qhs[k] = nodes["qs0"][k], nodes["qhs"][k]
            t.qx0[k], t.qhx[k] = nodes["qx0"][k], nodes["qhx"][k]
        self.handle = lib().hs_tables_create(C.byref(t), self.code)
        if not self.handle:
            raise ValueError("invalid host tables")

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hs_tables_free(self.handle, self.code)
            self.handle = None

    def rate(self, proc: int, chi) -> np.ndarray:
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        out = np.empty_like(chi)
        lib().hs_eval_rate(self.handle, self.code, proc, _ptr(chi), chi.size, _ptr(out))
        return out

    def sample(self, proc: int, chi, k) -> np.ndarray:
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.uint32), chi.shape))
        out = np.empty_like(chi)
        lib().hs_sample(self.handle, self.code, proc, _ptr(chi), _ptr(k), chi.size, _ptr(out))
        return out


class Store:
    """One species on the host, structure of arrays in the step's dtype."""

    def __init__(self, capacity: int, dtype=np.float32, photon=False, positions=False, appended=False):
        cap = max(int(capacity), 1)
        self.dtype = np.dtype(dtype)
        self.p = np.zeros((3, cap), dtype=self.dtype)
        self.x = np.zeros((3, cap), dtype=self.dtype) if positions else None
        self.w = np.zeros(cap, np.float32)
        self.tau = np.zeros(cap, np.float64)
        self.id = np.zeros(cap, np.uint64)
        self.alive = np.ones(cap, np.uint8) if photon else None
        self.nev = np.zeros(cap, np.int32)
        self.t_birth = np.zeros(cap, np.float64) if appended else None
        self.root = np.zeros(cap, np.uint32) if appended else None
        self.capacity = int(capacity)
        self.count = 0

    @classmethod
    def from_arrays(cls, p, w, tau, ids, dtype=np.float32, photon=False, x=None):
        n = len(ids)
        s = cls(n, dtype, photon, x is not None)
        s.p[:, :n] = np.asarray(p, dtype=np.float64).T
        if x is not None:
            s.x[:, :n] = np.asarray(x, dtype=np.float64).T
        s.w[:n] = w
        s.tau[:n] = tau
        s.id[:n] = ids
        s.count = n
        return s

    def c(self) -> Species:
        x = self.x if self.x is not None else None
        return Species(*[_ptr(self.p[k]) for k in range(3)],
                       *([_ptr(x[k]) for k in range(3)] if x is not None else [None] * 3),
                       _ptr(self.w), _ptr(self.tau), _ptr(self.id), _ptr(self.alive), _ptr(self.nev),
                       _ptr(self.t_birth), _ptr(self.root), self.count, self.capacity)


def fields_c(f: np.ndarray, dtype) -> tuple:
    """[n, 6] per particle or [1, 6] shared -> (FieldsC, the arrays it points to)."""
    a = [np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1, 6)[:, k], dtype=dtype) for k in range(6)]
    return FieldsC(*[_ptr(v) for v in a], 0 if a[0].size == 1 else 1), a


def step(tables: Tables, main: list, fields: list, app: list, dt: float, seed: int, step_index: int,
         emission=True, pair=True, push=False, positions=False, gamma_min=1.0, max_events=1 << 20,
         threads=0) -> tuple[int, Stats]:
    cfg = Cfg(tables.code, int(emission), int(pair), int(push), int(positions), float(gamma_min), int(max_events),
              int(threads))
    M = (Species * 3)(*[m.c() for m in main])
    A = (Species * 3)(*[a.c() for a in app])
    keep = []
    F = (FieldsC * 3)()
    for s in range(3):
        F[s], arrays = fields_c(fields[s], tables.dtype)
        keep.append(arrays)
    st = Stats()
    rc = lib().hs_step(tables.handle, C.byref(cfg), M, F, A, float(dt), C.c_uint64(seed), C.c_uint32(step_index),
                       C.byref(st))
    for s in range(3):
        app[s].count = int(A[s].count)
    return rc, st
