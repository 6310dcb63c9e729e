"""CPU oracle -- TEST INFRASTRUCTURE, never part of the product path.

A plain FP64 reference of the per-macroparticle SFQED event generator of
arXiv:2409.17299 (Sec. 3, Algorithms 1 and 2), written from the physics it
defers to (locally-constant-field nonlinear Compton and Breit-Wheeler spectra).
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library.

The C++ part (``sfqed_oracle.cpp``) holds the special functions, quadrature,
Philox4x32-10, rates, inverse CDFs and the ensemble step.  ``mlp.py`` holds the
FP64 numpy forward/backward of the surrogate network.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_DIR = Path(__file__).resolve().parent
_SRC = _DIR / "sfqed_oracle.cpp"
_LIB = _DIR / "liboracle.so"
# SFQED_ORACLE_LIB names another build of the same source (the tests build
# copies with a deliberate mistake planted, to show that the pins catch it)
_LIB_OVERRIDE = os.environ.get("SFQED_ORACLE_LIB")

ELECTRON, POSITRON, PHOTON = 0, 1, 2


def build(force: bool = True) -> Path:
    """Compile the oracle with g++ (host only, OpenMP)."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp")
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", str(_SRC), "-o", str(tmp)]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Species(C.Structure):
    _fields_ = [("state", C.POINTER(C.c_double)), ("id", C.POINTER(C.c_uint64)),
                ("root", C.POINTER(C.c_int32)), ("alive", C.POINTER(C.c_uint8)),
                ("nev", C.POINTER(C.c_int32)), ("count", C.c_int64), ("capacity", C.c_int64)]


class Fields(C.Structure):
    _fields_ = [("f", C.POINTER(C.c_double)), ("stride", C.c_int64)]


class Cfg(C.Structure):
    _fields_ = [("emission", C.c_int32), ("pair", C.c_int32), ("push", C.c_int32),
                ("positions", C.c_int32), ("max_events", C.c_int64), ("gamma_min", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("n_emit", C.c_int64), ("n_pair", C.c_int64), ("n_new", C.c_int64 * 3),
                ("n_rounds", C.c_int64), ("max_events", C.c_int64), ("overflow", C.c_int64),
                ("capped", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not _LIB.exists():
                build(force=False)
            L = C.CDLL(str(_LIB))
        d, i64, p = C.c_double, C.c_int64, C.c_void_p
        for name, res, args in [
            ("orc_philox", None, [p, p, p]),
            ("orc_philox_stream", None, [C.c_uint64, p, p, p, i64, p]),
            ("orc_alpha", d, []),
            ("orc_bessel_k", d, [d, d, C.c_int]),
            ("orc_bessel_ki", d, [d, d, C.c_int]),
            ("orc_spec_rad", d, [d, d, C.c_int]),
            ("orc_spec_pair", d, [d, d, C.c_int]),
            ("orc_spec_rad_many", None, [p, p, i64, p]),
            ("orc_spec_pair_many", None, [p, p, i64, p]),
            ("orc_rate_rad", d, [d, C.c_int]),
            ("orc_rate_pair", d, [d, C.c_int]),
            ("orc_rate_rad_many", None, [p, i64, p]),
            ("orc_rate_pair_many", None, [p, i64, p]),
            ("orc_cdf_rad", d, [d, d, C.c_int]),
            ("orc_cdf_pair", d, [d, d, C.c_int]),
            ("orc_sample_rad", None, [p, p, i64, p, p]),
            ("orc_sample_pair", None, [p, p, i64, p, p]),
            ("orc_sample_rad_r", None, [d, d, d, C.c_int, p, p]),
            ("orc_sample_pair_r", None, [d, d, d, C.c_int, p, p]),
            ("orc_sample_rad_grid", None, [p, i64, p, p, i64, p, p]),
            ("orc_chi", d, [p, d, p, p]),
            ("orc_boris", None, [p, d, p, p, d]),
            ("orc_init_tau", None, [C.POINTER(Species), C.c_uint64, C.c_uint32]),
            ("orc_step", C.c_int, [C.POINTER(Species), C.POINTER(Fields), C.POINTER(Species), d,
                                   C.c_uint64, C.c_uint32, C.POINTER(Cfg), C.POINTER(Stats)]),
            ("orc_merge", C.c_int, [C.POINTER(Species), C.POINTER(Species)]),
        ]:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


ALPHA = 7.2973525693e-3


# ---------------------------------------------------------------- RNG
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(o))
    return o


def philox_stream(seed: int, ids, steps, js) -> np.ndarray:
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    n = ids.size
    st = np.ascontiguousarray(np.broadcast_to(np.asarray(steps, dtype=np.uint32), (n,)))
    jj = np.ascontiguousarray(np.broadcast_to(np.asarray(js, dtype=np.uint32), (n,)))
    out = np.zeros((n, 4), dtype=np.uint32)
    lib().orc_philox_stream(C.c_uint64(seed), _ptr(ids), _ptr(st), _ptr(jj), n, _ptr(out))
    return out


# ---------------------------------------------------------------- special functions / spectra
def bessel_k(nu: float, x: float, definition: bool = True) -> float:
    return lib().orc_bessel_k(nu, x, int(definition))


def bessel_ki(nu: float, x: float, definition: bool = True) -> float:
    return lib().orc_bessel_ki(nu, x, int(definition))


def spec_rad(chi: float, delta: float, definition: bool = False) -> float:
    """dW_rad/d(delta) * gamma/alpha."""
    return lib().orc_spec_rad(chi, delta, int(definition))


def spec_pair(chi: float, xi: float, definition: bool = False) -> float:
    """dW_pair/d(xi) * eps/alpha."""
    return lib().orc_spec_pair(chi, xi, int(definition))


def spec_rad_many(chi, delta) -> np.ndarray:
    c = np.ascontiguousarray(chi, dtype=np.float64)
    d = np.ascontiguousarray(np.broadcast_to(np.asarray(delta, dtype=np.float64), c.shape))
    o = np.empty_like(d)
    lib().orc_spec_rad_many(_ptr(c), _ptr(d), d.size, _ptr(o))
    return o


def spec_pair_many(chi, xi) -> np.ndarray:
    """dW_pair/d(xi) * eps/alpha at many (chi, xi)."""
    c = np.ascontiguousarray(chi, dtype=np.float64)
    x = np.ascontiguousarray(np.broadcast_to(np.asarray(xi, dtype=np.float64), c.shape))
    o = np.empty_like(x)
    lib().orc_spec_pair_many(_ptr(c), _ptr(x), x.size, _ptr(o))
    return o


def rate_rad_reduced(chi: float, definition: bool = False) -> float:
    """W_rad * gamma / alpha."""
    return lib().orc_rate_rad(chi, int(definition))


def rate_pair_reduced(chi: float, definition: bool = False) -> float:
    """W_pair * eps / alpha."""
    return lib().orc_rate_pair(chi, int(definition))


def rate_rad_reduced_many(chi) -> np.ndarray:
    c = np.ascontiguousarray(chi, dtype=np.float64)
    o = np.empty_like(c)
    lib().orc_rate_rad_many(_ptr(c), c.size, _ptr(o))
    return o


def rate_pair_reduced_many(chi) -> np.ndarray:
    c = np.ascontiguousarray(chi, dtype=np.float64)
    o = np.empty_like(c)
    lib().orc_rate_pair_many(_ptr(c), c.size, _ptr(o))
    return o


def cdf_rad(chi: float, delta: float, definition: bool = False) -> float:
    return lib().orc_cdf_rad(chi, delta, int(definition))


def cdf_pair(chi: float, xi: float, definition: bool = False) -> float:
    return lib().orc_cdf_pair(chi, xi, int(definition))


def sample_rad(chi, k) -> tuple[np.ndarray, np.ndarray]:
    """delta and 1-delta for raw 32-bit uniforms k (r = (k+1/2)/2^32)."""
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.uint32), chi.shape))
    d = np.empty_like(chi)
    o = np.empty_like(chi)
    lib().orc_sample_rad(_ptr(chi), _ptr(k), chi.size, _ptr(d), _ptr(o))
    return d, o


def sample_pair(chi, k) -> tuple[np.ndarray, np.ndarray]:
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.uint32), chi.shape))
    d = np.empty_like(chi)
    o = np.empty_like(chi)
    lib().orc_sample_pair(_ptr(chi), _ptr(k), chi.size, _ptr(d), _ptr(o))
    return d, o


def sample_rad_r(chi: float, r: float, definition: bool = False, rc: float | None = None) -> float:
    """delta at uniform r (rc = 1 - r, pass it when r is close to 1)."""
    d = C.c_double()
    o = C.c_double()
    lib().orc_sample_rad_r(chi, r, 1.0 - r if rc is None else rc, int(definition), C.byref(d), C.byref(o))
    return d.value


def sample_rad_r2(chi: float, r: float, rc: float) -> tuple[float, float]:
    """delta and 1 - delta."""
    d = C.c_double()
    o = C.c_double()
    lib().orc_sample_rad_r(chi, r, rc, 0, C.byref(d), C.byref(o))
    return d.value, o.value


def sample_rad_grid(chi, r, rc=None) -> tuple[np.ndarray, np.ndarray]:
    """Emission draws on a chi grid: chi [m], r and rc = 1 - r [m, k] -> delta and 1 - delta [m, k]."""
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    rc = np.ascontiguousarray(1.0 - r if rc is None else rc, dtype=np.float64)
    m, k = r.shape
    assert chi.shape == (m,) and rc.shape == r.shape
    d = np.empty_like(r)
    o = np.empty_like(r)
    lib().orc_sample_rad_grid(_ptr(chi), m, _ptr(r), _ptr(rc), k, _ptr(d), _ptr(o))
    return d, o


def sample_pair_r(chi: float, r: float, definition: bool = False, rc: float | None = None) -> float:
    d = C.c_double()
    o = C.c_double()
    lib().orc_sample_pair_r(chi, r, 1.0 - r if rc is None else rc, int(definition), C.byref(d), C.byref(o))
    return d.value


def chi(p, energy, E, B) -> float:
    p = np.ascontiguousarray(p, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    return lib().orc_chi(_ptr(p), float(energy), _ptr(E), _ptr(B))


def boris(p, q, E, B, h) -> np.ndarray:
    p = np.array(p, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    lib().orc_boris(_ptr(p), float(q), _ptr(E), _ptr(B), float(h))
    return p


# ---------------------------------------------------------------- ensemble step
class Store:
    """One species, FP64 host SoA: state[:, 0:9] = px py pz x y z w tau t_birth."""

    def __init__(self, capacity: int):
        self.state = np.zeros((max(capacity, 1), 9), dtype=np.float64)
        self.id = np.zeros(max(capacity, 1), dtype=np.uint64)
        self.root = np.zeros(max(capacity, 1), dtype=np.int32)
        self.alive = np.ones(max(capacity, 1), dtype=np.uint8)
        self.nev = np.zeros(max(capacity, 1), dtype=np.int32)
        self.count = 0
        self.capacity = capacity

    @classmethod
    def from_arrays(cls, p, w, tau, ids, x=None, capacity=None, alive=None):
        n = len(ids)
        s = cls(capacity if capacity is not None else n)
        s.state[:n, 0:3] = p
        if x is not None:
            s.state[:n, 3:6] = x
        s.state[:n, 6] = w
        s.state[:n, 7] = tau
        s.id[:n] = ids
        if alive is not None:
            s.alive[:n] = alive
        s.count = n
        return s

    def c(self) -> Species:
        return Species(self.state.ctypes.data_as(C.POINTER(C.c_double)),
                       self.id.ctypes.data_as(C.POINTER(C.c_uint64)),
                       self.root.ctypes.data_as(C.POINTER(C.c_int32)),
                       self.alive.ctypes.data_as(C.POINTER(C.c_uint8)),
                       self.nev.ctypes.data_as(C.POINTER(C.c_int32)),
                       self.count, self.capacity)

    # views of the live part
    @property
    def p(self):
        return self.state[:self.count, 0:3]

    @property
    def x(self):
        return self.state[:self.count, 3:6]

    @property
    def w(self):
        return self.state[:self.count, 6]

    @property
    def tau(self):
        return self.state[:self.count, 7]

    @property
    def t_birth(self):
        return self.state[:self.count, 8]


def step(main: list[Store], fields: list[np.ndarray], app: list[Store], dt: float, seed: int,
         step_index: int, emission=True, pair=True, push=False, positions=False,
         max_events: int = 1 << 20, gamma_min: float = 1.0) -> tuple[int, Stats]:
    """One global step of the ensemble (Alg. 2 for every particle).

    fields[s] is an [n, 6] FP64 array (ex ey ez bx by bz) per particle of
    species s, or a [1, 6] array for one field shared by all.
    """
    M = (Species * 3)(*[m.c() for m in main])
    A = (Species * 3)(*[a.c() for a in app])
    F = (Fields * 3)()
    keep = []
    for s in range(3):
        f = np.ascontiguousarray(fields[s], dtype=np.float64).reshape(-1, 6)
        keep.append(f)
        F[s] = Fields(f.ctypes.data_as(C.POINTER(C.c_double)), 0 if f.shape[0] == 1 else 1)
    cfg = Cfg(int(emission), int(pair), int(push), int(positions), max_events, float(gamma_min))
    st = Stats()
    rc = lib().orc_step(M, F, A, float(dt), C.c_uint64(seed), C.c_uint32(step_index), C.byref(cfg),
                        C.byref(st))
    for s in range(3):
        app[s].count = A[s].count
    return rc, st


def merge(main: list[Store], app: list[Store]) -> int:
    M = (Species * 3)(*[m.c() for m in main])
    A = (Species * 3)(*[a.c() for a in app])
    rc = lib().orc_merge(M, A)
    for s in range(3):
        main[s].count = M[s].count
    return rc


def init_tau(store: Store, seed: int, step_index: int) -> None:
    S = store.c()
    lib().orc_init_tau(C.byref(S), C.c_uint64(seed), C.c_uint32(step_index))
