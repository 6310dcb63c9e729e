"""MI355X (gfx950) per-macroparticle strong-field QED event generator.

Python binding of libsfqed (``include/sfqed.h``): argument marshalling only.
Every step of the generator runs in the library's HIP kernels; PyTorch provides
device memory and the stream.  Importing works without a GPU; the first call
that needs the library raises ``SfqedError`` if ``libsfqed.so`` was not built
(``python -m paper_2409_17299_amd.build``).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libsfqed.so"

ELECTRON, POSITRON, PHOTON = 0, 1, 2
EMISSION, PAIR = 0, 1
F32, F64 = 0, 1
STATUS = {0: "ok", 1: "invalid argument", 2: "capacity exceeded", 3: "HIP runtime error", 4: "invalid state",
          5: "max_events reached"}


class SfqedError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


# ----------------------------------------------------------------------------- C structs
class TableCfg(C.Structure):
    _fields_ = [("rate_chi_min", C.c_double), ("rate_chi_max", C.c_double), ("rate_nodes", C.c_int32),
                ("rad_chi_min", C.c_double), ("rad_chi_max", C.c_double), ("rad_rows", C.c_int32),
                ("rad_cols", C.c_int32), ("rad_x_min", C.c_double), ("rad_x_max", C.c_double),
                ("pair_chi_min", C.c_double), ("pair_chi_max", C.c_double), ("pair_rows", C.c_int32),
                ("pair_cols", C.c_int32), ("pair_x_min", C.c_double), ("f64_refine", C.c_int32)]


class CSpecies(C.Structure):
    _fields_ = [("px", C.c_void_p), ("py", C.c_void_p), ("pz", C.c_void_p), ("x", C.c_void_p),
                ("y", C.c_void_p), ("z", C.c_void_p), ("w", C.c_void_p), ("tau", C.c_void_p),
                ("id", C.c_void_p), ("alive", C.c_void_p), ("nev", C.c_void_p), ("count", C.c_int64),
                ("capacity", C.c_int64)]


class CAppend(C.Structure):
    _fields_ = [("rec", C.c_void_p), ("pos", C.c_void_p), ("count", C.c_int64), ("capacity", C.c_int64)]


def record_dtype(float_dtype) -> np.dtype:
    """numpy layout of one appended record (qed_rec32 / qed_rec64)."""
    f = np.dtype(float_dtype)
    return np.dtype([("px", f), ("py", f), ("pz", f), ("t_birth", f), ("tau", np.float64), ("id", np.uint64),
                     ("w", np.float32), ("root", np.uint32), ("nev", np.int32), ("alive", np.uint32)])


class CFields(C.Structure):
    _fields_ = [("ex", C.c_void_p), ("ey", C.c_void_p), ("ez", C.c_void_p), ("bx", C.c_void_p),
                ("by", C.c_void_p), ("bz", C.c_void_p), ("stride", C.c_int64), ("n", C.c_int64)]


class CEnsemble(C.Structure):
    _fields_ = [("dtype", C.c_int), ("s", CSpecies * 3), ("f", CFields * 3)]


class StepCfg(C.Structure):
    _fields_ = [("emission", C.c_int32), ("pair", C.c_int32), ("push", C.c_int32), ("gamma_min", C.c_double),
                ("max_events", C.c_int64), ("profile", C.c_int32), ("nev", C.c_int32),
                ("validate", C.c_int32)]


class StepStats(C.Structure):
    _fields_ = [("n_emit", C.c_int64), ("n_pair", C.c_int64), ("n_new", C.c_int64 * 3), ("n_rounds", C.c_int64),
                ("max_events", C.c_int64), ("required_capacity", C.c_int64 * 3), ("n_launches", C.c_int64),
                ("kernel_ms", C.c_double * 5), ("kernel_launches", C.c_int64 * 5),
                ("kernel_particles", C.c_int64 * 5), ("event_particles", C.c_int64 * 2),
                ("log_replays", C.c_int64), ("log_reruns", C.c_int64)]

    KERNELS = ("count_lepton", "scan", "write_lepton", "count_photon", "write_photon")

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if hasattr(v, "__len__") else v
        return d


class ResampleCfg(C.Structure):
    _fields_ = [("photon_energy_min", C.c_double), ("target", C.c_int64 * 3), ("seed", C.c_uint64),
                ("step", C.c_uint32)]


class ResampleStats(C.Structure):
    _fields_ = [("count_before", C.c_int64 * 3), ("count_after", C.c_int64 * 3), ("filtered", C.c_int64),
                ("w_threshold", C.c_double * 3), ("iterations", C.c_int32 * 3)]

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if hasattr(v, "__len__") else v
        return d


class CGrid1d(C.Structure):
    _fields_ = [("dtype", C.c_int), ("nx", C.c_int64), ("x0", C.c_double), ("length", C.c_double)] + \
               [(k, C.c_void_p) for k in ("ex", "ey", "ez", "bx", "by", "bz")]


class CBox(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("len", C.c_double * 3)]


class CFieldArrays(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ex", "ey", "ez", "bx", "by", "bz")] + [("n", C.c_int64)]


_lib = None


MLP_PARAMS = 4417


class MlpCfg(C.Structure):
    _fields_ = [(k, C.c_float) for k in ("chi_min", "chi_max", "f1_scale", "f1_shift", "f2_scale", "out_scale")]


class TrainCfg(C.Structure):
    _fields_ = [("steps", C.c_int64), ("batch", C.c_int64), ("schedule_start", C.c_int64),
                ("schedule_len", C.c_int64), ("lr_max", C.c_float), ("lr_min", C.c_float),
                ("warmup", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("seed", C.c_uint64), ("shuffle", C.c_int32)]


def lib():
    """The loaded libsfqed (raises SfqedError if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise SfqedError(4, f"{LIB_PATH} is missing: build it with python -m paper_2409_17299_amd.build")
        L = C.CDLL(str(LIB_PATH))
        v, p, i64 = C.c_void_p, C.c_void_p, C.c_int64
        sig = {
            "qed_table_cfg_default": (None, [C.POINTER(TableCfg)]),
            "qed_build_rate_tables": (C.c_int, [C.POINTER(TableCfg), v, C.POINTER(v)]),
            "qed_tables_free": (None, [v]),
            "qed_tables_export": (C.c_int, [v, C.c_int, v, C.POINTER(C.c_size_t)]),
            "qed_tables_geometry": (C.c_int, [v, C.POINTER(C.c_double), C.c_int]),
            "qed_step_cfg_default": (None, [C.POINTER(StepCfg)]),
            "qed_init_tau": (C.c_int, [C.POINTER(CEnsemble), C.c_uint64, C.c_uint32, v]),
            "qed_step": (C.c_int, [v, C.POINTER(StepCfg), C.POINTER(CEnsemble), C.POINTER(CAppend), C.c_double,
                                   C.c_uint64, C.c_uint32, C.POINTER(StepStats), v]),
            "qed_merge": (C.c_int, [C.POINTER(CEnsemble), C.POINTER(CAppend), v]),
            "qed_merge_noalloc": (C.c_int, [C.POINTER(CEnsemble), C.POINTER(CAppend), v]),
            "qed_validate": (C.c_int, [C.POINTER(CEnsemble), C.POINTER(C.c_int64), v]),
            "qed_step_merged": (C.c_int, [v, C.POINTER(StepCfg), C.POINTER(CEnsemble), C.POINTER(CAppend),
                                          C.c_double, C.c_uint64, C.c_uint32, C.POINTER(StepStats), v]),
            "qed_resample_cfg_default": (None, [C.POINTER(ResampleCfg)]),
            "qed_resample": (C.c_int, [C.POINTER(CEnsemble), C.POINTER(ResampleCfg), C.POINTER(ResampleStats), v]),
            "qed_grid_standing_wave": (C.c_int, [C.POINTER(CGrid1d), C.c_double, C.c_double, C.c_double,
                                                 C.c_double, C.c_double, v]),
            "qed_gather_fields": (C.c_int, [C.POINTER(CEnsemble), C.POINTER(CGrid1d), C.POINTER(CBox),
                                            C.POINTER(CFieldArrays), v]),
            "qed_eval_rate": (C.c_int, [v, C.c_int, C.c_int, p, p, p, i64, v]),
            "qed_eval_particles": (C.c_int, [v, C.c_int, C.c_int, p, p, p, C.POINTER(CFields), i64, p, p, v]),
            "qed_sample": (C.c_int, [v, C.c_int, C.c_int, p, p, p, i64, v]),
            "qed_mlp_cfg_default": (None, [C.POINTER(MlpCfg)]),
            "qed_mlp_train_cfg_default": (None, [C.POINTER(TrainCfg)]),
            "qed_mlp_create": (C.c_int, [C.POINTER(MlpCfg), C.POINTER(v)]),
            "qed_mlp_free": (None, [v]),
            "qed_mlp_get_cfg": (C.c_int, [v, C.POINTER(MlpCfg)]),
            "qed_mlp_set_params": (C.c_int, [v, p, v]),
            "qed_mlp_get_params": (C.c_int, [v, p, v]),
            "qed_mlp_forward": (C.c_int, [v, p, p, i64, v]),
            "qed_mlp_grad": (C.c_int, [v, p, p, i64, p, p, v]),
            "qed_mlp_train": (C.c_int, [v, p, p, i64, C.POINTER(TrainCfg), p, v]),
            "qed_sample_mlp": (C.c_int, [v, v, p, p, p, i64, v]),
            "qed_status_str": (C.c_char_p, [C.c_int]),
            "qed_last_error": (C.c_char_p, []),
            "qed_abi_version": (C.c_int32, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise SfqedError(rc, lib().qed_last_error().decode(errors="replace"))


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ----------------------------------------------------------------------------- tables
def default_table_cfg(**overrides) -> TableCfg:
    cfg = TableCfg()
    lib().qed_table_cfg_default(C.byref(cfg))
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


TABLE_PARTS = {"cheb_rad": 0, "cheb_pair": 1, "herm_rad": 2, "herm_pair": 3, "cdf32_rad": 4, "cdf32_pair": 5,
               "cdf64_rad": 6, "cdf64_pair": 7}


class Tables:
    """Rate and inverse-CDF tables built on the current device (blocking)."""

    def __init__(self, cfg: TableCfg | None = None, stream=None):
        self.cfg = cfg if cfg is not None else default_table_cfg()
        h = C.c_void_p()
        _check(lib().qed_build_rate_tables(C.byref(self.cfg), _stream(stream), C.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.qed_tables_free(h)
            self.handle = None

    def export(self, part: str) -> np.ndarray:
        which = TABLE_PARTS[part]
        n = C.c_size_t(0)
        _check(lib().qed_tables_export(self.handle, which, None, C.byref(n)))
        dt = np.float64 if which in (0, 1, 6, 7) else np.float32
        out = np.empty(n.value // np.dtype(dt).itemsize, dtype=dt)
        _check(lib().qed_tables_export(self.handle, which, out.ctypes.data_as(C.c_void_p), C.byref(n)))
        g = self.geometry()
        if which in (0, 1):
            return out.reshape(-1, 17)
        if which in (2, 3):
            return out.reshape(-1, 2)
        p = which % 2
        rows, cols = (g[f"rows32_{p}"], g[f"cols32_{p}"]) if which in (4, 5) else (g[f"rows64_{p}"], g[f"cols64_{p}"])
        return out.reshape(rows, cols)

    def geometry(self) -> dict:
        v = (C.c_double * 21)()
        _check(lib().qed_tables_geometry(self.handle, v, 21))
        names = ["nseg_0", "s_lo_0", "nseg_1", "s_lo_1", "herm_n"]
        for p in (0, 1):
            names += [f"rows32_{p}", f"cols32_{p}", f"rows64_{p}", f"cols64_{p}", f"s0_{p}", f"s1_{p}", f"x0_{p}",
                      f"x1_{p}"]
        return {k: (int(x) if k.startswith(("nseg", "herm", "rows", "cols")) else float(x)) for k, x in zip(names, v)}


# ----------------------------------------------------------------------------- particle stores
@dataclass
class Store:
    """One species in device memory (structure of arrays, torch tensors)."""
    px: object
    py: object
    pz: object
    w: object
    tau: object
    id: object
    alive: object = None
    nev: object = None
    x: object = None
    y: object = None
    z: object = None
    count: int = 0
    cap: int | None = None  # capacity passed to the library (default: the tensor length)

    @property
    def capacity(self) -> int:
        return int(self.px.numel()) if self.cap is None else int(self.cap)

    @property
    def dtype(self):
        return self.px.dtype

    @classmethod
    def empty(cls, capacity: int, dtype=None, photon: bool = False, positions: bool = False, nev: bool = True,
              device="cuda"):
        torch = _torch()
        dtype = dtype or torch.float32
        cap = max(int(capacity), 0)
        z = lambda dt: torch.zeros(cap, dtype=dt, device=device)  # noqa: E731
        s = cls(z(dtype), z(dtype), z(dtype), z(torch.float32), z(torch.float64), z(torch.int64))
        if photon:
            s.alive = torch.ones(cap, dtype=torch.uint8, device=device)
        if nev:
            s.nev = z(torch.int32)
        if positions:
            s.x, s.y, s.z = z(dtype), z(dtype), z(dtype)
        return s

    @classmethod
    def from_arrays(cls, p, w, tau, ids, dtype=None, capacity=None, photon=False, positions=None, x=None,
                    device="cuda"):
        torch = _torch()
        dtype = dtype or torch.float32
        n = len(ids)
        s = cls.empty(capacity if capacity is not None else n, dtype, photon=photon, positions=x is not None,
                      device=device)
        p = torch.as_tensor(np.asarray(p, dtype=np.float64))
        s.px[:n] = p[:, 0].to(dtype)
        s.py[:n] = p[:, 1].to(dtype)
        s.pz[:n] = p[:, 2].to(dtype)
        s.w[:n] = torch.as_tensor(np.asarray(w, dtype=np.float32))
        s.tau[:n] = torch.as_tensor(np.asarray(tau, dtype=np.float64))
        s.id[:n] = torch.as_tensor(np.asarray(ids, dtype=np.uint64).view(np.int64))
        if x is not None:
            xx = torch.as_tensor(np.asarray(x, dtype=np.float64))
            s.x[:n], s.y[:n], s.z[:n] = xx[:, 0].to(dtype), xx[:, 1].to(dtype), xx[:, 2].to(dtype)
        s.count = n
        return s

    def c(self) -> CSpecies:
        return CSpecies(*[_ptr(t) for t in (self.px, self.py, self.pz, self.x, self.y, self.z, self.w, self.tau,
                                            self.id, self.alive, self.nev)],
                        self.count, self.capacity)

    def host(self) -> dict:
        """Live part copied to host numpy arrays (momenta as [n, 3] float64)."""
        n = self.count
        out = {"p": np.stack([t[:n].double().cpu().numpy() for t in (self.px, self.py, self.pz)], axis=1),
               "w": self.w[:n].cpu().numpy(), "tau": self.tau[:n].cpu().numpy(),
               "id": self.id[:n].cpu().numpy().view(np.uint64)}
        for name in ("alive", "nev"):
            t = getattr(self, name)
            if t is not None:
                out[name] = t[:n].cpu().numpy()
        if self.x is not None:
            out["x"] = np.stack([t[:n].double().cpu().numpy() for t in (self.x, self.y, self.z)], axis=1)
        return out


class AppendBuffer:
    """Appended particles of one species: 16-byte-aligned records (qed_rec32 or
    qed_rec64) in a torch uint8 tensor, plus optional positions (4 per record)."""

    def __init__(self, capacity: int, dtype=None, positions: bool = False, device="cuda"):
        torch = _torch()
        self.dtype = dtype or torch.float32
        self.np_float = np.float32 if self.dtype == torch.float32 else np.float64
        self.rec_dtype = record_dtype(self.np_float)
        cap = max(int(capacity), 0)
        self.data = torch.zeros(max(cap, 1) * self.rec_dtype.itemsize, dtype=torch.uint8, device=device)
        self.pos = torch.zeros(max(cap, 1) * 4, dtype=self.dtype, device=device) if positions else None
        self.cap = cap
        self.count = 0

    @property
    def capacity(self) -> int:
        return self.cap

    def c(self) -> CAppend:
        return CAppend(_ptr(self.data), _ptr(self.pos), self.count, self.capacity)

    def records(self, n: int | None = None) -> np.ndarray:
        n = self.count if n is None else n
        raw = self.data[: n * self.rec_dtype.itemsize].cpu().numpy()
        return raw.view(self.rec_dtype)

    def host(self) -> dict:
        r = self.records()
        out = {"p": np.stack([r["px"], r["py"], r["pz"]], axis=1).astype(np.float64), "w": r["w"].copy(),
               "tau": r["tau"].copy(), "id": r["id"].copy(), "root": r["root"].copy(),
               "t_birth": r["t_birth"].astype(np.float64), "nev": r["nev"].copy(),
               "alive": r["alive"].astype(np.uint8)}
        if self.pos is not None:
            out["x"] = self.pos[: 4 * self.count].double().cpu().numpy().reshape(-1, 4)[:, :3]
        return out


@dataclass
class Fields:
    """Per-particle (stride 1) or shared (stride 0) E and B of one species."""
    ex: object
    ey: object
    ez: object
    bx: object
    by: object
    bz: object
    stride: int = 1

    @classmethod
    def from_array(cls, f, dtype=None, device="cuda"):
        torch = _torch()
        dtype = dtype or torch.float32
        f = np.asarray(f, dtype=np.float64).reshape(-1, 6)
        t = torch.as_tensor(f).to(device=device, dtype=dtype)
        return cls(*[t[:, k].contiguous() for k in range(6)], stride=0 if f.shape[0] == 1 else 1)

    def c(self) -> CFields:
        ts = (self.ex, self.ey, self.ez, self.bx, self.by, self.bz)
        return CFields(*[_ptr(t) for t in ts], self.stride, min(t.numel() for t in ts))


def _dtype_code(t) -> int:
    torch = _torch()
    if t == torch.float32:
        return F32
    if t == torch.float64:
        return F64
    raise SfqedError(1, f"unsupported dtype {t}")


def _ensemble(main: list, fields: list) -> CEnsemble:
    e = CEnsemble()
    e.dtype = _dtype_code(main[0].dtype)
    for k in range(3):
        e.s[k] = main[k].c()
        e.f[k] = fields[k].c()
    return e


def step_cfg(emission=True, pair=True, push=True, gamma_min=1.0, max_events=1 << 20, profile=False,
             nev=True, validate=False) -> StepCfg:
    cfg = StepCfg()
    lib().qed_step_cfg_default(C.byref(cfg))
    cfg.emission, cfg.pair, cfg.push = int(emission), int(pair), int(push)
    cfg.gamma_min, cfg.max_events, cfg.profile = float(gamma_min), int(max_events), int(profile)
    cfg.nev = int(nev)
    cfg.validate = int(validate)
    return cfg


def init_tau(main: list, fields: list, seed: int, step_index: int, stream=None):
    e = _ensemble(main, fields)
    _check(lib().qed_init_tau(C.byref(e), C.c_uint64(seed), C.c_uint32(step_index), _stream(stream)))


def step(tables: Tables, main: list, fields: list, app: list, dt: float, seed: int, step_index: int,
         cfg: StepCfg | None = None, stream=None, check: bool = True) -> tuple[int, StepStats]:
    """One global step (Algorithms 1 and 2).  Updates main/app in place and app counts."""
    cfg = cfg if cfg is not None else step_cfg()
    e = _ensemble(main, fields)
    for s in app:
        s.count = 0
    a = (CAppend * 3)(*[s.c() for s in app])
    st = StepStats()
    rc = lib().qed_step(tables.handle, C.byref(cfg), C.byref(e), a, float(dt), C.c_uint64(seed),
                        C.c_uint32(step_index), C.byref(st), _stream(stream))
    for k in range(3):
        app[k].count = int(a[k].count)
    if check:
        _check(rc)
    return rc, st


def step_merged(tables: Tables, main: list, fields: list, app: list, dt: float, seed: int, step_index: int,
                cfg: StepCfg | None = None, stream=None, check: bool = True) -> tuple[int, StepStats]:
    """step() then merge() in one call, the photons merged inside the step
    (qed_step_merged); updates main counts and app counts."""
    cfg = cfg if cfg is not None else step_cfg()
    e = _ensemble(main, fields)
    for s in app:
        s.count = 0
    a = (CAppend * 3)(*[s.c() for s in app])
    st = StepStats()
    rc = lib().qed_step_merged(tables.handle, C.byref(cfg), C.byref(e), a, float(dt), C.c_uint64(seed),
                               C.c_uint32(step_index), C.byref(st), _stream(stream))
    for k in range(3):
        app[k].count = int(a[k].count)
        main[k].count = int(e.s[k].count)
    if check:
        _check(rc)
    return rc, st


def validate(main: list, fields: list, stream=None) -> tuple[int, list[int]]:
    """qed_validate: (status, particles with non-finite values per species)."""
    e = _ensemble(main, fields)
    bad = (C.c_int64 * 3)()
    rc = lib().qed_validate(C.byref(e), bad, _stream(stream))
    return rc, [int(b) for b in bad]


def merge(main: list, fields: list, app: list, stream=None, noalloc: bool = False):
    """qed_merge, or qed_merge_noalloc (scratch in a fixed device array) when noalloc is set."""
    e = _ensemble(main, fields)
    a = (CAppend * 3)(*[s.c() for s in app])
    fn = lib().qed_merge_noalloc if noalloc else lib().qed_merge
    _check(fn(C.byref(e), a, _stream(stream)))
    for k in range(3):
        main[k].count = int(e.s[k].count)


def resample_cfg(photon_energy_min: float = 0.0, target=(0, 0, 0), seed: int = 0, step: int = 0) -> ResampleCfg:
    cfg = ResampleCfg()
    lib().qed_resample_cfg_default(C.byref(cfg))
    cfg.photon_energy_min = float(photon_energy_min)
    for k in range(3):
        cfg.target[k] = int(target[k])
    cfg.seed, cfg.step = int(seed), int(step)
    return cfg


def resample(main: list, fields: list, cfg: ResampleCfg, stream=None) -> ResampleStats:
    """Photon energy filter and global leveling of the ensemble (after merge);
    updates the stores' counts."""
    e = _ensemble(main, fields)
    st = ResampleStats()
    _check(lib().qed_resample(C.byref(e), C.byref(cfg), C.byref(st), _stream(stream)))
    for k in range(3):
        main[k].count = int(e.s[k].count)
    return st


# ----------------------------------------------------------------------------- grid fields
class Grid1d:
    """Fields at nx nodes x_i = x0 + i length / nx of a periodic line along x
    (six device arrays of the step's dtype)."""

    def __init__(self, nx: int, x0: float, length: float, dtype=None, device="cuda"):
        torch = _torch()
        self.dtype = dtype or torch.float32
        self.nx, self.x0, self.length = int(nx), float(x0), float(length)
        self.g = [torch.zeros(max(self.nx, 1), dtype=self.dtype, device=device) for _ in range(6)]

    @classmethod
    def from_array(cls, nodes, x0: float, length: float, dtype=None, device="cuda"):
        """nodes: [nx, 6] (ex ey ez bx by bz) on the host."""
        torch = _torch()
        nodes = np.asarray(nodes, dtype=np.float64).reshape(-1, 6)
        g = cls(nodes.shape[0], x0, length, dtype, device)
        t = torch.as_tensor(nodes).to(device=device, dtype=g.dtype)
        for k in range(6):
            g.g[k].copy_(t[:, k])
        return g

    def c(self) -> CGrid1d:
        return CGrid1d(_dtype_code(self.dtype), self.nx, self.x0, self.length, *[_ptr(t) for t in self.g])

    def host(self) -> np.ndarray:
        return np.stack([t[:self.nx].double().cpu().numpy() for t in self.g], axis=1)


def box(lo=(0.0, 0.0, 0.0), length=(0.0, 0.0, 0.0)) -> CBox:
    """Periodic box [lo, lo + length) per axis; length 0 leaves an axis unwrapped."""
    b = CBox()
    for k in range(3):
        b.lo[k], b.len[k] = float(lo[k]), float(length[k])
    return b


def field_buffers(capacity: int, dtype=None, device="cuda") -> Fields:
    """Per-particle field arrays (stride 1) for gather_fields and step."""
    torch = _torch()
    dtype = dtype or torch.float32
    return Fields(*[torch.zeros(max(int(capacity), 1), dtype=dtype, device=device) for _ in range(6)], stride=1)


def standing_wave(grid: Grid1d, e0: float, k: float, omega: float, xc: float, t: float, stream=None):
    """Nodes of the standing circularly polarised wave at time t (qed_grid_standing_wave)."""
    g = grid.c()
    _check(lib().qed_grid_standing_wave(C.byref(g), float(e0), float(k), float(omega), float(xc), float(t),
                                        _stream(stream)))


def gather_fields(main: list, grid: Grid1d, box_: CBox, out: list, stream=None):
    """Wraps positions into the box and interpolates the grid at them into
    out[s] (Fields with stride 1, capacity >= count)."""
    for s in range(3):
        if main[s].count > 0 and (out[s].stride != 1 or out[s].ex.numel() < main[s].count):
            raise SfqedError(1, f"gather_fields: output of species {s} holds fewer than {main[s].count} particles")
    e = _ensemble(main, out)
    def arrays(f):
        ts = (f.ex, f.ey, f.ez, f.bx, f.by, f.bz)
        return CFieldArrays(*[_ptr(t) for t in ts], min(t.numel() for t in ts))

    o = (CFieldArrays * 3)(*[arrays(f) for f in out])
    g = grid.c()
    _check(lib().qed_gather_fields(C.byref(e), C.byref(g), C.byref(box_), o, _stream(stream)))


def eval_rate(tables: Tables, process: int, chi, energy, stream=None):
    torch = _torch()
    out = torch.empty_like(chi)
    _check(lib().qed_eval_rate(tables.handle, process, _dtype_code(chi.dtype), _ptr(chi), _ptr(energy), _ptr(out),
                               chi.numel(), _stream(stream)))
    return out


def eval_particles(tables: Tables, species: int, store: Store, fields: Fields, n: int | None = None, stream=None):
    torch = _torch()
    n = store.count if n is None else n
    chi = torch.empty(n, dtype=store.dtype, device=store.px.device)
    w = torch.empty_like(chi)
    f = fields.c()
    _check(lib().qed_eval_particles(tables.handle, species, _dtype_code(store.dtype), _ptr(store.px), _ptr(store.py),
                                    _ptr(store.pz), C.byref(f), n, _ptr(chi), _ptr(w), _stream(stream)))
    return chi, w


def sample(tables: Tables, process: int, chi, k, stream=None):
    """delta (emission) or xi (pairs) for raw 32-bit uniforms k (int32 tensor holding the bits)."""
    torch = _torch()
    out = torch.empty_like(chi)
    _check(lib().qed_sample(tables.handle, process, _dtype_code(chi.dtype), _ptr(chi), _ptr(k), _ptr(out),
                            chi.numel(), _stream(stream)))
    return out


# ----------------------------------------------------------------------------- surrogate
def mlp_cfg(**overrides) -> MlpCfg:
    cfg = MlpCfg()
    lib().qed_mlp_cfg_default(C.byref(cfg))
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


def train_cfg(**overrides) -> TrainCfg:
    cfg = TrainCfg()
    lib().qed_mlp_train_cfg_default(C.byref(cfg))
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


class Mlp:
    """The inverse-CDF surrogate network on the current device (qed_mlp)."""

    def __init__(self, params=None, cfg: MlpCfg | None = None, **cfg_overrides):
        h = C.c_void_p()
        self.cfg = cfg if cfg is not None else mlp_cfg(**cfg_overrides)
        _check(lib().qed_mlp_create(C.byref(self.cfg), C.byref(h)))
        self.handle = h
        if params is not None:
            self.set_params(params)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.qed_mlp_free(h)
            self.handle = None

    def set_params(self, params, stream=None):
        a = np.ascontiguousarray(params, dtype=np.float32)
        assert a.shape == (MLP_PARAMS,), a.shape
        _check(lib().qed_mlp_set_params(self.handle, a.ctypes.data_as(C.c_void_p), _stream(stream)))

    def params(self, stream=None) -> np.ndarray:
        a = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(lib().qed_mlp_get_params(self.handle, a.ctypes.data_as(C.c_void_p), _stream(stream)))
        return a

    def forward(self, x, stream=None):
        """Network outputs for a device float32 tensor x [n, 2]."""
        torch = _torch()
        assert x.dtype == torch.float32 and x.is_contiguous() and x.dim() == 2 and x.shape[1] == 2
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _check(lib().qed_mlp_forward(self.handle, _ptr(x), _ptr(y), x.shape[0], _stream(stream)))
        return y

    def grad(self, x, t, stream=None):
        """(gradient [4417], loss) of the mean squared error on device tensors x [n, 2], t [n]."""
        torch = _torch()
        assert x.dtype == torch.float32 and t.dtype == torch.float32 and x.is_contiguous() and t.is_contiguous()
        assert x.dim() == 2 and x.shape[1] == 2 and t.shape == (x.shape[0],)
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(lib().qed_mlp_grad(self.handle, _ptr(x), _ptr(t), x.shape[0], _ptr(g), _ptr(loss), _stream(stream)))
        return g, loss

    def train(self, x, t, cfg: TrainCfg, record_loss=True, stream=None):
        """cfg.steps Adam steps on device data; returns the per-step loss tensor (or None)."""
        torch = _torch()
        assert x.dtype == torch.float32 and t.dtype == torch.float32 and x.is_contiguous() and t.is_contiguous()
        assert x.dim() == 2 and x.shape[1] == 2 and t.shape == (x.shape[0],)
        loss = torch.empty(max(cfg.steps, 1), dtype=torch.float32, device=x.device) if record_loss else None
        _check(lib().qed_mlp_train(self.handle, _ptr(x), _ptr(t), x.shape[0], C.byref(cfg), _ptr(loss),
                                   _stream(stream)))
        return loss

    def sample(self, tables: "Tables", chi, k, stream=None):
        """Emission delta for float32 chi and raw uniforms k (int32 tensor holding the bits)."""
        torch = _torch()
        assert chi.dtype == torch.float32 and chi.is_contiguous() and k.is_contiguous() and k.numel() == chi.numel()
        out = torch.empty_like(chi)
        _check(lib().qed_sample_mlp(tables.handle, self.handle, _ptr(chi), _ptr(k), _ptr(out), chi.numel(),
                                    _stream(stream)))
        return out


def load_surrogate(path=None) -> np.ndarray:
    """Trained parameters shipped with the package (surrogate_rad.npz)."""
    path = Path(path) if path is not None else Path(__file__).resolve().parent / "surrogate_rad.npz"
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32)
