"""Helpers of the GPU parity tests: run one workload through the HIP library and
through the oracle on identical inputs, and compare the results."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def need_gpu():
    import pytest
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_17299_amd as sf
    sf.lib()  # raises if the HIP library is missing
    return torch, sf


def cast_inputs(wl: synth.Workload, np_dtype):
    """Round momenta and fields to the step dtype; both sides then see the same values."""
    out = []
    for sp in wl.species:
        out.append(dict(p=sp.p.astype(np_dtype).astype(np.float64),
                        fields=sp.fields.astype(np_dtype).astype(np.float64),
                        w=sp.w.astype(np.float32).astype(np.float64), tau=sp.tau.copy(), id=sp.id.copy()))
    return out


def _x(positions, x0, s, n):
    if not positions:
        return None
    return x0 if (x0 is not None and s == 0) else np.zeros((n, 3))


def run_gpu(sf, torch, tabs, wl, inputs, dtype, cap, cfg, seed=0, step_index=0, positions=False, x0=None):
    """x0: positions of the electrons (others start at 0) when positions are on."""
    main, fields, app = [], [], []
    for s, d in enumerate(inputs):
        n = d["id"].size
        main.append(sf.Store.from_arrays(d["p"], d["w"], d["tau"], d["id"], dtype=dtype, photon=s == 2,
                                         capacity=max(n, 1), x=_x(positions, x0, s, n)))
        fields.append(sf.Fields.from_array(d["fields"] if d["fields"].shape[0] else np.zeros((1, 6)), dtype))
        app.append(sf.AppendBuffer(cap[s], dtype, positions=positions))
    rc, st = sf.step(tabs, main, fields, app, wl.dt, seed, step_index, cfg, check=False)
    torch.cuda.synchronize()
    return rc, st, main, fields, app


def run_oracle(wl, inputs, cap, seed=0, step_index=0, x0=None, **kw):
    main, fields = [], []
    for s, d in enumerate(inputs):
        n = d["id"].size
        main.append(oracle.Store.from_arrays(d["p"], d["w"], d["tau"], d["id"], capacity=max(n, 1),
                                             x=_x(kw.get("positions", False), x0, s, n)))
        fields.append(d["fields"] if d["fields"].shape[0] else np.zeros((1, 6)))
    app = [oracle.Store(c) for c in cap]
    rc, st = oracle.step(main, fields, app, wl.dt, seed, step_index, **kw)
    return rc, st, main, app


def by_id(ids: np.ndarray) -> dict:
    return {int(v): i for i, v in enumerate(ids)}


def compare_species(g: dict, o_store, rtol_p, atol_tau, rtol_tb=None, check_order=True):
    """Element-wise comparison of one species; returns (n_matched, n_only_gpu, n_only_oracle, max rel p err)."""
    n_o = o_store.count
    o_ids = o_store.id[:n_o]
    g_ids = g["id"]
    if check_order and g_ids.size == n_o and np.array_equal(g_ids, o_ids):
        idx_g = np.arange(n_o)
        idx_o = np.arange(n_o)
    else:
        om = by_id(o_ids)
        pairs = [(i, om[int(v)]) for i, v in enumerate(g_ids) if int(v) in om]
        idx_g = np.array([a for a, _ in pairs], dtype=np.int64)
        idx_o = np.array([b for _, b in pairs], dtype=np.int64)
    pg, po = g["p"][idx_g], o_store.p[idx_o]
    scale = np.maximum(np.linalg.norm(po, axis=1), 1e-300)
    err = np.linalg.norm(pg - po, axis=1) / scale
    return idx_g, idx_o, err
