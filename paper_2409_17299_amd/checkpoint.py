"""Host save and restore of the particle ensemble between global steps
(checkpoint and resume of a long cascade run, Sec. 5).

Every random number a step draws is a function of (seed, particle id, step
index, event index) (Philox4x32-10, the counter-based generator of Sec. 3),
and the library keeps no other state from one step to the next.  An ensemble
saved after step k - 1 and restored into fresh device memory therefore
continues with step k exactly as the run that never stopped.  A checkpoint
holds the live part of every array of the three species bit for bit (in
their own dtypes), the counts and capacities, the seed and the index of the
next step, in one .npz file (no pickled objects)."""
from __future__ import annotations

import json
import os
from pathlib import Path

import numpy as np

from . import Store

_ARRAYS = ("px", "py", "pz", "x", "y", "z", "w", "tau", "id", "alive", "nev")
_FORMAT = 1


def save(path, main: list, next_step: int, seed: int, extra: dict | None = None) -> Path:
    """Writes the three stores (electrons, positrons, photons) to `path`
    (written to a temporary file first, then renamed over it).  extra: small
    JSON-serialisable values kept with the checkpoint."""
    path = Path(path)
    arrays = {}
    meta = {"format": _FORMAT, "next_step": int(next_step), "seed": int(seed), "extra": extra or {},
            "dtype": str(main[0].dtype).replace("torch.", ""), "species": []}
    for s, m in enumerate(main):
        have = [a for a in _ARRAYS if getattr(m, a) is not None]
        meta["species"].append({"count": int(m.count), "capacity": int(m.capacity), "arrays": have})
        for a in have:
            arrays[f"s{s}_{a}"] = getattr(m, a)[: m.count].cpu().numpy()
    arrays["meta"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    tmp = path.with_name(path.name + ".tmp.npz")
    np.savez(tmp, **arrays)
    os.replace(tmp, path)
    return path


def load(path, device="cuda") -> tuple[list, dict]:
    """The stores of a checkpoint, in new device memory with the saved
    capacities, and its metadata (next_step, seed, extra)."""
    import torch
    with np.load(Path(path), allow_pickle=False) as z:
        meta = json.loads(bytes(z["meta"]).decode())
        if meta.get("format") != _FORMAT:
            raise ValueError(f"unknown checkpoint format {meta.get('format')}")
        dtype = getattr(torch, meta["dtype"])
        main = []
        for s, sm in enumerate(meta["species"]):
            have = set(sm["arrays"])
            m = Store.empty(sm["capacity"], dtype, photon="alive" in have, positions="x" in have,
                            nev="nev" in have, device=device)
            n = sm["count"]
            for a in have:
                src = torch.from_numpy(np.ascontiguousarray(z[f"s{s}_{a}"]))
                dst = getattr(m, a)
                if src.dtype != dst.dtype or src.numel() != n:
                    raise ValueError(f"species {s} array {a}: {src.dtype}[{src.numel()}], expected {dst.dtype}[{n}]")
                dst[:n] = src.to(device)
            m.count = n
            main.append(m)
    return main, meta
