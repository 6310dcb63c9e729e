"""Trains the emission inverse-CDF surrogate on the GPU with the library's own
kernels (qed_mlp_train: BF16-MFMA forward and backward, FP32 Adam).

Reads a directory of draws (x.npy float32 [n, 2] network inputs, t.npy float32
[n] targets, as written by the FP64 draw generator) and writes an .npz with the
parameters (`params`, float32 [4417]), the input/output configuration and the
loss history.  Progress is printed after every chunk of steps.

    python -m paper_2409_17299_amd.train_surrogate --data DIR --out surrogate_rad.npz
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def initial_params(seed: int) -> np.ndarray:
    """Weights and biases uniform in +-1/sqrt(fan_in) (the usual dense-layer start)."""
    g = np.random.default_rng(seed)
    parts = []
    for shape, fan_in in (((64, 2), 2), ((64,), 2), ((64, 64), 64), ((64,), 64), ((64,), 64), ((1,), 64)):
        b = 1.0 / np.sqrt(fan_in)
        parts.append(g.uniform(-b, b, size=shape).ravel())
    return np.concatenate(parts).astype(np.float32)


def train(data: Path, out: Path, steps: int, batch: int, lr_max: float, lr_min: float, warmup: float, seed: int,
          chunk: int, init: str | None = None, limit: int | None = None):
    import torch

    import paper_2409_17299_amd as sf

    x = np.load(data / "x.npy", mmap_mode="r")
    t = np.load(data / "t.npy", mmap_mode="r")
    if limit:
        x, t = x[:limit], t[:limit]
    n = t.shape[0]
    xt = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    tt = torch.empty((n,), dtype=torch.float32, device="cuda")
    step_rows = 1 << 24
    for a in range(0, n, step_rows):  # upload in slices (host memory stays small)
        b = min(n, a + step_rows)
        xt[a:b].copy_(torch.from_numpy(np.ascontiguousarray(x[a:b])))
        tt[a:b].copy_(torch.from_numpy(np.ascontiguousarray(t[a:b])))
    torch.cuda.synchronize()
    p0 = sf.load_surrogate(init) if init else initial_params(seed)
    net = sf.Mlp(p0)
    losses = []
    t0 = time.time()
    for s0 in range(0, steps, chunk):
        cfg = sf.train_cfg(steps=min(chunk, steps - s0), batch=batch, schedule_start=s0, schedule_len=steps,
                           lr_max=lr_max, lr_min=lr_min, warmup=warmup, seed=seed, shuffle=1)
        loss = net.train(xt, tt, cfg)
        torch.cuda.synchronize()
        lv = loss.cpu().numpy()
        losses.append(lv)
        print(f"  steps {s0 + cfg.steps}/{steps}: loss {lv.mean():.4e} (last {lv[-min(100, lv.size):].mean():.4e}), "
              f"{time.time() - t0:.1f} s", flush=True)
    params = net.params()
    hist = np.concatenate(losses) if losses else np.zeros(0, np.float32)
    c = net.cfg
    meta = {"steps": steps, "batch": batch, "lr_max": lr_max, "lr_min": lr_min, "warmup": warmup, "seed": seed,
            "n_data": int(n), "seconds": time.time() - t0,
            "cfg": {k: float(getattr(c, k)) for k, _ in c._fields_}}
    out.parent.mkdir(parents=True, exist_ok=True)
    np.savez(out, params=params, loss=hist[:: max(1, hist.size // 2000)], meta=json.dumps(meta))
    print(f"wrote {out} ({meta['seconds']:.1f} s of training)", flush=True)
    return params, hist


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--data", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--steps", type=int, default=200_000)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr-max", type=float, default=3e-3)
    ap.add_argument("--lr-min", type=float, default=1e-6)
    ap.add_argument("--warmup", type=float, default=0.02)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=10_000)
    ap.add_argument("--init", default=None, help="start from the parameters of this .npz")
    ap.add_argument("--limit", type=int, default=None, help="use only the first LIMIT draws")
    a = ap.parse_args(argv)
    train(Path(a.data), Path(a.out), a.steps, a.batch, a.lr_max, a.lr_min, a.warmup, a.seed, a.chunk, a.init,
          a.limit)


if __name__ == "__main__":
    main()
