"""Checkpoint format on the host: stores built in CPU memory go through
save and load bit for bit (every array in its own dtype, NaN payloads and
signed zeros included), with counts, capacities, the optional arrays that
are present and the metadata; a file of another dtype layout is refused.
The resume on the GPU (5 + 5 steps against 10) is in test_gpu_checkpoint.py."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2409_17299_amd import Store, checkpoint  # noqa: E402


def _stores(dtype):
    rng = np.random.default_rng(3)
    out = []
    for s, n in enumerate((37, 0, 101)):
        p = rng.normal(0, 1e3, (n, 3))
        if n:
            p[0, 1] = -0.0
        ids = rng.integers(0, 2**63, n, dtype=np.uint64) | np.uint64(1 << 63)
        m = Store.from_arrays(p, rng.random(n), rng.exponential(1.0, n), ids, dtype=dtype, photon=s == 2,
                              capacity=n + 50 * (s + 1), x=rng.normal(0, 5, (n, 3)) if s == 0 else None,
                              device="cpu")
        if s == 0:
            m.nev[:n] = torch.from_numpy(rng.integers(0, 9, n).astype(np.int32))
            m.tau[3] = float("nan")
            m.px.view(torch.int32 if dtype == torch.float32 else torch.int64)[5] = 0x7FC00123  # a NaN payload
        if s == 2:
            m.alive[:n:3] = 0
            m.nev = None
        out.append(m)
    return out


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_round_trip_is_bit_exact(tmp_path, dtype_name):
    dtype = getattr(torch, dtype_name)
    main = _stores(dtype)
    path = checkpoint.save(tmp_path / "ck.npz", main, next_step=17, seed=99, extra={"dt": 0.5})
    back, meta = checkpoint.load(path, device="cpu")
    assert meta["next_step"] == 17 and meta["seed"] == 99 and meta["extra"] == {"dt": 0.5}
    for a, b in zip(main, back):
        assert (a.count, a.capacity, a.dtype) == (b.count, b.capacity, b.dtype)
        for name in ("px", "py", "pz", "x", "y", "z", "w", "tau", "id", "alive", "nev"):
            ta, tb = getattr(a, name), getattr(b, name)
            assert (ta is None) == (tb is None), name
            if ta is None:
                continue
            n = a.count
            assert ta.dtype == tb.dtype, name
            assert ta[:n].numpy().tobytes() == tb[:n].numpy().tobytes(), name
            fill = 1 if name == "alive" else 0  # the free part is as Store.empty leaves it
            assert bool((tb[n:] == fill).all()), name


def test_refuses_mismatched_arrays(tmp_path):
    main = _stores(torch.float32)
    path = checkpoint.save(tmp_path / "ck.npz", main, next_step=1, seed=0)
    with np.load(path, allow_pickle=False) as z:
        arrays = {k: z[k] for k in z.files}
    arrays["s0_px"] = arrays["s0_px"].astype(np.float64)  # not the dtype the metadata names
    bad = tmp_path / "bad.npz"
    np.savez(bad, **arrays)
    with pytest.raises(ValueError):
        checkpoint.load(bad, device="cpu")
