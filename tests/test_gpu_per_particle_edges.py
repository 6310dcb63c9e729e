"""Edges of the per-particle entry points (qed_eval_particles, qed_sample,
qed_eval_rate): fields shared by all particles (stride 0) give exactly what
the same field repeated per particle gives, and empty inputs are accepted."""
import numpy as np
import pytest

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, sf = need_gpu()
    return torch, sf, sf.Tables()


def _store(sf, torch, p, dtype, photon):
    n = p.shape[0]
    ids = np.arange(n, dtype=np.uint64)
    return sf.Store.from_arrays(p, np.ones(n), np.ones(n), ids, dtype=dtype, photon=photon, capacity=max(n, 1))


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_shared_fields_equal_repeated_fields(env, dtype_name):
    torch, sf, tabs = env
    dtype = getattr(torch, dtype_name)
    rng = np.random.default_rng(21)
    n = 1027
    for species in (0, 2):
        e = np.exp(rng.uniform(np.log(1e2), np.log(1e4), n))
        d = rng.normal(size=(n, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        p = d * (np.sqrt(e * e - 1.0) if species < 2 else e)[:, None]
        f = np.array([[1e-3, -2e-3, 5e-4, 3e-3, 1e-3, -2e-3]])
        st = _store(sf, torch, p, dtype, species == 2)
        shared = sf.Fields.from_array(f, dtype)
        repeated = sf.Fields.from_array(np.repeat(f, n, axis=0), dtype)
        assert shared.stride == 0 and repeated.stride == 1
        chi_a, w_a = sf.eval_particles(tabs, species, st, shared)
        chi_b, w_b = sf.eval_particles(tabs, species, st, repeated)
        a = torch.stack([chi_a, w_a]).cpu().numpy()
        b = torch.stack([chi_b, w_b]).cpu().numpy()
        assert np.all(np.isfinite(a)) and np.any(a[1] > 0)
        assert np.array_equal(a, b), (dtype_name, species)


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_empty_inputs(env, dtype_name):
    torch, sf, tabs = env
    dtype = getattr(torch, dtype_name)
    st = _store(sf, torch, np.zeros((0, 3)), dtype, False)
    f = sf.Fields.from_array(np.zeros((1, 6)), dtype)
    chi, w = sf.eval_particles(tabs, 0, st, f)
    assert chi.numel() == 0 and w.numel() == 0
    empty = torch.zeros(0, dtype=dtype, device="cuda")
    k = torch.zeros(0, dtype=torch.int32, device="cuda")
    for proc in (0, 1):
        assert sf.sample(tabs, proc, empty, k).numel() == 0
        assert sf.eval_rate(tabs, proc, empty, empty).numel() == 0
    torch.cuda.synchronize()
