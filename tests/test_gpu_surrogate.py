"""The trained emission surrogate shipped with the package, against the FP64
oracle on draws it was not trained on (seed 7; training used seed 0).

Spectral error: L1 = sum over 256 equal bins of log10(delta) in [-12, 0] of
|n_b(surrogate) - n_b(oracle)| / N with paired draws (the same chi and r on
both sides), chi log-uniform in [1e-2, 1e2].  Target: L1 <= 1e-3.

What the network gains over the table method is measured, not assumed: the
same draws go through a table of the network's size (its inference bytes:
BF16 W2 plus FP32 vectors) built by the library with the same interpolation
as the default table.  On this hardware the network gains neither accuracy at
equal memory nor speed; the test keeps both numbers honest.
"""
import numpy as np
import pytest

import oracle
import synth

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu
EDGES = np.linspace(-12.0, 0.0, 257)


@pytest.fixture(scope="module")
def draws():
    groups, per = 4000, 1000           # 4e6 paired draws
    chi, k = synth.surrogate_draws(np.arange(groups), per, seed=7)
    kk = k.astype(np.float64)
    r = (kk + 0.5) * 2.0**-32
    rc = ((2.0**32 - 1.0 - kk) + 0.5) * 2.0**-32
    d, _ = oracle.sample_rad_grid(chi.astype(np.float64), r, rc)
    return np.repeat(chi, per), k.ravel(), np.log(d.ravel())


def l1(ld_model, ld_ref):
    h, _ = np.histogram(ld_model / np.log(10.0), EDGES)
    h0, _ = np.histogram(ld_ref / np.log(10.0), EDGES)
    return np.abs(h - h0).sum() / ld_ref.size


def run(torch, fn, chi, k):
    c = torch.tensor(chi, device="cuda")
    kt = torch.tensor(k.view(np.int32), device="cuda")
    return np.log(fn(c, kt).double().cpu().numpy())


def test_shipped_surrogate_spectral_error(draws):
    torch, sf = need_gpu()
    chi, k, ld = draws
    tabs = sf.Tables()
    net = sf.Mlp(sf.load_surrogate())
    lm = run(torch, lambda c, kt: net.sample(tabs, c, kt), chi, k)
    lt = run(torch, lambda c, kt: sf.sample(tabs, 0, c, kt), chi, k)
    e_net, e_tab = l1(lm, ld), l1(lt, ld)
    print(f"paired L1: surrogate {e_net:.3e}, FP32 table {e_tab:.3e}; "
          f"rms d ln(delta): surrogate {np.sqrt(np.mean((lm - ld) ** 2)):.3e}")
    assert e_net <= 1e-3, e_net
    assert e_tab <= 1e-4, e_tab
    # per-draw agreement: the bulk within 0.5%, no draw off by more than 20% in delta
    e = np.abs(lm - ld)
    assert np.quantile(e, 0.99) < 5e-3 and e.max() < 0.2, (np.quantile(e, 0.99), e.max())


def test_gain_over_table_at_equal_memory(draws):
    torch, sf = need_gpu()
    chi, k, ld = draws
    net_bytes = 64 * 64 * 2 + (64 * 5 + 1) * 4   # BF16 W2 + FP32 W1, b1, b2, w3, b3
    rows, cols = 23, 103                          # 9476 bytes of FP32 nodes
    assert abs(rows * cols * 4 - net_bytes) <= 16
    small = sf.Tables(sf.default_table_cfg(rad_rows=rows, rad_cols=cols, rad_chi_min=1e-2, rad_chi_max=1e2))
    tabs = sf.Tables()
    net = sf.Mlp(sf.load_surrogate())
    lm = run(torch, lambda c, kt: net.sample(tabs, c, kt), chi, k)
    ls = run(torch, lambda c, kt: sf.sample(small, 0, c, kt), chi, k)
    e_net, e_small = l1(lm, ld), l1(ls, ld)
    r_net, r_small = np.sqrt(np.mean((lm - ld) ** 2)), np.sqrt(np.mean((ls - ld) ** 2))
    print(f"equal memory ({net_bytes} B): paired L1 surrogate {e_net:.3e} vs table {e_small:.3e}; "
          f"rms d ln(delta) {r_net:.3e} vs {r_small:.3e}")
    # measured outcome: the equal-size table is the more accurate sampler
    assert e_small <= e_net and r_small <= r_net
