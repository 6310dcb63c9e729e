"""qed_merge_noalloc (scratch in a fixed device array) against qed_merge.

Two calls in a row on the same device, the second on a smaller ensemble: the
fixed array keeps the first call's contents, so the second call must clear and
re-epoch what it needs.  Arrays, order and counts must equal qed_merge's bit
for bit.  (The size limit is checked on the CPU, in test_abi.py.)
"""
import numpy as np
import pytest

import synth
from gpu_util import cast_inputs, need_gpu, run_gpu

pytestmark = pytest.mark.gpu


def _stepped(sf, torch, tabs, stride, dtype_name):
    np_dtype = np.float32 if dtype_name == "float32" else np.float64
    dtype = getattr(torch, dtype_name)
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, stride)] * 2 +
                             [np.arange(0, 2_000_000, stride // 2)])
    inp = cast_inputs(wl, np_dtype)
    n = sum(d["id"].size for d in inp)
    cap = [n * 30, n * 30, n * 200]
    rc, st, gm, gf, ga = run_gpu(sf, torch, tabs, wl, inp, dtype, cap, sf.step_cfg(push=False, gamma_min=2.0))
    assert rc == 0 and st.n_pair > 0
    return gm, gf, ga, dtype


def _grown(sf, torch, gm, ga, dtype):
    out = []
    for s in range(3):
        h = gm[s].host()
        b = sf.Store.from_arrays(h["p"], h["w"], h["tau"], h["id"], dtype=dtype, photon=s == 2,
                                 capacity=gm[s].count + ga[s].count)
        if s == 2:
            b.alive[:gm[s].count] = gm[s].alive[:gm[s].count]
        out.append(b)
    return out


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_merge_noalloc_equals_merge(dtype_name):
    torch, sf = need_gpu()
    tabs = sf.Tables()
    for call, stride in enumerate([20_000, 80_000]):  # the second input is smaller
        gm, gf, ga, dtype = _stepped(sf, torch, tabs, stride, dtype_name)
        ref = _grown(sf, torch, gm, ga, dtype)
        got = _grown(sf, torch, gm, ga, dtype)
        sf.merge(ref, gf, ga)
        sf.merge(got, gf, ga, noalloc=True)
        torch.cuda.synchronize()
        for s in range(3):
            assert got[s].count == ref[s].count
            hr, hg = ref[s].host(), got[s].host()
            for k in hr:
                assert np.array_equal(hr[k], hg[k]), (call, s, k)
        print(f"{dtype_name} call {call}: merged counts {[b.count for b in got]} equal to qed_merge")

