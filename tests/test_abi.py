"""The C ABI without a GPU: the built library loads, exports every function
that include/sfqed.h declares, and its host-only calls behave as declared
(defaults, argument checks that fail before any device work)."""
import ctypes as C
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "sfqed.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(qed_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    import paper_2409_17299_amd as sf
    if not sf.LIB_PATH.exists():
        pytest.skip("libsfqed.so is not built")
    return sf.lib()


def test_header_parses():
    names = declared_functions()
    for must in ("qed_build_rate_tables", "qed_step", "qed_merge", "qed_sample", "qed_mlp_train", "qed_sample_mlp"):
        assert must in names
    assert len(names) >= 25


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_defaults_and_version(L):
    import paper_2409_17299_amd as sf
    assert L.qed_abi_version() == 1
    t = sf.default_table_cfg()
    assert t.rad_rows == 70 and t.rad_cols == 265 and t.f64_refine == 4
    m = sf.mlp_cfg()
    assert abs(m.chi_min - 1e-2) < 1e-9 and abs(m.chi_max - 1e2) < 1e-4 and m.out_scale == 10.0
    tc = sf.train_cfg()
    assert tc.batch > 0 and tc.steps > 0 and 0 < tc.beta1 < 1
    assert L.qed_status_str(0) == b"ok"


def test_argument_errors_without_device(L):
    import paper_2409_17299_amd as sf
    # null handles and bad configurations are rejected before any HIP call
    assert L.qed_step(None, None, None, None, 1.0, 0, 0, None, None) == 1
    assert L.qed_merge(None, None, None) == 1
    assert L.qed_validate(None, None, None) == 1
    c = sf.step_cfg()
    assert c.validate == 0 and sf.step_cfg(validate=True).validate == 1
    assert L.qed_mlp_create(None, None) == 1
    bad = sf.mlp_cfg(chi_min=-1.0)
    h = C.c_void_p()
    assert L.qed_mlp_create(C.byref(bad), C.byref(h)) == 1
    assert L.qed_sample_mlp(None, None, None, None, None, 0, None) == 1
    cfg = sf.default_table_cfg(rad_rows=2)
    assert L.qed_build_rate_tables(C.byref(cfg), None, C.byref(h)) == 1


def test_grid_argument_errors_without_device(L):
    import paper_2409_17299_amd as sf
    assert L.qed_grid_standing_wave(None, 1.0, 1.0, 1.0, 0.0, 0.0, None) == 1
    g = sf.CGrid1d(sf.F32, 0, 0.0, 1.0)             # no nodes, no arrays
    assert L.qed_grid_standing_wave(C.byref(g), 1.0, 1.0, 1.0, 0.0, 0.0, None) == 1
    assert L.qed_gather_fields(None, None, None, None, None) == 1
    e = sf.CEnsemble()
    b = sf.box()
    out = (sf.CFieldArrays * 3)()
    assert L.qed_gather_fields(C.byref(e), C.byref(g), C.byref(b), out, None) == 1
    b_bad = sf.box((0, 0, 0), (float("nan"), 0, 0))
    g_ok_shape = sf.CGrid1d(sf.F32, 8, 0.0, 1.0, *([C.c_void_p(16)] * 6))  # never dereferenced: the box fails first
    assert L.qed_gather_fields(C.byref(e), C.byref(g_ok_shape), C.byref(b_bad), out, None) == 1


def test_merge_noalloc_limit_without_device(L):
    """qed_merge_noalloc refuses more photons than its fixed scratch holds
    before any HIP call (the pointers below are never dereferenced)."""
    import paper_2409_17299_amd as sf
    fake = C.c_void_p(256)
    e = sf.CEnsemble()
    e.dtype = sf.F32
    for s in range(3):
        sp = e.s[s]
        sp.px = sp.py = sp.pz = sp.w = sp.tau = sp.id = sp.alive = fake
        sp.count, sp.capacity = 0, 1
    n = (1 << 28) + 1  # one photon past 2^17 tiles of 2048
    e.s[2].count = e.s[2].capacity = n
    a = (sf.CAppend * 3)(*[sf.CAppend(fake, None, 0, 1) for _ in range(3)])
    assert L.qed_merge_noalloc(C.byref(e), a, None) == 1
    assert b"limit" in L.qed_last_error()
    assert L.qed_merge_noalloc(None, None, None) == 1


def test_short_fields_rejected_without_device(L):
    """Per-particle fields (stride 1) must hold at least as many entries as
    the species has particles; the step, the merged step, the validation pass
    and qed_eval_particles refuse shorter ones before any HIP call (the
    pointers below are never dereferenced)."""
    import paper_2409_17299_amd as sf
    fake = C.c_void_p(256)
    e = sf.CEnsemble()
    e.dtype = sf.F32
    for s in range(3):
        sp = e.s[s]
        sp.px = sp.py = sp.pz = sp.w = sp.tau = sp.id = sp.alive = fake
        sp.count, sp.capacity = 0, 1
        e.f[s] = sf.CFields(*([fake] * 6), 0, 0)
    e.s[2].count = e.s[2].capacity = 100
    e.f[2] = sf.CFields(*([fake] * 6), 1, 99)
    a = (sf.CAppend * 3)(*[sf.CAppend(fake, None, 0, 1) for _ in range(3)])
    t = C.c_void_p(512)
    cfg = sf.step_cfg()
    st = sf.StepStats()
    for fn in (L.qed_step, L.qed_step_merged):
        assert fn(t, C.byref(cfg), C.byref(e), a, 1.0, 0, 0, C.byref(st), None) == 1
        assert b"fields of species 2" in L.qed_last_error()
    bad = (C.c_int64 * 3)()
    assert L.qed_validate(C.byref(e), bad, None) == 1
    assert b"fields of species 2" in L.qed_last_error()
    f = sf.CFields(*([fake] * 6), 1, 99)
    assert L.qed_eval_particles(t, 2, sf.F32, fake, fake, fake, C.byref(f), 100, fake, fake, None) == 1
    f2 = sf.CFields(*([fake] * 6), 2, 1000)  # a stride other than 0 or 1
    assert L.qed_eval_particles(t, 2, sf.F32, fake, fake, fake, C.byref(f2), 100, fake, fake, None) == 1


def test_short_gather_output_rejected_without_device(L):
    """qed_gather_fields refuses output arrays with fewer entries than
    particles before any HIP call (pointers never dereferenced)."""
    import paper_2409_17299_amd as sf
    fake = C.c_void_p(256)
    e = sf.CEnsemble()
    e.dtype = sf.F32
    for s in range(3):
        sp = e.s[s]
        sp.px = sp.py = sp.pz = sp.w = sp.tau = sp.id = sp.alive = sp.x = sp.y = sp.z = fake
        sp.count, sp.capacity = 0, 1
    e.s[1].count = e.s[1].capacity = 10
    g = sf.CGrid1d(sf.F32, 8, 0.0, 1.0, *([fake] * 6))
    b = sf.box((0, 0, 0), (1.0, 1.0, 1.0))
    out = (sf.CFieldArrays * 3)(*[sf.CFieldArrays(*([fake] * 6), 9) for _ in range(3)])
    assert L.qed_gather_fields(C.byref(e), C.byref(g), C.byref(b), out, None) == 1
    assert b"fewer entries" in L.qed_last_error()
