"""C-ABI contract checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2210_08024_amd import ism

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(ism_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = ism.lib()
    decl = declared_functions()
    assert "ism_chem_cool_step" in decl and "ism_columns6" in decl and "ism_rates" in decl
    for name in decl:
        assert hasattr(L, name), f"libism.so does not export {name}"


def test_params_default_matches_binding_defaults():
    p = ism._Params()
    ism.lib().ism_params_default(ctypes.byref(p))
    d = ism.Params()
    for f, _ in ism._Params._fields_:
        if f != "pad_":
            assert getattr(p, f) == getattr(d, f), f


def test_param_struct_layout():
    assert ctypes.sizeof(ism._Params) == 10 * 8 + 6 * 4
    assert ctypes.sizeof(ism._Grid) == 24


def test_diag_names():
    names = ism.diag_names()
    assert len(names) == ism.ndiag() == 39
    assert names[0] == "xCp" and names[-1] == "C_Hp" and "Lambda" in names
    assert ism.lib().ism_diag_name(99) is None


def _bad(p=None, prec=0):
    p = p or ism.Params()
    cp = p._c()
    rc = ism.lib().ism_chem_cool_step(ctypes.byref(cp), prec, 10, 1.0, *([None] * 17))
    return rc, ism.lib().ism_last_error().decode()


@pytest.mark.parametrize("field,value,msg", [("Zg", 0.0, "Zg"), ("Zd", -1.0, "Zd"), ("eps_sub", 0.0, "eps_sub"),
                                             ("fd_rel", 0.7, "fd_rel"), ("cr_mode", 5, "cr_mode"),
                                             ("max_substeps", 0, "max_substeps"), ("T_floor", 0.0, "T_floor"),
                                             ("order_cells", 3, "order_cells"), ("order_cells", -1, "order_cells")])
def test_invalid_params_rejected_before_launch(field, value, msg):
    p = ism.Params()
    setattr(p, field, value)
    rc, err = _bad(p)
    assert rc == -1 and msg in err


def test_invalid_precision_and_null_arrays():
    rc, err = _bad(prec=7)
    assert rc == -1 and "precision" in err
    rc, err = _bad()
    assert rc == -1 and "NULL" in err
    cp = ism.Params()._c()
    assert ism.lib().ism_chem_cool_step(ctypes.byref(cp), 0, -1, 1.0, *([None] * 17)) == -1
    assert ism.lib().ism_chem_cool_step(ctypes.byref(cp), 0, 10, float("nan"), *([None] * 17)) == -1
    # zero cells is a no-op that succeeds without touching the device
    assert ism.lib().ism_chem_cool_step(ctypes.byref(cp), 0, 0, 1.0, *([None] * 17)) == 0


def test_columns6_argument_checks():
    cp = ism.Params()._c()
    g = ism._Grid(0, 4, 4, 0, 1.0)
    assert ism.lib().ism_columns6(ctypes.byref(g), ctypes.byref(cp), 0, *([None] * 10)) == -1
    assert "grid" in ism.lib().ism_last_error().decode()
    g = ism._Grid(4, 4, 4, 0, -1.0)
    assert ism.lib().ism_columns6(ctypes.byref(g), ctypes.byref(cp), 0, *([None] * 10)) == -1
    g = ism._Grid(4, 4, 4, 0, 1.0)
    assert ism.lib().ism_columns6(ctypes.byref(g), ctypes.byref(cp), 0, *([None] * 10)) == -1
    assert "NULL" in ism.lib().ism_last_error().decode()


def test_init_rejects_missing_or_bad_coefficient_file(tmp_path):
    assert ism.lib().ism_init(0, b"/nonexistent/coeffs.json") == -5
    bad = tmp_path / "bad.json"
    bad.write_text('{"printed": {}, "standin": {}, "tables": {}}')
    assert ism.lib().ism_init(0, str(bad).encode()) == -5
    assert "missing coefficient" in ism.lib().ism_last_error().decode()


def test_surrogate_entry_points_reject_null_handles():
    L = ism.lib()
    assert L.ism_surrogate_create(None, 0) == -1
    assert L.ism_surrogate_destroy(None) == 0
    assert L.ism_surrogate_set_norm(None, None, None, None, None) == -1
    assert L.ism_surrogate_forward(None, None, None, 4, None) == -1
    assert "NULL" in L.ism_last_error().decode()
    assert L.ism_surrogate_backward(None, None, None, None, 4, None) == -1
    assert L.ism_surrogate_train_step(None, None, None, 4, ctypes.c_float(1e-3), None, None) == -1
    assert L.ism_surrogate_get_params(None, None, None) == -1
    assert L.ism_surrogate_set_params(None, None, None) == -1


def test_surrogate_sizes_match_the_reference_network():
    from oracle import mlp
    assert ism.SURR_NPARAM == mlp.n_params() == 34819
    text = open(os.path.join(ROOT, "include", "ism.h")).read()
    assert "#define ISM_SURR_NPARAM 34819" in text
    assert ism.SURR_STATE_FLOATS == 3 * 34819 + 27


def test_ray_trace_rejects_bad_options_before_launch():
    g = ism._Grid(8, 8, 8, 0, 3.0e18)
    cp = ism.Params()._c()
    src = (ism._Source * 1)(ism._Source(1e18, 1e18, 1e18, 1e49, 1e38))
    L = ism.lib()

    def call(opt, nsrc=1, arrays=None):
        o = None if opt is None else ctypes.cast(ctypes.pointer(ism._ArtOptions(*opt)), ctypes.c_void_p)
        rc = L.ism_ray_trace(ctypes.byref(g), ctypes.byref(cp), 0, nsrc, ctypes.cast(src, ctypes.c_void_p), o,
                             *(arrays or [None] * 11), None)
        return rc, L.ism_last_error().decode()

    assert ctypes.sizeof(ism._ArtOptions) == 24
    for opt, msg in (((5, 4, 4.0, 30.0), "level0"), ((0, 14, 4.0, 30.0), "max_level"),
                     ((-1, 4, 4.0, 30.0), "level0"), ((4, 13, 0.0, 30.0), "rays_per_cell"),
                     ((4, 13, float("inf"), 30.0), "rays_per_cell"), ((4, 13, 4.0, 0.0), "tau_max")):
        rc, err = call(opt)
        assert rc == -1 and msg in err, (opt, err)
    rc, err = call(None, nsrc=257)
    assert rc == -1 and "nsrc" in err
    rc, err = call(None)
    assert rc == -1 and "NULL" in err
    # no sources: a no-op that succeeds without touching the device
    assert call(None, nsrc=0)[0] == 0


def test_radiation_force_rejects_bad_arguments_before_launch():
    cp = ism.Params()._c()
    L = ism.lib()
    fake = ctypes.c_void_p(4096)  # never dereferenced: every case fails in the host checks

    def call(opt, ncell=8, arrays=None, dt=0.0, mom=None, etot=None):
        o = None if opt is None else ctypes.cast(ctypes.pointer(ism._ForceOptions(*opt)), ctypes.c_void_p)
        arr = arrays if arrays is not None else [fake] * 5
        rc = L.ism_radiation_force(ctypes.byref(cp), 0, ncell, *arr[:5], o, fake, None, dt, mom, etot, None)
        return rc, L.ism_last_error().decode()

    assert ctypes.sizeof(ism._ForceOptions) == 16
    for opt, msg in (((0.0, 50.0), "T_destroy"), ((float("nan"), 50.0), "T_destroy"),
                     ((1e6, -1.0), "prad_ratio_max"), ((1e6, float("nan")), "prad_ratio_max")):
        rc, err = call(opt)
        assert rc == -1 and msg in err, (opt, err)
    assert "dt_s" in call(None, dt=-1.0)[1]
    assert "dt_s" in call(None, dt=float("inf"))[1]
    assert "etot needs mom" in call(None, etot=fake)[1]
    assert "ncell" in call(None, ncell=-1)[1]
    assert "ncell" in call(None, ncell=1 << 33)[1]
    assert "NULL" in call(None, arrays=[fake, None, fake, fake, fake])[1]
    assert call(None, ncell=0)[0] == 0
