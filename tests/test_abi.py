"""CPU checks of the C-ABI boundary: the library loads without a GPU, exports every function
include/nb.h declares, and rejects invalid parameters before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2405_01420_amd import nb, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(nb_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = nb.lib()
    names = declared_functions()
    assert "nb_setup" in names and "nb_forces" in names and "nb_backward" in names
    for name in names:
        assert hasattr(lib, name), name


def test_every_declared_function_has_argument_types():
    """Without argtypes ctypes passes Python ints as 32-bit C ints, which truncates the context
    pointers; every declared function gets explicit argument types."""
    lib = nb.lib()
    for name in declared_functions():
        assert getattr(lib, name).argtypes is not None, name


def test_binding_names_match_header():
    for name in declared_functions():
        assert hasattr(nb, name), name


def base_params(**kw):
    t = synth.tiny()
    p = nb.Params.from_instance(t)
    for k, v in kw.items():
        setattr(p.c, k, v)
    return p


def test_valid_parameters_pass():
    assert nb.nb_validate_params(base_params()) == nb.NB_OK
    assert nb.nb_validate_params(base_params(cluster=4)) == nb.NB_OK


@pytest.mark.parametrize("field,value,code", [
    ("cutoff", 0.95, nb.NB_ERR_CUTOFF),      # rc >= L/2
    ("cutoff", -1.0, nb.NB_ERR_ARG),
    ("cutoff", float("nan"), nb.NB_ERR_ARG),
    ("buffer", -0.1, nb.NB_ERR_ARG),
    ("ewald_beta", 5.0, nb.NB_ERR_ARG),     # beta * rc beyond the erfc fit
    ("coulomb_const", 0.0, nb.NB_ERR_ARG),
    ("ntypes", 0, nb.NB_ERR_ARG),
    ("ntypes", 33, nb.NB_ERR_ARG),
    ("natoms", 0, nb.NB_ERR_ARG),
    ("cluster", 6, nb.NB_ERR_ARG),
    ("flags", 0x100, nb.NB_ERR_ARG),
    ("elec", 3, nb.NB_ERR_ARG),
    ("vdw", 5, nb.NB_ERR_ARG),
])
def test_invalid_parameters_are_rejected(field, value, code):
    assert nb.nb_validate_params(base_params(**{field: value})) == code
    assert nb.nb_last_error(None) != ""


@pytest.mark.parametrize("kw", [
    dict(vdw=1, rswitch=0.9),               # rswitch must lie below rc = 0.9
    dict(vdw=1, rswitch=-0.1),
    dict(elec=1, epsilon_rf=0.5),           # 0 (infinity) or >= 1
])
def test_invalid_flavour_parameters_are_rejected(kw):
    assert nb.nb_validate_params(base_params(**kw)) == nb.NB_ERR_ARG


def test_ewald_corrections_need_ewald_electrostatics():
    assert nb.nb_validate_params(base_params(flags=nb.NB_EWALD_CORR)) == nb.NB_OK
    assert nb.nb_validate_params(base_params(flags=nb.NB_EWALD_CORR, elec=1)) == nb.NB_ERR_ARG


def test_valid_flavours_pass():
    for kw in (dict(elec=1), dict(elec=1, epsilon_rf=78.0), dict(vdw=1, rswitch=0.7),
               dict(elec=1, vdw=1, rswitch=0.0)):
        assert nb.nb_validate_params(base_params(**kw)) == nb.NB_OK


def test_rlist_beyond_box_is_rejected():
    p = base_params(buffer=1.0)  # rc + rb = 1.9 > L = 1.862
    assert nb.nb_validate_params(p) == nb.NB_ERR_CUTOFF


def test_list_range_beyond_padding_spacing_is_rejected():
    # padding slots sit 16 nm apart (they are excluded by distance, not by the masks), so the
    # list range must stay below that even in a box large enough for it
    p = base_params(buffer=0.1)
    p.c.box[0] = p.c.box[1] = p.c.box[2] = 50.0
    p.c.ewald_beta = 0.2  # beta rc within the erfc fit's range
    p.c.cutoff = 15.95
    assert nb.nb_validate_params(p) == nb.NB_ERR_CUTOFF
    p.c.cutoff = 15.8
    assert nb.nb_validate_params(p) == nb.NB_OK


def test_bad_exclusions_are_rejected():
    t = synth.tiny()
    idx = t.excl_idx.copy()
    idx[3] = t.natoms  # out of range
    p = nb.Params.from_instance(t)
    p.excl_idx = idx
    p.c.excl_idx = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert nb.nb_validate_params(p) == nb.NB_ERR_ARG


def test_too_many_exclusions_per_atom_are_rejected():
    """Atom 0 gets NB_MAX_EXCL_PER_ATOM + 1 partners (symmetric lists)."""
    t = synth.tiny()
    n = t.natoms
    lists = [list(t.excl_idx[t.excl_off[i]:t.excl_off[i + 1]]) for i in range(n)]
    for k in range(1, nb.NB_MAX_EXCL_PER_ATOM + 2):
        j = 3 * k  # an oxygen of another molecule
        if j not in lists[0]:
            lists[0].append(j)
            lists[j].append(0)
    off = np.zeros(n + 1, np.int32)
    off[1:] = np.cumsum([len(l) for l in lists])
    idx = np.concatenate([np.asarray(l, np.int32) for l in lists]).astype(np.int32)
    assert off[1] - off[0] > nb.NB_MAX_EXCL_PER_ATOM
    p = nb.Params.from_instance(t)
    p.excl_off, p.excl_idx = off, idx
    p.c.excl_off = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    p.c.excl_idx = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert nb.nb_validate_params(p) == nb.NB_ERR_ARG
    assert "32" in nb.nb_last_error(None)


def test_setup_rejects_invalid_params_without_gpu():
    with pytest.raises(nb.NbError) as ei:
        nb.nb_setup(base_params(cutoff=0.95), stream=0)
    assert ei.value.code == nb.NB_ERR_CUTOFF


@pytest.mark.parametrize("kw", [dict(order=5), dict(order=10), dict(grid=(6, 32, 32)),
                                dict(beta=0.0), dict(natoms=0), dict(box=(2.0, -1.0, 2.0))])
def test_invalid_pme_parameters_are_rejected(kw):
    args = dict(box=2.0, beta=3.0, coulomb_const=138.935458, grid=(32, 32, 32), order=4, natoms=10)
    args.update(kw)
    with pytest.raises(nb.NbError) as ei:
        nb.nb_pme_setup(nb.pme_params(**args), stream=0)  # rejected before any device call
    assert ei.value.code == nb.NB_ERR_ARG
    assert nb.nb_pme_last_error(None) != ""


def test_tuner_size_buckets():
    """Host logic of the autotuner: logarithmic buckets over 3,000-30,000 atoms; sizes outside
    fall into the first and last buckets."""
    from paper_2405_01420_amd import tune
    e = tune.bucket_edges(3000, 30000, 5)
    assert len(e) == 6 and abs(e[0] - 3000) < 1e-9 and abs(e[-1] - 30000) < 1e-6
    assert all(abs(e[k + 1] / e[k] - 10 ** 0.2) < 1e-12 for k in range(5))
    assert tune.bucket_of(100, e) == 0 and tune.bucket_of(3000, e) == 0
    assert tune.bucket_of(4800, e) == 1 and tune.bucket_of(29999, e) == 4 and tune.bucket_of(10 ** 6, e) == 4


def test_null_handles_are_rejected_without_gpu():
    """Entry points given a NULL context return NB_ERR_ARG before touching the device."""
    L = nb.lib()
    assert L.nb_prune(None, None, 1.0) == nb.NB_ERR_ARG
    assert L.nb_forces(None, None, None, None, None, None) == nb.NB_ERR_ARG
    assert L.nb_pme_forces(None, None, None, None, None) == nb.NB_ERR_ARG
    assert L.nb_batch_tune_schedule(None, None, None, None, None, None, 1, None, None) == nb.NB_ERR_ARG
    assert L.nb_backward_noalloc(None, None, None, None, None, None, None, None, None, None) == nb.NB_ERR_ARG
    assert L.nb_set_timing(None, 7) == nb.NB_ERR_ARG
    assert L.nb_get_timing(None, None, None) == nb.NB_ERR_ARG


def test_autotune_rejects_bad_arguments_and_cache_without_gpu(tmp_path):
    """nb_autotune checks its arguments and reads its cache file before touching the device: a
    file that is not a tuning cache is NB_ERR_IO, a missing input NB_ERR_ARG."""
    L = nb.lib()
    res = nb.nb_tune_result()
    ao = np.array([0, 3000], dtype=np.int32)
    bx = np.array([6.7, 6.7, 6.7])
    p = base_params()
    cl = np.zeros(1, dtype=np.int32)
    assert L.nb_autotune(1, ao.ctypes.data, bx.ctypes.data, ctypes.byref(p.c), None, None, None, None,
                         None, cl.ctypes.data, ctypes.byref(res)) == nb.NB_ERR_ARG
    bad = tmp_path / "cache.json"
    for text in ("not json", '{"k": {"cluster": 4}', '{"k": [1, 2]}', '{"k": {"cluster": "four"}}'):
        bad.write_text(text)
        code = L.nb_autotune(1, ao.ctypes.data, bx.ctypes.data, ctypes.byref(p.c), 1, 1, 1,
                             str(bad).encode(), None, cl.ctypes.data, ctypes.byref(res))
        assert code == nb.NB_ERR_IO, text
        assert "tuning cache" in nb.nb_autotune_last_error()
