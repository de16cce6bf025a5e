"""Host-side checks of the C-ABI that need no GPU: the library loads, exports
every entry point the header declares, and rejects bad arguments before
touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2105_04884_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbl.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbl_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    try:
        return _lib.load()
    except _lib.LibraryMissing as e:
        pytest.fail(str(e))


def test_header_declares_expected_calls():
    names = _declared()
    for want in ("rbl_create", "rbl_build", "rbl_forces", "rbl_full_forces", "rbl_step",
                 "rbl_export_lists", "rbl_export_batches", "rbl_sync", "rbl_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert sorted(_lib.exported_names()) == _declared()


def test_config_defaults(lib):
    cfg = _lib.Config()
    lib.rbl_config_init(C.byref(cfg), 1000)
    assert cfg.n == 1000 and cfg.n_replicas == 1
    assert cfg.precision == _lib.PREC_FP64 and cfg.pair == _lib.PAIR_LJ
    assert cfg.lists == _lib.LIST_CORE | _lib.LIST_SHELL
    assert cfg.skin == 0.3 and cfg.shift == 1 and cfg.momentum_fix == 1 and cfg.predraw == 1
    assert cfg.capacity_factor == 1.25 and cfg.lanes == 0 and cfg.persistent == 0
    assert cfg.shell_source == _lib.SHELL_LIST and cfg.core_filter == 2
    assert lib.rbl_version().decode().startswith("librbl")


def _create(lib, **over):
    cfg = _lib.Config()
    lib.rbl_config_init(C.byref(cfg), over.pop("n", 100))
    offsets = over.pop("offsets", None)
    keep = None
    if offsets is not None:
        keep = (C.c_int64 * len(offsets))(*offsets)
        cfg.replica_offsets = C.cast(keep, C.POINTER(C.c_int64))
    for k, v in over.items():
        setattr(cfg, k, v)
    h = C.c_void_p()
    st = lib.rbl_create(C.byref(cfg), None, C.byref(h))
    return st, h


@pytest.mark.parametrize("over", [
    {"n": 0}, {"n": -5}, {"n_replicas": 0}, {"precision": 7}, {"pair": 3}, {"lists": 0},
    {"lists": 9}, {"skin": -0.1}, {"skin": float("nan")}, {"pair": 1, "alpha": 0.0},
    {"capacity_factor": 0.0}, {"lanes": 3}, {"lanes": -1}, {"persistent": 3}, {"persistent": -1},
    {"shell_source": 3}, {"shell_source": -1}, {"core_filter": 3}, {"core_filter": -1},
    {"n_replicas": 2},                                   # offsets missing
    {"n": 10, "n_replicas": 2, "offsets": [0, 4, 9]},    # does not end at n
    {"n": 10, "n_replicas": 2, "offsets": [0, 0, 10]},   # empty replica
])
def test_create_rejects_bad_config(lib, over):
    st, h = _create(lib, **over)
    assert st == _lib.RBL_E_ARG
    assert not h.value
    assert lib.rbl_last_error().decode()


def test_config_type_fields_default_off(lib):
    cfg = _lib.Config()
    lib.rbl_config_init(C.byref(cfg), 10)
    assert cfg.n_types == 0 and not cfg.types and not cfg.pair_coeffs
    # the pointers follow the two int32 words at the end of the C struct
    assert _lib.Config.types.offset == _lib.Config.n_types.offset + 4
    assert _lib.Config.types.offset % 8 == 0


def _typed(lib, types, table, **over):
    t = (C.c_int32 * len(types))(*types)
    flat = [v for row in table for pair in row for v in pair]
    e = (C.c_double * len(flat))(*flat)
    return _create(lib, n=len(types), n_types=len(table), types=C.cast(t, C.POINTER(C.c_int32)),
                   pair_coeffs=C.cast(e, C.POINTER(C.c_double)), **over)


GOOD2 = [[(1.0, 1.0), (1.0, 1.3)], [(1.0, 1.3), (1.0, 1.6)]]


@pytest.mark.parametrize("types,table,over", [
    ([0, 1, 2], GOOD2, {}),                                          # type out of range
    ([0, 1, -1], GOOD2, {}),
    ([0, 1, 1], [[(1.0, 1.0), (1.0, 1.3)], [(1.0, 1.2), (1.0, 1.6)]], {}),   # not symmetric
    ([0, 1, 1], [[(1.0, 1.0), (1.0, 0.0)], [(1.0, 0.0), (1.0, 1.6)]], {}),   # sigma 0
    ([0, 1, 1], [[(-1.0, 1.0), (1.0, 1.3)], [(1.0, 1.3), (1.0, 1.6)]], {}),  # epsilon < 0
    ([0, 1, 1], GOOD2, {"pair": 1, "alpha": 1.0}),                   # no charges with types
    ([0, 1, 1], GOOD2, {"shell_source": 1}),                         # shell rows only
    ([0] * 3, [[(1.0, 1.0)] * 5] * 5, {}),                           # more than 4 types
])
def test_create_rejects_bad_types(lib, types, table, over):
    st, h = _typed(lib, types, table, **over)
    assert st == _lib.RBL_E_ARG
    assert not h.value
    assert lib.rbl_last_error().decode()


def test_create_rejects_types_without_count(lib):
    t = (C.c_int32 * 3)(0, 0, 0)
    st, h = _create(lib, n=3, types=C.cast(t, C.POINTER(C.c_int32)))
    assert st == _lib.RBL_E_ARG and not h.value


def test_calls_reject_null_context(lib):
    box = (C.c_double * 3)(10.0, 10.0, 10.0)
    assert lib.rbl_build(None, None, box, 1.5, 3.5) == _lib.RBL_E_ARG
    assert lib.rbl_forces(None, 10, 1, 0, None, None, None) == _lib.RBL_E_ARG
    assert lib.rbl_full_forces(None, None, None, None) == _lib.RBL_E_ARG
    assert lib.rbl_step(None, None, None, None, 10, 0.005, 10, 1, 0, 10, 0, None) == _lib.RBL_E_ARG
    assert lib.rbl_sync(None) == _lib.RBL_E_ARG
    assert lib.rbl_set_profiling(None, 1) == _lib.RBL_E_ARG
    kt = (C.c_double * 1)(1.0)
    assert lib.rbl_set_thermostat(None, 1.0, kt) == _lib.RBL_E_ARG
    assert lib.rbl_unwrap(None, None, None) == _lib.RBL_E_ARG
    assert lib.rbl_msd(None, None, None, None) == _lib.RBL_E_ARG
    assert lib.rbl_rdf(None, None, 3.0, 100, None) == _lib.RBL_E_ARG
    out = (C.c_double * 4)()
    assert lib.rbl_thermo(None, None, None, out) == _lib.RBL_E_ARG
    assert lib.rbl_destroy(None) == _lib.RBL_OK
