"""The C-ABI library loads on a host without a GPU and exports every symbol
include/mp.h declares; argument checks that need no device answer without one.
No compute calls are made here."""
from __future__ import annotations

import ctypes

import pytest

from paper_0809_1833_amd import mp


def test_header_declares_the_boundary():
    names = mp.header_functions()
    for required in ("mp_create", "mp_solve", "mp_destroy", "mp_status_str", "mp_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = mp.library()
    missing = [f for f in mp.header_functions() if not hasattr(lib, f)]
    assert missing == []


def test_status_strings():
    assert mp.mp_status_str(mp.MP_OK) == "MP_OK"
    assert mp.mp_status_str(mp.MP_ENOTNORM) == "MP_ENOTNORM"
    assert mp.mp_status_str(99) == "MP_UNKNOWN"


@pytest.mark.parametrize("kw,detail", [
    (dict(psi=None), "psi is NULL"),
    (dict(n=0), "n and m"),
    (dict(m=0), "n and m"),
    (dict(ld=3), "ld must be"),
    (dict(n=16385, ld=16385), "16384"),
    (dict(m=2 ** 31), "2^31"),
    (dict(flags=0x10), "flags"),
    (dict(storage=7), "storage"),
])
def test_create_rejects_bad_arguments(kw, detail):
    args = dict(psi=0x1000, n=4, m=4, ld=4, storage=0, flags=0)
    args.update(kw)
    h = ctypes.c_void_p(123)
    st = mp.library().mp_create(ctypes.byref(h), args["psi"], args["n"], args["m"], args["ld"],
                                args["storage"], args["flags"], None)
    assert st == mp.MP_EINVAL
    assert h.value is None
    assert detail in mp.mp_last_error(None)


def test_create_null_out():
    assert mp.library().mp_create(None, 0x1000, 4, 4, 4, 0, 0, None) == mp.MP_EINVAL


def test_solve_and_destroy_accept_null_context():
    lib = mp.library()
    opts = mp.Opts(1e-5, 10, 0, 0)
    assert lib.mp_solve(None, 1, 1, None, ctypes.byref(opts), None, None, None) == mp.MP_EINVAL
    assert lib.mp_solve_result(None, None) == mp.MP_EINVAL
    lib.mp_destroy(None)


def test_create_without_device_reports_edevice():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = mp.library().mp_create(ctypes.byref(h), 0x1000, 4, 4, 4, 0, 0, None)
    assert st == mp.MP_EDEVICE


@pytest.mark.parametrize("kw,detail", [
    (dict(psi=None), "psi is NULL"),
    (dict(n=0), "n and m"),
    (dict(ld=3), "ld must be"),
    (dict(n=16385, ld=16385), "16384"),
    (dict(m=2 ** 31), "2^31"),
    (dict(flags=0x10), "flags"),
])
def test_create_f64_rejects_bad_arguments(kw, detail):
    args = dict(psi=0x1000, n=4, m=4, ld=4, flags=0)
    args.update(kw)
    h = ctypes.c_void_p(123)
    st = mp.library().mp_create_f64(ctypes.byref(h), args["psi"], args["n"], args["m"],
                                    args["ld"], args["flags"], None)
    assert st == mp.MP_EINVAL
    assert h.value is None
    assert detail in mp.mp_last_error(None)


def test_f64_storage_goes_through_its_own_entry_point():
    h = ctypes.c_void_p(123)
    st = mp.library().mp_create(ctypes.byref(h), 0x1000, 4, 4, 4, mp.MP_F64, 0, None)
    assert st == mp.MP_EINVAL and "mp_create_f64" in mp.mp_last_error(None)
    opts = mp.Opts(1e-5, 10, 0, 0)
    assert mp.library().mp_solve_f64(None, 1, 1, None, ctypes.byref(opts), None, None,
                                     None) == mp.MP_EINVAL


@pytest.mark.parametrize("kw,detail", [
    (dict(signs=None), "signs is NULL"),
    (dict(n=0), "n and m"),
    (dict(m=0), "n and m"),
    (dict(n=16385, ldw=600), "16384"),
    (dict(n=33, ldw=1), "ldw must be"),
    (dict(m=2 ** 31), "2^31"),
    (dict(flags=0x10), "flags"),
])
def test_create_signs_rejects_bad_arguments(kw, detail):
    args = dict(signs=0x1000, n=64, m=4, ldw=2, flags=0)
    args.update(kw)
    h = ctypes.c_void_p(123)
    st = mp.library().mp_create_signs(ctypes.byref(h), args["signs"], args["n"], args["m"],
                                      args["ldw"], args["flags"], None)
    assert st == mp.MP_EINVAL
    assert h.value is None
    assert detail in mp.mp_last_error(None)


def test_sign_storage_goes_through_its_own_entry_point():
    h = ctypes.c_void_p(123)
    st = mp.library().mp_create(ctypes.byref(h), 0x1000, 4, 4, 4, mp.MP_SIGN1, 0, None)
    assert st == mp.MP_EINVAL and "mp_create_signs" in mp.mp_last_error(None)


def _header_text():
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "include", "mp.h")) as f:
        return f.read()


def _struct_fields(text, name):
    """Member names of `typedef struct name { ... } name;` in declaration order."""
    import re
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    return [m.group(1) for m in re.finditer(r"\b(\w+)\s*;", body)]


def test_binding_flags_match_the_header():
    import re
    text = _header_text()
    for name in ("MP_SKIP_NORM_CHECK", "MP_SOLVE_STEP_LAUNCHES", "MP_SOLVE_ASYNC"):
        value = re.search(r"#define %s (0x[0-9a-fA-F]+)u" % name, text).group(1)
        assert getattr(mp, name) == int(value, 16), name


def test_binding_structs_match_the_header():
    text = _header_text()
    assert [f[0] for f in mp.Opts._fields_] == _struct_fields(text, "mp_opts")
    assert [f[0] for f in mp.Result._fields_] == _struct_fields(text, "mp_result")
    assert [f[0] for f in mp.Trace._fields_] == _struct_fields(text, "mp_trace")
    assert [f[0] for f in mp.TraceF64._fields_] == _struct_fields(text, "mp_trace_f64")
    assert ctypes.sizeof(mp.Result) == 32 and ctypes.sizeof(mp.Opts) == 24
    assert ctypes.sizeof(mp.Trace) == 48 and ctypes.sizeof(mp.TraceF64) == 48
    assert [f[0] for f in mp.BatchedConfig._fields_] == _struct_fields(text, "mp_batched_config")
    assert [f[0] for f in mp.RaggedConfig._fields_] == _struct_fields(text, "mp_ragged_config")


def test_batched_tile_rules_tried():
    """The tuner's switch-point pairs: each runs every tile it names (a
    64-atom switch at or below the 128-atom one, or none), and the library's
    default rule is among them."""
    from paper_0809_1833_amd import tune
    rules = tune.batched_rules()
    assert len(rules) == len(set(rules))
    for a128, a64, a32 in rules:
        assert (a64 <= a128 or a64 == tune.NEVER) and a32 == 0
    assert (tune.NEVER, 96, 0) in rules and (tune.NEVER, tune.NEVER, 0) in rules
    assert all(a > 0 for a in tune.ATOMS32_ABOVE)
