"""The C interface: the built library loads and exports every declared entry point.

These run without a GPU: loading the library and calling the argument checks
touches no device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "radio.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"RADIO_API\s+[\w\s\*]+?\b(radio_\w+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    import paper_2302_14812_amd as radio
    assert _declared() == sorted(radio.EXPORTS)


def _struct_fields(name):
    """Field names of `typedef struct name {...} name;` in the header, in order."""
    src = open(HEADER).read()
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), src, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        if not decl.strip():
            continue
        # "type a, b" declares a and b; drop array extents and pointer stars
        first, *rest = decl.split(",")
        for d in [first.split()[-1]] + [r.strip() for r in rest]:
            names.append(re.sub(r"\[.*\]", "", d).lstrip("*"))
    return names


@pytest.mark.parametrize("cname,pyname", [("radio_chunk", "_Chunk"), ("radio_detector_desc", "_Desc"), ("radio_push_desc", "_Push"),
                                          ("radio_stats", "_Stats"), ("radio_tuning", "_Tuning")])
def test_binding_structs_follow_the_header(cname, pyname):
    import paper_2302_14812_amd as radio
    assert [f for f, _ in getattr(radio, pyname)._fields_] == _struct_fields(cname)


def test_library_exports_every_declared_symbol():
    import paper_2302_14812_amd as radio
    lib = radio._lib()
    for name in _declared():
        assert hasattr(lib, name), name
    # exported with default visibility, i.e. visible to dlsym
    raw = ctypes.CDLL(radio.LIB_PATH)
    for name in _declared():
        getattr(raw, name)


def test_status_strings():
    import paper_2302_14812_amd as radio
    lib = radio._lib()
    assert lib.radio_status_string(0) == b"ok"
    assert lib.radio_status_string(-1) == b"invalid argument"
    assert lib.radio_status_string(12345) == b"unknown status"


def test_invalid_arguments_rejected_before_any_device_work():
    import paper_2302_14812_amd as radio
    lib = radio._lib()
    h = ctypes.c_void_p()
    d = radio._Desc()
    d.geometry = radio.GEOM_PLANE
    d.n1 = d.n2 = 4
    d.e1[:] = [1, 0, 0]
    d.e2[:] = [0, 1, 0]
    d.half1 = d.half2 = 1.0
    d.n_t = 16
    d.c = 1.0
    d.dt_det = 0.0  # invalid
    assert lib.radio_detector_create(ctypes.byref(d), None, ctypes.byref(h)) == radio.EINVAL
    d.dt_det = 0.1
    d.n_t = 0  # invalid
    assert lib.radio_detector_create(ctypes.byref(d), None, ctypes.byref(h)) == radio.EINVAL
    d.n_t = 16
    d.c = -1.0
    assert lib.radio_detector_create(ctypes.byref(d), None, ctypes.byref(h)) == radio.EINVAL
    d.c = 1.0
    d.precision = 7
    assert lib.radio_detector_create(ctypes.byref(d), None, ctypes.byref(h)) == radio.EINVAL
    d.precision = 0
    d.options = radio.HOLD_PREVIOUS | radio.HOLD_LINEAR  # two hold rules at once
    assert lib.radio_detector_create(ctypes.byref(d), None, ctypes.byref(h)) == radio.EINVAL
    d.options = radio.POTENTIALS | radio.ACCEL_ONLY  # potentials have no acceleration term
    assert lib.radio_detector_create(ctypes.byref(d), None, ctypes.byref(h)) == radio.EINVAL
    d.options = 32  # unknown option bit
    assert lib.radio_detector_create(ctypes.byref(d), None, ctypes.byref(h)) == radio.EINVAL
    d.options = radio.FAR_FIELD | radio.ACCEL_ONLY
    d.geometry = 9
    assert lib.radio_detector_create(ctypes.byref(d), None, ctypes.byref(h)) == radio.EINVAL
    d.geometry = radio.GEOM_EXPLICIT
    d.n_cells = 3
    d.cells = ctypes.POINTER(ctypes.c_double)()  # NULL
    assert lib.radio_detector_create(ctypes.byref(d), None, ctypes.byref(h)) == radio.EINVAL
    assert lib.radio_detector_create(None, None, ctypes.byref(h)) == radio.EINVAL
    ch = radio._Chunk(1, 1, 0.0, 0.1, 0, None, None, None)
    assert lib.radio_deposit_trajectory_chunk(None, ctypes.byref(ch), None) == radio.EINVAL
    assert lib.radio_read_detector(None, None, None, None) == radio.EINVAL
    assert lib.radio_detector_load(None, None, None, None) == radio.EINVAL
    assert lib.radio_detector_reset(None, None) == radio.EINVAL
    assert lib.radio_detector_destroy(None) == radio.OK
    assert lib.radio_deposit_batch(None, None, -1, None) == radio.EINVAL
    assert lib.radio_deposit_batch(None, None, 0, None) == radio.OK
    assert lib.radio_arrival_times(None, None, None, 5, 1.0, None, None) == radio.EINVAL
    assert lib.radio_arrival_times(None, None, None, 0, 0.0, None, None) == radio.EINVAL
    assert lib.radio_slot_coordinates(None, None, None, 5, 1.0, 0.0, 0.1, None, None) == radio.EINVAL
    assert lib.radio_slot_coordinates(None, None, None, 0, 1.0, 0.0, 0.0, None, None) == radio.EINVAL
    assert lib.radio_slot_coordinates(None, None, None, 0, 1.0, 0.0, 0.1, None, None) == radio.OK


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2302_14812_amd as radio
    monkeypatch.setattr(radio, "_LIB", None)
    monkeypatch.setattr(radio, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        radio._lib()
