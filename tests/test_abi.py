"""CPU checks of the C interface: the library loads without a GPU, exports
every function include/bl.h declares, and reports a missing device."""
import ctypes as C
import os
import re

import pytest

from paper_1909_10286_amd import bl

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "bl.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bl_[a-z_]+)\s*\(", text)))


def test_header_declares_binding_names():
    assert _declared() == bl.EXPORTED


def test_library_exports_every_declared_symbol():
    lib = bl.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_no_device_reports_edevice():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    lib = bl.load()
    h = C.c_void_p()
    assert lib.bl_create(0, C.byref(h)) == bl.EDEVICE
    assert lib.bl_status_str(bl.EDEVICE) == b"device error"
    assert lib.bl_status_str(bl.EINVAL) == b"invalid argument"
    with pytest.raises(bl.BlError):
        bl.Context(0)


def test_null_arguments_rejected_without_device():
    lib = bl.load()
    assert lib.bl_create(0, None) == bl.EINVAL
    assert lib.bl_set_stream(None, None) == bl.EINVAL
    assert lib.bl_timing_enable(None, 1) == bl.EINVAL
    assert lib.bl_instance_upload(None, None, None) == bl.EINVAL
    assert lib.bl_instance_info_get(None, 0, None) == bl.EINVAL
