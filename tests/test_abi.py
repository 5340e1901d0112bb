"""The C ABI library loads on the CPU and exports every entry point its header
declares (no GPU work is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(hsp_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared()
    for required in ("hsp_create", "hsp_sweep", "hsp_draws", "hsp_destroy", "hsp_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1608_04329_amd import hsp
    lib = hsp.load()
    for name in declared():
        assert hasattr(lib, name), name
    assert sorted(hsp.EXPORTS) == declared()


def test_host_only_entry_points():
    from paper_1608_04329_amd import hsp
    o = hsp.hsp_default_options()
    assert o.seed == 1 and o.thin == 1 and o.max_draws == 1024 and o.use_graph == 1
    assert hsp.hsp_max_p() >= 1000
    # the options struct has the C layout
    assert o.multi_chain_z == 1
    assert ctypes.sizeof(hsp.hsp_options) == 80


def test_create_rejects_bad_shapes_before_touching_a_device():
    from paper_1608_04329_amd import hsp
    import numpy as np
    X = np.zeros((1, 3), np.float32)
    y = np.zeros(1, np.uint8)
    opt = hsp.hsp_default_options()
    opt.x_on_host = 1
    with pytest.raises(hsp.HspError) as e:
        hsp.hsp_create(X.ctypes.data, y.ctypes.data, 1, 3, opt)
    assert e.value.code == hsp.HSP_EINVAL
    with pytest.raises(hsp.HspError) as e:
        hsp.hsp_create(X.ctypes.data, y.ctypes.data, 5, 1, opt)
    assert e.value.code == hsp.HSP_EINVAL
    with pytest.raises(hsp.HspError) as e:
        hsp.hsp_create(X.ctypes.data, y.ctypes.data, 5, hsp.hsp_max_p() + 1, opt)
    assert e.value.code == hsp.HSP_EINVAL
