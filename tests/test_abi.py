"""CPU-side checks of the C ABI: the library loads, exports every function
that include/tl.h declares, and rejects bad descriptors on the host before
touching a device."""
import ctypes as C
import re
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "tl.h"


def _lib():
    from paper_1208_4093_amd import tl
    if not Path(tl.LIB_PATH).exists():
        pytest.skip("libtl.so not built")
    return tl, tl.load()


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tl_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("tl_lattice_create", "tl_lattice_destroy", "tl_solve", "tl_solve_batch",
              "tl_submit", "tl_poll", "tl_server_create", "tl_server_destroy", "tl_strerror"):
        assert n in names


def test_library_exports_every_declared_function():
    tl, lib = _lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(tl.EXPORTS)


def test_strerror_is_total():
    tl, lib = _lib()
    for s in range(-8, 3):
        assert isinstance(tl.tl_strerror(s), str)
    assert tl.tl_strerror(0) == "ok"


@pytest.mark.parametrize("nx,ny,kw", [
    (1, 8, {}),                                    # too narrow
    (8, 1, {}),                                    # a one-row lattice is a mechanism
    (8, 8, {"set_edge": 24}),                      # unsupported set edge
    (8, 8, {"ea": "neg"}),                         # negative stiffness
    (8, 8, {"ea": "nan"}),                         # non-finite stiffness
    (8, 8, {"fixed": "one"}),                      # a single support cannot stop rotation
    (8, 8, {"ea": "isolated"}),                    # a free node with no rod
    (8, 8, {"ea": "collinear"}),                   # a free node held by horizontal rods only
])
def test_create_rejects_bad_descriptors_on_host(nx, ny, kw):
    tl, lib = _lib()
    ea = np.ones((3, ny, nx), np.float32)
    fixed = None
    if kw.get("ea") == "neg":
        ea[1, 2, 3] = -1.0
    if kw.get("ea") == "nan":
        ea[0, 1, 1] = np.nan
    if kw.get("ea") in ("isolated", "collinear"):
        # the six rods of node (i, j) = (3, 3): its three forward rods and the
        # forward rods of (2, 3), (3, 2) and (4, 2) that end on it ([d, j, i])
        ea[1, 3, 3] = ea[1, 2, 3] = ea[2, 3, 3] = ea[2, 2, 4] = 0.0
        if kw["ea"] == "isolated":
            ea[0, 3, 3] = ea[0, 3, 2] = 0.0
    if kw.get("fixed") == "one":
        fixed = np.zeros((ny, nx), np.uint8)
        fixed[0, 0] = 1
    with pytest.raises(tl.TLError) as ei:
        tl.tl_lattice_create(nx, ny, ea=ea, fixed=fixed, set_edge=kw.get("set_edge", 0))
    assert ei.value.status == tl.TL_E_INVAL


def test_null_arguments_are_rejected():
    tl, lib = _lib()
    assert lib.tl_lattice_create(None, None, None) == tl.TL_E_INVAL
    assert lib.tl_solve(None, None, None, None, None, None) == tl.TL_E_INVAL
    assert lib.tl_poll(None, 0, None) == tl.TL_E_INVAL
    assert lib.tl_submit(None, None, None, None, None, None, None) == tl.TL_E_INVAL
    assert lib.tl_solve_noalloc(None, None, None, None, None, None) == tl.TL_E_INVAL
    assert lib.tl_tune(None, None, None, None, None) == tl.TL_E_INVAL
    assert lib.tl_tune_lookup(64, 64, 0, None) == tl.TL_E_INVAL
    assert lib.tl_tune_load(None) == tl.TL_E_INVAL
    assert lib.tl_tune_save(None) == tl.TL_E_INVAL
    out = C.c_void_p()
    assert lib.tl_server_create(0, 1, C.byref(out)) == tl.TL_E_INVAL
    assert lib.tl_server_create(1 << 20, 0, C.byref(out)) == tl.TL_E_INVAL
