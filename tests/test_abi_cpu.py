"""C ABI checks that need no GPU: the library loads, exports every function
include/gw.h declares, and the host-only size query follows the mesh rules."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gw_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    import paper_1101_2065_amd.gw as gw

    names = _declared()
    assert "gw_build_chi0" in names and "gw_solve_W" in names and "gw_poll" in names
    assert "gw_build_A" in names and "gw_build_A_time" in names and "gw_solve_W_A" in names
    lib = ctypes.CDLL(gw.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(gw._SIGS), "binding and header disagree"


def test_query_sizes_follows_mesh_rules():
    import paper_1101_2065_amd.gw as gw

    eig = np.sort(np.random.default_rng(0).uniform(-1.0, 2.0, 520))
    eig = np.ascontiguousarray(eig)
    g = gw.make_grid(1024, -8.0, 8.0, 0.02)
    s = gw.query_sizes(520, 160, 2304, eig, g)
    assert s.n_pairs == 160 * 360
    dmax = eig[-1] - eig[0]
    assert s.n_hbins == min(512, int(np.floor(dmax * 64)) + 2)
    assert s.n_upper == 2304 * 2305 // 2
    assert s.hist_bytes == s.n_hbins * s.n_upper * 8
    assert s.chi0_bytes == 1024 * 2304 * 2304 * 16
    sk = gw.query_sizes(520, 160, 2304, eig, g, k=100)
    assert sk.n_upper == 100 * 101 // 2


@pytest.mark.parametrize("bad", [
    (1000, -8.0, 8.0, 0.02),   # not a power of two
    (1024, -8.0, 9.0, 0.02),   # not symmetric
    (1024, -8.0, 8.0, 0.0),    # eps must be positive
    (768, -6.0, 6.0, 0.02),    # spacing not a power of two (and n not either)
    (4096, -8.0, 8.0, 0.02),   # beyond the FFT size the kernel supports
    (1024, -5.0, 5.0, 0.02),   # spacing 10/1024 is not a power of two
])
def test_query_sizes_rejects_bad_mesh(bad):
    import paper_1101_2065_amd.gw as gw

    eig = np.ascontiguousarray(np.linspace(-1, 1, 10))
    with pytest.raises(gw.GwError) as e:
        gw.query_sizes(10, 5, 10, eig, gw.make_grid(*bad))
    assert e.value.status == gw.GW_E_INVALID


def test_create_without_gpu_reports_device_error():
    import torch

    import paper_1101_2065_amd.gw as gw

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert gw.lib.gw_create(0, 0, ctypes.byref(h)) == gw.GW_E_DEVICE
    assert gw.lib.gw_destroy(None) == gw.GW_E_INVALID
    assert gw.lib.gw_last_error(None) == b"NULL context"
    # the A route's entry points reject a NULL context before touching anything
    assert gw.lib.gw_build_A(None, None, None, None, None, None, None) == gw.GW_E_INVALID
    assert gw.lib.gw_build_A_compressed(None, None, None, None, 0, None, None, None, None) == gw.GW_E_INVALID
    assert gw.lib.gw_build_A_time(None, None, None, None, None, None, None, None) == gw.GW_E_INVALID
    assert gw.lib.gw_solve_W_A(None, None, 0, 1, None, 2, 0, 1e-7, None, None, None) == gw.GW_E_INVALID
    assert gw.lib.gw_solve_W_A_noalloc(None, None, 0, 1, None, 2, None, None, None) == gw.GW_E_INVALID


def test_oracle_is_not_imported_by_the_product():
    """The product package never reads, imports or links the oracle."""
    pkg = os.path.join(ROOT, "paper_1101_2065_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "hist_ref" not in txt, f
