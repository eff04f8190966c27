"""CPU-side checks of the C ABI: the library loads, exports what include/vk.h
declares, rejects bad arguments before touching a GPU, and the binding's
marshalling prepares consistent inputs."""
import ctypes

import numpy as np

import paper_2210_02690_amd as vk
from synth import build_problem


def test_header_symbols_exported():
    names = vk.header_functions()
    for must in ("vk_create", "vk_set_level", "vanka_setup", "vanka_smooth", "vcycle", "gmres_solve",
                 "vk_workspace_bytes", "vk_set_workspace", "vk_destroy", "vk_last_error"):
        assert must in names
    lib = vk.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_errors_without_gpu():
    lib = vk.lib()
    p = ctypes.c_void_p()
    assert lib.vk_create(None, 3, None) == vk.VK_ERR_ARG
    assert lib.vk_create(ctypes.byref(p), 0, None) == vk.VK_ERR_ARG
    assert lib.vk_create(ctypes.byref(p), 33, None) == vk.VK_ERR_ARG
    assert lib.vk_workspace_bytes(None, vk.VK_F64, 30) == 0
    assert lib.vk_last_error(None) == b"n_levels must be in [1, 32]"
    assert lib.vanka_setup(None, 0.7, 0, None, None) == vk.VK_ERR_ARG
    assert lib.vanka_smooth(None, 1, None, None, 1, 0) == vk.VK_ERR_ARG
    assert lib.vcycle(None, None, None, 2, 2) == vk.VK_ERR_ARG
    assert lib.gmres_solve(None, None, None, 30, 10, 1e-8, 0.0, 2, 2, None, None, None) == vk.VK_ERR_ARG
    assert lib.vk_timing_enable(None, 1, -1) == vk.VK_ERR_ARG
    lib.vk_destroy(None)


def test_upload_level_colour_order_cpu():
    P = build_problem("channel2d_44x8_k1", shape=(10, 6), levels=2)
    L = P.finest
    u = vk.upload_level(L, "cpu")
    order = u["colour_cells"].numpy()
    ptr = u["colour_ptr"]
    assert ptr[0] == 0 and ptr[-1] == L.mesh.n_cells and u["n_colours"] == 4
    for c in range(4):
        cells = order[ptr[c]:ptr[c + 1]]
        assert np.all(L.colours[cells] == c) and np.all(np.diff(cells) > 0)
    assert u["J"]["row_ptr"].dtype.itemsize == 8 and u["J"]["col"].dtype.itemsize == 4
    s = vk.csr_struct(u["J"])
    assert s.nnz == L.J.nnz and s.n_rows == L.n
