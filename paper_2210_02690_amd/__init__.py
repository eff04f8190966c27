"""Python binding of libvk, the MI355X (gfx950) Vanka / geometric-multigrid /
GMRES solver for Newton-linearised space-time Navier-Stokes systems.

The functions below carry the names of the C ABI in include/vk.h and only
marshal arguments: torch tensors (device memory) become pointers, Python
numbers become C scalars.  Every numerical step runs in the library's HIP
kernels.  There is no fallback: if libvk.so is missing the import fails.
"""
import ctypes
import os
import re

import numpy as np
# torch ships its own HIP runtime (libamdhip64.so.7).  It must be the one that
# satisfies libvk.so's dependency: loading libvk.so first would map the system
# runtime as well, and two HIP runtimes in one process do not share devices.
import torch  # noqa: F401

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvk.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "vk.h")
HEADERS = [HEADER, os.path.join(os.path.dirname(_PKG), "include", "vk_mlp.h")]

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2210_02690_amd/build.py`")
_lib = ctypes.CDLL(LIB_PATH)

VK_OK, VK_ERR_ARG, VK_ERR_HIP, VK_ERR_SINGULAR, VK_ERR_NOCONV, VK_ERR_BREAKDOWN, VK_ERR_WORKSPACE, VK_ERR_STATE = range(8)
STATUS_NAMES = ["VK_OK", "VK_ERR_ARG", "VK_ERR_HIP", "VK_ERR_SINGULAR", "VK_ERR_NOCONV", "VK_ERR_BREAKDOWN",
                "VK_ERR_WORKSPACE", "VK_ERR_STATE"]
VK_F64, VK_F32, VK_BF16 = 0, 1, 2
VK_ADDITIVE, VK_MULT_COLOURED = 0, 1
PRECISIONS = {"f64": VK_F64, "f32": VK_F32, "bf16": VK_BF16}
MODES = {"additive": VK_ADDITIVE, "multiplicative": VK_MULT_COLOURED}


class vk_csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class vk_cell_group(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32), ("n_K", ctypes.c_int32), ("cell_dofs", ctypes.c_void_p),
                ("colour_cells", ctypes.c_void_p), ("colour_ptr", ctypes.POINTER(ctypes.c_int32)),
                ("n_colours", ctypes.c_int32)]


_P = ctypes.c_void_p
_I32, _I64, _D, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_PI32, _PI64, _PD = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "vk_create": (ctypes.c_int, [ctypes.POINTER(_P), _I32, _P]),
    "vk_destroy": (None, [_P]),
    "vk_last_error": (ctypes.c_char_p, [_P]),
    "vk_set_level": (ctypes.c_int, [_P, _I32, ctypes.POINTER(vk_csr), ctypes.POINTER(vk_csr),
                                    ctypes.POINTER(vk_csr), _I32, _I32, _P, _P, _PI32, _I32]),
    "vk_workspace_bytes": (_SZ, [_P, ctypes.c_int, _I32]),
    "vk_set_workspace": (ctypes.c_int, [_P, _P, _SZ, ctypes.c_int, _I32]),
    "vanka_setup": (ctypes.c_int, [_P, _D, ctypes.c_int, _PI32, _PI32]),
    "vanka_smooth": (ctypes.c_int, [_P, _I32, _P, _P, _I32, _I32]),
    "vanka_smooth_noalloc": (ctypes.c_int, [_P, _I32, _P, _P, _I32, _I32]),
    "vcycle": (ctypes.c_int, [_P, _P, _P, _I32, _I32]),
    "gmres_solve": (ctypes.c_int, [_P, _P, _P, _I32, _I32, _D, _D, _I32, _I32, _PI32, _PD, _PD]),
    "vk_spmv": (ctypes.c_int, [_P, _I32, _D, _P, _D, _P, _P]),
    "vk_get_patch_inverses": (ctypes.c_int, [_P, _I32, _I32, _I32, _P]),
    "vk_get_coarse_inverse": (ctypes.c_int, [_P, _P]),
    "vk_set_patch_tile": (ctypes.c_int, [_P, _I32, _I32]),
    "vk_patch_layout": (ctypes.c_int, [_P, _I32, _PI64, _PI32]),
    "vk_timing_enable": (ctypes.c_int, [_P, _I32, _I32]),
    "vk_set_sweep_variant": (ctypes.c_int, [_P, _I32]),
    "vk_set_setup_variant": (ctypes.c_int, [_P, _I32]),
    "vk_set_coarse_pivoting": (ctypes.c_int, [_P, _I32]),
    "vk_set_coarse_solver": (ctypes.c_int, [_P, _I32]),
    "vk_set_spmv_format": (ctypes.c_int, [_P, _I32]),
    "vk_spmv_format": (ctypes.c_int, [_P, _I32]),
    "vk_spmv_bytes": (ctypes.c_double, [_P, _I32]),
    "vk_coarse_plan": (ctypes.c_int, [_P, _I32, _PD]),
    "vk_autotune": (ctypes.c_int, [_P, _I32]),
    "vk_set_graphs": (ctypes.c_int, [_P, _I32]),
    "vk_graph_stats": (ctypes.c_int, [_P, _PI64, _PI64]),
    "vk_set_level_groups": (ctypes.c_int, [_P, _I32, ctypes.POINTER(vk_csr), ctypes.POINTER(vk_csr),
                                           ctypes.POINTER(vk_csr), _I32, ctypes.POINTER(vk_cell_group), _I32,
                                           _PI64]),
    "vk_set_segments": (ctypes.c_int, [_P, _I32, _PI64]),
    "gmres_solve_batched": (ctypes.c_int, [_P, _P, _P, _I32, _I32, _D, _D, _I32, _I32, _PI32, _PD, _PI32]),
    "vk_timing_kinds": (ctypes.c_int, [_P, ctypes.c_uint32, _I32]),
    "vk_timing_read": (ctypes.c_int, [_P, _I32, _I32, _PI64, _PD]),
    # learned initial guess (vk_mlp.h)
    "vk_mlp_create": (ctypes.c_int, [ctypes.POINTER(_P), _I32, _I32, _I32, _I32, _I32, _P]),
    "vk_mlp_destroy": (None, [_P]),
    "vk_mlp_last_error": (ctypes.c_char_p, [_P]),
    "vk_mlp_param_count": (_I64, [_P]),
    "vk_mlp_workspace_bytes": (_SZ, [_P]),
    "vk_mlp_set_workspace": (ctypes.c_int, [_P, _P, _SZ]),
    "vk_mlp_set_params": (ctypes.c_int, [_P, _P]),
    "vk_mlp_get_params": (ctypes.c_int, [_P, _P]),
    "vk_mlp_forward": (ctypes.c_int, [_P, _I32, _P, _P, _P]),
    "vk_mlp_gradient": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _P]),
    "vk_mlp_adam": (ctypes.c_int, [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    "vk_mlp_patch_features": (ctypes.c_int, [_P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "vk_mlp_patch_targets": (ctypes.c_int, [_P, _I32, _I32, _P, _P, _P, _P, _P, _P]),
    "vk_mlp_patch_average": (ctypes.c_int, [_P, _I64, _P, _P, _I32, _P, _P, _P, _P, _P]),
    "vk_mlp_slab_extrapolate": (ctypes.c_int, [_P, _I64, _I32, _PD, _P, _P]),
}
KERNEL_KINDS = {"patch_apply": 0, "spmv": 1, "patch_setup": 2, "patch_residual": 3, "patch_gemv": 4,
                "dof_gather": 5, "sweep": 6, "block_invert": 7}
SWEEP_VARIANTS = {"dof_gather": 0, "coloured_scatter": 1, "dof_gather_offsets": 2}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def header_functions(paths=None):
    """Names of the functions declared in include/vk.h and include/vk_mlp.h."""
    names = set()
    for path in (HEADERS if paths is None else ([paths] if isinstance(paths, str) else paths)):
        with open(path) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(?:vk_status|void|size_t|int64_t|const char\*)\s+\*?(\w+)\s*\(", text))
    return sorted(names)


class VkError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def csr_struct(t):
    """vk_csr from a dict of device tensors {n_rows, n_cols, row_ptr, col, val}."""
    if t is None:
        return None
    return vk_csr(int(t["n_rows"]), int(t["n_cols"]), int(t["val"].numel()),
                  t["row_ptr"].data_ptr(), t["col"].data_ptr() if t["val"].numel() else None,
                  t["val"].data_ptr() if t["val"].numel() else None)


def upload_csr(A, device):
    """scipy CSR -> dict of device tensors (int64 row pointers, int32 columns, FP64 values)."""
    import torch
    A = A.tocsr()
    A.sort_indices()
    return {
        "n_rows": A.shape[0], "n_cols": A.shape[1],
        "row_ptr": torch.from_numpy(A.indptr.astype(np.int64)).to(device),
        "col": torch.from_numpy(A.indices.astype(np.int32)).to(device),
        "val": torch.from_numpy(A.data.astype(np.float64)).to(device),
    }


def upload_level(level, device):
    """Device tensors of one level (an object with J, P, R, cell_dofs, colours)."""
    import torch
    out = {"J": upload_csr(level.J, device),
           "P": upload_csr(level.P, device) if level.P is not None else None,
           "R": upload_csr(level.R, device) if level.R is not None else None}
    cd = np.ascontiguousarray(level.cell_dofs, dtype=np.int32)
    colours = np.asarray(level.colours, dtype=np.int32)
    order = np.argsort(colours, kind="stable").astype(np.int32)
    n_col = int(colours.max()) + 1 if colours.size else 1
    ptr = np.concatenate([[0], np.cumsum(np.bincount(colours, minlength=n_col))]).astype(np.int32)
    out.update(n_cells=cd.shape[0], n_K=cd.shape[1], cell_dofs=torch.from_numpy(cd).to(device),
               colour_cells=torch.from_numpy(order).to(device), colour_ptr=ptr, n_colours=n_col)
    return out


def _colour_order(colours):
    colours = np.asarray(colours, dtype=np.int32)
    order = np.argsort(colours, kind="stable").astype(np.int32)
    n_col = int(colours.max()) + 1 if colours.size else 1
    ptr = np.concatenate([[0], np.cumsum(np.bincount(colours, minlength=n_col))]).astype(np.int32)
    return order, ptr, n_col


def upload_packed_level(level, device):
    """Device tensors of one packed batch level (synth.batch.PackedLevel)."""
    import torch
    out = {"J": upload_csr(level.J, device),
           "P": upload_csr(level.P, device) if level.P is not None else None,
           "R": upload_csr(level.R, device) if level.R is not None else None,
           "groups": [], "blocks": np.asarray(level.blocks, dtype=np.int64)}
    for g in level.groups:
        order, ptr, n_col = _colour_order(g["colours"])
        cd = np.ascontiguousarray(g["cell_dofs"], dtype=np.int32)
        out["groups"].append(dict(n_cells=cd.shape[0], n_K=cd.shape[1], cell_dofs=torch.from_numpy(cd).to(device),
                                  colour_cells=torch.from_numpy(order).to(device), colour_ptr=ptr,
                                  n_colours=n_col))
    return out


class Solver:
    """Owns a vk_ctx and the device tensors it points to."""

    def __init__(self, levels, stream=None):
        self._keep = []
        self.levels = levels
        self.stream = stream
        ctx = _P()
        st = _lib.vk_create(ctypes.byref(ctx), len(levels), _stream_handle(stream))
        if st != VK_OK:
            raise VkError(st, "vk_create failed: " + _lib.vk_last_error(None).decode())
        self.ctx = ctx
        for l, lv in enumerate(levels):
            J = csr_struct(lv["J"])
            P = csr_struct(lv["P"]) if l > 0 else None
            R = csr_struct(lv["R"]) if l > 0 else None
            if "groups" in lv:
                gs = (vk_cell_group * max(1, len(lv["groups"])))()
                for i, g in enumerate(lv["groups"]):
                    ptr = np.ascontiguousarray(g["colour_ptr"], dtype=np.int32)
                    self._keep.append(ptr)
                    gs[i] = vk_cell_group(int(g["n_cells"]), int(g["n_K"]), g["cell_dofs"].data_ptr(),
                                          g["colour_cells"].data_ptr(), ptr.ctypes.data_as(_PI32),
                                          int(g["n_colours"]))
                blocks = np.ascontiguousarray(lv["blocks"], dtype=np.int64)
                self._keep += [gs, blocks]
                nb = max(0, len(blocks) - 1)
                self._check(_lib.vk_set_level_groups(
                    self.ctx, l, ctypes.byref(J), ctypes.byref(P) if P is not None else None,
                    ctypes.byref(R) if R is not None else None, len(lv["groups"]), gs, nb,
                    blocks.ctypes.data_as(_PI64) if nb else None))
                continue
            ptr = np.ascontiguousarray(lv["colour_ptr"], dtype=np.int32)
            self._keep.append(ptr)
            self._check(_lib.vk_set_level(
                self.ctx, l, ctypes.byref(J), ctypes.byref(P) if P is not None else None,
                ctypes.byref(R) if R is not None else None, int(lv["n_cells"]), int(lv["n_K"]),
                _ptr(lv["cell_dofs"]), _ptr(lv["colour_cells"]),
                ptr.ctypes.data_as(_PI32), int(lv["n_colours"])))
        self.workspace = None
        self.prec = None
        self.restart = None

    def _check(self, st):
        if st != VK_OK:
            raise VkError(st, _lib.vk_last_error(self.ctx).decode())
        return st

    def close(self):
        if getattr(self, "ctx", None):
            _lib.vk_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n(self):
        return int(self.levels[-1]["J"]["n_rows"])

    def vk_workspace_bytes(self, prec="f64", restart=30):
        return int(_lib.vk_workspace_bytes(self.ctx, PRECISIONS[prec], restart))

    def vk_set_workspace(self, prec="f64", restart=30, device="cuda"):
        import torch
        nbytes = self.vk_workspace_bytes(prec, restart)
        if nbytes == 0:
            raise VkError(VK_ERR_STATE, "levels inconsistent or arguments invalid")
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-ws.data_ptr()) % 256
        self._check(_lib.vk_set_workspace(self.ctx, ctypes.c_void_p(ws.data_ptr() + off), nbytes,
                                          PRECISIONS[prec], restart))
        self.workspace, self.prec, self.restart = ws, prec, restart

    def vanka_setup(self, omega=0.7, mode="additive"):
        bl, bc = _I32(-1), _I32(-1)
        st = _lib.vanka_setup(self.ctx, omega, MODES[mode], ctypes.byref(bl), ctypes.byref(bc))
        if st != VK_OK:
            err = VkError(st, _lib.vk_last_error(self.ctx).decode())
            err.bad_level, err.bad_cell = bl.value, bc.value
            raise err

    def vanka_smooth(self, l, b, d, sweeps, d_is_zero=False):
        self._check(_lib.vanka_smooth(self.ctx, l, _ptr(b), _ptr(d), sweeps, 1 if d_is_zero else 0))

    def vanka_smooth_noalloc(self, l, b, d, sweeps, d_is_zero=False):
        self._check(_lib.vanka_smooth_noalloc(self.ctx, l, _ptr(b), _ptr(d), sweeps, 1 if d_is_zero else 0))

    def vcycle(self, b, x, nu_pre=2, nu_post=2):
        self._check(_lib.vcycle(self.ctx, _ptr(b), _ptr(x), nu_pre, nu_post))

    def gmres_solve(self, b, x, restart=30, max_iter=300, rtol=1e-8, atol=0.0, nu_pre=2, nu_post=2,
                    raise_on_noconv=True):
        its = _I32(0)
        rel = _D(0.0)
        hist = (ctypes.c_double * (max_iter + 1))()
        st = _lib.gmres_solve(self.ctx, _ptr(b), _ptr(x), restart, max_iter, rtol, atol, nu_pre, nu_post,
                              ctypes.byref(its), ctypes.byref(rel), hist)
        if st != VK_OK and not (st == VK_ERR_NOCONV and not raise_on_noconv):
            raise VkError(st, _lib.vk_last_error(self.ctx).decode())
        return its.value, rel.value, np.array(hist[: its.value + 1]), st == VK_OK

    def vk_set_segments(self, seg_rows):
        seg = np.ascontiguousarray(seg_rows, dtype=np.int64)
        self._keep.append(seg)
        self._check(_lib.vk_set_segments(self.ctx, len(seg) - 1, seg.ctypes.data_as(_PI64)))
        self.n_seg = len(seg) - 1

    def gmres_solve_batched(self, b, x, restart=30, max_iter=300, rtol=1e-8, atol=0.0, nu_pre=2, nu_post=2,
                            raise_on_noconv=True):
        ns = getattr(self, "n_seg", 1)
        its = (ctypes.c_int32 * ns)()
        rel = (ctypes.c_double * ns)()
        conv = _I32(0)
        st = _lib.gmres_solve_batched(self.ctx, _ptr(b), _ptr(x), restart, max_iter, rtol, atol, nu_pre, nu_post,
                                      its, rel, ctypes.byref(conv))
        if st != VK_OK and not (st == VK_ERR_NOCONV and not raise_on_noconv):
            raise VkError(st, _lib.vk_last_error(self.ctx).decode())
        return np.array(its[:]), np.array(rel[:]), bool(conv.value)

    def vk_spmv(self, l, x, y, alpha=1.0, beta=0.0, z=None):
        self._check(_lib.vk_spmv(self.ctx, l, alpha, _ptr(x), beta, _ptr(z), _ptr(y)))

    def vk_get_patch_inverses(self, l, cell0, n, out):
        self._check(_lib.vk_get_patch_inverses(self.ctx, l, cell0, n, _ptr(out)))

    def vk_get_coarse_inverse(self, out):
        self._check(_lib.vk_get_coarse_inverse(self.ctx, _ptr(out)))

    def vk_set_patch_tile(self, l, cells_per_block):
        self._check(_lib.vk_set_patch_tile(self.ctx, l, cells_per_block))

    def vk_set_sweep_variant(self, variant):
        self._check(_lib.vk_set_sweep_variant(self.ctx, SWEEP_VARIANTS[variant]))

    def vk_set_setup_variant(self, variant):
        self._check(_lib.vk_set_setup_variant(self.ctx, variant))

    def vk_set_coarse_pivoting(self, mode):
        """0: tournament pivoting for blocks wider than 4096 rows; 1: partial pivoting over all rows;
        2: the tournament for every block."""
        self._check(_lib.vk_set_coarse_pivoting(self.ctx, mode))

    def vk_set_spmv_format(self, grouped):
        """1 (or True): grouped CSR for the J products of large levels, lanes per group chosen by
        the library (default); 4, 8, 16, 32 or 64: the grouped CSR with that many lanes per group;
        0 (or False): CSR everywhere."""
        self._check(_lib.vk_set_spmv_format(self.ctx, int(grouped)))

    def vk_spmv_format(self, level):
        """0: CSR; otherwise the lanes per row group of the grouped CSR in use on that level."""
        v = _lib.vk_spmv_format(self.ctx, level)
        if v < 0:
            raise VkError(VK_ERR_ARG, "invalid level")
        return int(v)

    def vk_spmv_bytes(self, level):
        """Algorithmic bytes of one product with level `level`'s J in the storage in use."""
        v = _lib.vk_spmv_bytes(self.ctx, level)
        if v < 0:
            raise VkError(VK_ERR_ARG, "invalid level")
        return float(v)

    def vk_set_coarse_solver(self, mode):
        """0: block-tridiagonal factorisation of a wide coarse block where its pattern allows; 1: dense inverse."""
        self._check(_lib.vk_set_coarse_solver(self.ctx, mode))

    def vk_coarse_plan(self, level=0):
        """(blocks of the level's block-tridiagonal factorisation, 0 for dense inverses; setup flops)."""
        f = _D(0.0)
        nb = _lib.vk_coarse_plan(self.ctx, level, ctypes.byref(f))
        if nb < 0:
            raise VkError(VK_ERR_ARG, "invalid level")
        return int(nb), float(f.value)

    def vk_autotune(self, reps=10):
        self._check(_lib.vk_autotune(self.ctx, reps))

    def vk_set_graphs(self, enable=True):
        self._check(_lib.vk_set_graphs(self.ctx, 1 if enable else 0))

    def vk_graph_stats(self):
        c, n = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(_lib.vk_graph_stats(self.ctx, ctypes.byref(c), ctypes.byref(n)))
        return c.value, n.value

    def vk_timing_enable(self, enable=True, level=-1):
        self._check(_lib.vk_timing_enable(self.ctx, 1 if enable else 0, level))

    def vk_timing_kinds(self, kinds=None, every=1):
        """Record only these kernel classes (names of KERNEL_KINDS; None: all), one launch in `every`."""
        mask = 0xFFFFFFFF if kinds is None else sum(1 << KERNEL_KINDS[k] for k in kinds)
        self._check(_lib.vk_timing_kinds(self.ctx, mask, every))

    def vk_timing_read(self, kind, l=-1):
        cnt, ms = _I64(0), _D(0.0)
        self._check(_lib.vk_timing_read(self.ctx, KERNEL_KINDS[kind], l, ctypes.byref(cnt), ctypes.byref(ms)))
        return cnt.value, ms.value

    def vk_patch_layout(self, l):
        b, ld = _I64(0), _I32(0)
        self._check(_lib.vk_patch_layout(self.ctx, l, ctypes.byref(b), ctypes.byref(ld)))
        return b.value, ld.value


def lib():
    return _lib


class MLP:
    """A vk_mlp context: the BF16 network of the learned initial guess and its patch kernels.

    Tensors passed in must live on the context's device; BF16 arrays are torch.bfloat16."""

    def __init__(self, n_in, width, n_hidden, n_out, max_batch, device="cuda", stream=None):
        import torch
        ctx = _P()
        st = _lib.vk_mlp_create(ctypes.byref(ctx), n_in, width, n_hidden, n_out, max_batch, _stream_handle(stream))
        if st != VK_OK:
            raise VkError(st, _lib.vk_mlp_last_error(None).decode())
        self.ctx = ctx
        self.shape = (n_in, width, n_hidden, n_out)
        self.n_params = int(_lib.vk_mlp_param_count(ctx))
        nbytes = int(_lib.vk_mlp_workspace_bytes(ctx))
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-ws.data_ptr()) % 256
        self._check(_lib.vk_mlp_set_workspace(ctx, ctypes.c_void_p(ws.data_ptr() + off), nbytes))
        self.workspace = ws
        self.device = device

    def _check(self, st):
        if st != VK_OK:
            raise VkError(st, _lib.vk_mlp_last_error(self.ctx).decode())
        return st

    def close(self):
        if getattr(self, "ctx", None):
            _lib.vk_mlp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        self._check(_lib.vk_mlp_set_params(self.ctx, _ptr(params)))

    def get_params(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        self._check(_lib.vk_mlp_get_params(self.ctx, _ptr(out)))
        return out

    def forward(self, x, rows=None, out=None):
        import torch
        batch = int(rows.numel()) if rows is not None else int(x.shape[0])
        if out is None:
            out = torch.empty((batch, self.shape[3]), dtype=torch.float32, device=self.device)
        self._check(_lib.vk_mlp_forward(self.ctx, batch, _ptr(x), _ptr(rows), _ptr(out)))
        return out

    def gradient(self, x, target, rows=None, want_grad=True):
        import torch
        batch = int(rows.numel()) if rows is not None else int(x.shape[0])
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        grad = torch.empty(self.n_params, dtype=torch.float32, device=self.device) if want_grad else None
        self._check(_lib.vk_mlp_gradient(self.ctx, batch, _ptr(x), _ptr(rows), _ptr(target), _ptr(loss),
                                         _ptr(grad)))
        return loss, grad

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(_lib.vk_mlp_adam(self.ctx, lr, beta1, beta2, eps))

    def patch_features(self, cell_dofs, X1, X2, B, mean, inv_std, out):
        n_cells, n_K = cell_dofs.shape
        self._check(_lib.vk_mlp_patch_features(self.ctx, n_cells, n_K, _ptr(cell_dofs), _ptr(X1), _ptr(X2),
                                               _ptr(B), _ptr(mean), _ptr(inv_std), _ptr(out)))

    def patch_targets(self, cell_dofs, X, base, mean, inv_std, out):
        n_cells, n_K = cell_dofs.shape
        self._check(_lib.vk_mlp_patch_targets(self.ctx, n_cells, n_K, _ptr(cell_dofs), _ptr(X), _ptr(base),
                                              _ptr(mean), _ptr(inv_std), _ptr(out)))

    def patch_average(self, dof_ptr, dof_list, n_K, pred, mean, std, base, out):
        self._check(_lib.vk_mlp_patch_average(self.ctx, int(base.numel()), _ptr(dof_ptr), _ptr(dof_list), n_K,
                                              _ptr(pred), _ptr(mean), _ptr(std), _ptr(base), _ptr(out)))

    def slab_extrapolate(self, E, X, out):
        Eh = np.ascontiguousarray(E, dtype=np.float64)
        n_time = Eh.shape[0]
        self._check(_lib.vk_mlp_slab_extrapolate(self.ctx, int(X.numel()) // n_time, n_time,
                                                 Eh.ctypes.data_as(_PD), _ptr(X), _ptr(out)))


def dof_entries(cell_dofs, n):
    """CSR of DoF -> patch entries (cell * n_K + local), ascending, for MLP.patch_average (host)."""
    cd = np.asarray(cell_dofs, dtype=np.int64)
    flat = cd.ravel()
    order = np.argsort(flat, kind="stable")
    ptr = np.concatenate([[0], np.cumsum(np.bincount(flat, minlength=n))]).astype(np.int64)
    return ptr, order.astype(np.int64)
