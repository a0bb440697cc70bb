"""Python binding of the CHERT C ABI (include/chert.h) for MI355X.

Argument marshalling only: every step of the hot path runs in the HIP
library ``libchert.so`` built from ``csrc/``.  PyTorch provides device memory
(tensors) and the stream.  Importing this module does not need a GPU; calling
a device entry point does, and there is no CPU fallback: a missing library
raises ``ChertError``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchert.so")

CHERT_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "HIP",
                4: "NO_CONVERGENCE", 5: "CAPACITY", 6: "UNREACHABLE", 7: "CYCLE", 8: "ABORTED"}
QP, QSV, QSH = 0, 1, 2
KERNEL_MEV, KERNEL_OEV = 0, 1
SAMPLE_RAY, SAMPLE_SLOWNESS = 0, 1
ST_OK, ST_NO_BRACKET, ST_ILL, ST_FLUID, ST_NONPHYS, ST_NOCONV = 0, 1, 2, 4, 8, 16
ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_NO_CONVERGENCE, ERR_ABORTED = 1, 2, 4, 8
FIELDS = ("V", "A", "Q", "rx", "rz", "thR", "thI", "res")
NF = len(FIELDS)
OUT_TAU_R, OUT_TAU_I, OUT_TSTAR, OUT_PRED_P, OUT_PRED_A = 1, 2, 4, 8, 16
OUT_ALL = 31
LAUNCH_PER_ROUND, LAUNCH_PERSISTENT, LAUNCH_FRONTIER = 0, 1, 2

EXPORTS = (
    "chert_class_from_thomsen", "chert_classes_from_thomsen", "chert_cache_layout_of",
    "chert_build_cache_workspace_bytes", "chert_build_cache",
    "chert_trace_workspace_bytes", "chert_trace_field",
    "chert_trace_batch_workspace_bytes", "chert_trace_batch",
    "chert_extract_raypath", "chert_star_2d", "chert_last_error",
    "chert_prof_enable", "chert_prof_read",
    "chert_surrogate_layout_of", "chert_surrogate_init", "chert_surrogate_dataset",
    "chert_surrogate_fit_norm", "chert_surrogate_grad_workspace_bytes", "chert_surrogate_grad",
    "chert_surrogate_adam", "chert_surrogate_infer",
    "chert_build_cache_surrogate_workspace_bytes", "chert_build_cache_surrogate",
    "chert_trace_graph_create", "chert_trace_graph_launch", "chert_trace_graph_finish",
    "chert_trace_graph_destroy", "chert_trace_autotune_workspace_bytes", "chert_trace_autotune",
    "chert_star_3d", "chert_build_cache_noalloc", "chert_build_cache_noalloc_max_bytes",
    "chert_trace_cells_workspace_bytes", "chert_trace_cells",
    "chert_trace_mspm_workspace_bytes", "chert_trace_mspm",
    "chert_trace_blocks_workspace_bytes", "chert_trace_blocks",
)
WARM_NSTATS = 10
# parameter blocks of the surrogate, in their order in the parameter vector
SURROGATE_SHAPES = [(16, 128), (128,), (128, 128), (128,), (128, 128), (128,), (128, 4), (4,)]
WARM_STATS = ("jobs", "fallback_jobs", "directions", "fold", "newton_fail", "slope",
              "theta_i_not_nearest", "rejected", "window_samples", "window_guard_failed")


class ChertError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class ChertClass(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "a11", "a13", "a33", "a44", "a66", "q11", "q13", "q33", "q44", "q66",
        "rho", "tilt", "azimuth")]

    def as_array(self):
        return np.array([getattr(self, n) for n, _ in self._fields_])


class CacheStats(ctypes.Structure):
    _fields_ = [("n_entries", ctypes.c_int64), ("n_converged", ctypes.c_int64),
                ("n_fallback", ctypes.c_int64), ("n_noconv", ctypes.c_int64),
                ("n_illcond", ctypes.c_int64), ("n_nobracket", ctypes.c_int64),
                ("n_unusable", ctypes.c_int64), ("max_resid", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


CACHE_STATS_BYTES = ctypes.sizeof(CacheStats)


class CacheDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_dirs", ctypes.c_int32),
                ("mode_mask", ctypes.c_uint32), ("kernel", ctypes.c_int32),
                ("n_sweep", ctypes.c_int32), ("n_subset", ctypes.c_int32),
                ("subset_host", ctypes.c_void_p), ("resid_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("sampling", ctypes.c_int32),
                ("stats_dev", ctypes.c_void_p)]

    @property
    def n_cols(self):
        return self.n_subset if self.n_subset else self.n_dirs


class CacheLayout(ctypes.Structure):
    _fields_ = [("fields_offset", ctypes.c_size_t), ("status_offset", ctypes.c_size_t),
                ("total_bytes", ctypes.c_size_t)]


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("nx", ctypes.c_int64), ("nz", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("hx", ctypes.c_double), ("hz", ctypes.c_double), ("hy", ctypes.c_double),
                ("class_id_dev", ctypes.c_void_p)]


class CellGrid(ctypes.Structure):
    _fields_ = [("ncx", ctypes.c_int32), ("ncz", ctypes.c_int32), ("cell_n", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("hx", ctypes.c_double), ("hz", ctypes.c_double),
                ("class_id_dev", ctypes.c_void_p)]


class BlockGrid(ctypes.Structure):
    _fields_ = [("ncx", ctypes.c_int32), ("ncy", ctypes.c_int32), ("ncz", ctypes.c_int32),
                ("block_n", ctypes.c_int32), ("hx", ctypes.c_double), ("hy", ctypes.c_double),
                ("hz", ctypes.c_double), ("class_id_dev", ctypes.c_void_p)]


class TraceJob(ctypes.Structure):
    _fields_ = [("d", ctypes.c_void_p), ("cache_dev", ctypes.c_void_p),
                ("n_classes", ctypes.c_int64), ("g", ctypes.c_void_p),
                ("mode", ctypes.c_int32), ("n_src", ctypes.c_int32),
                ("src_nodes_host", ctypes.c_void_p),
                ("tau_r_dev", ctypes.c_void_p), ("tau_i_dev", ctypes.c_void_p),
                ("tstar_dev", ctypes.c_void_p), ("pred_p_dev", ctypes.c_void_p),
                ("pred_a_dev", ctypes.c_void_p)]


class TraceStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32),
                ("tile_visits", ctypes.c_int64 * 3), ("edge_relaxations", ctypes.c_int64 * 3),
                ("levels_sum", ctypes.c_int64 * 3), ("levels_max", ctypes.c_int32 * 3),
                ("reserved2", ctypes.c_int32)]

    def as_dict(self):
        return {"rounds": list(self.rounds), "tile_visits": list(self.tile_visits),
                "edge_relaxations": list(self.edge_relaxations),
                "levels_sum": list(self.levels_sum), "levels_max": list(self.levels_max)}


class TraceOpts(ctypes.Structure):
    _fields_ = [("outputs", ctypes.c_uint32), ("tile_x", ctypes.c_int32),
                ("tile_z", ctypes.c_int32), ("max_rounds", ctypes.c_int32),
                ("push_group", ctypes.c_int32), ("launch", ctypes.c_int32),
                ("bucket_width", ctypes.c_double), ("stats_host", ctypes.c_void_p),
                ("abort_flag_host", ctypes.c_void_p)]


class SurrogateLayout(ctypes.Structure):
    _fields_ = [("total_bytes", ctypes.c_size_t), ("norm_offset", ctypes.c_size_t),
                ("params_offset", ctypes.c_size_t), ("adam_m_offset", ctypes.c_size_t),
                ("adam_v_offset", ctypes.c_size_t), ("n_params", ctypes.c_int32),
                ("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("n_out", ctypes.c_int32)]


class ProfEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


_lib = None


def lib():
    """Load libchert.so (after torch, so the HIP runtime is shared)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ChertError(2, f"HIP library not built: {LIB_PATH} "
                                "(run __graft_entry__.build())")
        try:
            import torch  # noqa: F401  (loads the HIP runtime the library links)
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, sz, d = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                              ctypes.c_size_t, ctypes.c_double)
        L.chert_last_error.restype = ctypes.c_char_p
        L.chert_class_from_thomsen.argtypes = [d] * 10 + [P]
        L.chert_classes_from_thomsen.argtypes = [P, i64, P, P]
        L.chert_cache_layout_of.argtypes = [P, i64, P]
        L.chert_build_cache_workspace_bytes.argtypes = [P, i64]
        L.chert_build_cache_workspace_bytes.restype = sz
        L.chert_build_cache.argtypes = [P, P, i64, P, P, sz, P]
        L.chert_build_cache_noalloc.argtypes = [P, P, i64, P, P]
        L.chert_build_cache_noalloc_max_bytes.argtypes = []
        L.chert_build_cache_noalloc_max_bytes.restype = sz
        L.chert_trace_workspace_bytes.argtypes = [P, i64, P, i32, P]
        L.chert_trace_workspace_bytes.restype = sz
        L.chert_trace_field.argtypes = [P, P, i64, P, i32, P, i32, P, P, P, P, P, P, P, sz, P]
        L.chert_trace_batch_workspace_bytes.argtypes = [P, i32, P]
        L.chert_trace_batch_workspace_bytes.restype = sz
        L.chert_trace_batch.argtypes = [P, i32, P, P, sz, P]
        L.chert_extract_raypath.argtypes = [P, i64, i64, i64, P, i64, P]
        L.chert_star_2d.argtypes = [i32, d, d, i32, P, P, P, P]
        L.chert_prof_enable.argtypes = [i32, ctypes.c_char_p]
        L.chert_prof_read.argtypes = [P, i32, P]
        L.chert_surrogate_layout_of.argtypes = [P]
        L.chert_surrogate_init.argtypes = [P, P, P]
        L.chert_surrogate_dataset.argtypes = [P, P, P, i64, P, P, P, P]
        L.chert_surrogate_fit_norm.argtypes = [P, P, P, P, i64, P]
        L.chert_surrogate_grad_workspace_bytes.argtypes = [i32]
        L.chert_surrogate_grad_workspace_bytes.restype = sz
        L.chert_surrogate_grad.argtypes = [P, P, P, P, i32, P, P, P, sz, P]
        L.chert_surrogate_adam.argtypes = [P, P, i32, ctypes.c_float, P]
        L.chert_surrogate_infer.argtypes = [P, P, i64, P, P]
        L.chert_build_cache_surrogate_workspace_bytes.argtypes = [P, i64]
        L.chert_build_cache_surrogate_workspace_bytes.restype = sz
        L.chert_build_cache_surrogate.argtypes = [P, P, i64, P, d, P, P, P, sz, P]
        L.chert_trace_graph_create.argtypes = [P, i32, P, P, sz, P, P]
        L.chert_trace_graph_launch.argtypes = [P, P]
        L.chert_trace_graph_finish.argtypes = [P, P, P]
        L.chert_trace_graph_destroy.argtypes = [P]
        L.chert_trace_autotune_workspace_bytes.argtypes = [P, i32, P]
        L.chert_trace_autotune_workspace_bytes.restype = sz
        L.chert_trace_autotune.argtypes = [P, i32, P, P, sz, P, P]
        L.chert_star_3d.argtypes = [i32, d, d, d, i32, P, P, P, P, P]
        L.chert_trace_cells_workspace_bytes.argtypes = [P, i64, P, i32, P]
        L.chert_trace_cells_workspace_bytes.restype = sz
        L.chert_trace_cells.argtypes = [P, P, i64, P, i32, P, i32, P, P, P, P, P, P, P, sz, P]
        L.chert_trace_blocks_workspace_bytes.argtypes = [P, i64, P, i32, P]
        L.chert_trace_blocks_workspace_bytes.restype = sz
        L.chert_trace_blocks.argtypes = [P, P, i64, P, i32, P, i32, P, P, P, P, P, P, P, sz, P]
        L.chert_trace_mspm_workspace_bytes.argtypes = [i64, P, i32, P]
        L.chert_trace_mspm_workspace_bytes.restype = sz
        L.chert_trace_mspm.argtypes = [P, i64, P, i32, i32, i32, P, i32, P, P, P, P, P, P, P,
                                       sz, P]
        _lib = L
    return _lib


def chert_last_error() -> str:
    return lib().chert_last_error().decode()


def _check(rc):
    if rc != CHERT_OK:
        raise ChertError(rc, chert_last_error())


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------- host calls --

def chert_class_from_thomsen(vp0, vs0, rho, eps, delta, gamma, tilt, azimuth, qp, qs):
    out = ChertClass()
    _check(lib().chert_class_from_thomsen(vp0, vs0, rho, eps, delta, gamma, tilt,
                                          azimuth, qp, qs, ctypes.byref(out)))
    return out


def cache_desc(n_dirs=360, modes=(QP, QSV, QSH), kernel=KERNEL_MEV, n_sweep=1440, dim=2,
               subset=None, resid_tol=0.0, max_iter=0, stats=None, sampling=0):
    """subset: ascending direction indices closed under reversal (kept
    referenced by the descriptor), e.g. star_subset(radius, hx, hz);
    resid_tol / max_iter: the solver's residual cap and bracket step cap
    (0 = library defaults); sampling: SAMPLE_RAY (ray-direction columns)
    or SAMPLE_SLOWNESS (slowness-angle columns); stats: a device tensor of at least
    CACHE_STATS_BYTES bytes that the build calls overwrite with a
    chert_cache_stats (read it with cache_stats_of)."""
    mask = 0
    for m in modes:
        mask |= 1 << m
    sp = stats.data_ptr() if stats is not None else None
    if subset is None:
        d = CacheDesc(dim, n_dirs, mask, kernel, n_sweep, 0, None, float(resid_tol),
                      int(max_iter), int(sampling), sp)
    else:
        sub = np.ascontiguousarray(subset, dtype=np.int32)
        d = CacheDesc(dim, n_dirs, mask, kernel, n_sweep, int(sub.size), sub.ctypes.data,
                      float(resid_tol), int(max_iter), int(sampling), sp)
        d._subset = sub
    d._stats = stats
    return d


def cache_stats_of(stats_dev):
    """chert_cache_stats from the device tensor a build wrote (synchronises)."""
    raw = bytes(stats_dev[:CACHE_STATS_BYTES].cpu().numpy().tobytes())
    return CacheStats.from_buffer_copy(raw)


def star_subset(radius, hx, hz, n_dirs=360):
    """Directions a forward star of this radius reads (sorted, unique)."""
    return np.unique(chert_star_2d(radius, hx, hz, n_dirs)[3]).astype(np.int32)


def chert_cache_layout_of(desc, n_classes):
    out = CacheLayout()
    _check(lib().chert_cache_layout_of(ctypes.byref(desc), n_classes, ctypes.byref(out)))
    return out


def chert_build_cache_workspace_bytes(desc, n_classes):
    return int(lib().chert_build_cache_workspace_bytes(ctypes.byref(desc), n_classes))


def chert_star_2d(radius, hx, hz, n_dirs=360):
    n = lib().chert_star_2d(radius, hx, hz, n_dirs, None, None, None, None)
    if n < 0:
        raise ChertError(1, chert_last_error())
    ox = np.zeros(n, np.int32)
    oz = np.zeros(n, np.int32)
    L = np.zeros(n)
    b = np.zeros(n, np.int32)
    lib().chert_star_2d(radius, hx, hz, n_dirs, ox.ctypes.data, oz.ctypes.data,
                        L.ctypes.data, b.ctypes.data)
    return ox, oz, L, b


def chert_star_3d(radius, hx, hy, hz, n_dirs=41253):
    """(ox, oy, oz, length, bin) of the 3D forward star (host)."""
    n = lib().chert_star_3d(radius, hx, hy, hz, n_dirs, None, None, None, None, None)
    if n < 0:
        _check(1)
    ox, oy, oz, b = (np.zeros(n, np.int32) for _ in range(4))
    L = np.zeros(n)
    p = lambda a: ctypes.c_void_p(a.ctypes.data)
    lib().chert_star_3d(radius, hx, hy, hz, n_dirs, p(ox), p(oy), p(oz), p(L), p(b))
    return ox, oy, oz, L, b


def make_grid3(nx, ny, nz, h, radius, class_id_dev, hy=None, hz=None):
    """3D grid: node ix + nx (iy + ny iz), spacing h (or hx=h, hy, hz)."""
    g = Grid(3, radius, nx, nz, ny, h, h if hz is None else hz, h if hy is None else hy,
             class_id_dev.data_ptr())
    g._keep = class_id_dev
    return g


def chert_extract_raypath(pred, src, rcv, capacity=None):
    """pred: host int32 array (numpy or CPU tensor).  Returns int64 path."""
    p = np.ascontiguousarray(np.asarray(pred), dtype=np.int32)
    n = p.size
    cap = n if capacity is None else capacity
    out = np.zeros(max(cap, 1), np.int64)
    ln = ctypes.c_int64(0)
    _check(lib().chert_extract_raypath(p.ctypes.data, n, src, rcv, out.ctypes.data, cap,
                                       ctypes.byref(ln)))
    return out[: ln.value].copy()


def raypath_length(pred, src, rcv):
    """Required capacity (the CAPACITY path of chert_extract_raypath)."""
    p = np.ascontiguousarray(np.asarray(pred), dtype=np.int32)
    ln = ctypes.c_int64(0)
    rc = lib().chert_extract_raypath(p.ctypes.data, p.size, src, rcv, None, 0, ctypes.byref(ln))
    if rc not in (CHERT_OK, 5):
        _check(rc)
    return ln.value


# ----------------------------------------------------------- device calls --

def chert_classes_from_thomsen(params_dev, classes_out_dev, stream=None):
    """params_dev: float64 device tensor [n, 10]; classes_out_dev: float64
    device tensor [n, 13] (the chert_class layout)."""
    n = params_dev.shape[0]
    _check(lib().chert_classes_from_thomsen(_ptr(params_dev), n, _ptr(classes_out_dev),
                                            _stream(stream)))

def chert_build_cache(desc, classes_dev, n_classes, cache_dev, workspace_dev, stream=None):
    """classes_dev: float64 device tensor [K, 13]; cache_dev: uint8 device
    tensor of the layout's total_bytes; workspace_dev: uint8 device tensor."""
    ws = workspace_dev.numel() * workspace_dev.element_size() if workspace_dev is not None else 0
    _check(lib().chert_build_cache(ctypes.byref(desc), _ptr(classes_dev), n_classes,
                                   _ptr(cache_dev), _ptr(workspace_dev), ws, _stream(stream)))


def chert_build_cache_noalloc(desc, classes_dev, n_classes, cache_dev, stream=None):
    """chert_build_cache with its scratch in the library's own device array
    (no workspace, no allocation); see include/chert.h."""
    _check(lib().chert_build_cache_noalloc(ctypes.byref(desc), _ptr(classes_dev), n_classes,
                                           _ptr(cache_dev), _stream(stream)))


def chert_build_cache_noalloc_max_bytes():
    return int(lib().chert_build_cache_noalloc_max_bytes())


def make_grid(nx, nz, hx, hz, radius, class_id_dev):
    """class_id_dev None: the cache holds one class per node (index = node)."""
    g = Grid(2, radius, nx, nz, 1, hx, hz, 0.0,
             class_id_dev.data_ptr() if class_id_dev is not None else None)
    g._keep = class_id_dev  # the struct holds a raw pointer
    return g


def trace_opts(outputs=OUT_ALL, tile_x=0, tile_z=0, max_rounds=0, stats=None, push_group=0,
               launch=0, bucket_width=0.0, abort_flag=None):
    """stats: a TraceStats to fill (kept referenced by the returned options);
    launch: LAUNCH_PER_ROUND, LAUNCH_PERSISTENT (2D tiles) or LAUNCH_FRONTIER
    (node frontier; always used in 3D); bucket_width: near/far bucket width
    of the frontier iteration (units of the smallest edge weight);
    abort_flag: a pinned host int32 tensor (torch pin_memory) whose first
    element, once non-zero, stops the relaxation (CHERT_ERR_ABORTED)."""
    o = TraceOpts(outputs, tile_x, tile_z, max_rounds, push_group, launch, float(bucket_width),
                  ctypes.addressof(stats) if stats is not None else None,
                  abort_flag.data_ptr() if abort_flag is not None else None)
    o._stats = stats
    o._abort = abort_flag
    return o


def chert_prof_enable(on=True, only=None):
    _check(lib().chert_prof_enable(1 if on else 0, only.encode() if only else None))


def chert_prof_read():
    """{kernel name: (launches, total_ms)} of the current profiling window."""
    n = ctypes.c_int32(0)
    _check(lib().chert_prof_read(None, 0, ctypes.byref(n)))
    arr = (ProfEntry * max(n.value, 1))()
    _check(lib().chert_prof_read(arr, n.value, ctypes.byref(n)))
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n.value)}


def chert_trace_workspace_bytes(desc, n_classes, grid, n_src, opts):
    return int(lib().chert_trace_workspace_bytes(ctypes.byref(desc), n_classes,
                                                 ctypes.byref(grid), n_src, ctypes.byref(opts)))


def make_cell_grid(ncx, ncz, cell_n, hx, hz, class_id_dev):
    """Cell network: ncx x ncz cells of cell_n intervals per side; the class
    map covers the (ncz cell_n + 1) x (ncx cell_n + 1) lattice."""
    g = CellGrid(ncx, ncz, cell_n, 0, hx, hz, class_id_dev.data_ptr())
    g._keep = class_id_dev
    return g


def chert_trace_cells_workspace_bytes(desc, n_classes, grid, n_src, opts):
    return int(lib().chert_trace_cells_workspace_bytes(ctypes.byref(desc), n_classes,
                                                       ctypes.byref(grid), n_src,
                                                       ctypes.byref(opts)))


def chert_trace_cells(desc, cache_dev, n_classes, grid, mode, src_nodes: Sequence[int], opts,
                      tau_r=None, tau_i=None, tstar=None, pred_p=None, pred_a=None,
                      workspace_dev=None, stream=None):
    src = np.ascontiguousarray(np.asarray(src_nodes, dtype=np.int64).reshape(-1))
    ws = workspace_dev.numel() * workspace_dev.element_size() if workspace_dev is not None else 0
    _check(lib().chert_trace_cells(
        ctypes.byref(desc), _ptr(cache_dev), n_classes, ctypes.byref(grid), mode,
        src.ctypes.data, int(src.size), ctypes.byref(opts), _ptr(tau_r), _ptr(tau_i),
        _ptr(tstar), _ptr(pred_p), _ptr(pred_a), _ptr(workspace_dev), ws, _stream(stream)))


def make_block_grid(ncx, ncy, ncz, block_n, hx, hy, hz, class_id_dev):
    """Block network: ncx x ncy x ncz blocks of block_n intervals per edge;
    the class map covers the (ncz n + 1) x (ncy n + 1) x (ncx n + 1) lattice."""
    g = BlockGrid(ncx, ncy, ncz, block_n, hx, hy, hz, class_id_dev.data_ptr())
    g._keep = class_id_dev
    return g


def chert_trace_blocks_workspace_bytes(desc, n_classes, grid, n_src, opts):
    return int(lib().chert_trace_blocks_workspace_bytes(ctypes.byref(desc), n_classes,
                                                        ctypes.byref(grid), n_src,
                                                        ctypes.byref(opts)))


def chert_trace_blocks(desc, cache_dev, n_classes, grid, mode, src_nodes: Sequence[int], opts,
                       tau_r=None, tau_i=None, tstar=None, pred_p=None, pred_a=None,
                       workspace_dev=None, stream=None):
    src = np.ascontiguousarray(np.asarray(src_nodes, dtype=np.int64).reshape(-1))
    ws = workspace_dev.numel() * workspace_dev.element_size() if workspace_dev is not None else 0
    _check(lib().chert_trace_blocks(
        ctypes.byref(desc), _ptr(cache_dev), n_classes, ctypes.byref(grid), mode,
        src.ctypes.data, int(src.size), ctypes.byref(opts), _ptr(tau_r), _ptr(tau_i),
        _ptr(tstar), _ptr(pred_p), _ptr(pred_a), _ptr(workspace_dev), ws, _stream(stream)))


def chert_trace_mspm_workspace_bytes(n_classes, grid, n_src, opts):
    return int(lib().chert_trace_mspm_workspace_bytes(n_classes, ctypes.byref(grid), n_src,
                                                      ctypes.byref(opts)))


def chert_trace_mspm(classes_dev, n_classes, grid, mode, src_nodes: Sequence[int], opts,
                     tau_r=None, tau_i=None, tstar=None, pred_p=None, pred_a=None,
                     workspace_dev=None, kernel=KERNEL_MEV, n_sweep=1440, stream=None):
    src = np.ascontiguousarray(np.asarray(src_nodes, dtype=np.int64).reshape(-1))
    ws = workspace_dev.numel() * workspace_dev.element_size() if workspace_dev is not None else 0
    _check(lib().chert_trace_mspm(
        _ptr(classes_dev), n_classes, ctypes.byref(grid), mode, kernel, n_sweep,
        src.ctypes.data, int(src.size), ctypes.byref(opts), _ptr(tau_r), _ptr(tau_i),
        _ptr(tstar), _ptr(pred_p), _ptr(pred_a), _ptr(workspace_dev), ws, _stream(stream)))


def chert_trace_field(desc, cache_dev, n_classes, grid, mode, src_nodes: Sequence[int], opts,
                      tau_r=None, tau_i=None, tstar=None, pred_p=None, pred_a=None,
                      workspace_dev=None, stream=None):
    src = np.ascontiguousarray(np.asarray(src_nodes, dtype=np.int64).reshape(-1))
    ws = workspace_dev.numel() * workspace_dev.element_size() if workspace_dev is not None else 0
    _check(lib().chert_trace_field(
        ctypes.byref(desc), _ptr(cache_dev), n_classes, ctypes.byref(grid), mode,
        src.ctypes.data, int(src.size), ctypes.byref(opts), _ptr(tau_r), _ptr(tau_i),
        _ptr(tstar), _ptr(pred_p), _ptr(pred_a), _ptr(workspace_dev), ws, _stream(stream)))


class Batch:
    """Marshals a list of trace jobs into the chert_trace_job array; keeps
    every referenced structure and array alive for the duration."""

    def __init__(self):
        self._jobs = []
        self._keep = []

    def add(self, desc, cache_dev, n_classes, grid, mode, src_nodes, tau_r=None, tau_i=None,
            tstar=None, pred_p=None, pred_a=None):
        src = np.ascontiguousarray(np.asarray(src_nodes, dtype=np.int64).reshape(-1))
        self._keep += [desc, grid, src, cache_dev, tau_r, tau_i, tstar, pred_p, pred_a]
        ptr = lambda t: None if t is None else t.data_ptr()
        self._jobs.append(TraceJob(ctypes.addressof(desc), cache_dev.data_ptr(), n_classes,
                                   ctypes.addressof(grid), mode, int(src.size), src.ctypes.data,
                                   ptr(tau_r), ptr(tau_i), ptr(tstar), ptr(pred_p), ptr(pred_a)))
        return self

    def array(self):
        arr = (TraceJob * len(self._jobs))(*self._jobs)
        self._keep.append(arr)
        return arr, len(self._jobs)


def chert_trace_batch_workspace_bytes(batch, opts):
    arr, n = batch.array()
    return int(lib().chert_trace_batch_workspace_bytes(arr, n, ctypes.byref(opts)))


def chert_trace_batch(batch, opts, workspace_dev, stream=None):
    arr, n = batch.array()
    ws = workspace_dev.numel() * workspace_dev.element_size() if workspace_dev is not None else 0
    _check(lib().chert_trace_batch(arr, n, ctypes.byref(opts), _ptr(workspace_dev), ws,
                                   _stream(stream)))


# -------------------------------------------------------------- surrogate --

def _nbytes(t):
    return 0 if t is None else t.numel() * t.element_size()


def chert_surrogate_layout_of():
    out = SurrogateLayout()
    _check(lib().chert_surrogate_layout_of(ctypes.byref(out)))
    return out


def chert_surrogate_init(blob_dev, params_dev, stream=None):
    """blob_dev: uint8 device tensor of total_bytes (256-byte aligned);
    params_dev: float32 device tensor [n_params]."""
    _check(lib().chert_surrogate_init(_ptr(blob_dev), _ptr(params_dev), _stream(stream)))


def chert_surrogate_dataset(desc, cache_dev, classes_dev, n_classes, x_dev, y_dev, ok_dev,
                            stream=None):
    """x_dev float32 [n, 16], y_dev float32 [n, 4], ok_dev int32 [n] with n =
    modes * n_classes * columns."""
    _check(lib().chert_surrogate_dataset(ctypes.byref(desc), _ptr(cache_dev), _ptr(classes_dev),
                                         n_classes, _ptr(x_dev), _ptr(y_dev), _ptr(ok_dev),
                                         _stream(stream)))


def chert_surrogate_fit_norm(blob_dev, x_dev, y_dev, ok_dev, stream=None):
    _check(lib().chert_surrogate_fit_norm(_ptr(blob_dev), _ptr(x_dev), _ptr(y_dev), _ptr(ok_dev),
                                          x_dev.shape[0], _stream(stream)))


def chert_surrogate_grad_workspace_bytes(batch):
    return lib().chert_surrogate_grad_workspace_bytes(batch)


def chert_surrogate_grad(blob_dev, x_dev, y_dev, idx_dev, grad_dev, loss_dev, workspace_dev,
                         stream=None):
    """idx_dev int32 [batch]; grad_dev float32 [n_params]; loss_dev float32
    [1] or None."""
    _check(lib().chert_surrogate_grad(_ptr(blob_dev), _ptr(x_dev), _ptr(y_dev), _ptr(idx_dev),
                                      idx_dev.numel(), _ptr(grad_dev), _ptr(loss_dev),
                                      _ptr(workspace_dev), _nbytes(workspace_dev),
                                      _stream(stream)))


def chert_surrogate_adam(blob_dev, grad_dev, step, lr, stream=None):
    _check(lib().chert_surrogate_adam(_ptr(blob_dev), _ptr(grad_dev), int(step), float(lr),
                                      _stream(stream)))


def chert_surrogate_infer(blob_dev, x_dev, y_dev, stream=None):
    _check(lib().chert_surrogate_infer(_ptr(blob_dev), _ptr(x_dev), x_dev.shape[0], _ptr(y_dev),
                                       _stream(stream)))


def chert_build_cache_surrogate_workspace_bytes(desc, n_classes):
    return lib().chert_build_cache_surrogate_workspace_bytes(ctypes.byref(desc), n_classes)


def chert_build_cache_surrogate(desc, classes_dev, n_classes, blob_dev, cache_dev, workspace_dev,
                                stats_dev=None, resid_tol=0.0, stream=None):
    """stats_dev: int64 device tensor [WARM_NSTATS] or None."""
    _check(lib().chert_build_cache_surrogate(ctypes.byref(desc), _ptr(classes_dev), n_classes,
                                             _ptr(blob_dev), float(resid_tol), _ptr(cache_dev),
                                             _ptr(stats_dev), _ptr(workspace_dev),
                                             _nbytes(workspace_dev), _stream(stream)))


def train_surrogate(blob_dev, x_dev, y_dev, ok_dev, steps, batch=2048, lr=2e-3, lr_end=2e-5,
                    seed=0, stream=None):
    """Minibatch Adam on the usable samples (ok_dev != 0): each epoch visits
    them in a fresh seeded permutation; the learning rate decays from lr to
    lr_end on a cosine.  Every step is one chert_surrogate_grad and one
    chert_surrogate_adam call; returns the per-step losses (device
    float32 tensor [steps]).  Starts from the blob's current weights and
    continues its Adam moments at step 1 (a fresh chert_surrogate_init
    resets them)."""
    import math
    t = _torch()
    valid = np.flatnonzero(ok_dev.cpu().numpy()).astype(np.int32)
    if valid.size == 0:
        raise ChertError(1, "no usable samples")
    batch = int(min(batch, valid.size))
    rng = np.random.default_rng(seed)
    dev = x_dev.device
    grad = t.empty(chert_surrogate_layout_of().n_params, dtype=t.float32, device=dev)
    losses = t.zeros(steps, dtype=t.float32, device=dev)
    ws = t.empty(chert_surrogate_grad_workspace_bytes(batch), dtype=t.uint8, device=dev)
    per_epoch = valid.size // batch
    perm = None
    for s in range(steps):
        e, b = divmod(s, per_epoch)
        if b == 0:
            perm = t.from_numpy(rng.permutation(valid)).to(dev)
        idx = perm[b * batch:(b + 1) * batch]
        chert_surrogate_grad(blob_dev, x_dev, y_dev, idx, grad, losses[s:s + 1], ws, stream)
        rate = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * s / max(steps - 1, 1)))
        chert_surrogate_adam(blob_dev, grad, s + 1, rate, stream)
    return losses


def surrogate_views(blob_dev):
    """(params, adam_m, adam_v, norm[40]) float32 views into a blob tensor,
    following the documented layout."""
    lay = chert_surrogate_layout_of()
    t = _torch()
    n = lay.n_params

    def v(off, k):
        return blob_dev[off: off + 4 * k].view(dtype=t.float32)
    return (v(lay.params_offset, n), v(lay.adam_m_offset, n), v(lay.adam_v_offset, n),
            v(lay.norm_offset, 40))


# ------------------------------------------------------------ cache views --

def chert_trace_autotune_workspace_bytes(batch, opts):
    arr, n = batch.array()
    return int(lib().chert_trace_autotune_workspace_bytes(arr, n, ctypes.byref(opts)))


def chert_trace_autotune(batch, opts, workspace_dev, stream=None):
    """Updates opts in place (tile, push group, launch); returns the probe's
    time in ms."""
    arr, n = batch.array()
    ms = ctypes.c_double(0.0)
    _check(lib().chert_trace_autotune(arr, n, ctypes.byref(opts), _ptr(workspace_dev),
                                      _nbytes(workspace_dev), _stream(stream), ctypes.byref(ms)))
    return ms.value


class TraceGraph:
    """A chert_trace_batch captured as one HIP graph (persistent phases, or
    per-round launches with a round budget).
    Keeps the batch, options and workspace referenced while it lives."""

    def __init__(self, batch, opts, workspace_dev, stream=None):
        import torch
        self._keep = (batch, opts, workspace_dev)
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        arr, n = batch.array()
        h = ctypes.c_void_p()
        _check(lib().chert_trace_graph_create(arr, n, ctypes.byref(opts),
                                              _ptr(workspace_dev), _nbytes(workspace_dev),
                                              _stream(stream), ctypes.byref(h)))
        self._arr = arr
        self.handle = h

    def launch(self, stream=None):
        _check(lib().chert_trace_graph_launch(self.handle, _stream(stream or self._stream)))

    def finish(self, stats=None, stream=None):
        _check(lib().chert_trace_graph_finish(
            self.handle, _stream(stream or self._stream),
            ctypes.byref(stats) if stats is not None else None))

    def close(self):
        if self.handle:
            lib().chert_trace_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cache_views(cache_dev, desc, n_classes):
    """(fields [NF][3][K][n_dirs] float64, status [3][K][n_dirs] int32) views
    into a cache blob tensor, following the documented layout."""
    lay = chert_cache_layout_of(desc, n_classes)
    n = 3 * n_classes * desc.n_cols
    f = cache_dev[lay.fields_offset: lay.fields_offset + NF * n * 8]
    s = cache_dev[lay.status_offset: lay.status_offset + n * 4]
    return (f.view(dtype=_torch().float64).view(NF, 3, n_classes, desc.n_cols),
            s.view(dtype=_torch().int32).view(3, n_classes, desc.n_cols))


def _torch():
    import torch
    return torch
