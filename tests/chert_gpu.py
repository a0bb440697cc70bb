"""Test-side helpers that drive the HIP library through its C ABI (the
Python binding) with torch device tensors.  No arithmetic of the method
lives here."""
import numpy as np
import torch

import paper_2609_26108_amd as C

DEV = torch.device("cuda:0")


def classes_from_layers(layers):
    """Host chert_class_from_thomsen per layer -> float64 [K, 13] device tensor."""
    rows = [C.chert_class_from_thomsen(*L.thomsen_args()).as_array() for L in layers]
    return torch.from_numpy(np.stack(rows)).to(DEV)


def classes_from_arrays(arr):
    return torch.from_numpy(np.ascontiguousarray(np.atleast_2d(arr), dtype=np.float64)).to(DEV)


def build_cache(classes_dev, desc):
    K = classes_dev.shape[0]
    lay = C.chert_cache_layout_of(desc, K)
    cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=DEV)
    ws = torch.empty(max(C.chert_build_cache_workspace_bytes(desc, K), 1),
                     dtype=torch.uint8, device=DEV)
    C.chert_build_cache(desc, classes_dev, K, cache, ws)
    torch.cuda.synchronize()
    return cache


def cache_to_numpy(cache, desc, K):
    f, s = C.cache_views(cache, desc, K)
    return f.cpu().numpy(), s.cpu().numpy()


def import_cache(fields_np, status_np, desc, K):
    """Write oracle-computed arrays into a cache blob with the documented layout."""
    lay = C.chert_cache_layout_of(desc, K)
    cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=DEV)
    f, s = C.cache_views(cache, desc, K)
    f.copy_(torch.from_numpy(np.ascontiguousarray(fields_np)))
    s.copy_(torch.from_numpy(np.ascontiguousarray(status_np, dtype=np.int32)))
    torch.cuda.synchronize()
    return cache


def trace(cache, desc, K, nx, nz, hx, hz, radius, class_id_np, mode, sources,
          outputs=C.OUT_ALL, tile_x=0, tile_z=0, launch=0, bucket_width=0.0, push_group=0):
    cid = None  # one class per node
    if class_id_np is not None:
        cid = torch.from_numpy(np.ascontiguousarray(class_id_np, dtype=np.int32).reshape(-1)).to(DEV)
    g = C.make_grid(nx, nz, hx, hz, radius, cid)
    o = C.trace_opts(outputs, tile_x, tile_z, launch=launch, bucket_width=bucket_width,
                     push_group=push_group)
    n = nx * nz
    S = len(sources)
    out = {
        "tauR": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TAU_R else None,
        "tauI": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TAU_I else None,
        "tstar": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TSTAR else None,
        "predP": torch.empty((S, n), dtype=torch.int32, device=DEV) if outputs & C.OUT_PRED_P else None,
        "predA": torch.empty((S, n), dtype=torch.int32, device=DEV) if outputs & C.OUT_PRED_A else None,
    }
    wsb = C.chert_trace_workspace_bytes(desc, K, g, S, o)
    assert wsb > 0, C.chert_last_error()
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    C.chert_trace_field(desc, cache, K, g, mode, sources, o, out["tauR"], out["tauI"],
                        out["tstar"], out["predP"], out["predA"], ws)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def trace_cells(cache, desc, K, ncx, ncz, cn, hx, hz, class_id_np, mode, sources,
                outputs=C.OUT_ALL, bucket_width=0.0, max_rounds=0, stats=None):
    cid = torch.from_numpy(np.ascontiguousarray(class_id_np, dtype=np.int32).reshape(-1)).to(DEV)
    g = C.make_cell_grid(ncx, ncz, cn, hx, hz, cid)
    o = C.trace_opts(outputs, bucket_width=bucket_width, max_rounds=max_rounds, stats=stats)
    n = (ncx * cn + 1) * (ncz * cn + 1)
    S = len(sources)
    out = {
        "tauR": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TAU_R else None,
        "tauI": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TAU_I else None,
        "tstar": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TSTAR else None,
        "predP": torch.empty((S, n), dtype=torch.int32, device=DEV) if outputs & C.OUT_PRED_P else None,
        "predA": torch.empty((S, n), dtype=torch.int32, device=DEV) if outputs & C.OUT_PRED_A else None,
    }
    wsb = C.chert_trace_cells_workspace_bytes(desc, K, g, S, o)
    assert wsb > 0, C.chert_last_error()
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    C.chert_trace_cells(desc, cache, K, g, mode, sources, o, out["tauR"], out["tauI"],
                        out["tstar"], out["predP"], out["predA"], ws)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def trace_blocks(cache, desc, K, ncx, ncy, ncz, cn, hx, hy, hz, class_id_np, mode, sources,
                 outputs=C.OUT_ALL, bucket_width=0.0, max_rounds=0, stats=None):
    cid = torch.from_numpy(np.ascontiguousarray(class_id_np, dtype=np.int32).reshape(-1)).to(DEV)
    g = C.make_block_grid(ncx, ncy, ncz, cn, hx, hy, hz, cid)
    o = C.trace_opts(outputs, bucket_width=bucket_width, max_rounds=max_rounds, stats=stats)
    n = (ncx * cn + 1) * (ncy * cn + 1) * (ncz * cn + 1)
    S = len(sources)
    out = {
        "tauR": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TAU_R else None,
        "tauI": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TAU_I else None,
        "tstar": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TSTAR else None,
        "predP": torch.empty((S, n), dtype=torch.int32, device=DEV) if outputs & C.OUT_PRED_P else None,
        "predA": torch.empty((S, n), dtype=torch.int32, device=DEV) if outputs & C.OUT_PRED_A else None,
    }
    wsb = C.chert_trace_blocks_workspace_bytes(desc, K, g, S, o)
    assert wsb > 0, C.chert_last_error()
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    C.chert_trace_blocks(desc, cache, K, g, mode, sources, o, out["tauR"], out["tauI"],
                         out["tstar"], out["predP"], out["predA"], ws)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def trace_mspm(classes_np, ncx, ncz, cn, hx, hz, class_id_np, mode, sources, outputs=C.OUT_ALL,
               bucket_width=0.0, kernel=C.KERNEL_MEV, n_sweep=1440, stats=None):
    cls = classes_from_arrays(classes_np)
    K = cls.shape[0]
    cid = torch.from_numpy(np.ascontiguousarray(class_id_np, dtype=np.int32).reshape(-1)).to(DEV)
    g = C.make_cell_grid(ncx, ncz, cn, hx, hz, cid)
    o = C.trace_opts(outputs, bucket_width=bucket_width, stats=stats)
    n = (ncx * cn + 1) * (ncz * cn + 1)
    S = len(sources)
    out = {
        "tauR": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TAU_R else None,
        "tauI": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TAU_I else None,
        "tstar": torch.empty((S, n), dtype=torch.float64, device=DEV) if outputs & C.OUT_TSTAR else None,
        "predP": torch.empty((S, n), dtype=torch.int32, device=DEV) if outputs & C.OUT_PRED_P else None,
        "predA": torch.empty((S, n), dtype=torch.int32, device=DEV) if outputs & C.OUT_PRED_A else None,
    }
    wsb = C.chert_trace_mspm_workspace_bytes(K, g, S, o)
    assert wsb > 0, C.chert_last_error()
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    C.chert_trace_mspm(cls, K, g, mode, sources, o, out["tauR"], out["tauI"], out["tstar"],
                       out["predP"], out["predA"], ws, kernel=kernel, n_sweep=n_sweep)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
