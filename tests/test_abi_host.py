"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every function include/chert.h declares, the host entry points agree with the
oracle, and device entry points reject bad arguments before launching."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2609_26108_amd as C
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "chert.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chert_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 9
    lib = ctypes.CDLL(C.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(C.EXPORTS) <= set(names)


def test_class_from_thomsen_matches_oracle():
    for L in W.config2().layers + W.config1().layers:
        a = C.chert_class_from_thomsen(*L.thomsen_args()).as_array()
        b = O.class_from_thomsen(*L.thomsen_args())
        assert np.array_equal(a, b)


@pytest.mark.parametrize("args", [
    (3000.0, 3100.0, 2000, 0.1, 0.0, 0.0, 0, 0, 50, 50),      # vs >= vp
    (3000.0, 2900.0, 2000, 0.1, -0.45, 0.0, 0, 0, 50, 50),    # negative radicand
    (3000.0, 1500.0, 2000, 0.1, 0.0, 0.0, 0, 0, 0.0, 50),     # Q <= 0
    (float("nan"), 1500.0, 2000, 0.1, 0.0, 0.0, 0, 0, 50, 50),
])
def test_class_from_thomsen_rejects(args):
    with pytest.raises(C.ChertError) as e:
        C.chert_class_from_thomsen(*args)
    assert e.value.code == 1


def test_star_matches_oracle_bitwise():
    for R in range(1, 9):
        for hx, hz in [(10.0, 10.0), (5.0, 7.5)]:
            for n_dirs in (360, 180, 90, 720, 36):
                a = C.chert_star_2d(R, hx, hz, n_dirs)
                b = O.star_2d(R, hx, hz, n_dirs)
                for x, y in zip(a, b):
                    assert np.array_equal(x, y)


def test_star_subset_closed_at_half_step_ties():
    """At a 2-degree step the diagonal offsets lie half-way between two
    directions; the star still reads bin(o) + n_dirs/2 for -o, so its
    subset is closed under reversal and a per-node cache descriptor with
    it is accepted."""
    for R in (1, 3, 5):
        ox, oz, L, b = C.chert_star_2d(R, 10.0, 10.0, 180)
        assert np.array_equal(b[::-1], (b + 90) % 180)
        sub = C.star_subset(R, 10.0, 10.0, 180)
        d = C.cache_desc(n_dirs=180, modes=(0,), subset=sub)
        C.chert_cache_layout_of(d, 4)


def test_layout():
    d = C.cache_desc(n_dirs=360, modes=(0, 1, 2))
    lay = C.chert_cache_layout_of(d, 5)
    n = 3 * 5 * 360
    assert lay.fields_offset == 256
    assert lay.status_offset == 256 + 8 * n * 8
    assert lay.total_bytes >= lay.status_offset + 4 * n and lay.total_bytes % 256 == 0
    for bad in [C.cache_desc(n_dirs=359), C.cache_desc(n_sweep=8), C.CacheDesc(2, 360, 8, 0, 1440, 0),
                C.CacheDesc(2, 360, 1, 5, 1440, 0)]:
        with pytest.raises(C.ChertError):
            C.chert_cache_layout_of(bad, 5)
    # 3D: every Fibonacci direction is a column; subsets are not supported
    d3 = C.cache_desc(dim=3, n_dirs=41253, modes=(0, 1))
    lay3 = C.chert_cache_layout_of(d3, 6)
    assert lay3.status_offset == 256 + 8 * (3 * 6 * 41253) * 8
    with pytest.raises(C.ChertError) as e:
        C.chert_cache_layout_of(C.cache_desc(dim=3, n_dirs=360, subset=[0, 180]), 5)
    assert e.value.code == 2
    with pytest.raises(C.ChertError) as e:
        C.chert_cache_layout_of(C.cache_desc(dim=4), 5)
    assert e.value.code == 1


def test_star_3d_matches_oracle():
    """The library's host 3D star (offsets, lengths, Fibonacci bins) is the
    oracle's, bitwise."""
    for args in ((3, 10.0, 10.0, 10.0), (2, 10.0, 12.0, 8.0)):
        a = C.chert_star_3d(*args)
        b = O.star_3d(*args)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_raypath_matches_oracle_and_errors():
    rng = np.random.default_rng(1)
    nx, nz = 15, 11
    V = np.concatenate([rng.uniform(2000, 3000, (2, 180))] * 2, 1)
    A = np.full((2, 360), 1e-4)
    st = np.zeros((2, 360), np.int32)
    cid = rng.integers(0, 2, nx * nz).astype(np.int32)
    r = O.trace_2d(nx, nz, 5.0, 5.0, cid, 3, V, A, st, 7)
    for rcv in range(nx * nz):
        p = C.chert_extract_raypath(r["predP"], 7, rcv)
        rc, q = O.raypath(r["predP"], 7, rcv)
        assert rc == 0 and np.array_equal(p, q)
    assert C.raypath_length(r["predP"], 7, nx * nz - 1) == len(
        C.chert_extract_raypath(r["predP"], 7, nx * nz - 1))
    with pytest.raises(C.ChertError) as e:
        C.chert_extract_raypath(r["predP"], 7, nx * nz - 1, capacity=1)
    assert e.value.code == 5
    pred = r["predP"].copy()
    pred[20] = -1
    with pytest.raises(C.ChertError) as e:
        C.chert_extract_raypath(pred, 7, 20)
    assert e.value.code == 6
    pred = np.full(nx * nz, -1, np.int32)
    pred[3], pred[4] = 4, 3
    with pytest.raises(C.ChertError) as e:
        C.chert_extract_raypath(pred, 7, 3)
    assert e.value.code == 7
    with pytest.raises(C.ChertError) as e:
        C.chert_extract_raypath(pred, 7, nx * nz)
    assert e.value.code == 1


class _FakeTensor:
    """Stands in for a device tensor in validation-only calls (never
    dereferenced: validation fails before any launch)."""
    def __init__(self, n=0):
        self.n = n

    def data_ptr(self):
        return 0

    def numel(self):
        return self.n

    def element_size(self):
        return 1


def test_device_calls_validate_before_launch():
    d = C.cache_desc(n_dirs=361)
    with pytest.raises(C.ChertError) as e:
        C.chert_build_cache(d, _FakeTensor(), 3, _FakeTensor(), _FakeTensor(), stream=0)
    assert e.value.code == 1
    d = C.cache_desc()
    with pytest.raises(C.ChertError) as e:  # null classes / cache
        C.chert_build_cache(d, _FakeTensor(), 3, _FakeTensor(), _FakeTensor(), stream=0)
    assert e.value.code == 1
    g = C.Grid(2, 0, 10, 10, 1, 5.0, 5.0, 0.0, None)
    o = C.trace_opts()
    with pytest.raises(C.ChertError) as e:  # radius 0
        C.chert_trace_field(d, _FakeTensor(), 3, g, 0, [0], o, workspace_dev=_FakeTensor(), stream=0)
    assert e.value.code == 1
    assert C.chert_trace_workspace_bytes(d, 3, g, 1, o) == 0
    g = C.Grid(2, 3, 10, 10, 1, 5.0, 5.0, 0.0, 1234)
    with pytest.raises(C.ChertError) as e:  # null outputs for the selected mask
        C.chert_trace_field(d, _FakeTensor(), 3, g, 0, [0], o, workspace_dev=_FakeTensor(), stream=0)
    assert e.value.code == 1
    with pytest.raises(C.ChertError) as e:  # source out of range
        C.chert_trace_field(d, _FakeTensor(), 3, g, 0, [100], o, workspace_dev=_FakeTensor(), stream=0)
    assert e.value.code == 1
    o2 = C.trace_opts(outputs=C.OUT_TSTAR)
    with pytest.raises(C.ChertError):  # t* without its inputs
        C.chert_trace_field(d, _FakeTensor(), 3, g, 0, [0], o2, workspace_dev=_FakeTensor(), stream=0)
    g3 = C.Grid(3, 3, 10, 10, 10, 5.0, 5.0, 5.0, 1234)
    with pytest.raises(C.ChertError) as e:  # 3D grid, 2D cache
        C.chert_trace_field(d, _FakeTensor(), 3, g3, 0, [0], o, workspace_dev=_FakeTensor(), stream=0)
    assert e.value.code == 1
    d3 = C.cache_desc(dim=3, n_dirs=41253, modes=(0, 1))
    with pytest.raises(C.ChertError) as e:  # 3D: null outputs for the selected mask
        C.chert_trace_field(d3, _FakeTensor(), 3, g3, 0, [0], o, workspace_dev=_FakeTensor(),
                            stream=0)
    assert e.value.code == 1
    with pytest.raises(C.ChertError) as e:  # 3D: t* without its inputs
        C.chert_trace_field(d3, _FakeTensor(), 3, g3, 0, [0], C.trace_opts(C.OUT_TSTAR),
                            workspace_dev=_FakeTensor(), stream=0)
    assert e.value.code == 1
    g3n = C.Grid(3, 3, 10, 10, 10, 5.0, 5.0, 5.0, None)
    with pytest.raises(C.ChertError) as e:  # 3D needs a class map
        C.chert_trace_field(d3, _FakeTensor(), 3, g3n, 0, [0], o, workspace_dev=_FakeTensor(),
                            stream=0)
    assert e.value.code == 2
    o3 = C.trace_opts(C.OUT_TAU_R | C.OUT_TAU_I)
    assert C.chert_trace_workspace_bytes(d3, 3, g3, 1, o3) > 0
    g3b = C.Grid(3, 5, 10, 10, 10, 5.0, 5.0, 5.0, 1234)
    assert C.chert_trace_workspace_bytes(d3, 3, g3b, 1, o3) == 0  # radius above 4
    # 3D: tiles (tile_x x tile_x x tile_z, per round or persistent) or the
    # node frontier
    for launch in (C.LAUNCH_FRONTIER, C.LAUNCH_PERSISTENT):
        of3 = C.trace_opts(C.OUT_TAU_R | C.OUT_TAU_I, launch=launch)
        assert C.chert_trace_workspace_bytes(d3, 3, g3, 1, of3) > 0
    for bad in (dict(tile_x=2, tile_z=8),
                dict(tile_x=16, tile_z=8), dict(push_group=3)):
        ob = C.trace_opts(C.OUT_TAU_R | C.OUT_TAU_I, **bad)
        assert C.chert_trace_workspace_bytes(d3, 3, g3, 1, ob) == 0, bad
    assert C.chert_trace_workspace_bytes(d, 3, g, 1, o) > 0


def test_frontier_launch_validation_and_sizes():
    """2D batches on the node frontier: same argument checks as the tiles,
    workspace sized by node counts (lists, stamps) and the weight tables;
    bad launch values and bucket widths are refused."""
    d = C.cache_desc()
    g = C.Grid(2, 3, 10, 10, 1, 5.0, 5.0, 0.0, 1234)
    of = C.trace_opts(launch=C.LAUNCH_FRONTIER)
    nf = C.chert_trace_workspace_bytes(d, 3, g, 1, of)
    nt = C.chert_trace_workspace_bytes(d, 3, g, 1, C.trace_opts())
    assert nf > 0 and nt > 0 and nf != nt
    ob = C.trace_opts(launch=C.LAUNCH_FRONTIER, bucket_width=16.0)
    assert C.chert_trace_workspace_bytes(d, 3, g, 1, ob) > nf  # far piles
    assert C.chert_trace_workspace_bytes(d, 3, g, 2, of) > nf
    assert C.chert_trace_workspace_bytes(
        d, 3, g, 1, C.trace_opts(launch=C.LAUNCH_FRONTIER, bucket_width=-1.0)) == 0
    assert C.chert_trace_workspace_bytes(d, 3, g, 1, C.trace_opts(launch=7)) == 0
    gr = C.Grid(2, 9, 10, 10, 1, 5.0, 5.0, 0.0, 1234)
    assert C.chert_trace_workspace_bytes(d, 3, gr, 1, of) == 0  # radius above 8
    gp = C.Grid(2, 3, 10, 10, 1, 5.0, 5.0, 0.0, None)  # per node: 100 cache rows
    assert C.chert_trace_workspace_bytes(d, 100, gp, 1, of) > 0
    assert C.chert_trace_workspace_bytes(d, 99, gp, 1, of) == 0
    for bad in ([100], [-1]):
        with pytest.raises(C.ChertError) as e:
            C.chert_trace_field(d, _FakeTensor(), 3, g, 0, bad, of, workspace_dev=_FakeTensor(),
                                stream=0)
        assert e.value.code == 1
    with pytest.raises(C.ChertError) as e:  # TSTAR without its inputs
        C.chert_trace_field(d, _FakeTensor(), 3, g, 0, [0], C.trace_opts(
            C.OUT_TSTAR, launch=C.LAUNCH_FRONTIER), workspace_dev=_FakeTensor(), stream=0)
    assert e.value.code == 1
    dsub = C.cache_desc(subset=C.star_subset(2, 5.0, 5.0))
    gr5 = C.Grid(2, 5, 10, 10, 1, 5.0, 5.0, 0.0, 1234)  # the subset lacks radius-5 bins
    with pytest.raises(C.ChertError) as e:
        C.chert_trace_field(dsub, _Ptr(0x1000), 3, gr5, 0, [0], C.trace_opts(
            C.OUT_TAU_R, launch=C.LAUNCH_FRONTIER), tau_r=_Ptr(0x2000),
            workspace_dev=_Ptr(0x3000, n=1 << 40), stream=0)
    assert e.value.code == 1


class _Ptr(_FakeTensor):
    """A fake device pointer value (never dereferenced)."""
    def __init__(self, addr, n=0, shape=(0,)):
        super().__init__(n)
        self.addr = addr
        self.shape = shape

    def data_ptr(self):
        return self.addr


def test_surrogate_layout_and_validation():
    lay = C.chert_surrogate_layout_of()
    assert (lay.n_params, lay.n_in, lay.n_hidden, lay.n_out) == (35716, 16, 128, 4)
    for off in (lay.norm_offset, lay.params_offset, lay.adam_m_offset, lay.adam_v_offset,
                lay.total_bytes):
        assert off % 256 == 0
    assert lay.adam_m_offset >= lay.params_offset + 4 * lay.n_params
    assert lay.adam_v_offset >= lay.adam_m_offset + 4 * lay.n_params
    assert lay.total_bytes > lay.adam_v_offset + 4 * lay.n_params
    ok = _Ptr(0x10000)
    for blob in (_FakeTensor(), _Ptr(0x10010)):  # null, unaligned
        with pytest.raises(C.ChertError) as e:
            C.chert_surrogate_init(blob, ok, stream=0)
        assert e.value.code == 1
    with pytest.raises(C.ChertError):  # null parameters
        C.chert_surrogate_init(ok, _FakeTensor(), stream=0)
    with pytest.raises(C.ChertError):  # step 0
        C.chert_surrogate_adam(ok, ok, 0, 1e-3, stream=0)
    with pytest.raises(C.ChertError):  # negative learning rate
        C.chert_surrogate_adam(ok, ok, 1, -1.0, stream=0)
    assert C.chert_surrogate_grad_workspace_bytes(0) == 0
    assert C.chert_surrogate_grad_workspace_bytes(33) == 2 * C.chert_surrogate_grad_workspace_bytes(32)
    idx = _Ptr(0x20000, n=64)
    with pytest.raises(C.ChertError):  # workspace too small
        C.chert_surrogate_grad(ok, ok, ok, idx, ok, None, _Ptr(0x30000, n=16), stream=0)
    d = C.cache_desc(subset=C.star_subset(5, 10.0, 10.0), modes=(1,))
    need = C.chert_build_cache_surrogate_workspace_bytes(d, 100)
    assert need >= 100 * 40 // 2 * 8
    with pytest.raises(C.ChertError):  # workspace too small
        C.chert_build_cache_surrogate(d, ok, 100, ok, ok, _Ptr(0x40000, n=need - 1), stream=0)
    with pytest.raises(C.ChertError):  # unaligned blob
        C.chert_build_cache_surrogate(d, ok, 100, _Ptr(0x10010), ok, _Ptr(0x40000, n=need),
                                      stream=0)
    with pytest.raises(C.ChertError):  # negative residual tolerance
        C.chert_build_cache_surrogate(d, ok, 100, ok, ok, _Ptr(0x40000, n=need),
                                      resid_tol=-1.0, stream=0)


def test_class_pair_table_index_limit():
    """The tile kernels index one field's class-pair weight table
    [K][K][|O|] in 32 bits, so K * K * |O| must stay below 2^31: at radius 5
    (|O| = 80) K = 5181 is accepted and K = 5182 rejected before any device
    work."""
    import torch
    cid = torch.zeros(16, dtype=torch.int32)  # never read: validation fails first
    grid = C.make_grid(4, 4, 10.0, 10.0, 5, cid)
    opts = C.trace_opts(C.OUT_TAU_R)
    d = C.cache_desc(n_dirs=360, modes=(0,))
    assert 5181 * 5181 * 80 < 2 ** 31 <= 5182 * 5182 * 80
    assert C.chert_trace_workspace_bytes(d, 5181, grid, 1, opts) > 0
    assert C.chert_trace_workspace_bytes(d, 5182, grid, 1, opts) == 0
    b = C.Batch()
    t = torch.zeros(16, dtype=torch.float64)
    b.add(d, t, 5182, grid, 0, [0], tau_r=t)
    with pytest.raises(C.ChertError) as e:
        C.chert_trace_batch(b, opts, None, stream=0)
    assert e.value.code == 2


def test_cache_desc_solver_fields_validated():
    """resid_tol must be finite and >= 0, max_iter >= 0 and sampling one of
    the two kinds; each violation is INVALID_ARG before any device work."""
    C.chert_cache_layout_of(C.cache_desc(resid_tol=1e-12, max_iter=3), 2)
    for kw in ({"resid_tol": -1e-9}, {"resid_tol": float("nan")}, {"resid_tol": float("inf")},
               {"max_iter": -1}):
        with pytest.raises(C.ChertError) as e:
            C.chert_cache_layout_of(C.cache_desc(**kw), 2)
        assert e.value.code == 1
    d = C.cache_desc()
    d.sampling = 7
    with pytest.raises(C.ChertError) as e:
        C.chert_cache_layout_of(d, 2)
    assert e.value.code == 1
    # slowness-sampled caches are 2D and hold every column
    C.chert_cache_layout_of(C.cache_desc(sampling=C.SAMPLE_SLOWNESS), 2)
    for bad in (C.cache_desc(sampling=1, dim=3, n_dirs=300),
                C.cache_desc(sampling=1, subset=C.star_subset(2, 10.0, 10.0))):
        with pytest.raises(C.ChertError) as e:
            C.chert_cache_layout_of(bad, 2)
        assert e.value.code == 2


def test_abi_struct_layouts_match_header(tmp_path):
    """Every structure the binding marshals has the size and field offsets
    that a C compiler gives the declarations in include/chert.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"chert_class": C.ChertClass, "chert_cache_desc": C.CacheDesc,
               "chert_cache_layout": C.CacheLayout, "chert_cache_stats": C.CacheStats,
               "chert_grid": C.Grid, "chert_trace_job": C.TraceJob,
               "chert_trace_stats": C.TraceStats, "chert_trace_opts": C.TraceOpts,
               "chert_cell_grid": C.CellGrid, "chert_block_grid": C.BlockGrid}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "chert.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    got = {(out[i], out[i + 1]): int(out[i + 2]) for i in range(0, len(out), 3)}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_cell_network_validation():
    """Host checks of the cell-network trace (no device call): workspace
    bytes for valid networks, 0 for bad ones; the workspace grows with the
    sources."""
    d = C.cache_desc(n_dirs=360, modes=(0, 1))
    o = C.trace_opts(C.OUT_ALL)
    fake = 0x1000  # never dereferenced by the size query

    def g(ncx=10, ncz=6, cn=5, hx=10.0, hz=10.0, cls=fake):
        return C.CellGrid(ncx, ncz, cn, 0, hx, hz, cls)

    b1 = C.chert_trace_cells_workspace_bytes(d, 3, g(), 1, o)
    b4 = C.chert_trace_cells_workspace_bytes(d, 3, g(), 4, o)
    assert 0 < b1 < b4
    assert C.chert_trace_cells_workspace_bytes(d, 3, g(cn=16), 1, o) > 0
    for bad in (g(cn=0), g(cn=17), g(ncx=0), g(hx=0.0), g(hz=float("nan")), g(cls=None)):
        assert C.chert_trace_cells_workspace_bytes(d, 3, bad, 1, o) == 0
    assert C.chert_trace_cells_workspace_bytes(C.cache_desc(dim=3, n_dirs=500), 3, g(), 1, o) == 0
    assert C.chert_trace_cells_workspace_bytes(d, 3, g(), 1, C.trace_opts(C.OUT_TSTAR)) == 0
    assert C.chert_trace_cells_workspace_bytes(
        C.cache_desc(n_dirs=72, modes=(2,), sampling=C.SAMPLE_SLOWNESS), 3, g(), 1, o) > 0


def test_block_network_validation():
    """Host checks of the block-network trace (no device call): workspace
    bytes for valid 3D networks with a 3D cache, 0 for a 2D cache, block_n
    outside 1..3, empty or unspaced grids and a missing class map."""
    d = C.cache_desc(n_dirs=500, modes=(0, 1), dim=3)
    o = C.trace_opts(C.OUT_ALL)
    fake = 0x1000  # never dereferenced by the size query

    def g(ncx=6, ncy=5, ncz=4, cn=3, hx=10.0, hy=10.0, hz=10.0, cls=fake):
        return C.BlockGrid(ncx, ncy, ncz, cn, hx, hy, hz, cls)

    b1 = C.chert_trace_blocks_workspace_bytes(d, 3, g(), 1, o)
    b4 = C.chert_trace_blocks_workspace_bytes(d, 3, g(), 4, o)
    assert 0 < b1 < b4
    for cn in (1, 2):
        assert C.chert_trace_blocks_workspace_bytes(d, 3, g(cn=cn), 1, o) > 0
    for bad in (g(cn=0), g(cn=4), g(ncy=0), g(hy=0.0), g(hz=float("inf")), g(cls=None)):
        assert C.chert_trace_blocks_workspace_bytes(d, 3, bad, 1, o) == 0
    assert C.chert_trace_blocks_workspace_bytes(C.cache_desc(n_dirs=360), 3, g(), 1, o) == 0
