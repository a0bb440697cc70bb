"""The allocation-free cache build (chert_build_cache_noalloc) against the
workspace build (chert_build_cache) through the C ABI: the same kernels on
the same inputs, so the blobs must be identical byte for byte -- on two
calls in a row, the second with a smaller input, and in 3D; sizes beyond
the library's scratch array are refused before any device work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import chert_gpu
    return chert_gpu


def _C():
    import paper_2609_26108_amd as C
    return C


def both(G, classes, desc):
    """(workspace build, allocation-free build) of the same inputs: the
    header bytes and every field and status slot of the built modes (the
    bytes the build writes; other mode slots and the layout's padding are
    left as they were), as host arrays."""
    C = _C()
    K = classes.shape[0]
    ref = G.build_cache(classes, desc)
    lay = C.chert_cache_layout_of(desc, K)
    out = torch.full((lay.total_bytes,), 0x5A, dtype=torch.uint8, device=G.DEV)
    C.chert_build_cache_noalloc(desc, classes, K, out)
    torch.cuda.synchronize()
    modes = [m for m in range(3) if desc.mode_mask & (1 << m)]

    def written(blob):
        f, s = C.cache_views(blob, desc, K)
        return (blob[:256].cpu().numpy(), f[:, modes].cpu().numpy().view(np.uint64),
                s[modes].cpu().numpy())
    return written(ref), written(out)


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_noalloc_equals_workspace_build_twice_then_smaller(G):
    C = _C()
    assert C.chert_build_cache_noalloc_max_bytes() == 16 << 20
    big = W.config2()
    classes = G.classes_from_layers(big.layers)
    desc = C.cache_desc(n_dirs=360, modes=(0, 1, 2))
    ref, out = both(G, classes, desc)
    assert same(ref, out)
    # second call: fewer classes, fewer modes, a shorter sweep
    small = W.small_layered(n_layers=2, seed=9)
    classes2 = G.classes_from_layers(small.layers)
    desc2 = C.cache_desc(n_dirs=360, modes=(1,), n_sweep=720)
    ref2, out2 = both(G, classes2, desc2)
    assert same(ref2, out2)
    f2, s2 = out2[1].view(np.float64), out2[2]
    assert np.all(s2 == 0) and np.all(np.isfinite(f2[0]))


def test_noalloc_equals_workspace_build_3d(G):
    C = _C()
    m = W.config5(nx=8, ny=8, nz=8)
    classes = G.classes_from_layers(m.layers)
    desc = C.cache_desc(dim=3, n_dirs=2000, modes=(0, 1), n_sweep=720)
    ref, out = both(G, classes, desc)
    assert same(ref, out)


def test_noalloc_refuses_sweep_tables_beyond_its_array(G):
    C = _C()
    rows = W.surrogate_training_rows(255, seed=3)
    K = rows.shape[0]
    classes = torch.empty((K, 13), dtype=torch.float64, device=G.DEV)
    C.chert_classes_from_thomsen(torch.from_numpy(rows).to(G.DEV), classes)
    desc = C.cache_desc(n_dirs=360, modes=(0, 1), n_sweep=4096)
    assert C.chert_build_cache_workspace_bytes(desc, K) > C.chert_build_cache_noalloc_max_bytes()
    lay = C.chert_cache_layout_of(desc, K)
    out = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=G.DEV)
    with pytest.raises(C.ChertError) as e:
        C.chert_build_cache_noalloc(desc, classes, K, out)
    assert e.value.code == 5
    torch.cuda.synchronize()
    assert int(out.sum().item()) == 0
