"""The Python binding validates tensors before it calls into the library:
dtype, contiguity, byte size and device, for every launch kind.  A wrong
buffer never reaches a kernel (CPU-only: every call here is rejected)."""
import pytest

torch = pytest.importorskip("torch")

from paper_2208_11617_amd import binding as smap  # noqa: E402


@pytest.fixture
def no_library(monkeypatch):
    """Fail the test if any call reaches the C library."""
    def boom():
        raise AssertionError("the library was called")
    monkeypatch.setattr(smap, "lib", boom)


def _err(fn, *a, **k):
    with pytest.raises(smap.SimplexMapError) as e:
        fn(*a, **k)
    assert e.value.status == smap.EINVAL
    return str(e.value)


def test_launch_checks(no_library):
    n = 40
    u8 = torch.zeros((n + 1) ** 2, dtype=torch.uint8)
    for launch in (smap.map_launch, smap.bb_launch):
        assert "dtype" in _err(launch, 2, n, "ca2", u8.to(torch.int32), u8)
        assert "dtype" in _err(launch, 2, n, "ca2", u8, u8.to(torch.float64))
        assert "contiguous" in _err(launch, 2, n, "ca2", u8.view(n + 1, n + 1).t(), u8)
        assert "bytes" in _err(launch, 2, n, "ca2", u8[:-1], u8.clone())
        assert "device" in _err(launch, 2, n, "ca2", u8, u8.clone())
        w = torch.zeros((n + 1) ** 2, dtype=torch.int32)
        assert "dtype" in _err(launch, 2, n, "accum", u8, w)
        assert "bytes" in _err(launch, 2, n, "accum", w, w[:10])
        assert "bytes" in _err(launch, 2, n, "hash", None, w[:-1])
        assert "device" in _err(launch, 2, n, "hits", None, w)
        pts = torch.zeros((n + 1, 3), dtype=torch.float32)
        assert "bytes" in _err(launch, 2, n, "edm", pts[:-1], w)
        assert "dtype" in _err(launch, 2, n, "edm", pts.to(torch.float64), w)
        assert "device" in _err(launch, 2, n, "edm", pts, w)
        assert "torch tensor" in _err(launch, 2, n, "ca2", bytearray(10), u8)


def test_3d_and_4d_sizes(no_library):
    u8 = torch.zeros(11 ** 3, dtype=torch.uint8)
    assert "bytes" in _err(smap.map_launch, 3, 10, "ca3", u8, u8[:-1])
    w = torch.zeros(9 ** 4, dtype=torch.int32)
    assert "bytes" in _err(smap.map_launch, 4, 8, "hash", None, w[:-1])
    assert "device" in _err(smap.map_launch, 4, 8, "hash", None, w)


def test_steps_graph_tune_batch_serve_checks(no_library):
    n = 30
    u8 = torch.zeros((n + 1) ** 2, dtype=torch.uint8)
    assert "bytes" in _err(smap.map_launch_steps, 2, n, "ca2", 4, u8[:5], u8)
    assert "device" in _err(smap.bb_launch_steps, 2, n, "ca2", 4, u8, u8.clone())
    assert "device" in _err(smap.autotune, 2, n, "ca2", u8, u8.clone())
    assert "device" in _err(smap.Graph, 2, n, "ca2", u8, u8.clone(), steps=2)
    assert "bytes" in _err(smap.batch_launch, [(2, "ca2", n, u8, u8[:3])])
    assert "dtype" in _err(smap.queue_launch, [(2, "ca2", n, u8.to(torch.int32), u8)])
    assert "device" in _err(smap.QueueGraph, [(2, "ca2", n, u8, u8.clone())])
    arena = torch.zeros(1 << 12, dtype=torch.uint8)
    assert "device" in _err(smap.serve_run, [(2, "ca2", n, u8, 0.0)], arena, smap.SERVE_BATCHED)
    assert "contiguous" in _err(smap.serve_run, [], arena.view(64, 64).t(), smap.SERVE_BATCHED)
    assert "bytes" in _err(smap.serve_run, [(2, "ca2", n, u8[:7], 0.0)],
                           torch.zeros(1, dtype=torch.uint8), smap.SERVE_BATCHED)
