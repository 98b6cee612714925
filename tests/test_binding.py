"""The Python binding rejects ill-formed tensors on the host, before anything
reaches the library (which would hand raw pointers to kernels reading N x 3
or m x 9 doubles).  CPU only: the library loader is replaced by one that
fails, and the device check by one that accepts host tensors, so each case
shows the check that stops it."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


@pytest.fixture
def hq(monkeypatch):
    import paper_1708_08427_amd as hq
    from paper_1708_08427_amd import _lib

    def no_library():
        raise AssertionError("the library was reached")

    monkeypatch.setattr(_lib, "load", no_library)
    return hq


def handle(hq):
    # bodies of 4 and 6 beads: N = 10, m = 2, rows = 18
    h = hq.Handle(None, np.array([0, 4, 10]))
    h._raw = object()  # never dereferenced: every case fails before the call
    return h


def test_host_tensors_rejected(hq):
    h = handle(hq)
    pos = torch.zeros((10, 3), dtype=torch.float64)
    with pytest.raises(TypeError):
        h.rebuild(pos)
    with pytest.raises(TypeError):
        h.rigid_update(pos, torch.zeros(18, dtype=torch.float64), torch.zeros(6, dtype=torch.float64))
    with pytest.raises(TypeError):
        h.apply(torch.zeros((30, 1)))


def test_shapes_and_dtypes_rejected(hq, monkeypatch):
    import paper_1708_08427_amd as pkg

    def host_ok(t, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError(name)
        if not t.is_contiguous():
            raise ValueError(name)

    monkeypatch.setattr(pkg, "_check_dev", host_ok)
    h = handle(hq)
    f64 = torch.float64
    good_pos = torch.zeros((10, 3), dtype=f64)
    good_rot = torch.zeros((2, 9), dtype=f64)
    good_tr = torch.zeros((2, 3), dtype=f64)
    # positions: float64, (N, 3)
    with pytest.raises(TypeError):
        h.rebuild(torch.zeros((10, 3), dtype=torch.float32))
    with pytest.raises(ValueError):
        h.rebuild(torch.zeros((9, 3), dtype=f64))
    with pytest.raises(ValueError):
        h.rebuild(torch.zeros((30,), dtype=f64))
    with pytest.raises(ValueError):
        h.rebuild(torch.zeros((3, 10), dtype=f64).t())  # not contiguous
    # rigid motion tables: float64, 9m and 3m values
    with pytest.raises(TypeError):
        h.rigid_update(torch.zeros((10, 3), dtype=torch.float32), good_rot, good_tr)
    with pytest.raises(ValueError):
        h.rigid_update(good_pos, torch.zeros((1, 9), dtype=f64), good_tr)
    with pytest.raises(TypeError):
        h.rigid_update(good_pos, good_rot.float(), good_tr)
    with pytest.raises(ValueError):
        h.rigid_update(good_pos, good_rot, torch.zeros(5, dtype=f64))
    with pytest.raises(TypeError):
        h.rigid_update(good_pos, good_rot, good_tr.float())
    # rotated products: the rotation table and the out / work tensors
    v = torch.zeros((30, 2), dtype=f64)
    with pytest.raises(ValueError):
        h.apply_rotated(torch.zeros((3, 9), dtype=f64), v)
    with pytest.raises(ValueError):
        h.apply_rotated(good_rot, v, out=torch.zeros((11, 2), dtype=f64))
    with pytest.raises(ValueError):
        h.apply_rotated(good_rot, v, work=torch.zeros((30, 3), dtype=f64))
    # full Q: out and root shapes
    with pytest.raises(ValueError):
        h.apply_full(v, out=torch.zeros((12, 1), dtype=f64))
    with pytest.raises(ValueError):
        h.apply_full(v, root=torch.zeros((12, 3), dtype=f64))
    # apply: rows and dtypes
    with pytest.raises(ValueError):
        h.apply(torch.zeros((29, 2), dtype=f64))
    with pytest.raises(TypeError):
        h.apply(v, out=torch.zeros((18, 2), dtype=torch.float32))
