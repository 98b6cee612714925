"""The constrained Brownian-dynamics solve (hq_constrained_solve, Eqs. 1.5 and
1.6): conjugate gradients on Q~ D Q~^T with the GPU sweeps and a dense test
mobility D, against the dense LAPACK solution in the hierarchical oracle's
basis (oracle.bd).

* FP64, three bodies, 1 to 40 right-hand sides (narrow and wide sweeps), both
  layouts: V and g <= 1e-9 relative, with CG run to a 1e-12 residual.
* FP32, 1 to 8 right-hand sides, both layouts (the 16-byte and the
  one-element CG vector passes): <= 1e-4 relative.
* A D that is not positive definite is reported as HQ_E_INVALID; a failing
  callback's exception reaches the caller.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hq():
    import paper_1708_08427_amd as hq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return hq


def to_layout(a, layout):
    if layout == "rows":
        return np.ascontiguousarray(a)
    return np.ascontiguousarray(a.reshape(a.shape[0] // 3, 3, a.shape[1]).transpose(0, 2, 1))


def from_layout(t, layout):
    if layout == "rows":
        return t
    return np.ascontiguousarray(t.transpose(0, 2, 1).reshape(3 * t.shape[0], t.shape[1]))


def problem(seed, sizes, R):
    w = W.small_batch(seed, sizes)
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((3 * w.N, 3 * w.N))
    D = np.eye(3 * w.N) + 0.3 * (M @ M.T) / np.linalg.norm(M, 2) ** 2
    F = rng.standard_normal((6 * w.m, R))
    return w, D, F


def dense_dapply(Dd, layout):
    def f(x, y):
        if layout == "rows":
            torch.matmul(Dd, x, out=y)
        else:
            N, R = x.shape[0], x.shape[1]
            xr = x.permute(0, 2, 1).reshape(3 * N, R)
            y.copy_(torch.matmul(Dd, xr).reshape(N, 3, R).permute(0, 2, 1))
    return f


@pytest.mark.parametrize("R,layout", [(1, "rows"), (4, "triples"), (32, "rows"), (40, "triples")])
def test_constrained_solve_fp64(hq, R, layout):
    w, D, F = problem(51, [9, 40, 130], R)
    V_o, g_o = bd.constrained_solve(w.pos, w.offsets, D, F)
    print(f"[gpu] krylov FP64 R={R} {layout} N={w.N}", flush=True)
    h = hq.build(torch.from_numpy(w.pos).cuda(), w.offsets)
    Dd = torch.from_numpy(D).cuda()
    V, g, info = hq.constrained_solve(h, dense_dapply(Dd, layout), torch.from_numpy(to_layout(F, layout)).cuda(),
                                      layout=layout, rtol=1e-12, max_iter=200)
    V = from_layout(V.cpu().numpy(), layout)
    g = from_layout(g.cpu().numpy(), layout)
    assert info["max_rel_residual"] <= 1e-12 and info["iters"] < 200
    assert np.abs(V - V_o).max() <= 1e-9 * np.abs(V_o).max()
    assert np.abs(g - g_o).max() <= 1e-9 * np.abs(g_o).max()
    assert h.query()["device_flags"] == 0


# 855 constraint rows: rows x R is a whole number of 16-byte units for R = 8
# and R = 4 (the 16-byte CG passes), not for R = 1 and R = 6 (the one-element
# passes)
@pytest.mark.parametrize("R,layout", [(8, "rows"), (1, "rows"), (6, "triples"), (4, "triples")])
def test_constrained_solve_fp32(hq, R, layout):
    w, D, F = problem(52, [20, 70, 201], R)
    assert w.rows == 855
    V_o, g_o = bd.constrained_solve(w.pos, w.offsets, D, F)
    h = hq.build(torch.from_numpy(w.pos).cuda(), w.offsets)
    Dd = torch.from_numpy(D).float().cuda()
    V, g, info = hq.constrained_solve(h, dense_dapply(Dd, layout), torch.from_numpy(to_layout(F, layout)).float().cuda(),
                                      layout=layout, rtol=1e-6)
    V = from_layout(V.cpu().numpy(), layout)
    g = from_layout(g.cpu().numpy(), layout)
    assert info["max_rel_residual"] <= 1e-6
    assert np.abs(V - V_o).max() <= 1e-4 * np.abs(V_o).max()
    assert np.abs(g - g_o).max() <= 1e-4 * np.abs(g_o).max()


def test_constrained_solve_errors(hq):
    w, D, F = problem(53, [10, 12], 2)
    h = hq.build(torch.from_numpy(w.pos).cuda(), w.offsets)
    Fd = torch.from_numpy(F).cuda()
    # negative definite D: p^T A p < 0 on the first iteration
    Dn = -torch.from_numpy(D).cuda()
    with pytest.raises(hq.HQError):
        hq.constrained_solve(h, dense_dapply(Dn, "rows"), Fd)

    def boom(x, y):
        raise RuntimeError("mobility failed")
    with pytest.raises(RuntimeError, match="mobility failed"):
        hq.constrained_solve(h, boom, Fd)
    with pytest.raises(ValueError):
        hq.constrained_solve(h, dense_dapply(torch.from_numpy(D).cuda(), "rows"), Fd[:5])
    assert h.query()["device_flags"] == 0


def test_constrained_solve_check_interval(hq):
    """The CG scalars live on the device and converged columns take zero
    steps, so the host's check interval changes neither the iterations each
    column takes nor the solution (beyond the order of the dot products'
    atomic partial sums)."""
    w, D, F = problem(54, [15, 60, 150], 5)
    # columns of very different size converge at different iterations
    F = F * np.array([1.0, 1e3, 1e-3, 1.0, 10.0])
    h = hq.build(torch.from_numpy(w.pos).cuda(), w.offsets)
    Dd = torch.from_numpy(D).cuda()
    Fd = torch.from_numpy(F).cuda()
    res = [hq.constrained_solve(h, dense_dapply(Dd, "rows"), Fd, rtol=1e-10, check_every=c) for c in (1, 3, 16)]
    V0, g0, i0 = res[0]
    for V, g, info in res[1:]:
        assert info["iters"] == i0["iters"]
        assert float((V - V0).norm() / V0.norm()) <= 1e-12
        assert float((g - g0).norm() / g0.norm()) <= 1e-12
    V_o, g_o = bd.constrained_solve(w.pos, w.offsets, D, F)
    assert np.abs(V0.cpu().numpy() - V_o).max() <= 1e-8 * np.abs(V_o).max()
    with pytest.raises(ValueError):
        hq.constrained_solve(h, dense_dapply(Dd, "rows"), Fd, check_every=0)
