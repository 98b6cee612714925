"""Checks that pin the FP64 oracle to facts fixed outside the oracle itself.

Each check returns the worst error it found; the callers compare it with a
bound.  They are shared by the oracle tests and the planted-mistake tests.
"""
from __future__ import annotations

import numpy as np

from oracle import dense


def cross(r):
    return dense.cross_matrix(r)


# ---------------------------------------------------------------------------
# tree: the literal nested-box bisection of Section 2.1 (z, then y, then x)
# ---------------------------------------------------------------------------


def bisection_tree(pos):
    """Internal nodes of the literal recursive midpoint bisection on FP64
    coordinates: a set of (all, lower-half, upper-half) frozensets of bead ids.
    Halves with no bead are pruned; a box whose beads all fall in one half is
    replaced by that half."""
    pos = np.asarray(pos, dtype=np.float64)
    lo = pos.min(axis=0)
    h = float((pos.max(axis=0) - lo).max())
    out = set()
    axes = (2, 1, 0)
    stack = [(tuple(range(len(pos))), lo.copy(), np.array([h, h, h]), 0)]
    while stack:
        ids, blo, bsz, step = stack.pop()
        if len(ids) <= 1:
            continue
        if step > 3 * 40:
            raise ValueError("beads too close for the literal bisection")
        ax = axes[step % 3]
        mid = blo[ax] + bsz[ax] / 2.0
        low = tuple(i for i in ids if pos[i, ax] < mid)
        up = tuple(i for i in ids if pos[i, ax] >= mid)
        nsz = bsz.copy()
        nsz[ax] = bsz[ax] / 2.0
        ulo = blo.copy()
        ulo[ax] = mid
        if low and up:
            out.add((frozenset(ids), frozenset(low), frozenset(up)))
        if low:
            stack.append((low, blo.copy(), nsz, step + 1))
        if up:
            stack.append((up, ulo, nsz, step + 1))
    return out


def oracle_tree(body):
    perm = body.perm()
    out = set()
    for nd in body.nodes():
        allb = frozenset(int(perm[s]) for s in range(nd.first, nd.last + 1))
        if nd.x >= 0:
            xn = body.node(nd.x)
            lowb = frozenset(int(perm[s]) for s in range(xn.first, xn.last + 1))
        else:
            lowb = frozenset([int(perm[-(nd.x + 1)])])
        out.add((allb, lowb, allb - lowb))
    return out


# ---------------------------------------------------------------------------
# per-node checks
# ---------------------------------------------------------------------------


def infoset_identity_error(body, rng):
    """Definition 4.1 with Eq. 3.3: for every internal node p and any f,
    sum_{k in p} f_k = sqrt(n_p) M_p(1:3) and
    sum_{k in p} (r_k - c_p) x f_k = T22_p M_p(4:6), with c_p the mean of p's
    beads.  Returns the worst relative error."""
    f = rng.standard_normal(3 * body.n)
    _, M = body.up_infosets(f)
    perm = body.perm()
    F = f.reshape(-1, 3)
    worst = 0.0
    for i, nd in enumerate(body.nodes()):
        ids = perm[nd.first:nd.last + 1]
        r = body.pos[ids]
        c = r.mean(axis=0)
        force = F[ids].sum(axis=0)
        torque = np.cross(r - c, F[ids]).sum(axis=0)
        e1 = np.linalg.norm(force - np.sqrt(nd.n) * M[i, 0:3])
        e2 = np.linalg.norm(torque - nd.T22 @ M[i, 3:6])
        scale = np.linalg.norm(F[ids]) * (1.0 + np.abs(r - c).max())
        worst = max(worst, (e1 + e2) / scale)
    return worst


def lapack_convention_error(body):
    """At every node, K = [T22_x | T22_y | sqrt(n_x n_y / n) [c_x - c_y]x]
    (leaf blocks absent) must factor as LAPACK's Householder QR of K^T:
    T22 = R(1:3,1:3)^T and G = Q^T (numpy.linalg.qr).  Returns the worst
    relative deviation, skipping nodes where the factor is not determined
    (a zero tail in some column, or an ill-conditioned K)."""
    nodes = body.nodes()
    perm = body.perm()
    worst = 0.0
    for nd in nodes:
        blocks = []
        if nd.x >= 0:
            xn = nodes[nd.x]
            blocks.append(xn.T22)
            cx, nx = xn.c, xn.n
        else:
            cx, nx = body.pos[perm[-(nd.x + 1)]] - body.pos.min(axis=0), 1
        if nd.y >= 0:
            yn = nodes[nd.y]
            blocks.append(yn.T22)
            cy, ny = yn.c, yn.n
        else:
            cy, ny = body.pos[perm[-(nd.y + 1)]] - body.pos.min(axis=0), 1
        n = nx + ny
        blocks.append(np.sqrt(nx * ny / n) * cross(cx - cy))
        K = np.hstack(blocks)
        if nd.k == 3 or nd.kappa > 1e6:
            continue
        Qn, Rn = np.linalg.qr(K.T, mode="complete")
        scale = np.abs(K).max()
        worst = max(worst, np.abs(nd.T22 - Rn[:3, :3].T).max() / scale)
        worst = max(worst, np.abs(nd.G - Qn.T).max())
    return worst


def factor_error(body):
    """K = [T22 | 0] G and G G^T = I and T22 lower triangular, per node."""
    nodes = body.nodes()
    perm = body.perm()
    lo = body.pos.min(axis=0)
    worst = 0.0
    for nd in nodes:
        blocks = []
        if nd.x >= 0:
            blocks.append(nodes[nd.x].T22)
            cx, nx = nodes[nd.x].c, nodes[nd.x].n
        else:
            cx, nx = body.pos[perm[-(nd.x + 1)]] - lo, 1
        if nd.y >= 0:
            blocks.append(nodes[nd.y].T22)
            cy, ny = nodes[nd.y].c, nodes[nd.y].n
        else:
            cy, ny = body.pos[perm[-(nd.y + 1)]] - lo, 1
        n = nx + ny
        blocks.append(np.sqrt(nx * ny / n) * cross(cx - cy))
        K = np.hstack(blocks)
        T0 = np.zeros((3, nd.k))
        T0[:, :3] = nd.T22
        worst = max(worst, np.abs(T0 @ nd.G - K).max() / max(np.abs(K).max(), 1e-300))
        worst = max(worst, np.abs(nd.G @ nd.G.T - np.eye(nd.k)).max())
        worst = max(worst, np.abs(np.triu(nd.T22, 1)).max())
    return worst


# ---------------------------------------------------------------------------
# whole-body checks
# ---------------------------------------------------------------------------


def projector_error(body, rng, nrhs=3):
    """Q~^T (Q~ f) = P f with P from LAPACK's QR of Z^T."""
    f = rng.standard_normal((3 * body.n, nrhs))
    got = body.apply(body.apply(f), transpose=True)
    want = dense.project(body.pos, f)
    return np.abs(got - want).max() / np.abs(f).max()


def roundtrip_error(body, rng, nrhs=3):
    """Q~ (Q~^T w) = w (orthonormal rows)."""
    w = rng.standard_normal((body.rows, nrhs))
    return np.abs(body.apply(body.apply(w, transpose=True)) - w).max()


def leak_error(body, rng, nrhs=3):
    """Z Q~^T w = 0."""
    w = rng.standard_normal((body.rows, nrhs))
    return float(dense.leak(body.pos, body.apply(w, transpose=True)).max())


def norm_error(body, rng):
    """The full Q = [Q_Z; Q~] is orthogonal: ||M_root||^2 + ||eps||^2 = ||f||^2."""
    f = rng.standard_normal((3 * body.n, 1))
    root = np.zeros((6, 1))
    eps, root = body.apply(f, root=root)
    return abs(np.sum(root ** 2) + np.sum(eps ** 2) - np.sum(f ** 2)) / np.sum(f ** 2)


def full_q_inverse_error(body, rng, nrhs=3):
    """The full Q = [Q_Z; Q~] (Algorithms 2 and 3 with the root kept) is
    orthogonal: Q^T (Q f) = f, and Q (Q^T [r; w]) = [r; w] for any root
    Velocity-set r."""
    f = rng.standard_normal((3 * body.n, nrhs))
    eps, root = body.apply(f, root=np.zeros((6, nrhs)))
    back, _ = body.apply(eps, transpose=True, root=root)
    e1 = np.abs(back - f).max() / np.abs(f).max()
    r = rng.standard_normal((6, nrhs))
    w = rng.standard_normal((body.rows, nrhs))
    g, _ = body.apply(w, transpose=True, root=r)
    w2, r2 = body.apply(g, root=np.zeros((6, nrhs)))
    amax = lambda x: float(np.abs(x).max()) if x.size else 0.0  # noqa: E731 (two-bead bodies have no rows)
    e2 = max(amax(w2 - w), amax(r2 - r)) / max(amax(w), amax(r))
    return max(e1, e2)


def root_rows_error(body):
    """The six root rows Q_Z, assembled column by column from unit vectors:
    orthonormal, spanning the row space of Z (Q_Z^T Q_Z = I - P with P the
    LAPACK projector onto the complement), and the first three rows are the
    normalised sum [I ... I] / sqrt(n) (Definition 4.1 at the root)."""
    n3 = 3 * body.n
    _, Qz = body.apply(np.eye(n3), root=np.zeros((6, n3)))
    P = dense.projector(body.pos)
    e1 = np.abs(Qz @ Qz.T - np.eye(6)).max()
    e2 = np.abs(Qz.T @ Qz - (np.eye(n3) - P)).max()
    e3 = np.abs(Qz[0:3] - np.tile(np.eye(3), body.n) / np.sqrt(body.n)).max()
    return max(e1, e2, e3)


def explicit_error(body, rng, nrhs=2):
    """Explicit Q~ (Algorithm 1) against the implicit sweeps (Algorithms 2-3)."""
    Q = body.explicit()
    v = rng.standard_normal((3 * body.n, nrhs))
    w = rng.standard_normal((body.rows, nrhs))
    e1 = np.abs(Q @ v - body.apply(v)).max()
    e2 = np.abs(Q.T @ w - body.apply(w, transpose=True)).max()
    e3 = np.abs(Q @ Q.T - np.eye(body.rows)).max()
    return max(e1, e2, e3)


def block_structure_error(body, tol=1e-13):
    """The rows of Q~ follow Q~_p = [Residue_p; diag(Q~_x, Q~_y)] (Section 3):
    node p's residue rows, then x's subtree rows, then y's, with every row
    supported inside its node's beads.  Returns the largest entry found
    outside the expected support (0 when the layout holds)."""
    Q = body.explicit()
    perm = body.perm()
    nodes = body.nodes()
    worst = 0.0

    def rows_of(c):
        return 0 if c < 0 else 3 * nodes[c].n - 6

    def walk(i, off):
        nonlocal worst
        nd = nodes[i]
        if nd.off != off:
            worst = max(worst, 1.0)
        cols = np.zeros(3 * body.n, dtype=bool)
        for s in range(nd.first, nd.last + 1):
            cols[3 * perm[s]:3 * perm[s] + 3] = True
        blk = Q[off:off + nd.dim][:, ~cols]
        if blk.size:
            worst = max(worst, np.abs(blk).max())
        nxt = off + nd.dim
        if nd.x >= 0:
            walk(nd.x, nxt)
        nxt += rows_of(nd.x)
        if nd.y >= 0:
            walk(nd.y, nxt)

    walk(0, 0)
    return worst


def bucket_lapack_error(body):
    """Every leaf box of 2..s beads against LAPACK: its transform is
    G = diag(-1,-1,-1,1,...,1) Q^T from numpy's Householder QR of the 3n x 6
    matrix X = [U_t^T | Z_r^T] (U_t = [I ... I] / sqrt(n); Z_r = [A_1 ... A_n],
    A_k = [r_k - c]x about the leaf's centroid), beads in the tree's order.
    Checks the leaf's residue rows of the explicit Q~ (G's rows 7..3n) and
    T22 = R(4:6,4:6)^T, skipping ill-conditioned leaves (whose last
    reflectors are fixed only up to rounding).  Returns the worst deviation."""
    Q = body.explicit()
    perm = body.perm()
    worst = 0.0
    for nd in body.nodes():
        if not nd.bucket:
            continue
        ids = perm[nd.first:nd.last + 1]
        n = len(ids)
        r = body.pos[ids] - body.pos[ids].mean(axis=0)
        X = np.zeros((3 * n, 6))
        for b in range(n):
            X[3 * b:3 * b + 3, 0:3] = np.eye(3) / np.sqrt(n)
            X[3 * b:3 * b + 3, 3:6] = cross(r[b]).T
        Qn, Rn = np.linalg.qr(X, mode="complete")
        if n >= 3 and nd.kappa > 1e6:
            continue
        T = Rn[3:6, 3:6].T.copy()
        if n == 2:
            T[2, 2] = 0.0
        worst = max(worst, np.abs(nd.T22 - T).max() / max(np.abs(T).max(), 1e-300))
        cols = (3 * ids[:, None] + np.arange(3)[None, :]).reshape(-1)
        got = Q[nd.off:nd.off + nd.dim][:, cols]
        if got.size:
            worst = max(worst, np.abs(got - Qn.T[6:]).max())
    return worst


def case1_closed_form(a, b, c):
    """T22 and U printed for two beads at (a,b,c) and (-a,-b,-c) (Eqs.
    3.9-3.10, valid as printed for b > 0, c > 0)."""
    s2 = b * b + c * c
    rho2 = a * a + s2
    T22 = np.array([
        [np.sqrt(2 * s2), 0.0, 0.0],
        [-np.sqrt(2) * a * b / np.sqrt(s2), np.sqrt(2 * c * c * rho2 / s2), 0.0],
        [-np.sqrt(2) * a * c / np.sqrt(s2), -np.sqrt(2 * b * b * rho2 / s2), 0.0],
    ])
    U = np.array([
        np.array([0, -c, b, 0, c, -b]) / np.sqrt(2 * s2),
        np.array([s2, -a * b, -a * c, -s2, a * b, a * c]) / np.sqrt(2 * rho2 * s2),
        np.array([-a, -b, -c, a, b, c]) / np.sqrt(2 * rho2),
    ])
    return T22, U


def case1_error(body_cls, a, b, c, lib=None):
    """The oracle's root T22 and U for the two-bead body against Eqs.
    3.9-3.10, equal up to the sign of each U row (and T22 column)."""
    pos = np.array([[a, b, c], [-a, -b, -c]])
    body = body_cls(pos, lib=lib) if lib is not None else body_cls(pos)
    _, U = body.explicit(with_root_u=True)
    T22 = body.node(0).T22
    Tp, Up = case1_closed_form(a, b, c)
    worst = 0.0
    for i in range(3):
        s = 1.0 if np.dot(U[i], Up[i]) >= 0 else -1.0
        worst = max(worst, np.abs(s * U[i] - Up[i]).max())
        worst = max(worst, np.abs(s * T22[:, i] - Tp[:, i]).max() / np.abs(Tp).max())
    return worst
