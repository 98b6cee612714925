"""Dense FP64 oracle (numpy / LAPACK) of the basis-free quantities.

TEST INFRASTRUCTURE ONLY.

For one rigid body with beads r_k the Z-matrix of Eq. 1.2 is the 6 x 3n matrix
[I ... I; A_1 ... A_n] with A_k f = r_k x f.  Q~ is fixed only up to an
orthogonal change of its rows; what the problem fixes is

* Z Q~^T = 0 and Q~ Q~^T = I (the rows are an orthonormal basis of the
  orthogonal complement of Z's row space, Section 1 and the abstract), hence
* the orthogonal projector Q~^T Q~ = P = I - Z^T (Z Z^T)^{-1} Z.

P is computed stably from a QR factorisation of Z^T (LAPACK via numpy).
"""
from __future__ import annotations

import numpy as np


def cross_matrix(r):
    """A with A f = r x f (the A_k of Eq. 1.2)."""
    x, y, z = r
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def zmatrix(pos, center=None):
    """The 6 x 3n Z-matrix of one body.  With ``center`` the cross-product
    blocks use r_k - center (the row space does not change)."""
    pos = np.asarray(pos, dtype=np.float64)
    if center is not None:
        pos = pos - np.asarray(center, dtype=np.float64)
    n = len(pos)
    Z = np.zeros((6, 3 * n))
    for k in range(n):
        Z[0:3, 3 * k:3 * k + 3] = np.eye(3)
        Z[3:6, 3 * k:3 * k + 3] = cross_matrix(pos[k])
    return Z


def zmatrix_centroid(pos):
    pos = np.asarray(pos, dtype=np.float64)
    return zmatrix(pos, pos.mean(axis=0))


def rank(pos, tol=1e-10):
    Z = zmatrix_centroid(pos)
    s = np.linalg.svd(Z, compute_uv=False)
    return int(np.sum(s > tol * s[0]))


def row_space_basis(pos):
    """Orthonormal basis (3n x r) of Z's row space via QR of Z^T."""
    Z = zmatrix_centroid(pos)
    Q, R = np.linalg.qr(Z.T, mode="reduced")
    d = np.abs(np.diag(R))
    keep = d > 1e-12 * max(d.max(), 1e-300)
    if keep.all():
        return Q
    # rank-deficient body (collinear beads): use the SVD instead
    U, s, _ = np.linalg.svd(Z.T, full_matrices=False)
    r = int(np.sum(s > 1e-12 * s[0]))
    return U[:, :r]


def projector(pos):
    """P = I - Z^T (Z Z^T)^+ Z, the projector onto the complement of Z's rows."""
    Q1 = row_space_basis(pos)
    return np.eye(Q1.shape[0]) - Q1 @ Q1.T


def project(pos, f):
    """P f for f (3n x R) without forming the 3n x 3n projector."""
    Q1 = row_space_basis(pos)
    f = np.asarray(f, dtype=np.float64).reshape(Q1.shape[0], -1)
    return f - Q1 @ (Q1.T @ f)


def complement_basis(pos):
    """A reference Q~_d ((3n-6) x 3n): the last 3n-6 columns of the full QR of
    Z^T, transposed.  Any orthogonal row rotation of it is equally valid."""
    Z = zmatrix_centroid(pos)
    Q, _ = np.linalg.qr(Z.T, mode="complete")
    return Q[:, 6:].T


def leak(pos, x):
    """||Z x|| / (||Z||_2 ||x||) per column of x (3n x R), Z about the
    centroid."""
    Z = zmatrix_centroid(pos)
    x = np.asarray(x, dtype=np.float64).reshape(Z.shape[1], -1)
    nz = np.linalg.norm(Z, 2)
    return np.linalg.norm(Z @ x, axis=0) / (nz * np.maximum(np.linalg.norm(x, axis=0), 1e-300))


# ---------------------------------------------------------------------------
# The same quantities for bodies too large to form Z (millions of beads):
# Z x, Z^T y and the 6 x 6 Gram matrix Z Z^T straight from the definition of
# Eq. 1.2 in O(n).  Z is taken about the centroid as above; the projector is
# P f = f - Z^T (Z Z^T)^{-1} Z f, which for a body that spans 3D has a
# well-conditioned 6 x 6 Gram matrix.
# ---------------------------------------------------------------------------
def _centred(pos):
    pos = np.asarray(pos, dtype=np.float64)
    return pos - pos.mean(axis=0)


def zmul(pos, x):
    """Z x (6 x R) for x (3n x R): [sum_k x_k; sum_k r_k x x_k]."""
    r = _centred(pos)
    x = np.asarray(x, dtype=np.float64).reshape(len(r), 3, -1)
    top = x.sum(axis=0)
    bot = np.cross(r[:, :, None], x, axisa=1, axisb=1, axisc=1).sum(axis=0)
    return np.concatenate([top, bot], axis=0)


def zmul_t(pos, y):
    """Z^T y (3n x R) for y (6 x R): block k is y_t + A_k^T y_r = y_t - r_k x y_r."""
    r = _centred(pos)
    y = np.asarray(y, dtype=np.float64).reshape(6, -1)
    yt, yr = y[0:3], y[3:6]
    blk = yt[None, :, :] - np.cross(r[:, :, None], yr[None, :, :], axisa=1, axisb=1, axisc=1)
    return blk.reshape(3 * len(r), -1)


def gram(pos):
    """Z Z^T (6 x 6) about the centroid: [[n I, 0], [0, sum_k A_k A_k^T]]."""
    r = _centred(pos)
    G = np.zeros((6, 6))
    G[0:3, 0:3] = len(r) * np.eye(3)
    # A_k A_k^T = |r_k|^2 I - r_k r_k^T; the off-diagonal blocks sum_k A_k^T
    # vanish about the centroid (sum_k r_k = 0) up to rounding
    G[3:6, 3:6] = (r * r).sum() * np.eye(3) - r.T @ r
    S = np.zeros((3, 3))
    sx = r.sum(axis=0)
    S[:] = cross_matrix(sx).T
    G[0:3, 3:6] = S
    G[3:6, 0:3] = S.T
    return G


def project_large(pos, f):
    """P f (3n x R) in O(n)."""
    f = np.asarray(f, dtype=np.float64).reshape(3 * len(pos), -1)
    return f - zmul_t(pos, np.linalg.solve(gram(pos), zmul(pos, f)))


def leak_large(pos, x):
    """||Z x|| / (||Z||_2 ||x||) per column, in O(n)."""
    x = np.asarray(x, dtype=np.float64).reshape(3 * len(pos), -1)
    nz = np.sqrt(np.linalg.eigvalsh(gram(pos)).max())
    return np.linalg.norm(zmul(pos, x), axis=0) / (nz * np.maximum(np.linalg.norm(x, axis=0), 1e-300))
