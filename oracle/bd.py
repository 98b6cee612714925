"""Dense FP64 reference of the constrained Brownian-dynamics solve of
Section 1 (Eqs. 1.4-1.6), for small systems.

TEST INFRASTRUCTURE ONLY.

With the full orthogonal Q = [Q_Z; Q~] of every body (block diagonal over
bodies), the mobility problem Q D^-1 Q^T [V; 0] = [F; g] (Eq. 1.4) splits
into the constraint-force equation 0 = Q~ D Q_Z^T F + Q~ D Q~^T g (Eq. 1.5)
and the velocity formula V = Q_Z D (Q_Z^T F + Q~^T g) (Eq. 1.6).  Q~ is fixed
only up to an orthogonal change of rows; g and V are expressed in the basis
of the hierarchical oracle (``oracle.hier``), whose particular Q_Z and Q~ are
assembled densely here, and the system is solved with LAPACK.
"""
from __future__ import annotations

import numpy as np

from oracle import hier


def full_q(pos, offsets):
    """(Q_Z, Q~): 6m x 3N and rows x 3N, block diagonal over the bodies, rows
    of each body in the oracle's order; Q_Z is read off column by column from
    the upward sweep's root Info-sets (Algorithm 2 with the root kept)."""
    pos = np.asarray(pos, dtype=np.float64)
    offsets = np.asarray(offsets, dtype=np.int64)
    m = len(offsets) - 1
    N = int(offsets[-1])
    rows = int(np.sum(3 * np.diff(offsets) - 6))
    Qz = np.zeros((6 * m, 3 * N))
    Qt = np.zeros((rows, 3 * N))
    r0 = 0
    for j in range(m):
        b0, b1 = int(offsets[j]), int(offsets[j + 1])
        body = hier.Body(pos[b0:b1])
        n3 = 3 * (b1 - b0)
        _, qz = body.apply(np.eye(n3), root=np.zeros((6, n3)))
        Qz[6 * j:6 * j + 6, 3 * b0:3 * b1] = qz
        Qt[r0:r0 + body.rows, 3 * b0:3 * b1] = body.explicit()
        r0 += body.rows
    return Qz, Qt


def constrained_solve(pos, offsets, D, F):
    """g from Eq. 1.5 and V from Eq. 1.6 (F: 6m x R in Q_Z's coordinates)."""
    Qz, Qt = full_q(pos, offsets)
    F = np.asarray(F, dtype=np.float64)
    A = Qt @ D @ Qt.T
    b = -(Qt @ (D @ (Qz.T @ F)))
    g = np.linalg.solve(A, b)
    V = Qz @ (D @ (Qz.T @ F + Qt.T @ g))
    return V, g
