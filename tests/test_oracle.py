"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks it against a
library routine (LAPACK QR), a closed form printed in the paper, a brute-force
definition (literal box bisection, direct sums over beads), or an invariant.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dense, hier
from tests import pins


@pytest.fixture(scope="module")
def c1():
    w = W.sphere_n64()
    return w, hier.Body(w.pos)


def rand_body(seed, n, kind="ellipsoid"):
    rng = np.random.default_rng(seed)
    if kind == "sphere":
        pos = W.sphere(rng, n, 5.0, rng.uniform(-3, 3, 3))
    elif kind == "cube":
        pos = rng.uniform(-2, 7, (n, 3))
    else:
        pos = W.ellipsoid_body(rng, n, rng.uniform(5, 30, 3), jitter=0.3, center=rng.uniform(-50, 50, 3))
    return pos


# --------------------------------------------------------------------------
# C1: the n=64 sphere, against the dense projector
# --------------------------------------------------------------------------


def test_c1_against_dense(c1):
    w, b = c1
    Q = b.explicit()
    assert Q.shape == (186, 192)
    Z = dense.zmatrix(w.pos)
    P = dense.projector(w.pos)
    assert np.abs(Q @ Q.T - np.eye(186)).max() < 1e-14
    assert np.abs(Z @ Q.T).max() / np.linalg.norm(Z, 2) < 1e-14
    assert np.abs(Q.T @ Q - P).max() < 1e-14
    # Q~ Q~_d^T is orthogonal for the reference LAPACK basis
    Qd = dense.complement_basis(w.pos)
    O = Q @ Qd.T
    assert np.abs(O @ O.T - np.eye(186)).max() < 1e-13


def test_c1_products(c1):
    w, b = c1
    v, wv = w.draw_vectors()
    rng = np.random.default_rng(11)
    assert pins.projector_error(b, rng) < 1e-14
    assert pins.roundtrip_error(b, rng) < 1e-14
    assert pins.leak_error(b, rng) < 1e-14
    assert pins.norm_error(b, rng) < 1e-14
    assert pins.explicit_error(b, rng) < 1e-14


# --------------------------------------------------------------------------
# per-node pins
# --------------------------------------------------------------------------


@pytest.mark.parametrize("seed,n,kind", [(0, 40, "ellipsoid"), (1, 100, "sphere"), (2, 257, "cube"),
                                         (3, 600, "ellipsoid")])
def test_infoset_identities(seed, n, kind):
    b = hier.Body(rand_body(seed, n, kind))
    assert pins.infoset_identity_error(b, np.random.default_rng(seed)) < 1e-13


@pytest.mark.parametrize("seed,n", [(4, 50), (5, 300)])
def test_householder_matches_lapack(seed, n):
    b = hier.Body(rand_body(seed, n))
    assert pins.lapack_convention_error(b) < 1e-12


@pytest.mark.parametrize("seed,n", [(6, 64), (7, 500)])
def test_node_factorisation(seed, n):
    b = hier.Body(rand_body(seed, n))
    assert pins.factor_error(b) < 1e-13


def test_node_kinds_and_residue_count():
    b = hier.Body(rand_body(8, 333))
    nodes = b.nodes()
    assert len(nodes) == 332
    for nd in nodes:
        assert nd.k == 3 + 3 * (nd.x >= 0) + 3 * (nd.y >= 0)
        assert nd.dim == nd.k - 3
        assert abs(nd.sx - np.sqrt((nd.n - (b.node(nd.y).n if nd.y >= 0 else 1)) / nd.n)) < 1e-15
    assert sum(nd.dim for nd in nodes) == 3 * 333 - 6


def test_kappa_matches_svd():
    b = hier.Body(rand_body(9, 200))
    for nd in b.nodes():
        if nd.k == 3:
            continue
        s = np.linalg.svd(nd.T22, compute_uv=False)
        assert abs(nd.kappa - s[0] / s[2]) <= 1e-8 * s[0] / s[2]


@pytest.mark.parametrize("abc", [(0.3, 0.7, 1.1), (2.0, 0.1, 0.5), (-1.0, 0.4, 0.2)])
def test_case1_closed_form(abc):
    """Two beads at +-(a,b,c): T22 and U of Eqs. 3.9-3.10 (b, c > 0)."""
    a, b, c = abc
    assert pins.case1_error(hier.Body, a, b, c) < 1e-14


def test_case1_closed_form_is_a_valid_factor():
    """The printed closed form itself reproduces Z(4:6,:) for b, c > 0."""
    a, b, c = 0.3, 0.7, 1.1
    T22, U = pins.case1_closed_form(a, b, c)
    Z = dense.zmatrix(np.array([[a, b, c], [-a, -b, -c]]))
    assert np.abs(T22 @ U - Z[3:6]).max() < 1e-14
    assert np.abs(U @ U.T - np.eye(3)).max() < 1e-14


# --------------------------------------------------------------------------
# tree
# --------------------------------------------------------------------------


@pytest.mark.parametrize("seed,n", [(10, 2), (11, 3), (12, 9), (13, 64), (14, 200)])
def test_tree_is_the_literal_bisection(seed, n):
    pos = rand_body(seed, n, "cube")
    b = hier.Body(pos)
    assert pins.oracle_tree(b) == pins.bisection_tree(pos)


def test_codes_zyx_order():
    # two beads differing only in z land in different halves at the first split
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.0], [1.0, 1.0, 0.1]])
    c = hier.codes(pos)
    assert c[1] >> np.uint64(62) == 1 and c[0] >> np.uint64(62) == 0
    # the maximum coordinate is clamped into the top cell
    assert (int(c[1]) >> 60) & 0x4 == 0x4


# --------------------------------------------------------------------------
# whole-body properties, Table 1 magnitudes
# --------------------------------------------------------------------------


@pytest.mark.parametrize("n", [500, 1000, 2000, 4000])
def test_table1_magnitudes(n):
    """Section 5.2: Q Q^T - I, round trips and explicit-vs-implicit errors are
    all near machine precision (the paper reports <= 1.2e-13, infinity norm)."""
    rng = np.random.default_rng(n)
    b = hier.Body(W.ellipsoid_body(rng, n, (30, 20, 10), jitter=0.2))
    assert pins.roundtrip_error(b, rng) < 1e-13
    assert pins.projector_error(b, rng) < 1e-13
    assert pins.norm_error(b, rng) < 1e-13
    assert pins.leak_error(b, rng) < 1e-13
    if n <= 1000:
        assert pins.explicit_error(b, rng) < 1e-13


@pytest.mark.parametrize("seed,n", [(20, 30), (21, 120)])
def test_block_structure(seed, n):
    b = hier.Body(rand_body(seed, n))
    assert pins.block_structure_error(b) < 1e-14


def test_translation_and_scale_invariance():
    pos = rand_body(30, 150)
    b0 = hier.Body(pos)
    Q0 = b0.explicit()
    b1 = hier.Body(pos + np.array([0.25, -0.5, 2.0]))
    b2 = hier.Body(pos * 4.0)
    assert np.abs(b1.explicit() - Q0).max() < 1e-12
    assert np.abs(b2.explicit() - Q0).max() < 1e-12


def test_permutation_covariance():
    pos = rand_body(31, 120)
    rng = np.random.default_rng(31)
    p = rng.permutation(len(pos))
    Q0 = hier.Body(pos).explicit()
    Q1 = hier.Body(pos[p]).explicit()
    cols = (3 * p[:, None] + np.arange(3)[None, :]).reshape(-1)
    assert np.abs(Q1 - Q0[:, cols]).max() < 1e-14


def test_rotation_covariance_of_projector():
    pos = rand_body(32, 90)
    rng = np.random.default_rng(32)
    R = W.random_rotation(rng)
    B = np.kron(np.eye(len(pos)), R)
    Q0 = hier.Body(pos).explicit()
    Q1 = hier.Body(pos @ R.T).explicit()
    assert np.abs(Q1.T @ Q1 - B @ (Q0.T @ Q0) @ B.T).max() < 1e-13


# --------------------------------------------------------------------------
# special and degenerate bodies
# --------------------------------------------------------------------------


@pytest.mark.parametrize("seed,n,kind", [(21, 2, "cube"), (22, 3, "cube"), (23, 64, "sphere"), (24, 300, "ellipsoid")])
def test_full_q_orthogonal(seed, n, kind):
    """Q = [Q_Z; Q~] with the root Info-set kept (Algorithm 2) and a given root
    Velocity-set (Algorithm 3) is orthogonal."""
    b = hier.Body(rand_body(seed, n, kind))
    assert pins.full_q_inverse_error(b, np.random.default_rng(seed)) < 1e-13


@pytest.mark.parametrize("seed,n,kind", [(25, 3, "cube"), (26, 5, "cube"), (27, 64, "sphere"), (28, 200, "ellipsoid")])
def test_root_rows_span_z(seed, n, kind):
    """(Two beads are collinear, rank Z = 5: their six root rows are a full
    6 x 6 orthogonal matrix instead, checked by the orthogonality pin.)"""
    b = hier.Body(rand_body(seed, n, kind))
    assert pins.root_rows_error(b) < 1e-13


@pytest.mark.parametrize("seed,sizes", [(33, [2, 9, 30]), (34, [3, 50])])
def test_constrained_solve_satisfies_block_system(seed, sizes):
    """Eqs. 1.5-1.6 solved densely reproduce the original mobility problem
    Q D^-1 Q^T [V; 0] = [F; g] (Eq. 1.4), which uses D^-1 instead of D, and
    the bead velocities Q_Z^T V are rigid motions (in the row space of Z)."""
    from oracle import bd
    rng = np.random.default_rng(seed)
    pos = np.concatenate([rand_body(seed + i, n, "cube") for i, n in enumerate(sizes)])
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    N, m = int(offsets[-1]), len(sizes)
    M = rng.standard_normal((3 * N, 3 * N))
    D = np.eye(3 * N) + 0.2 * (M @ M.T) / np.linalg.norm(M, 2) ** 2
    F = rng.standard_normal((6 * m, 3))
    V, g = bd.constrained_solve(pos, offsets, D, F)
    Qz, Qt = bd.full_q(pos, offsets)
    Q = np.vstack([Qz, Qt])
    lhs = Q @ np.linalg.inv(D) @ Q.T @ np.vstack([V, np.zeros_like(g)])
    assert np.abs(lhs - np.vstack([F, g])).max() < 1e-10 * max(1.0, np.abs(F).max())
    u = Qz.T @ V
    for j in range(m):
        b0, b1 = offsets[j], offsets[j + 1]
        if dense.rank(pos[b0:b1]) == 6:
            uj = u[3 * b0:3 * b1]
            assert np.abs(uj - (np.eye(3 * (b1 - b0)) - dense.projector(pos[b0:b1])) @ uj).max() < 1e-12


def test_two_beads():
    pos = np.array([[0.0, 1.0, 2.0], [1.0, -1.0, 0.5]])
    b = hier.Body(pos)
    assert b.rows == 0
    Q, U = b.explicit(with_root_u=True)
    F = np.vstack([np.tile(np.eye(3), 2) / np.sqrt(2), U])
    assert np.abs(F @ F.T - np.eye(6)).max() < 1e-15


def test_three_beads():
    pos = np.array([[0.0, 1.0, 2.0], [1.0, -1.0, 0.5], [0.3, 0.2, -1.0]])
    b = hier.Body(pos)
    Q = b.explicit()
    assert Q.shape == (3, 9)
    assert np.abs(Q.T @ Q - dense.projector(pos)).max() < 1e-14


def test_collinear_body():
    """Beads on a line: rank Z = 5 (Section 2.2).  Q~ stays orthonormal and
    orthogonal to Z but spans one dimension less than the complement."""
    t = np.linspace(0.0, 3.0, 20)
    pos = np.stack([1 + t, 2 - 0.5 * t, 0.25 * t], axis=1)
    assert dense.rank(pos) == 5
    b = hier.Body(pos)
    Q = b.explicit()
    assert np.abs(Q @ Q.T - np.eye(b.rows)).max() < 1e-12
    Z = dense.zmatrix_centroid(pos)
    assert np.abs(Z @ Q.T).max() / np.linalg.norm(Z, 2) < 1e-12
    P = dense.projector(pos)
    assert abs(np.trace(P) - np.trace(Q.T @ Q) - 1.0) < 1e-10


def test_coincident_beads():
    """Beads sharing a position share their code; the split falls back to the
    sorted position, and the result stays orthonormal and orthogonal to Z."""
    rng = np.random.default_rng(40)
    base = rng.uniform(0, 1, (12, 3))
    pos = np.concatenate([base, base[:5]], axis=0)
    b = hier.Body(pos)
    Q = b.explicit()
    assert np.abs(Q @ Q.T - np.eye(b.rows)).max() < 1e-12
    Z = dense.zmatrix_centroid(pos)
    assert np.abs(Z @ Q.T).max() / np.linalg.norm(Z, 2) < 1e-12
    assert np.abs(Q.T @ Q - dense.projector(pos)).max() < 1e-12


def test_batch_block_diagonal():
    w = W.small_batch(50, [3, 17, 64, 2, 150])
    bt = hier.Batch(w.pos, w.offsets)
    rng = np.random.default_rng(50)
    v = rng.standard_normal((3 * w.N, 2))
    out = bt.apply(v)
    assert out.shape == (w.rows, 2)
    for j, b in enumerate(bt.bodies):
        r0, r1 = bt.row_off[j], bt.row_off[j + 1]
        assert np.array_equal(out[r0:r1], b.apply(v[3 * w.offsets[j]:3 * w.offsets[j + 1]]))


def test_large_body_helpers_match_dense_definitions():
    """The O(n) forms of Z x, Z^T y, Z Z^T, P f and the leak (used for
    bodies too large for a dense Z) against the dense Z of Eq. 1.2."""
    rng = np.random.default_rng(21)
    for n in (3, 7, 64, 300):
        p = rng.standard_normal((n, 3)) * rng.uniform(1, 20, 3) + rng.uniform(-50, 50, 3)
        x = rng.standard_normal((3 * n, 3))
        y = rng.standard_normal((6, 3))
        Z = dense.zmatrix_centroid(p)
        scale = np.abs(Z).max() ** 2 * n
        assert np.abs(dense.zmul(p, x) - Z @ x).max() <= 1e-12 * np.abs(Z).max() * np.abs(x).sum(axis=0).max()
        assert np.abs(dense.zmul_t(p, y) - Z.T @ y).max() <= 1e-12 * np.abs(Z).max() * np.abs(y).sum()
        assert np.abs(dense.gram(p) - Z @ Z.T).max() <= 1e-12 * scale
        assert np.abs(dense.project_large(p, x) - dense.project(p, x)).max() <= 1e-10
        assert np.abs(dense.leak_large(p, x) - dense.leak(p, x)).max() <= 1e-12
        # the projector annihilates the row space and is idempotent
        px = dense.project_large(p, x)
        assert np.abs(dense.zmul(p, px)).max() <= 1e-9 * np.abs(Z).max() * np.abs(x).max() * n
        assert np.abs(dense.project_large(p, px) - px).max() <= 1e-10


# --------------------------------------------------------------------------
# leaf boxes of up to s beads (Section 2.1 allows s > 1)
# --------------------------------------------------------------------------


@pytest.mark.parametrize("s", [2, 3, 5, 8, 16])
@pytest.mark.parametrize("seed,n,kind", [(60, 300, "ellipsoid"), (61, 97, "sphere"), (62, 500, "cube")])
def test_leaf_buckets_basis_free(s, seed, n, kind):
    """Buckets keep every basis-free fact: rows orthonormal and orthogonal to
    Z, the LAPACK projector, the full Q orthogonal with Q_Z spanning row(Z),
    explicit = implicit, and the pre-order block layout."""
    b = hier.Body(rand_body(seed, n, kind), s=s)
    rng = np.random.default_rng(seed)
    assert sum(nd.bucket for nd in b.nodes()) > 0
    assert pins.projector_error(b, rng) < 1e-12
    assert pins.roundtrip_error(b, rng) < 1e-12
    assert pins.leak_error(b, rng) < 1e-14
    assert pins.full_q_inverse_error(b, rng) < 1e-12
    assert pins.root_rows_error(b) < 1e-12
    assert pins.explicit_error(b, rng) < 1e-13
    assert pins.block_structure_error(b) == 0.0


@pytest.mark.parametrize("s", [2, 4, 16])
def test_leaf_buckets_pinned_to_lapack(s):
    """Each bucket's transform against numpy's Householder QR of its 3n x 6
    matrix [U_t^T | Z_r^T], and its Info-set identities (Definition 4.1)."""
    b = hier.Body(rand_body(63, 400), s=s)
    assert pins.bucket_lapack_error(b) < 1e-12
    assert pins.infoset_identity_error(b, np.random.default_rng(63)) < 1e-13


def test_leaf_bucket_whole_body():
    """A body of n <= s beads is one leaf: Q~ is LAPACK's complement rows of
    [U_t^T | Z_r^T] (beads in tree order) and the rest of the tree is empty."""
    pos = rand_body(64, 12)
    b = hier.Body(pos, s=12)
    assert b.num_internal == 1 and b.node(0).bucket == 1
    assert pins.bucket_lapack_error(b) < 1e-13
    assert pins.projector_error(b, np.random.default_rng(64)) < 1e-13


def test_leaf_buckets_leave_s1_unchanged():
    """s = 1 is the one-bead-leaf tree, bit for bit."""
    pos = rand_body(65, 200)
    v = np.random.default_rng(65).standard_normal((600, 2))
    assert np.array_equal(hier.Body(pos).apply(v), hier.Body(pos, s=1).apply(v))


def test_leaf_bucket_degenerate_cases():
    """Two-bead leaves (rank-2 rotation rows, T22(3,3) = 0) and a collinear
    leaf keep the rows orthonormal and orthogonal to Z."""
    rng = np.random.default_rng(66)
    pos = np.concatenate([rand_body(66, 40), 50 + np.outer(rng.uniform(0, 1, 6), [1.0, 2.0, -0.5])])
    b = hier.Body(pos, s=6)
    for nd in b.nodes():
        if nd.bucket and nd.n == 2:
            assert nd.T22[2, 2] == 0.0
    Q = b.explicit()
    assert np.abs(Q @ Q.T - np.eye(b.rows)).max() < 1e-12
    Z = dense.zmatrix_centroid(pos)
    assert np.abs(Z @ Q.T).max() / np.linalg.norm(Z, 2) < 1e-12
