"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module draws random numbers only: bead positions of shell-bead rigid bodies
(beads spread over a closed surface, Section 1 of the paper), the right-hand
sides, and rigid motions.  It holds none of the method's arithmetic, so both the
FP64 oracle and the GPU path can consume exactly the same inputs.

Every generator uses numpy's PCG64 ``default_rng(seed)`` in FP64.  Draw order
inside a workload: positions, then v (3N x R), then w (sum(3n_j-6) x R).

The paper does not state the bead distribution of its experiments (Section 5),
so the workloads below stand in for it:

* ``sphere``     n beads uniform on a sphere (normalised Gaussian directions).
* ``ellipsoid``  area-uniform beads on an ellipsoid surface, by rejection, which
                 imitates evenly spaced shell beads; optional rotation, jitter.
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# primitive samplers
# --------------------------------------------------------------------------


def unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return u


def sphere(rng, n, radius=1.0, center=(0.0, 0.0, 0.0)):
    return unit_vectors(rng, n) * radius + np.asarray(center, dtype=np.float64)


def ellipsoid_surface(rng, n, axes):
    """Area-uniform points on the ellipsoid with semi-axes ``axes`` (rejection).

    A unit direction u maps to (a u_x, b u_y, c u_z); it is kept with
    probability sqrt((bc u_x)^2 + (ac u_y)^2 + (ab u_z)^2) / max(ab, bc, ca),
    which is proportional to the local area element of that map.
    """
    a, b, c = (float(t) for t in axes)
    pmax = max(a * b, b * c, c * a)
    out = np.empty((n, 3))
    got = 0
    while got < n:
        want = max(64, int(1.6 * (n - got)))
        u = unit_vectors(rng, want)
        w = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2) / pmax
        keep = rng.random(want) < w
        pts = u[keep] * np.array([a, b, c])
        take = min(len(pts), n - got)
        out[got:got + take] = pts[:take]
        got += take
    return out


def random_rotation(rng) -> np.ndarray:
    """Haar-random rotation from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def offsets_from_sizes(sizes) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(np.asarray(sizes, dtype=np.int64), out=off[1:])
    return off


def residue_rows(offsets) -> int:
    n = np.diff(np.asarray(offsets, dtype=np.int64))
    return int(np.sum(3 * n - 6))


class Workload:
    """Positions (N,3) FP64 in user bead order, body offsets (m+1), and RHS."""

    def __init__(self, name, pos, offsets, nrhs, rng):
        self.name = name
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.nrhs = int(nrhs)
        self.rng = rng

    @property
    def N(self):
        return int(self.offsets[-1])

    @property
    def m(self):
        return len(self.offsets) - 1

    @property
    def rows(self):
        return residue_rows(self.offsets)

    def draw_vectors(self):
        """v ~ N(0,1) of shape (3N, R) then w ~ N(0,1) of shape (rows, R)."""
        v = self.rng.standard_normal((3 * self.N, self.nrhs))
        w = self.rng.standard_normal((self.rows, self.nrhs))
        return v, w


# --------------------------------------------------------------------------
# the five workloads (sizes and distributions of the target configurations)
# --------------------------------------------------------------------------


def sphere_n64(seed=0):
    """One body, n=64 uniform on a sphere of radius 20 centred at (3,-2,5)."""
    rng = np.random.default_rng(seed)
    pos = sphere(rng, 64, 20.0, (3.0, -2.0, 5.0))
    return Workload("sphere_n64", pos, [0, 64], 1, rng)


def ellipsoid_body(rng, n, axes, jitter=0.0, center=(0.0, 0.0, 0.0)):
    p = ellipsoid_surface(rng, n, axes) @ random_rotation(rng).T
    if jitter > 0:
        p = p + jitter * rng.standard_normal(p.shape)
    return p + np.asarray(center, dtype=np.float64)


def ellipsoid_n65536(seed=1, n=65536, nrhs=16):
    """One body on a randomly rotated (40,25,15) ellipsoid, jitter 0.5."""
    rng = np.random.default_rng(seed)
    pos = ellipsoid_body(rng, n, (40.0, 25.0, 15.0), jitter=0.5)
    return Workload(f"ellipsoid_n{n}_R{nrhs}", pos, [0, n], nrhs, rng)


def _batched_bodies(rng, sizes, box=500.0):
    parts = []
    for n in sizes:
        axes = rng.uniform(10.0, 50.0, 3)
        off = rng.uniform(0.0, box, 3)
        parts.append(ellipsoid_body(rng, int(n), axes, center=off))
    return np.concatenate(parts, axis=0)


def batched_m1000(seed=2, m=1000, lo=200, hi=2000, nrhs=1):
    """m bodies, n_j uniform integer in [lo,hi], each on its own ellipsoid."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, m)
    pos = _batched_bodies(rng, sizes)
    return Workload(f"batched_m{m}_R{nrhs}", pos, offsets_from_sizes(sizes), nrhs, rng)


def bd_sizes(rng, m):
    return np.clip(np.rint(500.0 * np.exp(0.6 * rng.standard_normal(m))), 50, 20000).astype(np.int64)


def bd_m4096(seed=3, m=4096, nrhs=32):
    """BD-step workload: m bodies with lognormal sizes (median 500, sigma 0.6)."""
    rng = np.random.default_rng(seed)
    sizes = bd_sizes(rng, m)
    pos = _batched_bodies(rng, sizes)
    return Workload(f"bd_m{m}_R{nrhs}", pos, offsets_from_sizes(sizes), nrhs, rng)


def rigid_motions(rng, steps, m):
    """Per-step, per-body rigid motions: Haar rotation (3x3) and a translation
    uniform in [-1,1]^3.  Returns rot (steps,m,3,3), trans (steps,m,3)."""
    q = rng.standard_normal((steps, m, 4))
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = (q[..., i] for i in range(4))
    rot = np.empty((steps, m, 3, 3))
    rot[..., 0, 0] = 1 - 2 * (y * y + z * z)
    rot[..., 0, 1] = 2 * (x * y - z * w)
    rot[..., 0, 2] = 2 * (x * z + y * w)
    rot[..., 1, 0] = 2 * (x * y + z * w)
    rot[..., 1, 1] = 1 - 2 * (x * x + z * z)
    rot[..., 1, 2] = 2 * (y * z - x * w)
    rot[..., 2, 0] = 2 * (x * z - y * w)
    rot[..., 2, 1] = 2 * (y * z + x * w)
    rot[..., 2, 2] = 1 - 2 * (x * x + y * y)
    trans = rng.uniform(-1.0, 1.0, (steps, m, 3))
    return rot, trans


def large_clustered(seed=4, n=4194304, clusters=64, frac=0.05, seg_len=20.0, perp=1e-9):
    """One large body on a jittered (400,250,150) ellipsoid; a fraction ``frac``
    of its beads is replaced by ``clusters`` near-collinear segments."""
    rng = np.random.default_rng(seed)
    pos = ellipsoid_body(rng, n, (400.0, 250.0, 150.0), jitter=0.5)
    k = int(frac * n)
    idx = rng.choice(n, k, replace=False)
    per = np.array_split(idx, clusters)
    anchors = pos[rng.choice(n, clusters, replace=False)]
    for c, ids in enumerate(per):
        d = unit_vectors(rng, 1)[0]
        t = rng.uniform(0.0, seg_len, len(ids))
        pts = anchors[c] + t[:, None] * d[None, :]
        pos[ids] = pts + perp * rng.standard_normal((len(ids), 3))
    return Workload(f"clustered_n{n}", pos, [0, n], 1, rng)


def small_batch(seed, sizes, axes_lo=10.0, axes_hi=50.0, box=100.0, nrhs=1):
    """A few bodies of chosen sizes (test helper with the batched geometry)."""
    rng = np.random.default_rng(seed)
    parts = []
    for n in sizes:
        axes = rng.uniform(axes_lo, axes_hi, 3)
        off = rng.uniform(0.0, box, 3)
        parts.append(ellipsoid_body(rng, int(n), axes, center=off))
    pos = np.concatenate(parts, axis=0) if parts else np.zeros((0, 3))
    return Workload(f"small_batch_{seed}", pos, offsets_from_sizes(sizes), nrhs, rng)


# --------------------------------------------------------------------------
# degenerate and edge-case bodies (Section 2.2: collinear beads make Z rank 5;
# coincident beads share their finest box)
# --------------------------------------------------------------------------


def collinear_body(rng, n, length=30.0, center=(0.0, 0.0, 0.0)):
    """n beads at uniform positions along a random line segment."""
    d = unit_vectors(rng, 1)[0]
    t = rng.uniform(0.0, length, n)
    return np.asarray(center, dtype=np.float64) + t[:, None] * d[None, :]


def with_duplicates(rng, pos, ndup, group=1):
    """``pos`` plus ``ndup`` groups of ``group`` exact copies of randomly
    chosen beads, the whole body in a random bead order."""
    src = rng.choice(len(pos), ndup, replace=False)
    extra = np.repeat(pos[src], group, axis=0)
    allp = np.concatenate([pos, extra], axis=0)
    return allp[rng.permutation(len(allp))]


def mixed_batch(seed, parts, nrhs=1):
    """A batch of bodies from (kind, n) parts: "ellipsoid" (batched geometry),
    "collinear", "duplicates" (an ellipsoid body of n beads of which n // 5 are
    exact copies of others), "cluster" (an ellipsoid body with one point
    holding n // 10 coincident beads), "point" (all n beads at one point)."""
    rng = np.random.default_rng(seed)
    out, sizes = [], []
    for kind, n in parts:
        off = rng.uniform(0.0, 100.0, 3)
        if kind == "ellipsoid":
            p = ellipsoid_body(rng, n, rng.uniform(10.0, 50.0, 3), center=off)
        elif kind == "collinear":
            p = collinear_body(rng, n, center=off)
        elif kind == "duplicates":
            base = ellipsoid_body(rng, n - n // 5, rng.uniform(10.0, 50.0, 3), center=off)
            p = with_duplicates(rng, base, n // 5)
        elif kind == "cluster":
            base = ellipsoid_body(rng, n - n // 10 + 1, rng.uniform(10.0, 50.0, 3), center=off)
            p = with_duplicates(rng, base, 1, group=n // 10 - 1)
        elif kind == "point":
            p = np.repeat(off[None, :], n, axis=0)
        else:
            raise ValueError(kind)
        assert len(p) == n
        out.append(p)
        sizes.append(n)
    return Workload(f"mixed_{seed}", np.concatenate(out, axis=0), offsets_from_sizes(sizes), nrhs, rng)
