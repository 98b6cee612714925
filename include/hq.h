/*
 * hq.h -- C ABI of the MI355X (gfx950) library for the hierarchical
 * orthogonal complement of rigid-body Z-matrices.
 *
 * Fang, Huang, Huber, McCammon, Zhang, "Hierarchical Orthogonal Matrix
 * Generation and Matrix-Vector Multiplications in Rigid Body Simulations".
 *
 * A rigid body j has n_j beads at r_k.  Its Z-matrix (Eq. 1.2) is the
 * 6 x 3n_j matrix [I ... I; A_1 ... A_n] with A_k f = r_k x f.  For m bodies the
 * matrices are block diagonal (Section 1): Q~ = diag(Q~^1, ..., Q~^m), where
 * Q~^j has 3n_j - 6 orthonormal rows spanning the orthogonal complement of the
 * row space of Z^j.  The Problem Statement of Section 1 asks to construct Q~
 * (explicitly if needed) and to compute Q~ v and Q~^T v; this ABI exposes
 * exactly that:
 *
 *   hq_build    tree and FP64 local transforms (Sections 2.1, 3; Algorithm 1's
 *               generation part, Eqs. 3.4-3.13), O(n log n)
 *   hq_apply    Q~ v (Algorithm 2, Eqs. 4.2-4.3) or Q~^T w (Algorithm 3,
 *               Theorem 4.3), O(n) per right-hand side
 *   hq_explicit Q~ itself (Algorithm 1), dense per body or block-sparse
 *
 * Conventions (all bodies):
 *   - Bead vectors are row-major (3N x nrhs), the right-hand sides fastest;
 *     bead k of body j occupies rows 3(off_j + k) .. 3(off_j + k) + 2 in the
 *     caller's bead order (the paper's f = [f_1; ...; f_n], Section 1).
 *   - Residue vectors are row-major (rows x nrhs), rows = sum_j (3n_j - 6);
 *     body j's rows start at sum_{i<j} (3n_i - 6).  Inside a body the rows
 *     follow the block form Q~_p = [Residue_p; diag(Q~_x, Q~_y)] of Section 3:
 *     a node's residue rows, then its x subtree's, then its y subtree's.
 *   - The tree: per body, the cube with lower corner at the per-axis bead
 *     minimum and side equal to the largest extent; coordinates quantised to
 *     21 bits; boxes split at midpoints in z, then y, then x (Section 2.1);
 *     x = lower half; single-child boxes collapse; beads sharing all 63 bits
 *     split by the highest differing bit of their sorted position in the body.
 *   - Transforms: K = [T22_x | T22_y | sqrt(n_x n_y / n) [c_x - c_y]x] (leaf
 *     blocks absent) is factored by Householder reflections in LAPACK's sign
 *     convention, K = [T22 | 0] G; a two-bead node's rank-2 T22 has its
 *     third column set to exactly 0 (Eq. 3.9).
 *
 * Memory and streams: pointers documented "device" are HIP device memory
 * owned by the caller; "host" pointers are ordinary host memory.  Every call
 * that takes a stream is stream-ordered and asynchronous unless noted; the
 * caller synchronises before reading results.  A hq_stream is a hipStream_t
 * (NULL = the default stream).
 *
 * Errors: every function returns a status and never aborts.  hq_last_error()
 * returns a thread-local message for the last failing call on the thread.
 * Conditions found on the device (non-finite positions, an internal limit)
 * raise a per-handle device flag that hq_query() reports.
 */
#ifndef HQ_H
#define HQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hq_plan_s *hq_handle;
typedef void *hq_stream;

typedef enum {
    HQ_OK = 0,
    HQ_E_INVALID = 1,      /* bad argument, offsets, sizes, or non-finite input */
    HQ_E_DEGENERATE = 2,   /* reserved: degenerate bodies are flagged, not failed */
    HQ_E_NOMEM = 3,        /* device allocation failed */
    HQ_E_DEVICE = 4,       /* a HIP runtime call failed */
    HQ_E_UNSUPPORTED = 5   /* request outside a documented limit */
} hq_status;

typedef enum { HQ_FP64 = 0, HQ_FP32 = 1 } hq_precision;

/* Layout of a vector of nrhs right-hand sides whose rows come in triples (a
 * bead's x, y, z rows; each node's residue rows, Algorithm 2, fill whole
 * triples).  Row triple t, right-hand side r, component d:
 *   HQ_ROWS     element (3t + d) * nrhs + r: row-major rows x nrhs;
 *   HQ_TRIPLES  element (t * nrhs + r) * 3 + d: for each triple, nrhs
 *               contiguous 3-vectors (e.g. per-bead forces of nrhs
 *               independent systems stored as [bead][system][xyz]).
 * Both hold the same values; HQ_TRIPLES lets the sweeps move a lane's three
 * values in one access. */
typedef enum { HQ_ROWS = 0, HQ_TRIPLES = 1 } hq_layout;

/* Device flag bits reported by hq_query (hq_info.device_flags). */
#define HQ_FLAG_NONFINITE   1  /* a position was NaN or infinite */
#define HQ_FLAG_STACK       2  /* an internal per-tile stack limit was hit */
#define HQ_FLAG_BOUNDS      4  /* an internal index failed its bounds check */
#define HQ_FLAG_PHASES      8  /* a rebuilt tree needed more tile phases than reserved */

/* Per-body flag bits (hq_body_info). */
#define HQ_BODY_ILLCOND     1  /* some node with k > 3 has kappa(T22) > 1e4 */
#define HQ_BODY_DEGENERATE  2  /* rank Z < 6 (e.g. collinear beads, Section 2.2) */

typedef struct {
    int32_t tile_units;    /* max units (beads or sub-tile roots) per tile; 0 = 32; <= 1024 */
    int32_t store;         /* transforms kept: 1 = FP64, 2 = FP32, 3 or 0 = both */
    int32_t explicit_dense_max_n; /* largest n_j for hq_explicit; 0 = 4096 */
    int32_t max_phases;    /* tile phases reserved for hq_rebuild; 0 = found at build + 2 */
    int32_t run_nodes;     /* nodes per run of whole tiles swept by one lane group in the
                              first phase of a wide sweep (>= 32 RHS); 0 = 48; 8..4096 */
    int32_t waves_per_cu;  /* grid of the later tile phases' sweeps, in waves per compute
                              unit; 0 = 16; 1..64 */
    int32_t keep_node_data;/* 1: hq_rebuild also refreshes the per-node centroids and T22
                              that hq_node_data returns (hq_build always writes them);
                              0: it skips them (less memory traffic) */
    int32_t later_tile_units; /* max units per tile in the tile phases after the first,
                              whose units are the roots of earlier tiles; smaller tiles give
                              those short phases more parallel work at the cost of more
                              phases; 0 = tile_units; <= 1024 */
    int32_t first_waves_per_cu; /* grid of the first tile phase's wide sweeps (>= 32 RHS), in
                              waves per compute unit, grid-strided over the runs; 0 = one wave
                              per run pair (uncapped, fastest for a sweep on its own); 1..64.
                              A cap leaves compute-unit slots and LDS to work running
                              concurrently on another stream, e.g. the next step's hq_rebuild
                              on a second handle; results are the same bit for bit */
    int32_t max_nrhs;      /* hq_build_into: right-hand sides the sweeps' exchange entries in the
                              workspace hold (in the largest precision kept); 0 = 32.  Calls
                              with more fail with HQ_E_UNSUPPORTED.  Ignored by hq_build, whose
                              handle grows its own buffer */
    int32_t max_tiles;     /* hq_build_into: tiles the tile-indexed tables hold (plus 64); 0 =
                              one per internal node, a bound every tree meets (tiles are
                              disjoint and hold at least one node).  A smaller value saves
                              workspace; a tree with more tiles fails hq_build_into with
                              HQ_E_UNSUPPORTED and raises HQ_FLAG_BOUNDS on hq_rebuild */
    int32_t krylov_nrhs;   /* hq_build_into: right-hand sides of hq_constrained_solve whose
                              work vectors the workspace holds; 0 = none (the solve then fails
                              on the handle with HQ_E_UNSUPPORTED) */
    int32_t sweep_kernel;  /* Which sweep kernels run; results agree to rounding.
                              0 (automatic): the first tile phase with the wide sweeps (a
                              lane group per run of whole tiles, node records read once per
                              group and broadcast) for 8 or more right-hand sides when every
                              vector buffer stays below 2 GiB, else with a lane group per
                              tile; the later phases node-parallel (a lane per node and
                              right-hand side, a tile's levels resolved in LDS) where their
                              tiles fit a workgroup, else as the first.
                              1: a lane group per tile (lanes reading whole records) in
                              every phase.
                              2: node-parallel in every phase whose tiles hold at most 64
                              units (up to 8 right-hand sides per pass).
                              3: the wide sweeps in every phase, for any number of
                              right-hand sides (buffers below 2 GiB). */
    int32_t fused_upward;  /* 0: one launch per tile phase; 1: the wide upward sweep
                              (Algorithm 2) of up to 64 right-hand sides in one launch, each
                              later-phase tile swept by the workgroup whose child tile
                              finished last (arrival counters, no waiting).  Same results
                              bit for bit; measured slower on 4,096 bodies (the last tiles'
                              chains of later-phase nodes trail the launch).  The downward
                              sweep, leaf boxes and sweeps of more than 64 right-hand sides
                              take one launch per phase either way */
    int32_t leaf_size;     /* 0 or 1: leaves of one bead (the paper's s = 1); 2..16: the
                              bisection of Section 2.1 stops at boxes of at most leaf_size
                              beads, each factored densely as one leaf: the Householder QR
                              of its 3n x 6 matrix [U_t^T | Z_r^T] (translation rows
                              [I..I]/sqrt(n), rotation rows [A_1..A_n] about its centroid)
                              gives G = diag(-1,-1,-1,1,..,1) Q^T, whose rows 7..3n are the
                              leaf's residue rows.  tile_units then sizes the tiles above
                              the leaves.  hq_explicit, hq_explicit_blocks and the
                              geometry of hq_node_data are unavailable (HQ_E_UNSUPPORTED) */
} hq_options;

typedef struct {
    int64_t N;             /* beads */
    int64_t m;             /* bodies */
    int64_t rows;          /* sum_j (3 n_j - 6) */
    int64_t internal_nodes;/* N - m */
    int64_t tiles;         /* tiles of the last build */
    int32_t phases;        /* tile phases of the last build */
    int32_t device_flags;  /* HQ_FLAG_* raised since the handle was built */
    int32_t tile_units;
    int32_t store;
    double max_kappa;      /* max over bodies of the largest kappa(T22), k > 3 nodes */
    int64_t ill_conditioned_bodies;
    int64_t degenerate_bodies;
} hq_info;

/* Pick tile_units, later_tile_units, run_nodes, waves_per_cu and leaf_size for a workload
 * by measurement: the subtree sizes of Section 2's tree cut into tiles, and
 * the launch shape of the sweeps (Algorithms 2 and 3).  For every candidate,
 * builds a handle on the given positions, then times (median of 5 after 2
 * warm-up rounds, HIP events on the stream) one round of: hq_rebuild if
 * include_rebuild, an upward and a downward hq_apply_layout with nrhs
 * right-hand sides in precision prec and vector layout layout.
 * Stage 1: tile_units 16, 32, 64 x run_nodes 32, 48, 64 x waves_per_cu 8,
 * 16, 32 (later_tile_units = tile_units).
 * Stage 2, on the winner: later_tile_units 4, 8, 16 (those below its
 * tile_units) x waves_per_cu 8, 16, 32; kept only if faster.
 * Stage 3, on that winner (unless base fixes leaf_size): leaf_size 4, 8, 16
 * (Section 2.1's leaves of up to s beads) x waves_per_cu; kept only if
 * faster.
 *   positions, body_offsets, m  as for hq_build.
 *   base          host, may be NULL: the other options of the trial builds.
 *   best          host: receives base with the chosen fields set
 *                 (later_tile_units 0 when stage 2 kept tile_units).
 *   best_ms       host, may be NULL: the chosen candidate's time per round.
 * Allocates (and frees) trial handles and two vector buffers; synchronises
 * the stream.  Errors as for hq_build and hq_apply. */
hq_status hq_autotune(const double *positions, const int64_t *body_offsets, int64_t m, int64_t nrhs,
                      hq_precision prec, hq_layout layout, int include_rebuild, const hq_options *base, hq_stream stream,
                      hq_options *best, double *best_ms);

/* Build the tree and the FP64 local transforms of m bodies: Section 1's
 * Problem Statement (construct Q~), with Section 2.1's nested boxes and
 * Section 3's per-node factorisations (Eqs. 3.4-3.13; Algorithm 1 without
 * forming Q~).
 *   positions     device, N x 3 FP64, x,y,z interleaved, caller's bead order.
 *   body_offsets  host, m + 1 entries: [0] = 0, strictly increasing, so that
 *                 body j holds beads [off_j, off_{j+1}); every n_j >= 2.
 *   opt           host, may be NULL for the defaults.
 *   out           receives the handle, which owns all device memory it uses
 *                 (allocated here with hipMalloc).
 * Synchronises the stream once (to size the tile phases); the stream is the
 * handle's: the calls below that read device state synchronise it.  Errors:
 * HQ_E_INVALID for bad offsets, n_j < 2, NULL pointers or non-finite
 * positions (found on the device); HQ_E_NOMEM; HQ_E_DEVICE. */
hq_status hq_build(const double *positions, const int64_t *body_offsets, int64_t m,
                   const hq_options *opt, hq_stream stream, hq_handle *out);

/* Device bytes hq_build_into needs for these bodies and options (the
 * Problem Statement's Q~ construction, as hq_build, in caller memory): the
 * tree, tile and node tables, the transforms of the precisions kept, the
 * tile-root table and exchange entries (hq_options.max_tiles, max_nrhs), the
 * explicit-block offsets of the largest body and the Krylov vectors
 * (krylov_nrhs).  Host only: no device memory is touched.  Errors as for
 * hq_build's argument checks. */
hq_status hq_workspace_bytes(const int64_t *body_offsets, int64_t m, const hq_options *opt, size_t *bytes);

/* hq_build into caller-owned device memory: workspace (device, 256-byte
 * aligned, at least hq_workspace_bytes bytes, e.g. a torch tensor) holds
 * every piece of the handle's device state; the handle allocates no device
 * memory, now or in any later call on it (hq_apply* beyond max_nrhs and
 * hq_constrained_solve beyond krylov_nrhs fail with HQ_E_UNSUPPORTED instead
 * of allocating).  The caller keeps the workspace alive until hq_destroy,
 * which frees nothing on the device.  Results are bit for bit those of
 * hq_build.  Errors as for hq_build; HQ_E_INVALID for a NULL, misaligned or
 * too small workspace. */
hq_status hq_build_into(const double *positions, const int64_t *body_offsets, int64_t m,
                        const hq_options *opt, void *workspace, size_t bytes, hq_stream stream,
                        hq_handle *out);

/* Rebuild the same bodies (same offsets) from new positions (Section 2.1's
 * tree and Section 3's factorisations again, as after a Brownian-dynamics
 * step, Section 1): device, N x 3 FP64.  No allocation and no host
 * synchronisation, so a stream capture may record it; tile phases beyond the
 * reserved count raise HQ_FLAG_PHASES. */
hq_status hq_rebuild(hq_handle h, const double *positions, hq_stream stream);

/* Pre-allocate the per-tile exchange buffers of the sweeps (Algorithms 2-3
 * across tiles) for up to nrhs right-hand sides of precision prec, so that
 * later hq_apply calls allocate nothing (needed before a stream capture).
 * Synchronises the handle's stream.  On a workspace handle it allocates
 * nothing and fails with HQ_E_UNSUPPORTED beyond max_nrhs. */
hq_status hq_reserve(hq_handle h, int64_t nrhs, hq_precision prec);

/* Apply Q~ or Q~^T to nrhs right-hand sides.
 *   transpose = 0: v device (3N x nrhs) -> out device (rows x nrhs) = Q~ v
 *                  (Algorithm 2; each body's root Info-set is dropped).
 *   transpose = 1: v device (rows x nrhs) -> out device (3N x nrhs) = Q~^T v
 *                  (Algorithm 3 with a zero root Velocity-set).
 *   Elements are double for HQ_FP64, float for HQ_FP32; the transforms of that
 *   precision must have been kept (hq_options.store).  v and out must not
 *   overlap.  Allocates the exchange buffers on first use unless reserved. */
hq_status hq_apply(hq_handle h, const void *v, void *out, int transpose, int64_t nrhs,
                   hq_precision prec, hq_stream stream);

/* hq_apply with both vectors in the given layout (hq_layout): the same
 * products (Algorithms 2 and 3), element for element.  HQ_E_INVALID for an
 * unknown layout; other errors as for hq_apply. */
hq_status hq_apply_layout(hq_handle h, const void *v, void *out, int transpose, int64_t nrhs,
                          hq_precision prec, hq_layout layout, hq_stream stream);

/* hq_apply_layout for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same products from the same kernels, with the sweeps' exchange buffer
 * (one entry of 6 x nrhs values per tile, passing Info-sets and
 * Velocity-sets between tile phases) in a static device array of 128 MiB
 * instead of the handle's own, growable buffer.  No hipMalloc, hipFree or
 * other allocation; each GPU the library runs on holds its array until the
 * process ends.  Nothing in the array needs clearing between calls (every
 * entry a sweep reads was written earlier in the same call), but all calls on
 * one GPU share it: calls that overlap in time on one GPU (other streams,
 * other handles, other threads) race and give wrong results.
 * HQ_E_UNSUPPORTED when (tiles of the handle's hq_build + 64) x 6 x nrhs
 * elements exceed 128 MiB (e.g. beyond 174,000 tiles at 32 FP32 right-hand
 * sides); a rebuilt tree with more tiles than that raises HQ_FLAG_BOUNDS.
 * Other errors as for hq_apply_layout. */
hq_status hq_apply_noalloc(hq_handle h, const void *v, void *out, int transpose, int64_t nrhs,
                           hq_precision prec, hq_layout layout, hq_stream stream);

/* The full orthogonal Q = [Q_Z; Q~] of every body (Algorithms 2 and 3 with
 * the root kept; Q_Z's six rows span the row space of Z, Eq. 1.2).
 *   transpose = 0: out = Q~ v as hq_apply_layout, and root receives Q_Z v,
 *                  each body's root Info-set (Definition 4.1).
 *   transpose = 1: root supplies each body's root Velocity-set L_root:
 *                  out = Q_Z^T root + Q~^T v (Algorithm 3, Theorem 4.3).
 *   root  device, 6 rows per body (6m rows x nrhs) in the call's layout:
 *         HQ_ROWS (6m x nrhs row-major) or HQ_TRIPLES (2m x nrhs x 3); for
 *         body j, rows 6j..6j+2 hold the sum of its bead rows over
 *         sqrt(n_j) (the translation part) and rows 6j+3..6j+5 the
 *         rotational part.  Must not overlap v or out.
 * Errors as for hq_apply_layout; HQ_E_INVALID if root is NULL or equals v or
 * out. */
hq_status hq_apply_full(hq_handle h, const void *v, void *out, void *root, int transpose, int64_t nrhs,
                        hq_precision prec, hq_layout layout, hq_stream stream);

/* Mobility product for hq_constrained_solve: y = D x for nrhs vectors of 3N
 * rows (the caller's bead order) in the solve's precision and layout.  x and
 * y are the device buffers dx and dy given to the solve; the callback may
 * run on the stream or synchronously, and returns 0 on success. */
typedef int (*hq_dapply_fn)(const void *x, void *y, int64_t nrhs, void *user, hq_stream stream);

typedef struct {
    int32_t max_iter;          /* in: CG iteration limit; 0 = 500 */
    double rtol;               /* in: relative residual target per RHS; 0 = 1e-8 */
    int32_t iters;             /* out: most iterations taken by one RHS */
    double max_rel_residual;   /* out: largest ||r|| / ||b|| over the RHS */
    int32_t check_every;       /* in: iterations between the host's convergence checks
                                  (1..64; 0 = 4) */
} hq_krylov_info;

/* The constrained Brownian-dynamics solve of Section 1: the constraint forces
 * g from 0 = Q~ D Q_Z^T F + Q~ D Q~^T g (Eq. 1.5) by conjugate gradients on
 * Q~ D Q~^T (symmetric positive definite when D is), then the rigid-body
 * velocities V = Q_Z D (Q_Z^T F + Q~^T g) (Eq. 1.6).  Q_Z and Q~ are this
 * handle's full Q (hq_apply_full); D is the caller's mobility (dapply).
 *   F   device, 6m x nrhs in the given layout (as hq_apply_full's root): the
 *       generalised forces in Q_Z's coordinates.
 *   V   device out, 6m x nrhs: the rigid-body velocities in the same
 *       coordinates.  g  device out, rows x nrhs.
 *   dx, dy  device workspace, 3N x nrhs elements each (caller-owned): the
 *       solve writes D's input into dx and calls dapply(dx, dy, ...).
 *   info  host, in/out (limits and results).
 * The CG scalars (one CG per right-hand side, FP64) stay on the device: a
 * column that has converged takes zero steps while others go on, and the host
 * synchronises the stream once every check_every iterations to read how many
 * columns are still active (so the loop may run up to check_every - 1
 * iterations past convergence without changing the results).  Allocates and
 * frees its own workspace (four vectors of rows x nrhs and the scalars),
 * unless the handle was built into a workspace with krylov_nrhs.
 * HQ_E_INVALID if an argument is NULL, the callback fails or Q~ D Q~^T is
 * not positive definite (reported at the next check); other errors as for
 * hq_apply_full. */
hq_status hq_constrained_solve(hq_handle h, hq_dapply_fn dapply, void *user, const void *F, void *V, void *g,
                               int64_t nrhs, hq_precision prec, hq_layout layout, void *dx, void *dy,
                               hq_krylov_info *info, hq_stream stream);

/* Products of rigidly moved bodies without a rebuild (reuse of the handle's
 * transforms): if body j moved to Rot_j r + t_j since the handle's last
 * hq_build / hq_rebuild (positions r), then Q~(moved) = Q~ blockdiag(Rot_j^T)
 * over its beads is an orthonormal basis of the complement of the moved
 * body's Z (Eq. 1.2: Z of the moved body is diag(Rot_j, Rot_j) Z
 * blockdiag(Rot_j^T) plus multiples of its translation rows).  It differs
 * from the Q~ a rebuild would give by an orthogonal change of rows; the
 * projector Q~^T Q~ is the same.
 *   transpose = 0: out = Q~ (blockdiag(Rot^T) v); work (device, 3N x nrhs,
 *                  distinct from v and out) may receive the rotated v.
 *   transpose = 1: out = blockdiag(Rot) (Q~^T v); work unused (may be NULL).
 * With the wide sweeps (32 or more right-hand sides) the rotations are
 * applied inside the sweeps as the bead vectors are read and written (no
 * extra pass over the vectors); otherwise in separate passes.
 *   rot  device m x 9 FP64 row-major: each body's rotation since the last
 *        build or rebuild (translations do not matter).
 * Vectors as for hq_apply_layout.  Capturable (no allocation once the
 * exchange buffer is reserved). */
hq_status hq_apply_rotated(hq_handle h, const double *rot, const void *v, void *out, void *work, int transpose,
                           int64_t nrhs, hq_precision prec, hq_layout layout, hq_stream stream);

/* Measurement form of hq_apply_layout (Algorithms 2 and 3): the same sweep, with a
 * HIP event recorded on the stream before each tile phase's launch and after
 * the last; waits for them and returns each phase's launch time in ms in
 * phase_ms[phase - 1] (host, max_phases entries; the downward sweep runs the
 * phases in reverse, the entries are still by phase) and the number of
 * phases in *nphases.  Creates and destroys its events; not for stream
 * capture.  Errors as for hq_apply; HQ_E_INVALID if max_phases is below the
 * handle's phases. */
hq_status hq_apply_timed(hq_handle h, const void *v, void *out, int transpose, int64_t nrhs,
                         hq_precision prec, hq_layout layout, hq_stream stream, float *phase_ms, int32_t max_phases,
                         int32_t *nphases);

/* Measurement helper for the sweeps' HBM roofline (Algorithms 2-3 stream
 * their vectors and node records once): one launch of a streaming kernel
 * that reads read_bytes from src and writes write_bytes to dst (a copy of
 * the first write_bytes; the rest is only read), 16 bytes per access with
 * the sweeps' non-temporal cache policy, blocks x 256 threads.  src, dst
 * device (distinct), sink device (4 bytes, written only if the data holds a
 * marker value).  Byte counts multiples of 16, write_bytes <= read_bytes.
 * Stream-ordered; the caller times it. */
hq_status hq_stream_ceiling(const void *src, size_t read_bytes, void *dst, size_t write_bytes, int32_t blocks,
                            void *sink, hq_stream stream);

/* Tile phase of every internal node of Section 2.1's tree (host, N - m
 * entries, the handle's node order; 1 = first phase): the launch that sweeps
 * it in Algorithms 2-3.  Synchronises the handle's stream. */
hq_status hq_node_phase(hq_handle h, int32_t *phase);

/* Dense Q~ of one body (Algorithm 1): out device FP64, (3n_j - 6) rows with
 * leading dimension ld >= 3n_j, columns in the caller's bead order.  A
 * two-bead body has no rows: HQ_OK without touching out (which may be NULL).
 * HQ_E_UNSUPPORTED when n_j exceeds explicit_dense_max_n. */
hq_status hq_explicit(hq_handle h, int64_t body, double *out, int64_t ld, hq_stream stream);

/* Block-sparse Q~ of one body in O(n log n) storage (Section 3, Algorithm
 * complexity).  Each internal node p with residue rows owns one dense block of
 * dim_p rows and 3 n_p columns: the rows are body rows row_off[b] ..
 * row_off[b] + rows[b] - 1 and the columns are the beads
 * hq_sorted_beads()[bead_first[b] .. bead_first[b] + cols[b]/3 - 1] (each bead
 * three columns x,y,z).  Q~ is zero outside the blocks.
 * hq_explicit_blocks_size gives the block count and the total value count;
 * hq_explicit_blocks fills values (device, prec's element type, blocks
 * row-major and concatenated) and the host arrays val_off (nblocks + 1),
 * row_off, bead_first (nblocks), rows and cols (nblocks).  Synchronises. */
hq_status hq_explicit_blocks_size(hq_handle h, int64_t body, int64_t *nblocks, int64_t *nvalues);
hq_status hq_explicit_blocks(hq_handle h, int64_t body, hq_precision prec, void *values,
                             int64_t *val_off, int64_t *row_off, int64_t *bead_first,
                             int32_t *rows, int32_t *cols, hq_stream stream);

/* The tree order of one body's beads (the leaves of Section 2.1's nested
 * boxes): host, n_j entries, the caller's bead index (0-based within the
 * body) of each tree leaf left to right.  Synchronises the handle's stream. */
hq_status hq_sorted_beads(hq_handle h, int64_t body, int64_t *bead_index);

/* Rigid motion of every body (a Brownian-dynamics step's position update):
 * r <- Rot_j (r - c_j) + c_j + t_j for the beads of body j, with c_j the
 * body centroid computed by the handle's last hq_build / hq_rebuild (state of
 * the handle, so a replayed capture continues from the last rebuild).
 * positions device N x 3 FP64 (in place), rot device m x 9 FP64 row-major,
 * trans device m x 3 FP64.  Capturable. */
hq_status hq_rigid_update(hq_handle h, double *positions, const double *rot,
                          const double *trans, hq_stream stream);

/* The same rigid motion about given centres, into another buffer:
 * out_k <- Rot_j (r_k - c_j) + c_j + t_j for the beads of body j.
 * positions device N x 3 FP64 (read), out device N x 3 FP64 (written; may be
 * positions itself), rot device m x 9 FP64 row-major, trans and centers device
 * m x 3 FP64.  It reads no state of the handle's last rebuild (only its body
 * ranges), so the motion of one step need not wait for the previous step's
 * rebuild: with two position buffers, consecutive steps' rebuilds can run
 * concurrently.  HQ_E_INVALID for a NULL pointer.  Capturable. */
hq_status hq_rigid_motion(hq_handle h, const double *positions, double *out, const double *rot,
                          const double *trans, const double *centers, hq_stream stream);

/* Sizes (Section 1: Q~ of body j has 3n_j - 6 rows), phase and tile counts,
 * conditioning of the per-node factorisations (Section 3) and device flags.
 * Synchronises the handle's stream (work queued on other streams must be
 * complete). */
hq_status hq_query(hq_handle h, hq_info *info);

/* Per-body flags and largest kappa(T22) over the nodes of Section 3's
 * factorisation (rank-5 bodies, Section 2.2): host arrays of m entries
 * (either may be NULL).  Synchronises the handle's stream. */
hq_status hq_body_info(hq_handle h, int32_t *flags, double *kappa);

/* Per-node data of Section 3's factorisation for tests, host arrays of N - m
 * entries in the handle's node order (any may be NULL): first/last sorted bead position within the body,
 * the children (>= 0: node index; < 0: -(sorted position within body) - 1),
 * body index, beads below, centroid (3, body-local: relative to the body's
 * lower corner), T22 (9, row-major), G (81, row-major k x k in the top-left),
 * k, and the first residue row within the body.  Synchronises.  Centroids and
 * T22 after an hq_rebuild need hq_options.keep_node_data (else HQ_E_INVALID).  Synchronises the handle's stream. */
hq_status hq_node_data(hq_handle h, int32_t *first, int32_t *last, int32_t *xchild,
                       int32_t *ychild, int32_t *body, int32_t *nbeads, double *centroid,
                       double *T22, double *G, int32_t *k, int32_t *row);

/* Stream capture helpers for repeated Brownian-dynamics steps (Section 1:
 * Q~ v and Q~^T v once per step): hipStreamBeginCapture / EndCapture /
 * hipGraphInstantiate / hipGraphLaunch; everything enqueued between begin
 * and end on the stream is recorded into *graph_exec, which replays it. */
hq_status hq_capture_begin(hq_stream stream);
hq_status hq_capture_end(hq_stream stream, void **graph_exec);
hq_status hq_graph_launch(void *graph_exec, hq_stream stream);
void hq_graph_destroy(void *graph_exec);

/* Destroy a handle (the end of Section 1's Q~ object): synchronise its
 * stream and free what it allocated (nothing on the device for a workspace
 * handle; NULL is accepted). */
void hq_destroy(hq_handle h);

/* The name of a status, and the thread's message of its last failing call
 * (the error behaviour stated at the top of this header). */
const char *hq_status_string(hq_status s);
const char *hq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HQ_H */
