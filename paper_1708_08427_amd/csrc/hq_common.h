// Internal declarations of the hq library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hq.h"

namespace hq {

// ---------------------------------------------------------------------------
// limits and layout constants
// ---------------------------------------------------------------------------
constexpr int kQBits = 21;              // quantisation bits per axis
constexpr int kSortChunk = 2048;        // largest segment sorted by one block (LDS bitonic sort)
constexpr int kMaxTileUnits = 1024;     // largest tile (units) supported
constexpr int kMaxPhases = 64;          // phase table capacity
constexpr int kRecWords = 32;           // elements (float or double) per node record
constexpr int kMaxDepth = 256;          // bound on tree depth walks (63 code bits + 32 index bits)
constexpr int kGenWords = 10;           // n, c[3], T22[6] per LDS slot and lane, and per tile root

// A node record (one per internal node, in schedule order) holds the three
// Householder reflectors of G in a zero-padded length-9 layout, the two
// translation weights and the links:
//   [0,8)   tail of reflector 0 (entries 1..8 of v_0; v_0[0] = 1)
//   [8,15)  tail of reflector 1 (entries 2..8 of v_1; v_1[1] = 1)
//   [15,21) tail of reflector 2 (entries 3..8 of v_2; v_2[2] = 1)
//   [21,24) tau_0, tau_1, tau_2
//   [24]    sx = sqrt(n_x / n)       [25]  sy = sqrt(n_y / n)
//   then six int32 links from element 26 on (the bytes of elements 26..31 of
//   a float record, 26..28 of a double record): xref, yref, off, meta,
//   slots (x slot | y slot << 8 | own slot << 16, LDS slots of the wide
//   sweeps), and the node's body (the row of its rigid-motion rotation).
constexpr int kRecTau = 21;
constexpr int kRecSx = 24;
constexpr int kRecSy = 25;
constexpr int kRecLinks = 26;
constexpr int kLinkInts = 6;

// Child references in the links:
//   ref >= 0   a bead: the caller's global bead index (vector row 3*ref)
//   ref == -1  an internal node of the same tile: taken from the tile stack
//   ref <= -2  the root of an earlier tile: exchange slot (-2 - ref)
constexpr int kRefStack = -1;
__host__ __device__ inline int ref_slot(int ref) { return -2 - ref; }

// meta bits
constexpr int kMetaTileRoot = 1;
constexpr int kMetaBodyRoot = 2;
constexpr int kMetaYFirst = 4;      // y's subtree is evaluated before x's
constexpr int kMetaSlotShift = 3;   // tile id (exchange slot) of a tile root

// device error flags (public values in hq.h)
constexpr int kFlagNonFinite = HQ_FLAG_NONFINITE;
constexpr int kFlagStack = HQ_FLAG_STACK;
constexpr int kFlagBounds = HQ_FLAG_BOUNDS;
constexpr int kFlagPhases = HQ_FLAG_PHASES;

// device counters (int32 array d_cnt)
enum Counter {
    kCntTiles = 0,      // tiles created so far
    kCntNodes = 1,      // internal nodes covered so far
    kCntPhases = 2,     // phases with at least one tile
    kCntRemain = 3,     // internal nodes still uncovered after the last phase
    kCntRemList = 4,    // length of the list of nodes left uncovered by the first phase
    kCntRuns = 5,       // run-table entries used so far
    kCntNum = 8
};

// Householder reflectors of a node record: tails start at element 0, 8, 15.
__host__ __device__ constexpr int tail_off(int j) { return j == 0 ? 0 : (j == 1 ? 8 : 15); }

// t <- G t = H_2 H_1 H_0 t on the first K entries (H_j = I - tau_j v_j v_j^T,
// v_j = e_j + tail_j on entries j+1 .. K-1).
template <int K, typename T>
__device__ __forceinline__ void house_fwd(T (&t)[9], const T *__restrict__ g) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const T *tl = g + tail_off(j);
        T w = t[j];
#pragma unroll
        for (int i = j + 1; i < K; ++i) w += tl[i - j - 1] * t[i];
        w *= g[kRecTau + j];
        t[j] -= w;
#pragma unroll
        for (int i = j + 1; i < K; ++i) t[i] -= w * tl[i - j - 1];
    }
}

// t <- G^T t = H_0 H_1 H_2 t on the first K entries.
template <int K, typename T>
__device__ __forceinline__ void house_bwd(T (&t)[9], const T *__restrict__ g) {
#pragma unroll
    for (int j = 2; j >= 0; --j) {
        const T *tl = g + tail_off(j);
        T w = t[j];
#pragma unroll
        for (int i = j + 1; i < K; ++i) w += tl[i - j - 1] * t[i];
        w *= g[kRecTau + j];
        t[j] -= w;
#pragma unroll
        for (int i = j + 1; i < K; ++i) t[i] -= w * tl[i - j - 1];
    }
}

inline int floor_log2(int v) {
    int r = -1;
    while (v) { v >>= 1; ++r; }
    return r;
}

// LDS stack depth for tiles of at most S units: heavy-first post-order needs
// at most floor(log2 S) + 1 pending results; one spare entry.
inline int stack_depth(int S) { return floor_log2(S) + 2; }

// Wide sweeps address LDS by slot: slots 0 .. floor(log2 S) hold the pending
// results of a tile.
inline int stack_slots(int S) { return floor_log2(S) + 1; }

// Leaf boxes: largest leaf size, and the values of one leaf record for
// leaves of up to smax beads (column-major 3 smax x 6 reflectors, 6 taus, pad)
constexpr int kMaxLeaf = 16;
inline int bucket_stride(int smax) { return 6 * 3 * smax + 8; }

// Run table: per phase (node begin, node end, first entry, runs, run length)
// at stride kPrunStride; a phase is cut into at least ~kRunTarget runs when it
// has that many tiles; run length 0: one run per tile (later phases of at most
// kRunTarget tiles).
constexpr int kPrunStride = 8;
constexpr int kRunTarget = 16384;

// ---------------------------------------------------------------------------
// the plan behind a handle
// ---------------------------------------------------------------------------
struct Plan {
    uint32_t magic = 0;
    int64_t N = 0, m = 0, NI = 0, rows = 0;
    int S = 256;   // tile size (units) of the first phase
    int S2 = 256;  // tile size of the later phases
    int smax() const { return S > S2 ? S : S2; }
    int store = 3;
    int dense_max_n = 4096;
    int phases_reserved = 0;  // phases launched by hq_rebuild
    int phases_built = 0;     // phases found by the last hq_build
    int64_t tiles_built = 0;
    int64_t tiles_ph[kMaxPhases] = {};  // tiles of each phase found by the last hq_build
    int max_n = 0;
    int run_nodes = 48;       // target nodes per run of whole tiles (wide sweeps)
    int waves_per_cu = 16;    // grid of the later phases' sweeps, waves per CU
    int first_wpc = 0;        // grid cap of the first phase's wide sweeps, waves per CU (0: none)
    int sweep_kernel = 0;     // 0: automatic; 1: a lane group per tile; 2: node-parallel; 3: wide
    int fused_up = 0;         // 1: the wide upward sweep in one launch; 0: one launch per tile phase
    int leaf_s = 1;           // leaf boxes hold up to leaf_s beads (>1: the first tile phase is leaves)
    int leaf_smax() const { return leaf_s <= 8 ? 8 : 16; }  // leaf-record layout and kernel instance
    int64_t tiles1_built = 0; // first-phase tiles (leaf boxes) of the last hq_build
    int64_t bucket_cap = 0;   // leaf-box records held
    double *d_brec64 = nullptr;  // leaf-box records (bucket_stride values each)
    float *d_brec32 = nullptr;
    int ncu = 256;            // compute units of the device
    bool keep_node_data = false;  // hq_rebuild writes per-node centroids and T22
    bool node_data_fresh = false; // they describe the last (re)build
    int64_t run_cap = 0;      // entries of d_run
    int64_t troot_cap = 0;    // tile-root table entries (twice the tiles of hq_build)

    std::vector<int64_t> offsets;  // host copy, m + 1
    std::vector<int64_t> row_off;  // host, m + 1

    // sort plan (host-side, static per handle)
    struct SortSegs { int nseg = 0; int32_t *d_seg = nullptr; };
    SortSegs sort_segs;    // (start, len, body or ~body for a chunk of a large body), longest first
    int large_passes = 0;                // merge passes for large bodies
    int64_t large_elems = 0;
    int nlarge = 0;
    int32_t *d_large = nullptr;          // (body index) list of large bodies
    int64_t *d_large_prefix = nullptr;   // prefix of element counts over the list

    // chunk table for per-bead body kernels: (body, begin, end) triples
    int nchunks = 0;
    int32_t *d_chunks = nullptr;

    // body level
    int32_t *d_bead_off = nullptr;   // m + 1
    int32_t *d_node_off = nullptr;   // m + 1 (internal node base: bead_off[j] - j)
    int32_t *d_row_off = nullptr;    // m + 1
    unsigned long long *d_bmin = nullptr, *d_bmax = nullptr;  // m x 3 ordered keys
    double *d_lo = nullptr;          // m x 3
    double *d_h = nullptr;           // m
    double *d_cen = nullptr;         // m x 3: centroid of the last build (absolute)
    unsigned long long *d_kappa = nullptr;  // m: bits of max kappa
    int32_t *d_bflags = nullptr;     // m

    // bead level
    unsigned long long *d_keyA = nullptr, *d_keyB = nullptr;
    int32_t *d_valA = nullptr, *d_valB = nullptr;
    unsigned long long *d_scode = nullptr;  // sorted codes
    int32_t *d_perm = nullptr;       // sorted global position -> caller's global bead index
    int32_t *d_leafpar = nullptr;    // sorted global position -> parent node
    int32_t *d_mark = nullptr, *d_msum = nullptr;  // flags and their scan (compaction)

    // node level (node g = internal node, Karras order per body)
    int32_t *d_lc = nullptr, *d_rc = nullptr, *d_par = nullptr;
    int32_t *d_first = nullptr, *d_last = nullptr;
    int32_t *d_nbody = nullptr;      // body of node
    int32_t *d_cov = nullptr;        // phase covering the node (0 = none yet)
    int32_t *d_units = nullptr;      // units below (current phase)
    int32_t *d_tileof = nullptr;
    int32_t *d_sched = nullptr;      // schedule index of node
    int32_t *d_yfirst = nullptr;
    int32_t *d_slot = nullptr;       // stack slot of the node's result inside its tile
    int2 *d_aw = nullptr;            // walk to the tile root: (parent, packed position step)
    int2 *d_lw = nullptr;            // walk to the body root: (parent, residue rows added)
    long long *d_trval = nullptr, *d_trscan = nullptr;  // packed (flag << 32 | len) and its scan
    int32_t *d_rem = nullptr;        // nodes left uncovered by the first phase, tree order
    int32_t *d_tord = nullptr;       // first-phase tiles, longest first (generation order)
    int32_t *d_lhist = nullptr, *d_lincl = nullptr;  // S x 256 length histograms and their scan
    int32_t *d_nn = nullptr;         // beads below
    double *d_ncen = nullptr;        // NI x 3 in schedule order, body-local
    double *d_T22 = nullptr;         // NI x 6 in schedule order, lower triangle packed (00,10,11,20,21,22)

    // tiles and schedule
    int32_t *d_tile_root = nullptr, *d_tile_base = nullptr, *d_tile_len = nullptr;
    int32_t *d_sched_node = nullptr; // schedule index -> node
    int32_t *d_ptile = nullptr;      // tile -> tile holding its root's parent (-1 at a body root)
    int32_t *d_tcnt = nullptr;       // tile -> child tiles yet to arrive in the fused upward sweep
    int32_t *d_tcnt0 = nullptr;      // tile -> child tiles (the counters' value between sweeps)
    int32_t *d_links = nullptr;      // schedule index -> int32[kLinkInts] links
    float *d_rec32 = nullptr;        // NI x 32
    double *d_rec64 = nullptr;       // NI x 32
    double *d_troot = nullptr;       // troot_cap x 10: (n, c[3], T22[6]) of each tile root

    int32_t *d_phase = nullptr;      // 2 x kMaxPhases: [begin, end) tile ids per phase
    int32_t *d_prun = nullptr;       // kPrunStride x kMaxPhases: node begin, node end, first run entry, runs, run length
    int32_t *d_run = nullptr;        // run_cap: first schedule index of each run (+ one end entry per phase)
    int32_t *d_cnt = nullptr;        // counters
    int32_t *d_err = nullptr;        // device error flags

    // scan scratch
    long long *d_scan_blk = nullptr;
    int64_t scan_blk_cap = 0;

    // exchange buffers
    void *d_xch = nullptr;
    float *d_rotf = nullptr;  // m x 9: the FP32 copy of a rigid-motion rotation table
    size_t xch_bytes = 0;

    // Device memory comes either from hipMalloc, one allocation per buffer
    // (hq_build; the handle frees them), or from one caller-owned workspace
    // carved into aligned pieces (hq_build_into; nothing is allocated, and
    // requests beyond the reserved sizes fail instead of growing a buffer).
    // sizing: only count the bytes the pieces take (hq_workspace_bytes).
    bool sizing = false;
    char *ws = nullptr;
    size_t ws_bytes = 0, ws_used = 0;
    int64_t *d_blk = nullptr;        // workspace: explicit-block offsets (max_n entries)
    void *d_kry = nullptr;           // workspace: Krylov vectors and scalars
    size_t kry_bytes = 0;
    hipStream_t stream = nullptr;    // the stream of hq_build / hq_build_into

    std::vector<void *> allocs;
};

// The plan behind a handle (nullptr, with the error set, for an invalid one).
Plan *plan_of(hq_handle h);
// Device memory of a handle: count elements from its workspace, or allocate.
hq_status plan_alloc(Plan &P, void **p, size_t bytes);

constexpr uint32_t kPlanMagic = 0x48514c42u;  // "HQLB"

// ---------------------------------------------------------------------------
// error handling helpers (host)
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);

#define HQ_HIP(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            ::hq::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            return HQ_E_DEVICE;                                               \
        }                                                                     \
    } while (0)

#define HQ_TRY(expr)                     \
    do {                                 \
        hq_status s_ = (expr);           \
        if (s_ != HQ_OK) return s_;      \
    } while (0)

// ---------------------------------------------------------------------------
// entry points between the library's own source files
// ---------------------------------------------------------------------------
hq_status scan_i32_inclusive(Plan &P, const int32_t *in, int32_t *out, int64_t n, hipStream_t s,
                             const int32_t *gate = nullptr);
hq_status scan_i64_exclusive(Plan &P, const long long *in, long long *out, int64_t n, hipStream_t s,
                             const int32_t *gate = nullptr, const int32_t *dn = nullptr);

hq_status build_device(Plan &P, const double *pos, hipStream_t s, bool probe_phases);
// rot: each body's rigid-motion rotation (m x 9 FP64, device) fused into the
// wide sweeps; HQ_E_UNSUPPORTED (nothing launched) when the sweeps are narrow
// xch, xch_bytes: the exchange buffer of the sweeps (nullptr: the handle's own)
hq_status apply_device(Plan &P, const void *v, void *out, void *root, int transpose, int64_t nrhs, int prec,
                       int layout, hipStream_t s, hipEvent_t *ev = nullptr, const double *rot = nullptr,
                       void *xch = nullptr, size_t xch_bytes = 0);
hq_status explicit_dense(Plan &P, int64_t body, double *out, int64_t ld, hipStream_t s);
hq_status explicit_blocks_launch(Plan &P, int64_t body, int prec, void *values, const int64_t *d_blk_off,
                                 hipStream_t s);
int64_t scan_blocks_needed(int64_t n);
// device bytes of the Krylov solve's work vectors and scalars
size_t krylov_bytes(int64_t rows, int64_t nrhs, size_t elem);
int lanes_per_tile(int64_t nrhs);
hq_status rigid_update(Plan &P, double *pos, const double *rot, const double *trans, hipStream_t s);
hq_status rigid_motion(Plan &P, const double *pin, double *pout, const double *rot, const double *trans,
                       const double *cen, hipStream_t s);
// in or out times blockdiag(Rot_j^T) (transpose = 1) or blockdiag(Rot_j) per body; in may equal out
hq_status rotate_vectors(Plan &P, const double *rot, const void *in, void *out, int64_t nrhs, int prec, int layout,
                         int transpose, hipStream_t s);

}  // namespace hq
