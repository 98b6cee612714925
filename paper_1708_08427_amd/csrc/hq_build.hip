// Setup of the hierarchical transforms on the GPU (Sections 2.1 and 3).
//
//   1. per-body bounding cube and 21-bit z-y-x interleaved box codes
//   2. per-body sort of (code, position in body): bitonic sort in LDS of up
//      to 2048 pairs per block, one launch for all bodies; larger bodies are
//      sorted in chunks of 2048 and merged pairwise
//   3. binary radix tree per body (Karras' construction on the sorted codes,
//      which is the nested-box bisection with empty halves pruned)
//   4. tiles: the tree is cut into connected pieces of at most S "units"
//      (beads or roots of earlier tiles); phase 1 takes the maximal subtrees
//      of at most S beads, later phases repeat on what remains.  Inside a tile
//      nodes are ordered by a post-order that visits the child with more
//      units first, so a sweep needs at most floor(log2 S) + 1 pending results.
//   5. per node in FP64: centroid, K = [T22_x | T22_y | sqrt(n_x n_y/n)
//      [c_x - c_y]x] (Eq. 3.5 with the leaf cases of Cases I and II) and its
//      Householder QR, giving T22 and G (Eqs. 3.6-3.8); FP64 and FP32 records
//      in schedule order.
#include "hq_buffer.h"
#include "hq_common.h"

#include <algorithm>
#include <climits>

namespace hq {

namespace {

constexpr int kThreads = 256;

__device__ inline unsigned long long ord_key(double x) {
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

__device__ inline double ord_val(unsigned long long k) {
    unsigned long long b = (k & 0x8000000000000000ull) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return __longlong_as_double((long long)b);
}

__device__ inline void raise_flag(int32_t *err, int f) { atomicOr(err, f); }

// ---------------------------------------------------------------------------
// initialisation
// ---------------------------------------------------------------------------

// Per-build reset of the node arrays the tiling fills in, the counters and
// the phase tables.
__global__ void k_init_nodes(int64_t NI, int32_t *cov, int32_t *tileof, int32_t *sched_node, int32_t *cnt,
                             int32_t *phase_tab, int32_t *prun) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t g = i0; g < NI; g += (int64_t)gridDim.x * blockDim.x) {
        cov[g] = 0;
        tileof[g] = -1;
        sched_node[g] = -1;
    }
    for (int64_t i = i0; i < kPrunStride * kMaxPhases; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < kCntNum) cnt[i] = 0;
        if (i < 2 * kMaxPhases) phase_tab[i] = 0;
        prun[i] = 0;
    }
}

__global__ void k_init_bodies(int64_t m, unsigned long long *bmin, unsigned long long *bmax,
                              unsigned long long *kappa, int32_t *bflags) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        for (int d = 0; d < 3; ++d) {
            bmin[3 * j + d] = ~0ull;
            bmax[3 * j + d] = 0ull;
        }
        kappa[j] = 0ull;
        bflags[j] = 0;
    }
}

// ---------------------------------------------------------------------------
// 1. bounding boxes and codes
// ---------------------------------------------------------------------------
__device__ inline double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ void __launch_bounds__(kThreads) k_bbox(const int32_t *__restrict__ chunks, const double *__restrict__ pos,
                                                   unsigned long long *bmin, unsigned long long *bmax, int32_t *err) {
    __shared__ double smn[3][kThreads / 64], smx[3][kThreads / 64];
    const int body = chunks[3 * blockIdx.x], b0 = chunks[3 * blockIdx.x + 1], b1 = chunks[3 * blockIdx.x + 2];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int i = b0 + threadIdx.x; i < b1; i += kThreads) {
        for (int d = 0; d < 3; ++d) {
            double x = pos[3 * (int64_t)i + d];
            if (!isfinite(x)) bad = true;
            mn[d] = fmin(mn[d], x);
            mx[d] = fmax(mx[d], x);
        }
    }
    if (bad) raise_flag(err, kFlagNonFinite);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int d = 0; d < 3; ++d) {
        double a = wave_min(mn[d]), b = wave_max(mx[d]);
        if (lane == 0) { smn[d][wid] = a; smx[d][wid] = b; }
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int d = threadIdx.x;
        double a = smn[d][0], b = smx[d][0];
        for (int w = 1; w < kThreads / 64; ++w) { a = fmin(a, smn[d][w]); b = fmax(b, smx[d][w]); }
        if (a <= b) {
            atomicMin(&bmin[3 * body + d], ord_key(a));
            atomicMax(&bmax[3 * body + d], ord_key(b));
        }
    }
}

// Spread the low 21 bits of x to every third bit.
__device__ inline unsigned long long spread3(unsigned long long x) {
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ inline unsigned int quantise(double x, double lo, double h) {
    if (!(h > 0.0)) return 0u;
    double t = ((x - lo) / h) * 2097152.0;  // 2^21
    double f = floor(t);
    f = fmin(fmax(f, 0.0), 2097151.0);
    return (unsigned int)f;
}

__global__ void __launch_bounds__(kThreads) k_codes(const int32_t *__restrict__ chunks, const int32_t *__restrict__ bead_off,
                                                    const double *__restrict__ pos, const unsigned long long *__restrict__ bmin,
                                                    const unsigned long long *__restrict__ bmax, double *lo_out, double *h_out,
                                                    unsigned long long *__restrict__ key, int32_t *__restrict__ val) {
    const int body = chunks[3 * blockIdx.x], b0 = chunks[3 * blockIdx.x + 1], b1 = chunks[3 * blockIdx.x + 2];
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = ord_val(bmin[3 * body + d]);
        hi[d] = ord_val(bmax[3 * body + d]);
    }
    double h = 0.0;
    for (int d = 0; d < 3; ++d) h = fmax(h, hi[d] - lo[d]);
    if (!(h >= 0.0)) h = 0.0;
    const int start = bead_off[body];
    if (b0 == start && threadIdx.x == 0) {
        for (int d = 0; d < 3; ++d) lo_out[3 * body + d] = lo[d];
        h_out[body] = h;
    }
    for (int i = b0 + threadIdx.x; i < b1; i += kThreads) {
        unsigned int qx = quantise(pos[3 * (int64_t)i + 0], lo[0], h);
        unsigned int qy = quantise(pos[3 * (int64_t)i + 1], lo[1], h);
        unsigned int qz = quantise(pos[3 * (int64_t)i + 2], lo[2], h);
        key[i] = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
        val[i] = i - start;
    }
}

// ---------------------------------------------------------------------------
// 2. per-body sort of (code, position in body)
// ---------------------------------------------------------------------------
__device__ inline bool key_less(unsigned long long ka, unsigned int va, unsigned long long kb, unsigned int vb) {
    return ka < kb || (ka == kb && va < vb);
}

// Length of the common prefix of the keys (code, position in the body) at i
// and j; -1 outside the body.
template <typename CodePtr>
__device__ inline int prefix_len(CodePtr sc, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    unsigned long long a = sc[i], b = sc[j];
    if (a != b) return __clzll((long long)(a ^ b));
    return 64 + __clz(i ^ j);
}

// Internal node i of one body in Karras' construction over the body's sorted
// codes sc (global memory or LDS), n beads, first bead base, first internal
// node g0: its children, parent links, bead range and walk words.
template <typename CodePtr>
__device__ __forceinline__ void karras_node(CodePtr sc, int n, int i, int base, int g0, int j, int32_t *lc,
                                            int32_t *rc, int32_t *par, int32_t *first, int32_t *last, int32_t *nn,
                                            int32_t *nbody, int32_t *leafpar, int2 *lw) {
    const int g = g0 + i;
    const int d = (prefix_len(sc, n, i, i + 1) - prefix_len(sc, n, i, i - 1)) > 0 ? 1 : -1;
    const int dmin = prefix_len(sc, n, i, i - d);
    int lmax = 2;
    while (prefix_len(sc, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(sc, n, i, i + (l + t) * d) > dmin) l += t;
    const int jj = i + l * d;
    const int dnode = prefix_len(sc, n, i, jj);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(sc, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int gamma = i + s * d + min(d, 0);
    const int lo = min(i, jj), hi = max(i, jj);
    int left, right;
    if (lo == gamma) {
        left = -(base + gamma) - 1;
        leafpar[base + gamma] = g;
    } else {
        left = g0 + gamma;
        par[left] = g;
    }
    if (hi == gamma + 1) {
        right = -(base + gamma + 1) - 1;
        leafpar[base + gamma + 1] = g;
    } else {
        right = g0 + gamma + 1;
        par[right] = g;
    }
    lc[g] = left;
    rc[g] = right;
    first[g] = base + lo;
    last[g] = base + hi;
    nn[g] = hi - lo + 1;
    nbody[g] = j;
    if (i == 0) {
        par[g] = -1;
        lw[g] = make_int2(-1, 0);
    }
    // residue rows that a walk from a child up to this node adds: this
    // node's own residue rows, and the x subtree's rows for the y child
    // (pre-order rows, Q~_p = [Residue_p; diag(Q~_x, Q~_y)])
    const int xi = left >= 0, yi = right >= 0;
    const int own = 3 * xi + 3 * yi;
    if (xi) lw[left] = make_int2(g, own);
    if (yi) lw[right] = make_int2(g, own + (xi ? 3 * (gamma - lo + 1) - 6 : 0));
}

// seg: (start, len, body) triples, len <= kSortChunk, longest first.  One block
// of kSortThreads threads per segment pads it to the next power of two (at
// least 128) and sorts it bitonically in LDS.  Pair p of a step with stride j
// is (i, i + j) with i = 2j floor(p / j) + p mod j; a thread takes pairs p,
// p + kSortThreads, ..., so for strides up to 64 the pairs of a wave stay
// inside 128-element blocks no other wave touches: those steps need no block
// barrier, only the wave's own ordering.  One launch covers all sizes, so the
// latency of the longest segments overlaps the work on the short ones.
// A segment of a whole body (body >= 0) writes sorted codes and the caller's
// bead index and builds the body's tree from the codes in LDS; a chunk of a
// larger body (stored as ~body) writes keys and values back in place for the
// merge passes (its tree is built after them).
constexpr int kSortThreads = 256;

__global__ void __launch_bounds__(kSortThreads) k_lds_sort(const int32_t *__restrict__ seg,
                                                           unsigned long long *keys, int32_t *vals,
                                                           const int32_t *__restrict__ bead_off,
                                                           unsigned long long *scode, int32_t *perm, int32_t *lc,
                                                           int32_t *rc, int32_t *par, int32_t *first,
                                                           int32_t *last, int32_t *nn, int32_t *nbody,
                                                           int32_t *leafpar, int2 *lw) {
    __shared__ unsigned long long K[kSortChunk];
    __shared__ unsigned int V[kSortChunk];
    const int start = seg[3 * blockIdx.x], len = seg[3 * blockIdx.x + 1], bcode = seg[3 * blockIdx.x + 2];
    const bool final_out = bcode >= 0;
    const int body = final_out ? bcode : ~bcode;
    int npad = 128;
    while (npad < len) npad <<= 1;
    if (npad > kSortChunk) return;  // never: segments are cut on the host
    for (int i = threadIdx.x; i < npad; i += kSortThreads) {
        if (i < len) {
            K[i] = keys[start + i];
            V[i] = (unsigned int)vals[start + i];
        } else {
            K[i] = ~0ull;
            V[i] = 0xffffffffu;
        }
    }
    __syncthreads();
    const int half = npad >> 1;
    for (int k = 2; k <= npad; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int lj = 31 - __builtin_clz(j);
            for (int p = threadIdx.x; p < half; p += kSortThreads) {
                const int i = ((p >> lj) << (lj + 1)) | (p & (j - 1)), ixj = i + j;
                const unsigned long long ka = K[i], kb = K[ixj];
                const unsigned int va = V[i], vb = V[ixj];
                const bool up = (i & k) == 0;
                if (key_less(kb, vb, ka, va) == up) {
                    K[i] = kb;
                    K[ixj] = ka;
                    V[i] = vb;
                    V[ixj] = va;
                }
            }
            const int jn = (j > 1) ? (j >> 1) : k;  // stride of the next step
            if (j >= 128 || jn >= 128) {
                __syncthreads();
            } else {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    __syncthreads();
    if (final_out) {
        const int base = bead_off[body];
        for (int i = threadIdx.x; i < len; i += kSortThreads) {
            scode[start + i] = K[i];
            perm[start + i] = base + (int)V[i];
        }
        // the body's tree, from the sorted codes still in LDS
        for (int i = threadIdx.x; i < len - 1; i += kSortThreads)
            karras_node(K, len, i, base, base - body, body, lc, rc, par, first, last, nn, nbody, leafpar, lw);
    } else {
        for (int i = threadIdx.x; i < len; i += kSortThreads) {
            keys[start + i] = K[i];
            vals[start + i] = (int)V[i];
        }
    }
}

__device__ inline int find_large(const int64_t *prefix, int nlarge, int64_t e) {
    int lo = 0, hi = nlarge - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// One pairwise merge of sorted runs of length L inside each large body; an
// element's output position is its rank in its run plus the number of smaller
// elements in the partner run (keys are unique).
__global__ void k_merge_pass(const int32_t *__restrict__ large, const int64_t *__restrict__ prefix, int nlarge,
                             int64_t total, const int32_t *__restrict__ bead_off, int L,
                             const unsigned long long *__restrict__ kin, const int32_t *__restrict__ vin,
                             unsigned long long *__restrict__ kout, int32_t *__restrict__ vout) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int li = find_large(prefix, nlarge, e);
        const int body = large[li];
        const int start = bead_off[body], n = bead_off[body + 1] - start;
        const int i = (int)(e - prefix[li]);
        const int r = i / L, partner = r ^ 1;
        const int pstart = partner * L;
        const unsigned long long k = kin[start + i];
        const int v = vin[start + i];
        if (pstart >= n) {
            kout[start + i] = k;
            vout[start + i] = v;
            continue;
        }
        const int plen = min(L, n - pstart);
        int lo = 0, hi = plen;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            unsigned long long pk = kin[start + pstart + mid];
            unsigned int pv = (unsigned int)vin[start + pstart + mid];
            if (key_less(pk, pv, k, (unsigned int)v)) lo = mid + 1; else hi = mid;
        }
        const int out = min(r, partner) * L + (i - r * L) + lo;
        kout[start + out] = k;
        vout[start + out] = v;
    }
}

__global__ void k_large_final(const int32_t *__restrict__ large, const int64_t *__restrict__ prefix, int nlarge,
                              int64_t total, const int32_t *__restrict__ bead_off,
                              const unsigned long long *__restrict__ kin, const int32_t *__restrict__ vin,
                              unsigned long long *__restrict__ scode, int32_t *__restrict__ perm) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int li = find_large(prefix, nlarge, e);
        const int body = large[li];
        const int start = bead_off[body];
        const int i = (int)(e - prefix[li]);
        scode[start + i] = kin[start + i];
        perm[start + i] = start + vin[start + i];
    }
}

// ---------------------------------------------------------------------------
// 3. binary radix tree (Karras 2012) over each body's sorted keys
// ---------------------------------------------------------------------------
// Trees of the bodies sorted in chunks and merged (the large-body list with
// its bead prefix; body li holds n - 1 internal nodes).
__global__ void k_tree_large(const int32_t *__restrict__ large, const int64_t *__restrict__ prefix, int nlarge,
                             int64_t total_nodes, const int32_t *__restrict__ bead_off,
                             const unsigned long long *__restrict__ scode, int32_t *lc, int32_t *rc, int32_t *par,
                             int32_t *first, int32_t *last, int32_t *nn, int32_t *nbody, int32_t *leafpar,
                             int2 *lw) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total_nodes;
         e += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = nlarge - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] - mid <= e) lo = mid; else hi = mid - 1;
        }
        const int j = large[lo];
        const int base = bead_off[j], n = bead_off[j + 1] - base;
        karras_node(scode + base, n, (int)(e - (prefix[lo] - lo)), base, base - j, j, lc, rc, par, first, last, nn,
                    nbody, leafpar, lw);
    }
}

// ---------------------------------------------------------------------------
// 4. tiles
// ---------------------------------------------------------------------------
// units of a child of an uncovered node: a bead or an earlier tile's root
// counts as one unit
__device__ inline int child_units(int c, const int32_t *cov, const int32_t *units) {
    if (c < 0) return 1;
    if (cov[c] != 0) return 1;
    return units[c];
}

// Later phases iterate over the nodes the first phase left uncovered (a few
// percent of all nodes), listed once in tree order: rem = null means all nodes
// in order.  dn holds the list's length on the device.
__device__ __forceinline__ int64_t node_count(int64_t NI, const int32_t *dn) {
    return dn ? min(NI, (int64_t)max(*dn, 0)) : NI;
}
__device__ __forceinline__ int node_at(int64_t i, const int32_t *rem) { return rem ? rem[i] : (int)i; }

__global__ void k_rem_scatter(int64_t NI, const int32_t *cov, const int32_t *pos, int32_t *rem, int32_t *cnt,
                              const int32_t *gate) {
    if (gate && *gate == 0) return;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < NI; g += (int64_t)gridDim.x * blockDim.x) {
        if (cov[g] == 0) rem[pos[g] - 1] = (int)g;
        if (g == NI - 1) cnt[kCntRemList] = pos[g];
    }
}

// Units of the uncovered nodes after the first phase (beads and roots of
// earlier tiles count one each): every uncovered node adds the units among its
// own children to itself and to all its ancestors, which are uncovered too.
__device__ __forceinline__ void units_walk_at(int64_t i, int64_t NI, const int32_t *rem, const int32_t *cov,
                                              const int32_t *lc, const int32_t *rc, const int32_t *par,
                                              int32_t *units, int32_t *err) {
    const int g = node_at(i, rem);
    if (cov[g] != 0) return;
    const int x = lc[g], y = rc[g];
    const int c = ((x < 0 || cov[x] != 0) ? 1 : 0) + ((y < 0 || cov[y] != 0) ? 1 : 0);
    if (c == 0) return;
    int q = g;
    for (int guard = 0; q >= 0; ++guard) {
        if (guard == kMaxDepth || q >= NI) {
            raise_flag(err, kFlagBounds);
            break;
        }
        atomicAdd(&units[q], c);
        q = par[q];
    }
}

__global__ void k_units_walk(int64_t NI, const int32_t *rem, const int32_t *dn, const int32_t *cov,
                             const int32_t *lc, const int32_t *rc, const int32_t *par, int32_t *units,
                             int32_t *err, const int32_t *gate) {
    if (gate && *gate == 0) return;
    const int64_t n = node_count(NI, dn);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        units_walk_at(i, NI, rem, cov, lc, rc, par, units, err);
}

__device__ __forceinline__ void tile_roots_at(int64_t i, const int32_t *rem, int phase, int S, const int32_t *cov,
                                              const int32_t *par, const int32_t *nn, int32_t *units,
                                              long long *trval) {
    const int g = node_at(i, rem);
    if (cov[g] != 0) {
        trval[i] = 0;
        return;
    }
    // first phase: every bead is a unit; later: counted by k_units_walk
    const int u = (phase == 1) ? nn[g] : units[g];
    const int p = par[g];
    const int up = (p < 0) ? INT_MAX : ((phase == 1) ? nn[p] : units[p]);
    if (phase == 1) units[g] = u;
    const bool root = (u <= S) && (up > S);
    trval[i] = root ? ((1ll << 32) | (long long)(u - 1)) : 0ll;
}

__global__ void k_tile_roots(int64_t NI, const int32_t *rem, const int32_t *dn, int phase, int S,
                             const int32_t *cov, const int32_t *par, const int32_t *nn, int32_t *units,
                             long long *trval, const int32_t *gate) {
    if (gate && *gate == 0) return;
    const int64_t n = node_count(NI, dn);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        tile_roots_at(i, rem, phase, S, cov, par, nn, units, trval);
}

// Per uncovered node: evaluation order of its children (the one with more
// units first) and the step of the walk up to its tile root: its parent, the
// post-order positions skipped when it is its parent's second child (the
// first child's subtree), whether that first child is an internal node of the
// tile (one more pending result on the stack), and whether it is a tile root.
// Word layout: bits 0..28 positions skipped (clamped: only walks that end in a
// tile use the value, and there it is below the tile size), bit 29 the pending
// flag, bit 30 the tile-root flag.
constexpr int kAwPend = 1 << 29, kAwRoot = 1 << 30, kAwSkip = (1 << 29) - 1;

// A tile root also enters its tile in the tile tables: root, node count and
// first schedule index (from the scan of the root flags and node counts).
__device__ __forceinline__ void assign_prep_at(int64_t i, const int32_t *rem, const int32_t *cov,
                                               const int32_t *par, const int32_t *lc, const int32_t *rc,
                                               const int32_t *units, const long long *trval,
                                               const long long *trscan, int tiles0, int nodes0, int32_t *tile_root,
                                               int32_t *tile_len, int32_t *tile_base, int32_t *tileof,
                                               int32_t *yfirst, int2 *aw) {
    const int g = node_at(i, rem);
    if (cov[g] != 0) return;
    const long long tv = trval[i];
    if (tv != 0) {
        const long long sc = trscan[i];
        const int t = tiles0 + (int)(sc >> 32);
        tile_root[t] = g;
        tile_len[t] = (int)(tv & 0xffffffffll);
        tile_base[t] = nodes0 + (int)(sc & 0xffffffffll);
        tileof[g] = t;
    }
    {
        const int ux = child_units(lc[g], cov, units), uy = child_units(rc[g], cov, units);
        yfirst[g] = (uy > ux) ? 1 : 0;
    }
    const int p = par[g];
    int word = (tv != 0) ? kAwRoot : 0;
    if (p >= 0) {
        const int x = lc[p], y = rc[p];
        const int ux = child_units(x, cov, units), uy = child_units(y, cov, units);
        const bool y_first = uy > ux;
        if (g == (y_first ? x : y)) {
            const int ufirst = y_first ? uy : ux;
            word |= min(ufirst - 1, kAwSkip) | ((ufirst > 1) ? kAwPend : 0);
        }
    }
    aw[g] = make_int2(p, word);
}

__global__ void k_assign_prep(int64_t NI, const int32_t *rem, const int32_t *dn, const int32_t *cov,
                              const int32_t *par, const int32_t *lc, const int32_t *rc, const int32_t *units,
                              const long long *trval, const long long *trscan, const int32_t *cnt,
                              int32_t *tile_root, int32_t *tile_len, int32_t *tile_base, int32_t *tileof,
                              int32_t *yfirst, int2 *aw, const int32_t *gate) {
    if (gate && *gate == 0) return;
    const int tiles0 = cnt[kCntTiles], nodes0 = cnt[kCntNodes];
    const int64_t n = node_count(NI, dn);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        assign_prep_at(i, rem, cov, par, lc, rc, units, trval, trscan, tiles0, nodes0, tile_root, tile_len, tile_base,
                       tileof, yfirst, aw);
}

// The first phase in two passes instead of three.  With every node still
// uncovered, a node's units are its bead count (nn), so the per-node steps of
// k_assign_prep (child order, the walk word) need no earlier pass and join
// k_tile_roots; and k_assign finds a tile's index and first schedule slot in
// the scan of the root flags at the root itself (the list of nodes is the
// identity in the first phase), where the root also enters its tile.  It
// also flags the nodes it leaves for the later phases (left), the input of
// their list.
__device__ __forceinline__ int first_units(int c, const int32_t *nn) { return c < 0 ? 1 : nn[c]; }

__global__ void k_tile_roots1(int64_t NI, int S, const int32_t *par, const int32_t *lc, const int32_t *rc,
                              const int32_t *nn, int32_t *units, long long *trval, int32_t *yfirst, int2 *aw) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NI; i += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)i;
        const int u = nn[g];
        const int p = par[g];
        const int up = (p < 0) ? INT_MAX : nn[p];
        units[g] = u;
        const bool root = (u <= S) && (up > S);
        trval[i] = root ? ((1ll << 32) | (long long)(u - 1)) : 0ll;
        yfirst[g] = (first_units(rc[g], nn) > first_units(lc[g], nn)) ? 1 : 0;
        int word = root ? kAwRoot : 0;
        if (p >= 0) {
            const int x = lc[p], y = rc[p];
            const int ux = first_units(x, nn), uy = first_units(y, nn);
            const bool y_first = uy > ux;
            if (g == (y_first ? x : y)) {
                const int ufirst = y_first ? uy : ux;
                word |= min(ufirst - 1, kAwSkip) | ((ufirst > 1) ? kAwPend : 0);
            }
        }
        aw[g] = make_int2(p, word);
    }
}

__global__ void k_assign1(int64_t NI, int32_t *cov, int32_t *units, const int2 *aw, const long long *trval,
                          const long long *trscan, const int32_t *cnt, int32_t *tile_root, int32_t *tile_len,
                          int32_t *tile_base, int32_t *tileof, int32_t *sched, int32_t *sched_node,
                          int32_t *depth_slot, int32_t *left, int32_t *err, int64_t sched_cap) {
    const int tiles0 = cnt[kCntTiles], nodes0 = cnt[kCntNodes];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NI; i += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)i;
        int pos = units[g] - 2, pend = 0;
        int q = g;
        bool found = false;
        bool too_deep = true;
        for (int guard = 0; guard < kMaxDepth; ++guard) {
            const int2 w = aw[q];
            if (w.y & kAwRoot) { found = true; too_deep = false; break; }
            if (w.x < 0) { too_deep = false; break; }
            pos += w.y & kAwSkip;
            pend += (w.y & kAwPend) ? 1 : 0;
            q = w.x;
        }
        if (too_deep) raise_flag(err, kFlagBounds);
        // a node above every tile root is left for the next phase, which
        // counts its units afresh
        if (!found) {
            units[g] = 0;
            left[g] = 1;
            continue;
        }
        const long long sc = trscan[q];
        const int t = tiles0 + (int)(sc >> 32);
        const int64_t base = (int64_t)nodes0 + (int)(sc & 0xffffffffll);
        const int64_t s = base + pos;
        if (t < 0 || t >= NI || pos < 0 || s < 0 || s >= sched_cap) {
            raise_flag(err, kFlagBounds);
            units[g] = 0;
            left[g] = 1;
            continue;
        }
        left[g] = 0;
        if (q == g) {
            tile_root[t] = g;
            tile_len[t] = (int)(trval[g] & 0xffffffffll);
            tile_base[t] = (int)base;
        }
        tileof[g] = t;
        depth_slot[g] = pend;
        sched[g] = (int)s;
        sched_node[s] = g;
        cov[g] = 1;
    }
}

// The later phases likewise (after k_units_walk, every unit count is
// final): k_tile_roots_l adds the per-node steps of k_assign_prep and records
// each root's place in the node list (ridx), and k_assign_l reads the root's
// tile index and base from the scan there.
__global__ void k_tile_roots_l(int64_t NI, const int32_t *rem, const int32_t *dn, int S, const int32_t *cov,
                               const int32_t *par, const int32_t *lc, const int32_t *rc, const int32_t *units,
                               long long *trval, int32_t *yfirst, int2 *aw, int32_t *ridx, const int32_t *gate) {
    if (gate && *gate == 0) return;
    const int64_t n = node_count(NI, dn);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int g = node_at(i, rem);
        if (cov[g] != 0) {
            trval[i] = 0;
            continue;
        }
        const int u = units[g];
        const int p = par[g];
        const int up = (p < 0) ? INT_MAX : units[p];
        const bool root = (u <= S) && (up > S);
        trval[i] = root ? ((1ll << 32) | (long long)(u - 1)) : 0ll;
        if (root) ridx[g] = (int)i;
        {
            const int ux = child_units(lc[g], cov, units), uy = child_units(rc[g], cov, units);
            yfirst[g] = (uy > ux) ? 1 : 0;
        }
        int word = root ? kAwRoot : 0;
        if (p >= 0) {
            const int x = lc[p], y = rc[p];
            const int ux = child_units(x, cov, units), uy = child_units(y, cov, units);
            const bool y_first = uy > ux;
            if (g == (y_first ? x : y)) {
                const int ufirst = y_first ? uy : ux;
                word |= min(ufirst - 1, kAwSkip) | ((ufirst > 1) ? kAwPend : 0);
            }
        }
        aw[g] = make_int2(p, word);
    }
}

__global__ void k_assign_l(int64_t NI, const int32_t *rem, const int32_t *dn, int phase, int32_t *cov,
                           int32_t *units, const int2 *aw, const long long *trval, const long long *trscan,
                           const int32_t *ridx, const int32_t *cnt, int32_t *tile_root, int32_t *tile_len,
                           int32_t *tile_base, int32_t *tileof, int32_t *sched, int32_t *sched_node,
                           int32_t *depth_slot, int32_t *err, int64_t sched_cap, const int32_t *gate) {
    if (gate && *gate == 0) return;
    const int tiles0 = cnt[kCntTiles], nodes0 = cnt[kCntNodes];
    const int64_t n = node_count(NI, dn);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int g = node_at(i, rem);
        if (cov[g] != 0) continue;
        int pos = units[g] - 2, pend = 0;
        int q = g;
        bool found = false;
        bool too_deep = true;
        for (int guard = 0; guard < kMaxDepth; ++guard) {
            const int2 w = aw[q];
            if (w.y & kAwRoot) { found = true; too_deep = false; break; }
            if (w.x < 0) { too_deep = false; break; }
            pos += w.y & kAwSkip;
            pend += (w.y & kAwPend) ? 1 : 0;
            q = w.x;
        }
        if (too_deep) raise_flag(err, kFlagBounds);
        const int iq = found ? ridx[q] : -1;
        if (!found || iq < 0 || iq >= n) {
            if (found) raise_flag(err, kFlagBounds);
            units[g] = 0;
            continue;
        }
        const long long sc = trscan[iq];
        const int t = tiles0 + (int)(sc >> 32);
        const int64_t base = (int64_t)nodes0 + (int)(sc & 0xffffffffll);
        const int64_t s = base + pos;
        if (t < 0 || t >= NI || pos < 0 || s < 0 || s >= sched_cap) {
            raise_flag(err, kFlagBounds);
            units[g] = 0;
            continue;
        }
        if (q == g) {
            tile_root[t] = g;
            tile_len[t] = (int)(trval[i] & 0xffffffffll);
            tile_base[t] = (int)base;
        }
        tileof[g] = t;
        depth_slot[g] = pend;
        sched[g] = (int)s;
        sched_node[s] = g;
        cov[g] = phase;
    }
}

// Post-order position of every uncovered node inside the tile whose root it
// reaches first going up (the child with more units is evaluated first), and
// the stack slot that receives its result (results of the tile pending while
// its subtree is swept).  A node placed in a tile is covered by this phase; a
// node left over gets its unit count cleared for the next phase's count.
__device__ __forceinline__ void assign_at(int64_t i, int64_t NI, const int32_t *rem, int phase, int32_t *cov,
                                          int32_t *units, const int2 *aw, const int32_t *tile_base, int32_t *tileof,
                                          int32_t *sched, int32_t *sched_node, int32_t *depth_slot, int32_t *err,
                                          int64_t sched_cap) {
    const int g = node_at(i, rem);
    if (cov[g] != 0) return;
    int pos = units[g] - 2, pend = 0;
    int q = g;
    bool found = false;
    bool too_deep = true;
    for (int guard = 0; guard < kMaxDepth; ++guard) {
        const int2 w = aw[q];
        if (w.y & kAwRoot) { found = true; too_deep = false; break; }
        if (w.x < 0) { too_deep = false; break; }
        pos += w.y & kAwSkip;
        pend += (w.y & kAwPend) ? 1 : 0;
        q = w.x;
    }
    if (too_deep) raise_flag(err, kFlagBounds);
    bool placed = false;
    if (found) {
        const int t = tileof[q];
        const int64_t s = (t >= 0 && t < NI) ? (int64_t)tile_base[t] + pos : -1;
        if (t < 0 || t >= NI || pos < 0 || s < 0 || s >= sched_cap) {
            raise_flag(err, kFlagBounds);
        } else {
            tileof[g] = t;
            depth_slot[g] = pend;
            sched[g] = (int)s;
            sched_node[s] = g;
            cov[g] = phase;
            placed = true;
        }
    }
    if (!placed) units[g] = 0;
}

__global__ void k_assign(int64_t NI, const int32_t *rem, const int32_t *dn, int phase, int32_t *cov,
                         int32_t *units, const int2 *aw, const int32_t *tile_base, int32_t *tileof,
                         int32_t *sched, int32_t *sched_node, int32_t *depth_slot, int32_t *err, int64_t sched_cap,
                         const int32_t *gate) {
    if (gate && *gate == 0) return;
    const int64_t n = node_count(NI, dn);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        assign_at(i, NI, rem, phase, cov, units, aw, tile_base, tileof, sched, sched_node, depth_slot, err, sched_cap);
}

__device__ __forceinline__ void phase_close_one(int64_t NI, const int32_t *dn, int phase, const long long *trval,
                                                const long long *trscan, int32_t *cnt, int32_t *phase_tab,
                                                int run_nodes, int32_t *prun, int64_t run_cap, int32_t *err) {
    const int64_t n = node_count(NI, dn);
    const long long tot = (n > 0) ? trscan[n - 1] + trval[n - 1] : 0;
    const int ntiles = (int)(tot >> 32), nnodes = (int)(tot & 0xffffffffll);
    phase_tab[2 * phase] = cnt[kCntTiles];
    phase_tab[2 * phase + 1] = cnt[kCntTiles] + ntiles;
    // runs: the first phase's schedule range cut at tile starts every ~tp
    // nodes (a small phase gets shorter runs so that it still spreads over
    // kRunTarget lane groups).  A later phase of at most kRunTarget tiles gets
    // exactly one run per tile (tp = 0): cut every tp nodes, its tiles of
    // 10-31 nodes left empty runs between them, so most waves swept one tile
    // with half their lanes idle and the phase needed two rounds of waves
    const bool per_tile = phase > 1 && ntiles <= kRunTarget;
    const int tp = per_tile ? 0 : max(1, min(run_nodes, (nnodes + kRunTarget - 1) / kRunTarget));
    const int p0 = cnt[kCntNodes], c0 = cnt[kCntRuns];
    int nrun = per_tile ? ntiles : (nnodes + tp - 1) / tp;
    if ((int64_t)c0 + nrun + 1 > run_cap) {
        raise_flag(err, kFlagBounds);
        nrun = -1;
    }
    prun[kPrunStride * phase] = p0;
    prun[kPrunStride * phase + 1] = p0 + nnodes;
    prun[kPrunStride * phase + 2] = c0;
    prun[kPrunStride * phase + 3] = max(nrun, 0);
    prun[kPrunStride * phase + 4] = tp;
    if (nrun >= 0) cnt[kCntRuns] = c0 + nrun + 1;
    cnt[kCntTiles] += ntiles;
    cnt[kCntNodes] += nnodes;
    if (ntiles > 0) cnt[kCntPhases] = phase;
    cnt[kCntRemain] = (int)(NI - cnt[kCntNodes]);
}

__global__ void k_phase_close(int64_t NI, const int32_t *dn, int phase, const long long *trval,
                              const long long *trscan, int32_t *cnt, int32_t *phase_tab, int run_nodes,
                              int32_t *prun, int64_t run_cap, int32_t *err, const int32_t *gate) {
    if (gate && *gate == 0) return;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    phase_close_one(NI, dn, phase, trval, trscan, cnt, phase_tab, run_nodes, prun, run_cap, err);
}

// Run starts of one phase: run c begins at the first tile that starts at or
// after node c * tp of the phase (phase end if none), so every run holds
// whole tiles and a lane group can sweep it as one node stream; with tp = 0
// run c is tile c of the phase.
__device__ __forceinline__ void runs_range(int phase, const int32_t *phase_tab, const int32_t *tile_base,
                                           const int32_t *prun, int32_t *run, int64_t first, int64_t stride) {
    const int tb = phase_tab[2 * phase], te = phase_tab[2 * phase + 1];
    const int *pr = prun + kPrunStride * phase;
    const int p0 = pr[0], p1 = pr[1], c0 = pr[2], nrun = pr[3], tp = max(pr[4], 1);
    if (nrun == 0 && p1 > p0) return;  // table full: flagged by k_phase_close
    if (pr[4] == 0) {
        for (int64_t tt = first; tt <= te - tb; tt += stride) {
            const int t = tb + (int)tt;
            run[c0 + tt] = (t < te) ? tile_base[t] : p1;
        }
        return;
    }
    for (int64_t tt = first; tt <= te - tb; tt += stride) {
        const int t = tb + (int)tt;
        const int st = (t < te) ? tile_base[t] - p0 : p1 - p0;
        const int lo = (t == tb) ? 0 : (tile_base[t - 1] - p0) / tp + 1;
        const int hi = (t < te) ? min(st / tp, nrun - 1) : nrun;
        for (int c = lo; c <= hi; ++c) run[c0 + c] = p0 + st;
    }
}

__global__ void k_runs(int phase, const int32_t *phase_tab, const int32_t *tile_base, const int32_t *prun,
                       int32_t *run, const int32_t *gate) {
    if (gate && *gate == 0) return;
    runs_range(phase, phase_tab, tile_base, prun, run, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
               (int64_t)gridDim.x * blockDim.x);
}

// Exclusive scan of in[0, n) into out by one workgroup (every thread calls
// it): a contiguous chunk per thread, the chunk sums scanned in LDS.
__device__ void block_exscan_i64(const long long *in, long long *out, int64_t n, long long *part) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t chunk = (n + nt - 1) / nt;
    const int64_t b = tid * chunk, e = min(n, b + chunk);
    long long sum = 0;
    for (int64_t i = b; i < e; ++i) sum += in[i];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const long long v = (tid >= off) ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    long long run = (tid > 0) ? part[tid - 1] : 0;
    for (int64_t i = b; i < e; ++i) {
        out[i] = run;
        run += in[i];
    }
}

// Tile phases ph0..ph1 of a rebuild in one workgroup (one launch instead of
// about nine per phase), for the reserved phases: a phase without nodes ends
// at once.  The same per-node steps as the multi-workgroup kernels, separated
// by workgroup barriers; the phase loop stops when no node is left.
constexpr int kTailThreads = 1024;

__global__ void __launch_bounds__(kTailThreads) k_tail_phases(
    int ph0, int ph1, int64_t NI, const int32_t *rem, const int32_t *dn, int S, int32_t *cov, const int32_t *par,
    const int32_t *lc, const int32_t *rc, const int32_t *nn, int32_t *units, long long *trval, long long *trscan,
    int32_t *cnt, int32_t *tile_root, int32_t *tile_len, int32_t *tile_base, int32_t *tileof, int32_t *yfirst,
    int2 *aw, int32_t *sched, int32_t *sched_node, int32_t *depth_slot, int64_t sched_cap, int32_t *phase_tab,
    int run_nodes, int32_t *prun, int64_t run_cap, int32_t *run, int32_t *err) {
    __shared__ long long part[kTailThreads];
    __shared__ int live;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int ph = ph0; ph <= ph1; ++ph) {
        __syncthreads();
        if (tid == 0) live = cnt[kCntRemain];
        __syncthreads();
        if (live == 0) break;
        const int64_t n = node_count(NI, dn);
        for (int64_t i = tid; i < n; i += nt) units_walk_at(i, NI, rem, cov, lc, rc, par, units, err);
        __syncthreads();
        for (int64_t i = tid; i < n; i += nt) tile_roots_at(i, rem, ph, S, cov, par, nn, units, trval);
        __syncthreads();
        block_exscan_i64(trval, trscan, n, part);
        __syncthreads();
        const int tiles0 = cnt[kCntTiles], nodes0 = cnt[kCntNodes];
        for (int64_t i = tid; i < n; i += nt)
            assign_prep_at(i, rem, cov, par, lc, rc, units, trval, trscan, tiles0, nodes0, tile_root, tile_len,
                           tile_base, tileof, yfirst, aw);
        __syncthreads();
        for (int64_t i = tid; i < n; i += nt)
            assign_at(i, NI, rem, ph, cov, units, aw, tile_base, tileof, sched, sched_node, depth_slot, err,
                      sched_cap);
        __syncthreads();
        if (tid == 0) phase_close_one(NI, dn, ph, trval, trscan, cnt, phase_tab, run_nodes, prun, run_cap, err);
        __syncthreads();
        if (prun[kPrunStride * ph + 1] != 0) runs_range(ph, phase_tab, tile_base, prun, run, tid, nt);
    }
}

// First residue row of every tile root (pre-order rows, Section 3's
// Q~_p = [Residue_p; diag(Q~_x, Q~_y)]): its walk up to the body root.  Other
// nodes then only walk up to their own tile root.
__global__ void k_troot_off(int64_t NI, const int32_t *cnt, const int32_t *tile_root, const int2 *lw,
                            const int32_t *nbody, const int32_t *row_off, int32_t *toff, int32_t *err) {
    // (also the check that the phases covered every node)
    if (blockIdx.x == 0 && threadIdx.x == 0 && cnt[kCntRemain] != 0) raise_flag(err, kFlagPhases);
    const int nt = cnt[kCntTiles];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
        const int r = tile_root[t];
        if (r < 0 || r >= NI) {
            raise_flag(err, kFlagBounds);
            continue;
        }
        int off = 0, q = r;
        for (int guard = 0;; ++guard) {
            if (guard == kMaxDepth) {
                raise_flag(err, kFlagBounds);
                break;
            }
            const int2 w = lw[q];
            if (w.x < 0) break;
            off += w.y;
            q = w.x;
        }
        toff[t] = off + row_off[nbody[r]];
    }
}

// Links of every node: child references, residue row (pre-order, Section 3's
// Q~_p = [Residue_p; diag(Q~_x, Q~_y)]) and flags.
__global__ void k_links(int64_t NI, const int32_t *cov, const int32_t *tileof, const int32_t *sched,
                        const int32_t *lc, const int32_t *rc, const int32_t *par, const int32_t *nn,
                        const int32_t *nbody, const int32_t *yfirst, const int32_t *tile_root,
                        const int32_t *perm, const int32_t *toff, const int32_t *depth_slot, int dstack,
                        const int2 *lw, int32_t *links, int32_t *err) {
    for (int64_t gg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gg < NI; gg += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)gg;
        if (cov[g] == 0) continue;
        const int t = tileof[g];
        int ref[2];
        const int ch[2] = {lc[g], rc[g]};
        for (int c = 0; c < 2; ++c) {
            const int x = ch[c];
            if (x < 0) ref[c] = perm[-(x + 1)];
            else if (cov[x] == cov[g] && tileof[x] == t) ref[c] = kRefStack;
            else ref[c] = -2 - tileof[x];
        }
        // residue rows before this node: the walk up to its tile root, plus
        // the tile root's own offset
        const int r = (t >= 0 && t < NI) ? tile_root[t] : -1;
        int off = 0, q = g;
        for (int guard = 0; q != r; ++guard) {
            if (guard == kMaxDepth || q < 0) {
                raise_flag(err, kFlagBounds);
                break;
            }
            const int2 w = lw[q];
            off += w.y;
            q = w.x;
        }
        if (r >= 0) off += toff[t];
        int meta = 0;
        if (tile_root[t] == g) meta |= kMetaTileRoot | (t << kMetaSlotShift);
        if (par[g] < 0) meta |= kMetaBodyRoot;
        if (yfirst[g]) meta |= kMetaYFirst;
        // LDS slots of the wide sweeps (dstack of them): the child evaluated
        // first sits in this node's own slot, the second one above it; bead
        // and earlier-tile children, and the result of a tile root, name
        // slot 0, which the sweeps never write for them
        const int own = depth_slot[g];
        const bool xin = ref[0] == kRefStack, yin = ref[1] == kRefStack;
        const bool yf = yfirst[g] != 0;
        const bool fin = yf ? yin : xin;
        int xs = 0, ys = 0;
        if (xin) xs = yf ? own + (fin ? 1 : 0) : own;
        if (yin) ys = yf ? own : own + (fin ? 1 : 0);
        const bool troot = (meta & kMetaTileRoot) != 0;
        const int os = troot ? 0 : own;
        if ((xin && xs >= dstack) || (yin && ys >= dstack) || (!troot && own >= dstack)) raise_flag(err, kFlagStack);
        const int s = sched[g];
        links[kLinkInts * s + 0] = ref[0];
        links[kLinkInts * s + 1] = ref[1];
        links[kLinkInts * s + 2] = off;
        links[kLinkInts * s + 3] = meta;
        links[kLinkInts * s + 4] = xs | (ys << 8) | (os << 16);
        links[kLinkInts * s + 5] = nbody[g];
    }
}

// ---------------------------------------------------------------------------
// 5. FP64 transforms (Eqs. 3.4-3.13)
// ---------------------------------------------------------------------------
// Reciprocal and square root from the hardware approximations refined by
// Newton steps (two for the reciprocal, one coupled step for the root),
// which leaves them within about an ulp of the rounded values at a third of
// the instructions of the IEEE sequences; arguments here are positive and
// normal.
__device__ __forceinline__ double rcp_nr(double b) {
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double sqrt_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    g = fma(d, h, g);
    return x > 0.0 ? g : 0.0;
}

// Condition number of the lower-triangular T22 (its singular values are
// those of K).  With S = T^T T, the smallest eigenvalue is the first root of
// the characteristic cubic, approached from 0 by Newton's method: the cubic
// is convex there, so the iterates stay below the root and the result stays
// an upper bound (six steps leave it within 4% of the converged value, also
// for a double root).  The largest is bounded by trace(S).  Returns
// sqrt(trace / lambda_min), an upper bound of sigma_1 / sigma_3 within a
// factor 1.04 sqrt(3); a huge value for a singular T22.
__device__ double cond_bound3(const double T[6]) {
    const double a = T[0], b = T[1], c = T[2], d = T[3], e = T[4], f = T[5];
    const double s00 = a * a + b * b + d * d, s01 = b * c + d * e, s02 = d * f;
    const double s11 = c * c + e * e, s12 = e * f, s22 = f * f;
    const double c2 = s00 + s11 + s22;
    const double c1 = s00 * s11 - s01 * s01 + s00 * s22 - s02 * s02 + s11 * s22 - s12 * s12;
    const double det = a * c * f;
    const double c0 = det * det;
    if (!(c0 > 0.0) || !(c2 > 0.0)) return 1e300;
    double lam = 0.0;
#pragma unroll
    for (int it = 0; it < 6; ++it) {
        const double p = ((-lam + c2) * lam - c1) * lam + c0;
        const double dp = (-3.0 * lam + 2.0 * c2) * lam - c1;
        lam = fma(-p, rcp_nr(dp), lam);
    }
    if (!(lam > 0.0)) return 1e300;
    return sqrt_nr(c2 * rcp_nr(lam));
}

// Transforms of one node (Eqs. 3.4-3.13).  A = K^T with the blocks of
// internal children first, then the shift block D = sqrt(n_x n_y / n)
// [c_x - c_y]x; rows beyond k stay zero, so reflectors of length 9 act as
// the length-k ones.
__device__ __forceinline__ void put_lower(double (&A)[9][3], int r0, const double *T) {
    // K block column jj = column jj of the lower-triangular T22 -> A row r0+jj
    A[r0 + 0][0] = T[0]; A[r0 + 0][1] = T[1]; A[r0 + 0][2] = T[3];
    A[r0 + 1][0] = 0.0;  A[r0 + 1][1] = T[2]; A[r0 + 1][2] = T[4];
    A[r0 + 2][0] = 0.0;  A[r0 + 2][1] = 0.0;  A[r0 + 2][2] = T[5];
}

__device__ __forceinline__ void put_shift(double (&A)[9][3], int r0, double sc, const double *dv) {
    A[r0 + 0][0] = 0.0;          A[r0 + 0][1] = sc * dv[2];   A[r0 + 0][2] = -sc * dv[1];
    A[r0 + 1][0] = -sc * dv[2];  A[r0 + 1][1] = 0.0;          A[r0 + 1][2] = sc * dv[0];
    A[r0 + 2][0] = sc * dv[1];   A[r0 + 2][1] = -sc * dv[0];  A[r0 + 2][2] = 0.0;
}

// Householder QR of A (9 x 3, rows beyond k zero) in place, LAPACK sign
// convention (tau = 0 for a zero tail): the scaled tail of reflector j
// replaces column j below the diagonal; T = R^T packed lower-triangular.
__device__ __forceinline__ void householder_qr(double (&A)[9][3], double (&tau)[3], double (&T)[6], int k) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double alpha = A[j][j];
        double xs = 0.0;
#pragma unroll
        for (int r = j + 1; r < 9; ++r) xs = fma(A[r][j], A[r][j], xs);
        if (xs == 0.0) {
            tau[j] = 0.0;
            continue;
        }
        const double nrm = sqrt_nr(fma(alpha, alpha, xs));
        const double beta = (alpha >= 0.0) ? -nrm : nrm;
        tau[j] = (beta - alpha) * rcp_nr(beta);
        const double scal = rcp_nr(alpha - beta);
#pragma unroll
        for (int r = j + 1; r < 9; ++r) A[r][j] *= scal;
        A[j][j] = beta;
#pragma unroll
        for (int l = j + 1; l < 3; ++l) {
            double w = A[j][l];
#pragma unroll
            for (int r = j + 1; r < 9; ++r) w = fma(A[r][j], A[r][l], w);
            w *= tau[j];
            A[j][l] -= w;
#pragma unroll
            for (int r = j + 1; r < 9; ++r) A[r][l] = fma(-w, A[r][j], A[r][l]);
        }
    }
    T[0] = A[0][0];
    T[1] = A[0][1];
    T[2] = A[1][1];
    T[3] = A[0][2];
    T[4] = A[1][2];
    T[5] = (k == 3) ? 0.0 : A[2][2];  // Case I: rank 2, third column exactly 0 (Eq. 3.9)
}

// Tiles of one phase ordered longest first (a counting sort on the node
// count, kLenBlocks blocks each taking a contiguous share of the tiles), so
// that the lanes of a generation wave walk tiles of about the same length.
constexpr int kLenBlocks = 256;

__global__ void __launch_bounds__(256) k_len_hist(int phase, const int32_t *phase_tab, const int32_t *tile_len,
                                                  int nbins, int32_t *hist) {
    __shared__ int32_t h[kMaxTileUnits];
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int tb = phase_tab[2 * phase], te = phase_tab[2 * phase + 1];
    const int C = (te - tb + kLenBlocks - 1) / kLenBlocks;
    const int a = tb + blockIdx.x * C, b = min(te, a + C);
    for (int t = a + threadIdx.x; t < b; t += blockDim.x)
        atomicAdd(&h[nbins - 1 - min(max(tile_len[t], 0), nbins - 1)], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) hist[i * kLenBlocks + blockIdx.x] = h[i];
}

__global__ void __launch_bounds__(256) k_len_scatter(int phase, const int32_t *phase_tab, const int32_t *tile_len,
                                                     int nbins, const int32_t *hist, const int32_t *incl,
                                                     int32_t *tord) {
    __shared__ int32_t cur[kMaxTileUnits];
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) {
        const int q = i * kLenBlocks + blockIdx.x;
        cur[i] = incl[q] - hist[q];
    }
    __syncthreads();
    const int tb = phase_tab[2 * phase], te = phase_tab[2 * phase + 1];
    const int C = (te - tb + kLenBlocks - 1) / kLenBlocks;
    const int a = tb + blockIdx.x * C, b = min(te, a + C);
    for (int t = a + threadIdx.x; t < b; t += blockDim.x)
        tord[tb + atomicAdd(&cur[nbins - 1 - min(max(tile_len[t], 0), nbins - 1)], 1)] = t;
}

// ---------------------------------------------------------------------------
// Transforms tile by tile: one lane per tile of a phase walks the tile's nodes
// in schedule order (children before parents, the order of the upward sweep).
// A child of the same tile is read from the lane's LDS slot (the slot numbers
// of the wide sweeps), the root of an earlier phase's tile from the tile-root
// table, a bead from the positions.  The loop is software-pipelined: while a
// node is computed, the children of the next node and the links of the one
// after it are in flight.
// ---------------------------------------------------------------------------
constexpr int kStageStride = 36;  // words per lane row of the record staging area (144 B)
constexpr size_t kStageBytes = (size_t)64 * kStageStride * 4 + 64 * 4;  // rows + schedule offsets

struct GenIn {
    double n, c[3], T[6];
};

__device__ __forceinline__ void gen_slot_put(double *lds, int slot, int lane, double n, const double (&c)[3],
                                             const double (&T)[6]) {
    double *p = lds + slot * kGenWords * 64 + lane;
    p[0] = n;
#pragma unroll
    for (int d = 0; d < 3; ++d) p[(1 + d) * 64] = c[d];
#pragma unroll
    for (int d = 0; d < 6; ++d) p[(4 + d) * 64] = T[d];
}

__device__ __forceinline__ void gen_slot_get(const double *lds, int slot, int lane, GenIn &o) {
    const double *p = lds + slot * kGenWords * 64 + lane;
    o.n = p[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) o.c[d] = p[(1 + d) * 64];
#pragma unroll
    for (int d = 0; d < 6; ++d) o.T[d] = p[(4 + d) * 64];
}

// Child data that lives in HBM: a bead (n = 1, absolute position, T22 = 0)
// or, after the first phase, an earlier tile's root (n, body-local centroid,
// T22).  The loads are issued unconditionally from clamped addresses and the
// result is selected afterwards, so no branch separates a load from its use
// (a same-tile child is replaced by the LDS read at compute time).
template <bool kLater>
__device__ __forceinline__ void gen_fetch(int ref, const double *pos, const double *troot, int64_t N, int64_t ntr,
                                          GenIn &o, bool &bad) {
    const bool bead = ref >= 0;
    bad |= ref >= N || (!kLater && ref < kRefStack) || (ref < kRefStack && ref_slot(ref) >= ntr);
    const int64_t u = bead ? min((int64_t)ref, N - 1) : 0;
    double p[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) p[d] = pos[3 * u + d];
    if (!kLater) {
        o.n = 1.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) o.c[d] = p[d];
#pragma unroll
        for (int d = 0; d < 6; ++d) o.T[d] = 0.0;
        return;
    }
    const int64_t t = (ref < kRefStack) ? min((int64_t)ref_slot(ref), ntr - 1) : 0;
    const double *q = troot + kGenWords * t;
    double w[kGenWords];
#pragma unroll
    for (int e = 0; e < kGenWords; ++e) w[e] = q[e];
    o.n = bead ? 1.0 : w[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) o.c[d] = bead ? p[d] : w[1 + d];
#pragma unroll
    for (int d = 0; d < 6; ++d) o.T[d] = bead ? 0.0 : w[4 + d];
}

// A same-tile child from the LDS slot (read unconditionally, then selected);
// a bead's position made body-local.
__device__ __forceinline__ void gen_child_fix(int ref, int slot, const double *lds, int lane, const double (&lo3)[3],
                                              GenIn &o) {
    GenIn l;
    gen_slot_get(lds, slot, lane, l);
    const bool st = ref == kRefStack, bead = ref >= 0;
    o.n = st ? l.n : o.n;
#pragma unroll
    for (int d = 0; d < 3; ++d) o.c[d] = st ? l.c[d] : (bead ? o.c[d] - lo3[d] : o.c[d]);
#pragma unroll
    for (int d = 0; d < 6; ++d) o.T[d] = st ? l.T[d] : o.T[d];
}

__device__ __forceinline__ void load_links(const int32_t *links, int64_t s, int32_t (&li)[kLinkInts]) {
    const int4 a = *reinterpret_cast<const int4 *>(links + kLinkInts * s);
    const int2 b = *reinterpret_cast<const int2 *>(links + kLinkInts * s + 4);
    li[0] = a.x;
    li[1] = a.y;
    li[2] = a.z;
    li[3] = a.w;
    li[4] = b.x;
    li[5] = b.y;
}

// One node's transform from its two children (Eqs. 3.4-3.13): its bead
// count and body-local centroid, the Householder QR of its k x 3 block K
// (the children's T22 blocks, or nothing for a bead, above the scaled
// centroid difference), its T22, the 26 record words (reflectors below the
// diagonal, tau, the two child weights sqrt(n_x / n) and sqrt(n_y / n)) and
// a bound on the condition number of T22.
__device__ __forceinline__ void gen_node(const GenIn &cx, const GenIn &cy, bool xi, bool yi, double &n,
                                         double (&cp)[3], double (&T)[6], double (&w64)[26], double &kap, int &k) {
    n = cx.n + cy.n;
    const double rn = rcp_nr(n);
    double dv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        cp[d] = (cx.n * cx.c[d] + cy.n * cy.c[d]) * rn;
        dv[d] = cx.c[d] - cy.c[d];
    }
    const double sc = sqrt_nr(cx.n * cy.n * rn);
    double A[9][3];
#pragma unroll
    for (int r = 0; r < 9; ++r) A[r][0] = A[r][1] = A[r][2] = 0.0;
    if (xi && yi) {
        put_lower(A, 0, cx.T);
        put_lower(A, 3, cy.T);
        put_shift(A, 6, sc, dv);
        k = 9;
    } else if (xi) {
        put_lower(A, 0, cx.T);
        put_shift(A, 3, sc, dv);
        k = 6;
    } else if (yi) {
        put_lower(A, 0, cy.T);
        put_shift(A, 3, sc, dv);
        k = 6;
    } else {
        put_shift(A, 0, sc, dv);
        k = 3;
    }
    double tau[3];
    householder_qr(A, tau, T, k);
    const double sx = sqrt_nr(cx.n * rn), sy = sqrt_nr(cy.n * rn);
    kap = (k > 3) ? cond_bound3(T) : 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) w64[e] = A[1 + e][0];
#pragma unroll
    for (int e = 8; e < 15; ++e) w64[e] = A[2 + (e - 8)][1];
#pragma unroll
    for (int e = 15; e < 21; ++e) w64[e] = A[3 + (e - 15)][2];
#pragma unroll
    for (int e = 21; e < 24; ++e) w64[e] = tau[e - 21];
    w64[24] = sx;
    w64[25] = sy;
}

// The stores of one node; an index of kOOB switches a group off.  The
// prologue of the node loop issues the same stores switched off, so that the
// compiler sees the same number of stores in flight on entry to the loop as
// on its back edge and waits for loads only.
template <int kStore, bool kNodes>
__device__ __forceinline__ void gen_store(rsrc_t r32, rsrc_t r64, rsrc_t rcen, rsrc_t rt22, rsrc_t rtr, rsrc_t rbc,
                                          uint32_t *stage, uint32_t *srel, int lane, uint32_t rel, uint32_t trel,
                                          uint32_t brel, const float (&w32)[26],
                                          const double (&w64)[26], const int32_t (&li)[kLinkInts],
                                          const double (&cp)[3], const double (&T)[6], const double (&tv)[kGenWords],
                                          const double (&bc)[3]) {
    auto scaled = [](uint32_t i, uint32_t b) { return i == kOOB ? kOOB : i * b; };
    if (kStore & 2) {
        // the 64 lanes' float records pass through LDS (one row per lane) and
        // leave as whole 128-byte lines: lanes 8i..8i+7 write record i of the
        // step, eight records per store
        u32x4 *row = reinterpret_cast<u32x4 *>(stage + kStageStride * lane);
#pragma unroll
        for (int q = 0; q < 6; ++q)
            row[q] = u32x4{__float_as_uint(w32[4 * q]), __float_as_uint(w32[4 * q + 1]),
                           __float_as_uint(w32[4 * q + 2]), __float_as_uint(w32[4 * q + 3])};
        row[6] = u32x4{__float_as_uint(w32[24]), __float_as_uint(w32[25]), (uint32_t)li[0], (uint32_t)li[1]};
        row[7] = u32x4{(uint32_t)li[2], (uint32_t)li[3], (uint32_t)li[4], (uint32_t)li[5]};
        srel[lane] = rel;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int c = lane & 7;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int r = 8 * q + (lane >> 3);
            const u32x4 v = reinterpret_cast<const u32x4 *>(stage + kStageStride * r)[c];
            const uint32_t rr = srel[r];
            __builtin_amdgcn_raw_buffer_store_b128(v, r32, rr == kOOB ? kOOB : rr * 128u + 16u * c, 0, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if (kStore & 1) {
        const uint32_t o = scaled(rel, 256u);
#pragma unroll
        for (int e = 0; e < 13; ++e) {
            const u32x2 a = __builtin_bit_cast(u32x2, w64[2 * e]), b = __builtin_bit_cast(u32x2, w64[2 * e + 1]);
            __builtin_amdgcn_raw_buffer_store_b128(u32x4{a.x, a.y, b.x, b.y}, r64, o + 16 * e, 0, 0);
        }
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{(uint32_t)li[0], (uint32_t)li[1], (uint32_t)li[2], (uint32_t)li[3]},
                                               r64, o + 208, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b64(u32x2{(uint32_t)li[4], (uint32_t)li[5]}, r64, o + 224, 0, 0);
    }
    auto pair = [](double a, double b) {
        const u32x2 x = __builtin_bit_cast(u32x2, a), y = __builtin_bit_cast(u32x2, b);
        return u32x4{x.x, x.y, y.x, y.y};
    };
    if (kNodes) {
        const uint32_t oc = scaled(rel, 24u), ot = scaled(rel, 48u);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, cp[0]), rcen, oc, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b128(pair(cp[1], cp[2]), rcen, oc + 8, 0, 0);
#pragma unroll
        for (int d = 0; d < 3; ++d) __builtin_amdgcn_raw_buffer_store_b128(pair(T[2 * d], T[2 * d + 1]), rt22, ot + 16 * d, 0, 0);
    }
    // tile root: (n, c, T22) for the phases above
    const uint32_t otr = scaled(trel, 80u);
#pragma unroll
    for (int e = 0; e < kGenWords / 2; ++e)
        __builtin_amdgcn_raw_buffer_store_b128(pair(tv[2 * e], tv[2 * e + 1]), rtr, otr + 16 * e, 0, 0);
    // body root: the body's centroid (absolute)
    const uint32_t ob = scaled(brel, 24u);
    __builtin_amdgcn_raw_buffer_store_b128(pair(bc[0], bc[1]), rbc, ob, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, bc[2]), rbc, ob + 16, 0, 0);
}

// Records, node data and tile-root entries leave through buffer stores whose
// resources start at the wave's first tile (all of a wave's tiles follow it
// in schedule order, tile order and body order, so offsets stay far below
// 2 GiB); a lane with nothing to write gets the offset kOOB.  Every store is
// therefore issued unconditionally and waiting for the next node's children
// never waits for this node's stores.
template <bool kLater, int kStore, bool kNodes>
__global__ void __launch_bounds__(64) k_gen_tile(int phase, const int32_t *phase_tab, const int32_t *tile_base,
                                                 const int32_t *tile_len, const int32_t *tile_root,
                                                 const int32_t *links, const int32_t *nbody, const double *pos,
                                                 const double *lo, double *troot, int64_t ntr, int nslot,
                                                 double *ncen, double *T22, float *rec32, double *rec64,
                                                 double *bcen, unsigned long long *kappa, int32_t *bflags,
                                                 const int32_t *tord, int64_t m, int64_t N, int64_t NI,
                                                 int32_t *err) {
    extern __shared__ unsigned char smem_raw[];
    double *lds = reinterpret_cast<double *>(smem_raw);
    // record staging after the nslot slots of pending results
    uint32_t *stage = reinterpret_cast<uint32_t *>(smem_raw + (size_t)nslot * kGenWords * 64 * sizeof(double));
    uint32_t *srel = stage + 64 * kStageStride;
    const int lane = threadIdx.x;
    const int tb = phase_tab[2 * phase], te = phase_tab[2 * phase + 1];
    // tord: the phase's tiles longest first (then every buffer is addressed
    // from its start, which the host checked stays below 2 GiB); otherwise
    // tiles in order, addressed from the wave's first tile
    const bool sorted = tord != nullptr;
    bool bad = false;
    for (int t0 = tb + blockIdx.x * 64; t0 < te; t0 += gridDim.x * 64) {
        const int t = (sorted && t0 + lane < te) ? tord[t0 + lane] : t0 + lane;
        int s = 0, se = 0, body = 0;
        if (t < te) {
            const int base = tile_base[t], len = tile_len[t], r = tile_root[t];
            if (base < 0 || len < 1 || (int64_t)base + len > NI || r < 0 || r >= NI) {
                bad = true;
            } else {
                s = base;
                se = base + len;
                body = nbody[r];
            }
        }
        if (body < 0 || body >= m) {
            bad = true;
            s = se = body = 0;
        }
        // wave-uniform bases: the first tile's schedule index, tile id, body
        const int s0 = sorted ? 0 : __builtin_amdgcn_readfirstlane(s);
        const int b0 = sorted ? 0 : __builtin_amdgcn_readfirstlane(body);
        const int tr0 = sorted ? 0 : t0;
        // every offset below stays under 2 GiB: at most 2^23 records of 256 B
        // and 2^24 bodies of 24 B from the wave's bases
        if (s < se && (s < s0 || se - s0 > (1 << 23) || body < b0 || body - b0 > (1 << 24) || t < tr0 ||
                       t - tr0 > (1 << 24))) {
            bad = true;
            s = se = 0;
        }
        // byte sizes in integer arithmetic, capped below 2 GiB
        auto cap = [](int64_t bytes) -> uint32_t {
            return bytes <= 0 ? 0u : (bytes >= 0x7fffffffll ? 0x7fffffffu : (uint32_t)bytes);
        };
        const int64_t t0c = tr0 < ntr ? tr0 : ntr;
        const rsrc_t r32 = make_rsrc_uniform(rec32 + (int64_t)kRecWords * s0, cap((NI - s0) * 128));
        const rsrc_t r64 = make_rsrc_uniform(rec64 + (int64_t)kRecWords * s0, cap((NI - s0) * 256));
        const rsrc_t rcen = make_rsrc_uniform(ncen + 3 * (int64_t)s0, cap((NI - s0) * 24));
        const rsrc_t rt22 = make_rsrc_uniform(T22 + 6 * (int64_t)s0, cap((NI - s0) * 48));
        const rsrc_t rtr = make_rsrc_uniform(troot + kGenWords * t0c, cap((ntr - t0c) * 80));
        const rsrc_t rbc = make_rsrc_uniform(bcen + 3 * (int64_t)b0, cap((m - b0) * 24));
        double lo3[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) lo3[d] = lo[3 * body + d];
        double kmax = 0.0;
        bool deg = false;
        // pipeline: the links two nodes ahead and the children one node ahead
        // are in flight while a node is computed
        int32_t li[kLinkInts], ln[kLinkInts];
        load_links(links, min((int64_t)s, NI - 1), li);
        GenIn cx, cy;
        bool bad0 = false;
        gen_fetch<kLater>(li[0], pos, troot, N, ntr, cx, bad0);
        gen_fetch<kLater>(li[1], pos, troot, N, ntr, cy, bad0);
        bad |= s < se && bad0;
        load_links(links, min((int64_t)s + 1, NI - 1), ln);
        {
            const float z32[26] = {};
            const double z64[26] = {}, z3[3] = {}, z6[6] = {}, z10[kGenWords] = {};
            gen_store<kStore, kNodes>(r32, r64, rcen, rt22, rtr, rbc, stage, srel, lane, kOOB, kOOB, kOOB, z32, z64, li, z3, z6,
                                      z10, z3);
        }
        while (__ballot(s < se)) {
            const bool act = s < se, actn = s + 1 < se;
            GenIn cxn, cyn;
            bool badn = false;
            gen_fetch<kLater>(ln[0], pos, troot, N, ntr, cxn, badn);
            gen_fetch<kLater>(ln[1], pos, troot, N, ntr, cyn, badn);
            bad |= actn && badn;
            int32_t lnn[kLinkInts];
            load_links(links, min((int64_t)s + 2, NI - 1), lnn);
            // --- this node (Eqs. 3.4-3.13)
            const int xs = min(li[4] & 0xff, nslot - 1), ys = min((li[4] >> 8) & 0xff, nslot - 1);
            const int os = min((li[4] >> 16) & 0xff, nslot - 1);
            gen_child_fix(li[0], xs, lds, lane, lo3, cx);
            gen_child_fix(li[1], ys, lds, lane, lo3, cy);
            const bool xi = li[0] < 0, yi = li[1] < 0;
            double n, cp[3], T[6], w64[26], kap;
            int k;
            gen_node(cx, cy, xi, yi, n, cp, T, w64, kap, k);
            const bool troot_node = (li[3] & kMetaTileRoot) != 0, body_root = (li[3] & kMetaBodyRoot) != 0;
            // the result waits in the node's slot for its parent (a tile
            // root's slot is never read again, nor is an idle lane's)
            gen_slot_put(lds, os, lane, n, cp, T);
            if (act) {
                kmax = fmax(kmax, kap);
                deg |= body_root && (k == 3 || kap > 1e12);
            }
            // --- stores of this node
            {
                float w32[26];
#pragma unroll
                for (int e = 0; e < 26; ++e) w32[e] = (float)w64[e];
                const int64_t tr = li[3] >> kMetaSlotShift;
                const bool wr = act && troot_node && tr == t && t < ntr;
                bad |= act && troot_node && (tr != t || t >= ntr);
                const uint32_t rel = (uint32_t)(s - s0);
                const double tv[kGenWords] = {n, cp[0], cp[1], cp[2], T[0], T[1], T[2], T[3], T[4], T[5]};
                const double bc[3] = {cp[0] + lo3[0], cp[1] + lo3[1], cp[2] + lo3[2]};
                gen_store<kStore, kNodes>(r32, r64, rcen, rt22, rtr, rbc, stage, srel, lane, act ? rel : kOOB, wr ? (uint32_t)(t - tr0) : kOOB,
                                  (act && body_root) ? (uint32_t)(body - b0) : kOOB, w32, w64, li, cp, T, tv, bc);
            }
#pragma unroll
            for (int q = 0; q < kLinkInts; ++q) {
                li[q] = ln[q];
                ln[q] = lnn[q];
            }
            cx = cxn;
            cy = cyn;
            ++s;
        }
        if (t < te && kmax > 0.0) {
            atomicMax(&kappa[body], (unsigned long long)__double_as_longlong(kmax));
            if (kmax > 1e4) atomicOr(&bflags[body], HQ_BODY_ILLCOND);
        }
        if (deg) atomicOr(&bflags[body], HQ_BODY_DEGENERATE);
    }
    if (bad) raise_flag(err, kFlagBounds);
}

// Slots of a node's same-tile children in the post-order schedule, from the
// subtree size z2 of the slot before the node (-1: a child elsewhere): the
// child taken second sits just before the node, the other one just before
// that child's subtree.
__device__ __forceinline__ int2 gen_children(int q, int xref, int yref, int meta, int z2) {
    const bool xs = xref == kRefStack, ys = yref == kRefStack;
    int xq = -1, yq = -1;
    if (xs && ys) {
        if (meta & kMetaYFirst) {
            xq = q - 1;
            yq = q - 1 - z2;
        } else {
            yq = q - 1;
            xq = q - 1 - z2;
        }
    } else if (xs) {
        xq = q - 1;
    } else if (ys) {
        yq = q - 1;
    }
    return make_int2(xq, yq);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The later tile phases, node-parallel: a lane per node, TS lanes per tile
// and 64 / TS tiles per wave.  A later phase holds few nodes, in tiles that
// are chains of up to S2 - 1 dependent nodes; one lane per tile walked them
// at about 4 us per node (FP64 dependency latency), so the phase took as long
// as its longest tile.  Here every node of a tile loads its links and its
// children from HBM at once, and the tile resolves level by level: a node
// computes in the round after its same-tile children have published their
// (n, centroid, T22) in LDS and the sizes of their subtrees, which locate
// the children in the post-order schedule.  A tile takes one round per
// level (at most TS rounds; a node left over is flagged).  The stores leave
// once, after the rounds, as in k_gen_tile.
template <int kStore, bool kNodes, int TS>
__global__ void __launch_bounds__(64) k_gen_np(int phase, const int32_t *phase_tab, const int32_t *tile_base,
                                               const int32_t *tile_len, const int32_t *tile_root,
                                               const int32_t *links, const int32_t *nbody, const double *pos,
                                               const double *lo, double *troot, int64_t ntr, double *ncen,
                                               double *T22, float *rec32, double *rec64, double *bcen,
                                               unsigned long long *kappa, int32_t *bflags, int64_t m, int64_t N,
                                               int64_t NI, int32_t *err) {
    static_assert(TS == 32 || TS == 64, "tiles of 32 or 64 lanes");
    constexpr int TPW = 64 / TS;
    extern __shared__ unsigned char smem_raw[];
    double *lds = reinterpret_cast<double *>(smem_raw);  // [word][lane]: each node's (n, c, T22)
    int *ssz = reinterpret_cast<int *>(smem_raw + (size_t)kGenWords * 64 * sizeof(double));
    uint32_t *stage = reinterpret_cast<uint32_t *>(ssz + 64);
    uint32_t *srel = stage + 64 * kStageStride;
    const int lane = threadIdx.x, tl = lane / TS, i = lane - tl * TS, q0 = tl * TS;
    const int tb = phase_tab[2 * phase], te = phase_tab[2 * phase + 1];
    bool bad = false;
    for (int t0 = tb + blockIdx.x * TPW; t0 < te; t0 += gridDim.x * TPW) {
        const int t = t0 + tl;
        int base = 0, len = 0, body = 0;
        if (t < te) {
            const int b = tile_base[t], l = tile_len[t], r = tile_root[t];
            if (b < 0 || l < 1 || l > TS || (int64_t)b + l > NI || r < 0 || r >= NI) {
                bad = true;
            } else {
                base = b;
                len = l;
                body = nbody[r];
            }
        }
        if (body < 0 || body >= m) {
            bad = true;
            base = len = body = 0;
        }
        // wave-uniform bases: tile t0's (the wave's tiles follow it in
        // schedule, tile and body order); offsets from them stay below 2 GiB
        const int s0 = __builtin_amdgcn_readfirstlane(base);
        const int b0 = __builtin_amdgcn_readfirstlane(body);
        if (len > 0 && (base < s0 || base + len - s0 > (1 << 23) || body < b0 || body - b0 > (1 << 24))) {
            bad = true;
            len = 0;
        }
        const bool act = i < len;
        const int s = base + (act ? i : 0);
        auto cap = [](int64_t bytes) -> uint32_t {
            return bytes <= 0 ? 0u : (bytes >= 0x7fffffffll ? 0x7fffffffu : (uint32_t)bytes);
        };
        const int64_t t0c = t0 < ntr ? t0 : ntr;
        const rsrc_t r32 = make_rsrc_uniform(rec32 + (int64_t)kRecWords * s0, cap((NI - s0) * 128));
        const rsrc_t r64 = make_rsrc_uniform(rec64 + (int64_t)kRecWords * s0, cap((NI - s0) * 256));
        const rsrc_t rcen = make_rsrc_uniform(ncen + 3 * (int64_t)s0, cap((NI - s0) * 24));
        const rsrc_t rt22 = make_rsrc_uniform(T22 + 6 * (int64_t)s0, cap((NI - s0) * 48));
        const rsrc_t rtr = make_rsrc_uniform(troot + kGenWords * t0c, cap((ntr - t0c) * 80));
        const rsrc_t rbc = make_rsrc_uniform(bcen + 3 * (int64_t)b0, cap((m - b0) * 24));
        double lo3[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) lo3[d] = lo[3 * body + d];
        // links and the children held in HBM, for every node at once
        int32_t li[kLinkInts];
        load_links(links, min((int64_t)s, NI - 1), li);
        GenIn cx, cy;
        bool fbad = false;
        gen_fetch<true>(li[0], pos, troot, N, ntr, cx, fbad);
        gen_fetch<true>(li[1], pos, troot, N, ntr, cy, fbad);
        bad |= act && fbad;
        const int xref = li[0], yref = li[1], meta = li[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            cx.c[d] = xref >= 0 ? cx.c[d] - lo3[d] : cx.c[d];
            cy.c[d] = yref >= 0 ? cy.c[d] - lo3[d] : cy.c[d];
        }
        const int nst = (int)(xref == kRefStack) + (int)(yref == kRefStack);
        // a tile's first node has no node of its own tile before it
        const bool first_bad = act && nst > 0 && i == 0;
        bad |= first_bad;
        bool done = !act || first_bad, fin = false;
        double n = 0.0, cp[3] = {0.0, 0.0, 0.0}, T[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, w64[26], kap = 0.0;
        int k = 3;
#pragma unroll
        for (int e = 0; e < 26; ++e) w64[e] = 0.0;
        wave_sync();  // the previous group's reads of ssz and the slots are over
        ssz[lane] = 0;
        for (int round = 0; round <= TS; ++round) {
            wave_sync();
            if (!__ballot(!done)) break;
            int z2 = 0, z1 = 0;
            int2 ch = make_int2(-1, -1);
            bool ready = false;
            if (!done) {
                if (nst == 0) {
                    ready = true;
                } else {
                    z2 = ssz[lane - 1];
                    if (z2 > 0) {
                        ch = gen_children(lane, xref, yref, meta, z2);
                        if (nst == 1) {
                            ready = true;
                        } else {
                            const int q1 = lane - 1 - z2;
                            if (q1 < q0) {
                                bad = true;
                                done = true;
                            } else {
                                z1 = ssz[q1];
                                ready = z1 > 0;
                            }
                        }
                    }
                }
            }
            wave_sync();  // this round's reads before its writes
            if (ready) {
                GenIn ax = cx, ay = cy;
                if (ch.x >= 0) gen_slot_get(lds, 0, ch.x, ax);
                if (ch.y >= 0) gen_slot_get(lds, 0, ch.y, ay);
                gen_node(ax, ay, xref < 0, yref < 0, n, cp, T, w64, kap, k);
                gen_slot_put(lds, 0, lane, n, cp, T);
                ssz[lane] = 1 + z2 + z1;
                done = true;
                fin = true;
            }
        }
        bad |= act && !fin;
        // --- stores
        const bool troot_node = (meta & kMetaTileRoot) != 0, body_root = (meta & kMetaBodyRoot) != 0;
        {
            float w32[26];
#pragma unroll
            for (int e = 0; e < 26; ++e) w32[e] = (float)w64[e];
            const int64_t tr = meta >> kMetaSlotShift;
            const bool wr = fin && troot_node && tr == t && t < ntr;
            bad |= fin && troot_node && (tr != t || t >= ntr);
            const uint32_t rel = (uint32_t)(s - s0);
            const double tv[kGenWords] = {n, cp[0], cp[1], cp[2], T[0], T[1], T[2], T[3], T[4], T[5]};
            const double bc[3] = {cp[0] + lo3[0], cp[1] + lo3[1], cp[2] + lo3[2]};
            gen_store<kStore, kNodes>(r32, r64, rcen, rt22, rtr, rbc, stage, srel, lane, fin ? rel : kOOB,
                                      wr ? (uint32_t)(t - t0) : kOOB, (fin && body_root) ? (uint32_t)(body - b0) : kOOB,
                                      w32, w64, li, cp, T, tv, bc);
        }
        // the tile's largest condition bound and its degeneracy, once per tile
        double km = fin ? kap : 0.0;
#pragma unroll
        for (int o = 1; o < TS; o <<= 1) km = fmax(km, __shfl_xor(km, o, 64));
        const unsigned long long dm = __ballot(fin && body_root && (k == 3 || kap > 1e12));
        const bool tdeg = TS == 64 ? dm != 0 : ((dm >> q0) & 0xffffffffull) != 0;
        if (i == 0 && len > 0) {
            if (km > 0.0) {
                atomicMax(&kappa[body], (unsigned long long)__double_as_longlong(km));
                if (km > 1e4) atomicOr(&bflags[body], HQ_BODY_ILLCOND);
            }
            if (tdeg) atomicOr(&bflags[body], HQ_BODY_DEGENERATE);
        }
    }
    if (bad) raise_flag(err, kFlagBounds);
}

// ---------------------------------------------------------------------------
// Leaf boxes of up to s beads (Section 2.1 lets the bisection stop at boxes
// of at most s beads).  They are the first tile phase's tiles of a handle
// with leaf_size s (a tile of at most s bead units is a maximal subtree of at
// most s beads, a leaf box), and each is factored densely: its 3n x 6 matrix
// X = [U_t^T | Z_r^T] (translation rows [I ... I] / sqrt(n), rotation rows
// [A_1 ... A_n] about the leaf's centroid, beads in tree order) by six
// Householder reflections in the convention of the nodes.  Its transform is
// diag(-1,-1,-1,1,...,1) Q^T: rows 1-3 the translation rows, rows 4-6 the
// rotation rows with T22 = R(4:6,4:6)^T, rows 7..3n its residue rows.  The
// tiles above it see the leaf as an earlier tile's root: (n, c, T22) in the
// tile-root table, its Info-set in the exchange buffer.
//
// Six lanes per leaf (lane j holds column j of X), ten leaves per wave; at
// step p lane p forms reflector p and hands it to lanes p+1..5 through LDS.
// Record of leaf b (the phase's b-th tile): column-major 3 s_max x 6 (entries
// below the diagonal of column j are reflector j's tail), then the six taus.
// ---------------------------------------------------------------------------
constexpr int kBucketLanes = 6;
constexpr int kBucketsPerWave = 10;

template <int SMAX, int kStore>
__global__ void __launch_bounds__(64) k_gen_bucket(const int32_t *__restrict__ phase_tab,
                                                   const int32_t *__restrict__ tile_root,
                                                   const int32_t *__restrict__ tile_base,
                                                   const int32_t *__restrict__ tile_len,
                                                   const int32_t *__restrict__ first, const int32_t *__restrict__ last,
                                                   const int32_t *__restrict__ nbody, const int32_t *__restrict__ perm,
                                                   const int32_t *__restrict__ links, const double *__restrict__ pos,
                                                   const double *__restrict__ lo, double *troot, int64_t ntr,
                                                   double *brec64, float *brec32, int64_t bcap, double *bcen,
                                                   unsigned long long *kappa, int32_t *bflags, int64_t m_bodies,
                                                   int64_t N, int64_t NI, int32_t *err) {
    constexpr int MS = 3 * SMAX, BS = 6 * MS + 8;
    __shared__ double vbuf[kBucketsPerWave][MS + 8];
    __shared__ double rbuf[kBucketsPerWave][9];
    const int lane = threadIdx.x;
    const int bq = lane / kBucketLanes, j = lane - bq * kBucketLanes;
    const int tb = phase_tab[2 * 1], te = phase_tab[2 * 1 + 1];
    bool bad = false;
    for (int t0 = tb + blockIdx.x * kBucketsPerWave; t0 < te; t0 += gridDim.x * kBucketsPerWave) {
        const int t = t0 + bq;
        const bool on = bq < kBucketsPerWave && t < te && (int64_t)(t - tb) < bcap;
        int f = 0, n = 0, body = 0, meta = 0;
        if (bq < kBucketsPerWave && t < te && !on) bad = true;
        if (on) {
            const int r = tile_root[t];
            const int sr = tile_base[t] + tile_len[t] - 1;
            if (r < 0 || r >= NI || sr < 0 || sr >= NI) {
                bad = true;
            } else {
                f = first[r];
                n = last[r] - f + 1;
                body = nbody[r];
                meta = links[(int64_t)kLinkInts * sr + 3];
                if (n < 2 || n > SMAX || f < 0 || (int64_t)f + n > N || body < 0 || body >= m_bodies) {
                    bad = true;
                    n = 0;
                }
            }
        }
        const int mrows = 3 * n;
        // the leaf's bead positions (body-local; zeros beyond n, loaded from
        // valid addresses), its centroid, and column j of X
        double c[3] = {0.0, 0.0, 0.0}, lo3[3] = {0.0, 0.0, 0.0};
        if (n > 0)
            for (int d = 0; d < 3; ++d) lo3[d] = lo[3 * body + d];
        double pb[SMAX][3];
#pragma unroll
        for (int k = 0; k < SMAX; ++k) {
            const bool ok = k < n;
            const int64_t u = perm[f + (ok ? k : 0)];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double x = pos[3 * u + d];
                pb[k][d] = ok ? x - lo3[d] : 0.0;
            }
        }
#pragma unroll
        for (int k = 0; k < SMAX; ++k)
#pragma unroll
            for (int d = 0; d < 3; ++d) c[d] += pb[k][d];
        for (int d = 0; d < 3; ++d) c[d] = n > 0 ? c[d] / (double)n : 0.0;
        const double rs = n > 0 ? 1.0 / sqrt((double)n) : 0.0;
        double col[MS];
#pragma unroll
        for (int k = 0; k < SMAX; ++k) {
            const bool ok = k < n;
            const double u0 = pb[k][0] - c[0], u1 = pb[k][1] - c[1], u2 = pb[k][2] - c[2];
            // column j < 3: U_t^T; column 3 + e: Z_r^T = A_k^T, A_k = [u]x
            // (rows {0, -u2, u1}, {u2, 0, -u0}, {-u1, u0, 0})
            const double e0 = j == 0 ? rs : (j == 4 ? u2 : (j == 5 ? -u1 : 0.0));
            const double e1 = j == 1 ? rs : (j == 3 ? -u2 : (j == 5 ? u0 : 0.0));
            const double e2 = j == 2 ? rs : (j == 3 ? u1 : (j == 4 ? -u0 : 0.0));
            col[3 * k] = ok ? e0 : 0.0;
            col[3 * k + 1] = ok ? e1 : 0.0;
            col[3 * k + 2] = ok ? e2 : 0.0;
        }
        double tau_j = 0.0;
        // unrolled, so that col[] is indexed by constants (a runtime index
        // would put the array in scratch memory)
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            if (j == p && n > 0) {
                const double alpha = col[p];
                double xs = 0.0;
#pragma unroll
                for (int i = 0; i < MS; ++i)
                    if (i > p && i < mrows) xs += col[i] * col[i];
                const double xnorm = sqrt(xs);
                if (xnorm == 0.0 || p >= mrows - 1) {
                    tau_j = 0.0;
                } else {
                    const double nrm = sqrt(alpha * alpha + xnorm * xnorm);
                    const double beta = (alpha >= 0.0) ? -nrm : nrm;
                    tau_j = (beta - alpha) / beta;
                    const double scal = 1.0 / (alpha - beta);
#pragma unroll
                    for (int i = 0; i < MS; ++i)
                        if (i > p && i < mrows) col[i] *= scal;
                    col[p] = beta;
                }
#pragma unroll
                for (int i = 0; i < MS; ++i)
                    if (i > p) vbuf[bq][i] = (i < mrows) ? col[i] : 0.0;
                vbuf[bq][MS] = tau_j;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (j > p && j < 6 && n > 0) {
                const double tp = vbuf[bq][MS];
                if (tp != 0.0) {
                    double w = col[p];
#pragma unroll
                    for (int i = 0; i < MS; ++i)
                        if (i > p) w += vbuf[bq][i] * col[i];
                    w *= tp;
                    col[p] -= w;
#pragma unroll
                    for (int i = 0; i < MS; ++i)
                        if (i > p) col[i] -= w * vbuf[bq][i];
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        // records: reflector j's tail and tau_j
        if (j < 6 && n > 0) {
            const int64_t base = (int64_t)(t - tb) * BS;
#pragma unroll
            for (int i = 0; i < MS; ++i) {
                const double x = (i > j && i < mrows) ? col[i] : 0.0;
                if (kStore & 1) brec64[base + j * MS + i] = x;
                if (kStore & 2) brec32[base + j * MS + i] = (float)x;
            }
            if (kStore & 1) brec64[base + 6 * MS + j] = tau_j;
            if (kStore & 2) brec32[base + 6 * MS + j] = (float)tau_j;
        }
        // T22 = R(4:6,4:6)^T: lane 3 + i holds R(3 .. 3 + i, 3 + i)
        if (j >= 3 && j < 6 && n > 0) {
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (q <= j - 3) rbuf[bq][(j - 3) * 3 + q] = col[3 + q];
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (j == 0 && n > 0) {
            double T[6] = {rbuf[bq][0], rbuf[bq][3], rbuf[bq][4], rbuf[bq][6], rbuf[bq][7], rbuf[bq][8]};
            if (n == 2) T[5] = 0.0;  // rank-2 rotation rows of two beads
            const double kap = (n >= 3) ? cond_bound3(T) : 0.0;
            if (t < ntr) {
                double *tr = troot + (int64_t)kGenWords * t;
                tr[0] = (double)n;
                for (int d = 0; d < 3; ++d) tr[1 + d] = c[d];
                for (int d = 0; d < 6; ++d) tr[4 + d] = T[d];
            } else {
                bad = true;
            }
            const bool body_root = (meta & kMetaBodyRoot) != 0;
            if (kap > 0.0) {
                atomicMax(&kappa[body], (unsigned long long)__double_as_longlong(kap));
                if (kap > 1e4) atomicOr(&bflags[body], HQ_BODY_ILLCOND);
            }
            if (body_root) {
                if (n == 2 || kap > 1e12) atomicOr(&bflags[body], HQ_BODY_DEGENERATE);
                for (int d = 0; d < 3; ++d) bcen[3 * body + d] = c[d] + lo3[d];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if (bad) raise_flag(err, kFlagBounds);
}

// Tile tables of the fused upward sweep: each tile's parent tile (the tile
// holding its root's parent node; -1 for a body root), and the child-tile
// counts, which the sweep's arrival counters start from.
__global__ void k_tile_zero(int64_t NI, const int32_t *__restrict__ cnt, int32_t *tcnt0) {
    const int64_t nt = min((int64_t)cnt[kCntTiles], NI);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x)
        tcnt0[t] = 0;
}

__global__ void k_tile_parents(int64_t NI, const int32_t *__restrict__ cnt, const int32_t *__restrict__ tile_root,
                               const int32_t *__restrict__ par, const int32_t *__restrict__ tileof, int32_t *ptile,
                               int32_t *tcnt0, int32_t *err) {
    const int64_t nt = min((int64_t)cnt[kCntTiles], NI);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
        const int r = tile_root[t];
        if (r < 0 || r >= NI) {
            raise_flag(err, kFlagBounds);
            ptile[t] = -1;
            continue;
        }
        const int p = par[r];
        const int pt = (p >= 0 && p < NI) ? tileof[p] : -1;
        ptile[t] = pt;
        if (pt >= 0 && pt < nt) atomicAdd(&tcnt0[pt], 1);
        else if (p >= 0) raise_flag(err, kFlagBounds);
    }
}

__global__ void k_tile_copy(int64_t NI, const int32_t *__restrict__ cnt, const int32_t *__restrict__ tcnt0,
                            int32_t *tcnt) {
    const int64_t nt = min((int64_t)cnt[kCntTiles], NI);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x)
        tcnt[t] = tcnt0[t];
}

// Rigid motion: r <- Rot (r - c) + c + t per body.
// pin and pout may be the same buffer: each thread reads a bead's position
// before it writes it.
__global__ void __launch_bounds__(kThreads) k_rigid(const int32_t *__restrict__ chunks, const double *pin,
                                                    double *pout, const double *__restrict__ rot,
                                                    const double *__restrict__ trans, const double *__restrict__ cen) {
    const int body = chunks[3 * blockIdx.x], b0 = chunks[3 * blockIdx.x + 1], b1 = chunks[3 * blockIdx.x + 2];
    double R[9], c[3], t[3];
    for (int i = 0; i < 9; ++i) R[i] = rot[9 * body + i];
    for (int d = 0; d < 3; ++d) { c[d] = cen[3 * body + d]; t[d] = trans[3 * body + d]; }
    for (int i = b0 + threadIdx.x; i < b1; i += kThreads) {
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = pin[3 * (int64_t)i + d] - c[d];
        for (int d = 0; d < 3; ++d)
            pout[3 * (int64_t)i + d] = R[3 * d] * x[0] + R[3 * d + 1] * x[1] + R[3 * d + 2] * x[2] + c[d] + t[d];
    }
}

// Vectors of a rigidly moved body (reuse of its transforms): Q~ of positions
// Rot_j r + t equals Q~ of r times blockdiag(Rot_j^T) over the body's beads,
// since Z of the moved body is diag(Rot_j, Rot_j) Z blockdiag(Rot_j^T) up to
// adding multiples of its translation rows to the others (Eq. 1.2).  Each
// bead's 3-vector of every right-hand side is multiplied by Rot_j^T
// (transpose = 1, before an upward sweep) or Rot_j (after a downward one);
// element (3i + d, r) at 3i R + r vlane + d vcomp.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_rotate(const int32_t *__restrict__ chunks, const double *__restrict__ rot,
                                                     const T *in, T *out, int R, int vlane, int vcomp, int transpose) {
    const int body = chunks[3 * blockIdx.x], b0 = chunks[3 * blockIdx.x + 1], b1 = chunks[3 * blockIdx.x + 2];
    double M[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = transpose ? rot[9 * body + 3 * b + a] : rot[9 * body + 3 * a + b];
    const int64_t cnt = (int64_t)(b1 - b0) * R;
    for (int64_t q = threadIdx.x; q < cnt; q += kThreads) {
        const int64_t i = b0 + q / R;
        const int r = (int)(q % R);
        const int64_t e = 3 * i * R + (int64_t)r * vlane;
        const double x0 = in[e], x1 = in[e + vcomp], x2 = in[e + 2 * vcomp];
        for (int d = 0; d < 3; ++d) out[e + d * vcomp] = (T)(M[3 * d] * x0 + M[3 * d + 1] * x1 + M[3 * d + 2] * x2);
    }
}

inline unsigned grid_for(int64_t n, int threads = kThreads) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 65535) b = 65535;
    return (unsigned)b;
}

}  // namespace

hq_status build_device(Plan &P, const double *pos, hipStream_t s, bool probe_phases) {
    const int64_t N = P.N, m = P.m, NI = P.NI;
    // --- init
    hipLaunchKernelGGL(k_init_bodies, dim3(grid_for(m)), dim3(kThreads), 0, s, m, P.d_bmin, P.d_bmax, P.d_kappa,
                       P.d_bflags);
    hipLaunchKernelGGL(k_init_nodes, dim3(grid_for(NI)), dim3(kThreads), 0, s, NI, P.d_cov, P.d_tileof,
                       P.d_sched_node, P.d_cnt, P.d_phase, P.d_prun);
    // --- 1. boxes and codes
    hipLaunchKernelGGL(k_bbox, dim3(P.nchunks), dim3(kThreads), 0, s, P.d_chunks, pos, P.d_bmin, P.d_bmax, P.d_err);
    hipLaunchKernelGGL(k_codes, dim3(P.nchunks), dim3(kThreads), 0, s, P.d_chunks, P.d_bead_off, pos, P.d_bmin,
                       P.d_bmax, P.d_lo, P.d_h, P.d_keyA, P.d_valA);
    // --- 2. sort (chunks of large bodies and whole bodies in one launch)
    if (P.sort_segs.nseg > 0)
        hipLaunchKernelGGL(k_lds_sort, dim3(P.sort_segs.nseg), dim3(kSortThreads), 0, s, P.sort_segs.d_seg, P.d_keyA,
                           P.d_valA, P.d_bead_off, P.d_scode, P.d_perm, P.d_lc, P.d_rc, P.d_par, P.d_first, P.d_last,
                           P.d_nn, P.d_nbody, P.d_leafpar, P.d_lw);
    HQ_HIP(hipGetLastError());
    if (P.nlarge > 0) {
        unsigned long long *kin = P.d_keyA, *kout = P.d_keyB;
        int32_t *vin = P.d_valA, *vout = P.d_valB;
        int L = kSortChunk;
        for (int p = 0; p < P.large_passes; ++p) {
            hipLaunchKernelGGL(k_merge_pass, dim3(grid_for(P.large_elems)), dim3(kThreads), 0, s, P.d_large,
                               P.d_large_prefix, P.nlarge, P.large_elems, P.d_bead_off, L, kin, vin, kout, vout);
            std::swap(kin, kout);
            std::swap(vin, vout);
            L *= 2;
        }
        hipLaunchKernelGGL(k_large_final, dim3(grid_for(P.large_elems)), dim3(kThreads), 0, s, P.d_large,
                           P.d_large_prefix, P.nlarge, P.large_elems, P.d_bead_off, kin, vin, P.d_scode, P.d_perm);
    }
    // --- 3. tree (bodies sorted whole got theirs in the sort kernel)
    if (P.nlarge > 0) {
        const int64_t large_nodes = P.large_elems - P.nlarge;
        hipLaunchKernelGGL(k_tree_large, dim3(grid_for(large_nodes)), dim3(kThreads), 0, s, P.d_large,
                           P.d_large_prefix, P.nlarge, large_nodes, P.d_bead_off, P.d_scode, P.d_lc, P.d_rc, P.d_par,
                           P.d_first, P.d_last, P.d_nn, P.d_nbody, P.d_leafpar, P.d_lw);
    }
    HQ_HIP(hipGetLastError());
    // --- 4. tiles
    int phases = 0;
    const int max_ph = probe_phases ? (kMaxPhases - 1) : P.phases_reserved;
    int64_t tiles_prev = 0;
    if (probe_phases) std::fill(P.tiles_ph, P.tiles_ph + kMaxPhases, (int64_t)0);
    for (int ph = 1; ph <= max_ph; ++ph) {
        if (!probe_phases && ph > std::max(P.phases_built, 2)) {
            // a rebuild's reserved phases (beyond those the first build
            // needed) in one single-workgroup launch: they are normally empty,
            // and about nine launches each cost their dispatch latency on the
            // rebuild's critical path.  (Taking a real phase this way is
            // slower than its multi-workgroup launches: a rebuild that needs
            // one more phase than the first build pays that, correctly.)
            hipLaunchKernelGGL(k_tail_phases, dim3(1), dim3(kTailThreads), 0, s, ph, max_ph, NI, P.d_rem,
                               P.d_cnt + kCntRemList, P.S2, P.d_cov, P.d_par, P.d_lc, P.d_rc, P.d_nn, P.d_units,
                               P.d_trval, P.d_trscan, P.d_cnt, P.d_tile_root, P.d_tile_len, P.d_tile_base,
                               P.d_tileof, P.d_yfirst, P.d_aw, P.d_sched, P.d_sched_node, P.d_slot, NI, P.d_phase,
                               P.run_nodes, P.d_prun, P.run_cap, P.d_run, P.d_err);
            HQ_HIP(hipGetLastError());
            phases = max_ph;
            break;
        }
        // a phase after the one that covered the last node is a no-op on the
        // device (reserved phases of a rebuild cost a few launches only)
        const int32_t *gate = (ph >= 2) ? P.d_cnt + kCntRemain : nullptr;
        // later phases work on the list of nodes the first phase left over
        const int32_t *rem = (ph >= 2) ? P.d_rem : nullptr;
        const int32_t *dn = (ph >= 2) ? P.d_cnt + kCntRemList : nullptr;
        const unsigned grid = (ph >= 2) ? std::min(grid_for(NI), 1024u) : grid_for(NI);
        if (ph == 2) {
            // the first phase's k_assign1 flagged the nodes it left (P.d_mark)
            HQ_TRY(scan_i32_inclusive(P, P.d_mark, P.d_msum, NI, s, gate));
            hipLaunchKernelGGL(k_rem_scatter, dim3(grid_for(NI)), dim3(kThreads), 0, s, NI, P.d_cov, P.d_msum,
                               P.d_rem, P.d_cnt, gate);
        }
        if (ph >= 2) {
            // (the previous phase's k_assign cleared the uncovered nodes' units)
            hipLaunchKernelGGL(k_units_walk, dim3(grid), dim3(kThreads), 0, s, NI, rem, dn, P.d_cov, P.d_lc, P.d_rc,
                               P.d_par, P.d_units, P.d_err, gate);
        }
        if (ph == 1) {
            hipLaunchKernelGGL(k_tile_roots1, dim3(grid), dim3(kThreads), 0, s, NI, P.S, P.d_par, P.d_lc, P.d_rc,
                               P.d_nn, P.d_units, P.d_trval, P.d_yfirst, P.d_aw);
            HQ_TRY(scan_i64_exclusive(P, P.d_trval, P.d_trscan, NI, s, gate, dn));
            hipLaunchKernelGGL(k_assign1, dim3(grid), dim3(kThreads), 0, s, NI, P.d_cov, P.d_units, P.d_aw,
                               P.d_trval, P.d_trscan, P.d_cnt, P.d_tile_root, P.d_tile_len, P.d_tile_base,
                               P.d_tileof, P.d_sched, P.d_sched_node, P.d_slot, P.d_mark, P.d_err, NI);
        } else {
            // (P.d_msum, the list's scan, is free once the list is built: it
            // holds the roots' places in the list)
            hipLaunchKernelGGL(k_tile_roots_l, dim3(grid), dim3(kThreads), 0, s, NI, rem, dn, P.S2, P.d_cov, P.d_par,
                               P.d_lc, P.d_rc, P.d_units, P.d_trval, P.d_yfirst, P.d_aw, P.d_msum, gate);
            HQ_TRY(scan_i64_exclusive(P, P.d_trval, P.d_trscan, NI, s, gate, dn));
            hipLaunchKernelGGL(k_assign_l, dim3(grid), dim3(kThreads), 0, s, NI, rem, dn, ph, P.d_cov, P.d_units,
                               P.d_aw, P.d_trval, P.d_trscan, P.d_msum, P.d_cnt, P.d_tile_root, P.d_tile_len,
                               P.d_tile_base, P.d_tileof, P.d_sched, P.d_sched_node, P.d_slot, P.d_err, NI, gate);
        }
        hipLaunchKernelGGL(k_phase_close, dim3(1), dim3(64), 0, s, NI, dn, ph, P.d_trval, P.d_trscan, P.d_cnt,
                           P.d_phase, P.run_nodes, P.d_prun, P.run_cap, P.d_err, gate);
        // the run table of a phase is built when the phase holds nodes
        hipLaunchKernelGGL(k_runs, dim3(std::min(grid_for(NI), 1024u)), dim3(kThreads), 0, s, ph, P.d_phase,
                           P.d_tile_base, P.d_prun, P.d_run, P.d_prun + kPrunStride * ph + 1);
        HQ_HIP(hipGetLastError());
        phases = ph;
        if (probe_phases) {
            int32_t cnt[kCntNum];
            HQ_HIP(hipMemcpyAsync(cnt, P.d_cnt, sizeof cnt, hipMemcpyDeviceToHost, s));
            HQ_HIP(hipStreamSynchronize(s));
            if (ph == 1) P.tiles1_built = cnt[kCntTiles];
            P.tiles_ph[ph] = cnt[kCntTiles] - tiles_prev;
            tiles_prev = cnt[kCntTiles];
            if (cnt[kCntRemain] == 0) {
                P.tiles_built = cnt[kCntTiles];
                break;
            }
            if (ph == max_ph) {
                set_error("tree needs more tile phases than supported");
                return HQ_E_UNSUPPORTED;
            }
        }
    }
    if (probe_phases) P.phases_built = phases;
    // the compaction flags are free again: they hold the tile roots' offsets
    int32_t *toff = P.d_mark;
    hipLaunchKernelGGL(k_troot_off, dim3(std::min(grid_for(NI), 2048u)), dim3(kThreads), 0, s, NI, P.d_cnt,
                       P.d_tile_root, P.d_lw, P.d_nbody, P.d_row_off, toff, P.d_err);
    hipLaunchKernelGGL(k_links, dim3(grid_for(NI)), dim3(kThreads), 0, s, NI, P.d_cov, P.d_tileof, P.d_sched,
                       P.d_lc, P.d_rc, P.d_par, P.d_nn, P.d_nbody, P.d_yfirst, P.d_tile_root, P.d_perm, toff,
                       P.d_slot, stack_slots(P.smax()), P.d_lw, P.d_links, P.d_err);
    if (P.fused_up) {
        // the fused upward sweep's tile tables (no other sweep reads them)
        const unsigned tg = std::min(grid_for(NI), 2048u);
        hipLaunchKernelGGL(k_tile_zero, dim3(tg), dim3(kThreads), 0, s, NI, P.d_cnt, P.d_tcnt0);
        hipLaunchKernelGGL(k_tile_parents, dim3(tg), dim3(kThreads), 0, s, NI, P.d_cnt, P.d_tile_root, P.d_par,
                           P.d_tileof, P.d_ptile, P.d_tcnt0, P.d_err);
        hipLaunchKernelGGL(k_tile_copy, dim3(tg), dim3(kThreads), 0, s, NI, P.d_cnt, P.d_tcnt0, P.d_tcnt);
    }
    // --- 5. transforms, one launch per tile phase; later phases read the
    // roots of earlier phases' tiles from the tile-root table (sized after
    // the first build: twice its tiles, the capacity of the exchange buffer)
    if (probe_phases && P.ws && P.troot_cap < P.tiles_built + 64) {
        set_error("the tree has more tiles than the workspace holds (hq_options.max_tiles)");
        return HQ_E_UNSUPPORTED;
    }
    if (probe_phases && !P.ws && P.troot_cap < 2 * P.tiles_built + 64) {
        const int64_t cap = 2 * P.tiles_built + 64;
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, (size_t)cap * kGenWords * sizeof(double));
        if (e != hipSuccess) {
            set_error(std::string("hipMalloc of the tile-root table: ") + hipGetErrorString(e));
            return HQ_E_NOMEM;
        }
        P.allocs.push_back(q);
        P.d_troot = reinterpret_cast<double *>(q);
        P.troot_cap = cap;
    }
    // leaf-box records: twice the first build's leaves (a rebuilt tree with
    // more raises HQ_FLAG_BOUNDS); a workspace handle has them already
    if (probe_phases && P.leaf_s > 1 && P.bucket_cap < 2 * P.tiles1_built + 64) {
        if (P.ws) {
            set_error("the tree has more leaf boxes than the workspace holds");
            return HQ_E_UNSUPPORTED;
        }
        const int64_t cap = 2 * P.tiles1_built + 64;
        const size_t per = (size_t)bucket_stride(P.leaf_smax());
        void *q = nullptr;
        if (P.store & 1) {
            HQ_TRY(plan_alloc(P, &q, (size_t)cap * per * sizeof(double)));
            P.d_brec64 = reinterpret_cast<double *>(q);
        }
        if (P.store & 2) {
            HQ_TRY(plan_alloc(P, &q, (size_t)cap * per * sizeof(float)));
            P.d_brec32 = reinterpret_cast<float *>(q);
        }
        P.bucket_cap = cap;
    }
    const int nslot = stack_slots(P.smax());
    const size_t gen_lds = (size_t)nslot * kGenWords * 64 * sizeof(double) + ((P.store & 2) ? kStageBytes : 0);
    const unsigned gen_grid = (unsigned)std::min<int64_t>((P.tiles_built + P.tiles_built / 4) / 64 + 1, 65535);
    using GenFn = decltype(&k_gen_tile<false, 0, false>);
    // [later phase][store][node data]
    const GenFn gen_fn[2][4][2] = {
        {{k_gen_tile<false, 0, false>, k_gen_tile<false, 0, true>}, {k_gen_tile<false, 1, false>, k_gen_tile<false, 1, true>},
         {k_gen_tile<false, 2, false>, k_gen_tile<false, 2, true>}, {k_gen_tile<false, 3, false>, k_gen_tile<false, 3, true>}},
        {{k_gen_tile<true, 0, false>, k_gen_tile<true, 0, true>}, {k_gen_tile<true, 1, false>, k_gen_tile<true, 1, true>},
         {k_gen_tile<true, 2, false>, k_gen_tile<true, 2, true>}, {k_gen_tile<true, 3, false>, k_gen_tile<true, 3, true>}}};
    // per-node centroids and T22 (introspection only): on hq_build, and on
    // hq_rebuild when the handle keeps them
    const bool nodes = probe_phases || P.keep_node_data;
    P.node_data_fresh = nodes;
    // the first phase's tiles longest first, when every buffer the generation
    // writes can be addressed from its start with 32-bit offsets
    const int64_t lim = 0x7fffffffll;
    const bool sort_tiles = P.leaf_s <= 1 && NI * 256 < lim && P.troot_cap * 80 < lim && m * 24 < lim;
    if (sort_tiles) {
        const int nbins = P.S;
        hipLaunchKernelGGL(k_len_hist, dim3(kLenBlocks), dim3(256), 0, s, 1, P.d_phase, P.d_tile_len, nbins, P.d_lhist);
        HQ_TRY(scan_i32_inclusive(P, P.d_lhist, P.d_lincl, (int64_t)nbins * kLenBlocks, s));
        hipLaunchKernelGGL(k_len_scatter, dim3(kLenBlocks), dim3(256), 0, s, 1, P.d_phase, P.d_tile_len, nbins,
                           P.d_lhist, P.d_lincl, P.d_tord);
    }
    for (int ph = 1; ph <= phases; ++ph) {
        const bool later = ph > 1;
        if (ph == 1 && P.leaf_s > 1) {
            const unsigned bg = (unsigned)std::min<int64_t>(P.bucket_cap / kBucketsPerWave + 1, 65535);
#define HQ_GEN_BUCKET(SM, ST)                                                                                   \
    hipLaunchKernelGGL((k_gen_bucket<SM, ST>), dim3(bg), dim3(64), 0, s, P.d_phase, P.d_tile_root, P.d_tile_base, \
                       P.d_tile_len, P.d_first, P.d_last, P.d_nbody, P.d_perm, P.d_links, pos, P.d_lo, P.d_troot, \
                       P.troot_cap, P.d_brec64, P.d_brec32, P.bucket_cap, P.d_cen, P.d_kappa, P.d_bflags, m, N, NI, \
                       P.d_err)
#define HQ_GEN_BUCKET_S(SM)                                    \
    do {                                                       \
        if ((P.store & 3) == 1) HQ_GEN_BUCKET(SM, 1);          \
        else if ((P.store & 3) == 2) HQ_GEN_BUCKET(SM, 2);     \
        else HQ_GEN_BUCKET(SM, 3);                             \
    } while (0)
            if (P.leaf_smax() == 8) HQ_GEN_BUCKET_S(8);
            else HQ_GEN_BUCKET_S(16);
#undef HQ_GEN_BUCKET_S
#undef HQ_GEN_BUCKET
            continue;
        }
        if (later && P.S2 <= 64) {
            // later phases node-parallel: tiles of up to 32 (two per wave) or
            // 64 lanes, a grid from the build's tiles in the phase
            const int ts = P.S2 <= 32 ? 32 : 64;
            const size_t lds_np = (size_t)kGenWords * 64 * sizeof(double) + 64 * sizeof(int) +
                                  ((P.store & 2) ? kStageBytes : 0);
            const int64_t groups = (2 * P.tiles_ph[ph] + 64 + 64 / ts - 1) / (64 / ts);
            const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(groups, P.ncu), 65535);
#define HQ_GEN_NP(ST, ND, TS)                                                                                     \
    hipLaunchKernelGGL((k_gen_np<ST, ND, TS>), dim3(g), dim3(64), lds_np, s, ph, P.d_phase, P.d_tile_base,        \
                       P.d_tile_len, P.d_tile_root, P.d_links, P.d_nbody, pos, P.d_lo, P.d_troot, P.troot_cap,   \
                       P.d_ncen, P.d_T22, P.d_rec32, P.d_rec64, P.d_cen, P.d_kappa, P.d_bflags, m, N, NI, P.d_err)
#define HQ_GEN_NP_S(TS)                                                  \
    do {                                                                 \
        switch ((P.store & 3) * 2 + (nodes ? 1 : 0)) {                   \
        case 2: HQ_GEN_NP(1, false, TS); break;                          \
        case 3: HQ_GEN_NP(1, true, TS); break;                           \
        case 4: HQ_GEN_NP(2, false, TS); break;                          \
        case 5: HQ_GEN_NP(2, true, TS); break;                           \
        case 6: HQ_GEN_NP(3, false, TS); break;                          \
        case 7: HQ_GEN_NP(3, true, TS); break;                           \
        default: HQ_GEN_NP(3, true, TS); break;                          \
        }                                                                \
    } while (0)
            if (ts == 32) HQ_GEN_NP_S(32);
            else HQ_GEN_NP_S(64);
#undef HQ_GEN_NP_S
#undef HQ_GEN_NP
            continue;
        }
        hipLaunchKernelGGL(gen_fn[later][P.store & 3][nodes ? 1 : 0], dim3(later ? std::min(gen_grid, 1024u) : gen_grid), dim3(64),
                           gen_lds, s, ph, P.d_phase, P.d_tile_base, P.d_tile_len, P.d_tile_root, P.d_links,
                           P.d_nbody, pos, P.d_lo, P.d_troot, P.troot_cap, nslot, P.d_ncen, P.d_T22, P.d_rec32,
                           P.d_rec64, P.d_cen, P.d_kappa, P.d_bflags,
                           (sort_tiles && !later) ? (const int32_t *)P.d_tord : nullptr, m, N, NI, P.d_err);
    }
    HQ_HIP(hipGetLastError());
    return HQ_OK;
}

hq_status rotate_vectors(Plan &P, const double *rot, const void *in, void *out, int64_t nrhs, int prec, int layout,
                         int transpose, hipStream_t s) {
    const int R = (int)nrhs;
    const int vlane = (layout == HQ_TRIPLES) ? 3 : 1, vcomp = (layout == HQ_TRIPLES) ? 1 : R;
    if (prec == HQ_FP64)
        hipLaunchKernelGGL(k_rotate<double>, dim3(P.nchunks), dim3(kThreads), 0, s, P.d_chunks, rot,
                           (const double *)in, (double *)out, R, vlane, vcomp, transpose);
    else
        hipLaunchKernelGGL(k_rotate<float>, dim3(P.nchunks), dim3(kThreads), 0, s, P.d_chunks, rot,
                           (const float *)in, (float *)out, R, vlane, vcomp, transpose);
    HQ_HIP(hipGetLastError());
    return HQ_OK;
}

hq_status rigid_update(Plan &P, double *pos, const double *rot, const double *trans, hipStream_t s) {
    hipLaunchKernelGGL(k_rigid, dim3(P.nchunks), dim3(kThreads), 0, s, P.d_chunks, pos, pos, rot, trans, P.d_cen);
    HQ_HIP(hipGetLastError());
    return HQ_OK;
}

hq_status rigid_motion(Plan &P, const double *pin, double *pout, const double *rot, const double *trans,
                       const double *cen, hipStream_t s) {
    hipLaunchKernelGGL(k_rigid, dim3(P.nchunks), dim3(kThreads), 0, s, P.d_chunks, pin, pout, rot, trans, cen);
    HQ_HIP(hipGetLastError());
    return HQ_OK;
}

}  // namespace hq
