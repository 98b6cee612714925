// The O(n) sweeps (Section 4).
//
// Upward, Q~ v (Algorithm 2, Eqs. 4.2-4.3): a leaf's Info-set is its bead
// vector; at a node with children x, y
//     M_p(1:3)          = sx M_x(1:3) + sy M_y(1:3)
//     [M_p(4:6); eps_p] = G [M_x(4:6)?; M_y(4:6)?; sy M_x(1:3) - sx M_y(1:3)]
// with sx = sqrt(n_x/n), sy = sqrt(n_y/n) and "?" present only for an
// internal child; eps_p are the node's residue rows of Q~ v.
//
// Downward, Q~^T w (Algorithm 3, Theorem 4.3): the root Velocity-set is 0;
//     s = G^T [L_p(4:6); w_p] = [s_x?; s_y?; s_t]
//     L_x = [sx L_p(1:3) + sy s_t; s_x],  L_y = [sy L_p(1:3) - sx s_t; s_y]
// and a leaf's velocity is L(1:3).
//
// G = H_2 H_1 H_0 is stored as three Householder reflectors.  Work is split
// into tiles (connected pieces of a body's tree); one group of LPT lanes
// sweeps one tile, each lane one right-hand side, through the tile's nodes in
// schedule order (reverse order downward).  Pending Info-sets / Velocity-sets
// of the tile live on a per-lane stack in LDS; a tile root exchanges its
// 6-vector with the tile above through a global exchange buffer.  Tiles of one
// phase are independent; phases run as separate launches.
#include "hq_buffer.h"
#include "hq_common.h"


namespace hq {

namespace {

struct Ctx {
    int64_t N, rows, nsched;
    int R, nchunks, dmax, xch_cap;
    int nslot;  // LDS slots per lane of the wide sweeps
    // vector layout: element (row0 + k, r) of a row triple (row0 a multiple of
    // 3, k < 3) sits at row0 * R + r * vlane + k * vcomp; rows (row-major
    // rows x R): vlane 1, vcomp R; triples (each column's three values of a
    // triple contiguous): vlane 3, vcomp 1
    int vlane, vcomp;
    int root_in;  // downward: body roots take their Velocity-set from the exchange buffer (full Q)
    int m;        // bodies (rows of the rotation table of the fused rigid-motion products)
    uint32_t in_bytes, out_bytes, xch_bytes;  // buffer sizes of the wide sweeps (each < 2 GiB)
    int bufs_ok;  // every vector buffer lies below 2 GiB (the sizes above are exact)
};

// Index of element (row0 + k, r) of a vector, row0 a multiple of 3.
__device__ __forceinline__ int64_t velem(int64_t row0, int k, int r, const Ctx &C) {
    return row0 * C.R + (int64_t)r * C.vlane + (int64_t)k * C.vcomp;
}

template <typename T>
__device__ __forceinline__ void push6(T *stk, int &sp, int dmax, const T (&m)[6], int lane, int32_t *err) {
    if (sp >= dmax) {
        atomicOr(err, kFlagStack);
        return;
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) stk[(sp * 6 + c) * 64 + lane] = m[c];
    ++sp;
}

template <typename T>
__device__ __forceinline__ void pop6(T *stk, int &sp, T (&m)[6], int lane, int32_t *err) {
    if (sp <= 0) {
        atomicOr(err, kFlagStack);
#pragma unroll
        for (int c = 0; c < 6; ++c) m[c] = T(0);
        return;
    }
    --sp;
#pragma unroll
    for (int c = 0; c < 6; ++c) m[c] = stk[(sp * 6 + c) * 64 + lane];
}

// Inputs of one node gathered ahead of its turn: links (child references,
// residue row, flags), the reflectors and weights, and the values that come
// from memory rather than from the tile stack.
template <typename T>
struct NodeIn {
    int4 lk;
    T g[26];
    T a[6];  // upward: x child (bead 3 / tile root 6); downward: residue coefficients w_p
    T b[6];  // upward: y child;                         downward: L_p of a tile root
};

template <typename T>
__device__ __forceinline__ void load_g(T (&g)[26], const T *__restrict__ src) {
#pragma unroll
    for (int q = 0; q < 26; ++q) g[q] = src[q];
}

template <>
__device__ __forceinline__ void load_g<float>(float (&g)[26], const float *__restrict__ src) {
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const float4 t = s4[q];
        g[4 * q] = t.x; g[4 * q + 1] = t.y; g[4 * q + 2] = t.z; g[4 * q + 3] = t.w;
    }
    const float2 t = reinterpret_cast<const float2 *>(src)[12];
    g[24] = t.x;
    g[25] = t.y;
}

template <>
__device__ __forceinline__ void load_g<double>(double (&g)[26], const double *__restrict__ src) {
    const double2 *s2 = reinterpret_cast<const double2 *>(src);
#pragma unroll
    for (int q = 0; q < 13; ++q) {
        const double2 t = s2[q];
        g[2 * q] = t.x;
        g[2 * q + 1] = t.y;
    }
}

__device__ __forceinline__ int4 load_links(const int32_t *__restrict__ links, int s) {
    const int2 *p = reinterpret_cast<const int2 *>(links + (int64_t)kLinkInts * s);
    const int2 a = p[0], b = p[1];
    return make_int4(a.x, a.y, b.x, b.y);
}

// Upward: values of the non-stack children of a node.
template <typename T>
__device__ __forceinline__ void fetch_child(int ref, T (&m)[6], const T *__restrict__ v, const T *__restrict__ xch,
                                            const Ctx &C, int r, bool act, int32_t *err) {
    if (ref >= 0) {
        if (ref >= C.N) {
            atomicOr(err, kFlagBounds);
        } else if (act) {
#pragma unroll
            for (int c = 0; c < 3; ++c) m[c] = v[velem((int64_t)3 * ref, c, r, C)];
        }
    } else if (ref != kRefStack) {
        const int slot = ref_slot(ref);
        if (slot < 0 || slot >= C.xch_cap) {
            atomicOr(err, kFlagBounds);
        } else if (act) {
#pragma unroll
            for (int c = 0; c < 6; ++c) m[c] = xch[((int64_t)slot * 6 + c) * C.R + r];
        }
    }
}

template <typename T>
__device__ __forceinline__ void fetch_up(NodeIn<T> &n, int s, const T *__restrict__ rec, const T *__restrict__ v,
                                         const T *__restrict__ xch, const Ctx &C, int r, bool act, int32_t *err) {
    load_g(n.g, rec + (int64_t)kRecWords * s);
#pragma unroll
    for (int c = 0; c < 6; ++c) n.a[c] = n.b[c] = T(0);
    fetch_child(n.lk.x, n.a, v, xch, C, r, act, err);
    fetch_child(n.lk.y, n.b, v, xch, C, r, act, err);
}

template <typename T>
__device__ __forceinline__ void node_up(const NodeIn<T> &n, T *stk, int &sp, T *__restrict__ out,
                                        T *__restrict__ xch, const Ctx &C, int r, bool act, int lane, int32_t *err) {
    const int xref = n.lk.x, yref = n.lk.y, off = n.lk.z, meta = n.lk.w;
    T mx[6], my[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        mx[c] = n.a[c];
        my[c] = n.b[c];
    }
    const bool xs = xref == kRefStack, ys = yref == kRefStack;
    if (xs && ys) {
        if (meta & kMetaYFirst) {
            pop6(stk, sp, mx, lane, err);
            pop6(stk, sp, my, lane, err);
        } else {
            pop6(stk, sp, my, lane, err);
            pop6(stk, sp, mx, lane, err);
        }
    } else if (xs) {
        pop6(stk, sp, mx, lane, err);
    } else if (ys) {
        pop6(stk, sp, my, lane, err);
    }
    const T sx = n.g[kRecSx], sy = n.g[kRecSy];
    const bool xi = xref < 0, yi = yref < 0;
    T mp[6], t9[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) mp[c] = sx * mx[c] + sy * my[c];
    int dim;
    if (xi && yi) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            t9[c] = mx[3 + c];
            t9[3 + c] = my[3 + c];
            t9[6 + c] = sy * mx[c] - sx * my[c];
        }
        house_fwd<9>(t9, n.g);
        dim = 6;
    } else if (xi || yi) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            t9[c] = xi ? mx[3 + c] : my[3 + c];
            t9[3 + c] = sy * mx[c] - sx * my[c];
        }
        house_fwd<6>(t9, n.g);
        dim = 3;
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) t9[c] = sy * mx[c] - sx * my[c];
        house_fwd<3>(t9, n.g);
        dim = 0;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) mp[3 + c] = t9[c];
    if (dim > 0) {
        if (off < 0 || (int64_t)off + dim > C.rows) {
            atomicOr(err, kFlagBounds);
        } else if (act) {
#pragma unroll
            for (int k = 0; k < 3; ++k) out[velem(off, k, r, C)] = t9[3 + k];
            if (dim == 6) {
#pragma unroll
                for (int k = 0; k < 3; ++k) out[velem(off + 3, k, r, C)] = t9[6 + k];
            }
        }
    }
    if (meta & kMetaTileRoot) {
        const int slot = meta >> kMetaSlotShift;
        if (slot >= C.xch_cap) {
            atomicOr(err, kFlagBounds);
        } else if (act) {
#pragma unroll
            for (int c = 0; c < 6; ++c) xch[((int64_t)slot * 6 + c) * C.R + r] = mp[c];
        }
    } else {
        push6(stk, sp, C.dmax, mp, lane, err);
    }
}

// One group of LPT lanes sweeps one tile; the loop is unrolled by two so the
// prefetched inputs alternate between two slots: at node i the links of node
// i+2 and the reflectors / memory inputs of node i+1 are in flight.
template <typename T, int LPT>
__global__ void __launch_bounds__(64) k_up(int phase, const int32_t *__restrict__ phase_tab,
                                           const int32_t *__restrict__ tile_base, const int32_t *__restrict__ tile_len,
                                           const int32_t *__restrict__ links, const T *__restrict__ rec,
                                           const T *__restrict__ v, T *__restrict__ out, T *__restrict__ xch, Ctx C,
                                           int32_t *err) {
    extern __shared__ unsigned char smem_raw[];
    T *stk = reinterpret_cast<T *>(smem_raw);
    constexpr int TPW = 64 / LPT;
    const int lane = threadIdx.x;
    const int tslot = lane / LPT, rl = lane % LPT;
    const int tb = phase_tab[2 * phase], te = phase_tab[2 * phase + 1];
    const int ngroups = (te - tb + TPW - 1) / TPW;
    const int items = ngroups * C.nchunks;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int grp = item / C.nchunks, chunk = item - grp * C.nchunks;
        const int t = tb + grp * TPW + tslot;
        const int r = chunk * LPT + rl;
        const bool tvalid = t < te;
        const bool act = tvalid && r < C.R;
        int base = 0, len = 0;
        if (tvalid) {
            base = tile_base[t];
            len = tile_len[t];
            if (base < 0 || len < 0 || (int64_t)base + len > C.nsched) {
                atomicOr(err, kFlagBounds);
                len = 0;
            }
        }
        int sp = 0;
        NodeIn<T> A, B;
        if (len > 0) {
            A.lk = load_links(links, base);
            fetch_up(A, base, rec, v, xch, C, r, act, err);
        }
        if (len > 1) B.lk = load_links(links, base + 1);
        for (int i = 0; i < len; i += 2) {
            {
                int4 lk2 = make_int4(0, 0, 0, 0);
                if (i + 2 < len) lk2 = load_links(links, base + i + 2);
                if (i + 1 < len) fetch_up(B, base + i + 1, rec, v, xch, C, r, act, err);
                node_up(A, stk, sp, out, xch, C, r, act, lane, err);
                A.lk = lk2;
            }
            if (i + 1 < len) {
                int4 lk2 = make_int4(0, 0, 0, 0);
                if (i + 3 < len) lk2 = load_links(links, base + i + 3);
                if (i + 2 < len) fetch_up(A, base + i + 2, rec, v, xch, C, r, act, err);
                node_up(B, stk, sp, out, xch, C, r, act, lane, err);
                B.lk = lk2;
            }
        }
    }
}

template <typename T>
__device__ __forceinline__ void fetch_down(NodeIn<T> &n, int s, const T *__restrict__ rec, const T *__restrict__ w,
                                           const T *__restrict__ xch, const Ctx &C, int r, bool act, int32_t *err) {
    load_g(n.g, rec + (int64_t)kRecWords * s);
    const int xref = n.lk.x, yref = n.lk.y, off = n.lk.z, meta = n.lk.w;
    const int dim = 3 * (int)(xref < 0) + 3 * (int)(yref < 0);
#pragma unroll
    for (int c = 0; c < 6; ++c) n.a[c] = n.b[c] = T(0);
    if (dim > 0) {
        if (off < 0 || (int64_t)off + dim > C.rows) {
            atomicOr(err, kFlagBounds);
        } else if (act) {
#pragma unroll
            for (int k = 0; k < 3; ++k) n.a[k] = w[velem(off, k, r, C)];
            if (dim == 6) {
#pragma unroll
                for (int k = 0; k < 3; ++k) n.a[3 + k] = w[velem(off + 3, k, r, C)];
            }
        }
    }
    if ((meta & kMetaTileRoot) && (!(meta & kMetaBodyRoot) || C.root_in)) {
        const int slot = meta >> kMetaSlotShift;
        if (slot >= C.xch_cap) {
            atomicOr(err, kFlagBounds);
        } else if (act) {
#pragma unroll
            for (int c = 0; c < 6; ++c) n.b[c] = xch[((int64_t)slot * 6 + c) * C.R + r];
        }
    }
}

template <typename T>
__device__ __forceinline__ void emit_child(int ref, const T (&L)[6], T *__restrict__ out, T *__restrict__ xch, T *stk,
                                           int &sp, const Ctx &C, int r, bool act, int lane, int32_t *err) {
    if (ref >= 0) {
        if (ref >= C.N) {
            atomicOr(err, kFlagBounds);
            return;
        }
        if (act) {
#pragma unroll
            for (int k = 0; k < 3; ++k) out[velem((int64_t)3 * ref, k, r, C)] = L[k];
        }
    } else if (ref == kRefStack) {
        push6(stk, sp, C.dmax, L, lane, err);
    } else {
        const int slot = ref_slot(ref);
        if (slot < 0 || slot >= C.xch_cap) {
            atomicOr(err, kFlagBounds);
            return;
        }
        if (act) {
#pragma unroll
            for (int c = 0; c < 6; ++c) xch[((int64_t)slot * 6 + c) * C.R + r] = L[c];
        }
    }
}

template <typename T>
__device__ __forceinline__ void node_down(const NodeIn<T> &n, T *stk, int &sp, T *__restrict__ out,
                                          T *__restrict__ xch, const Ctx &C, int r, bool act, int lane,
                                          int32_t *err) {
    const int xref = n.lk.x, yref = n.lk.y, meta = n.lk.w;
    T L[6];
    if (meta & kMetaTileRoot) {
        // from the exchange buffer; zeros for a body root unless the root
        // Velocity-set was given (full Q)
#pragma unroll
        for (int c = 0; c < 6; ++c) L[c] = n.b[c];
    } else {
        pop6(stk, sp, L, lane, err);
    }
    const T sx = n.g[kRecSx], sy = n.g[kRecSy];
    const bool xi = xref < 0, yi = yref < 0;
    T x9[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) x9[c] = L[3 + c];
#pragma unroll
    for (int c = 0; c < 6; ++c) x9[3 + c] = n.a[c];
    T st[3], Lx[6], Ly[6];
    if (xi && yi) {
        house_bwd<9>(x9, n.g);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Lx[3 + c] = x9[c];
            Ly[3 + c] = x9[3 + c];
            st[c] = x9[6 + c];
        }
    } else if (xi || yi) {
        house_bwd<6>(x9, n.g);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Lx[3 + c] = xi ? x9[c] : T(0);
            Ly[3 + c] = yi ? x9[c] : T(0);
            st[c] = x9[3 + c];
        }
    } else {
        house_bwd<3>(x9, n.g);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Lx[3 + c] = T(0);
            Ly[3 + c] = T(0);
            st[c] = x9[c];
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Lx[c] = sx * L[c] + sy * st[c];
        Ly[c] = sy * L[c] - sx * st[c];
    }
    // the child evaluated first upward is finished last downward
    if (meta & kMetaYFirst) {
        emit_child(yref, Ly, out, xch, stk, sp, C, r, act, lane, err);
        emit_child(xref, Lx, out, xch, stk, sp, C, r, act, lane, err);
    } else {
        emit_child(xref, Lx, out, xch, stk, sp, C, r, act, lane, err);
        emit_child(yref, Ly, out, xch, stk, sp, C, r, act, lane, err);
    }
}

template <typename T, int LPT>
__global__ void __launch_bounds__(64) k_down(int phase, const int32_t *__restrict__ phase_tab,
                                             const int32_t *__restrict__ tile_base,
                                             const int32_t *__restrict__ tile_len, const int32_t *__restrict__ links,
                                             const T *__restrict__ rec, const T *__restrict__ w, T *__restrict__ out,
                                             T *__restrict__ xch, Ctx C, int32_t *err) {
    extern __shared__ unsigned char smem_raw[];
    T *stk = reinterpret_cast<T *>(smem_raw);
    constexpr int TPW = 64 / LPT;
    const int lane = threadIdx.x;
    const int tslot = lane / LPT, rl = lane % LPT;
    const int tb = phase_tab[2 * phase], te = phase_tab[2 * phase + 1];
    const int ngroups = (te - tb + TPW - 1) / TPW;
    const int items = ngroups * C.nchunks;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int grp = item / C.nchunks, chunk = item - grp * C.nchunks;
        const int t = tb + grp * TPW + tslot;
        const int r = chunk * LPT + rl;
        const bool tvalid = t < te;
        const bool act = tvalid && r < C.R;
        int base = 0, len = 0;
        if (tvalid) {
            base = tile_base[t];
            len = tile_len[t];
            if (base < 0 || len < 0 || (int64_t)base + len > C.nsched) {
                atomicOr(err, kFlagBounds);
                len = 0;
            }
        }
        // node j of the sweep is schedule index last - j (reverse order)
        const int last = base + len - 1;
        int sp = 0;
        NodeIn<T> A, B;
        if (len > 0) {
            A.lk = load_links(links, last);
            fetch_down(A, last, rec, w, xch, C, r, act, err);
        }
        if (len > 1) B.lk = load_links(links, last - 1);
        for (int j = 0; j < len; j += 2) {
            {
                int4 lk2 = make_int4(0, 0, 0, 0);
                if (j + 2 < len) lk2 = load_links(links, last - j - 2);
                if (j + 1 < len) fetch_down(B, last - j - 1, rec, w, xch, C, r, act, err);
                node_down(A, stk, sp, out, xch, C, r, act, lane, err);
                A.lk = lk2;
            }
            if (j + 1 < len) {
                int4 lk2 = make_int4(0, 0, 0, 0);
                if (j + 3 < len) lk2 = load_links(links, last - j - 3);
                if (j + 2 < len) fetch_down(A, last - j - 2, rec, w, xch, C, r, act, err);
                node_down(B, stk, sp, out, xch, C, r, act, lane, err);
                B.lk = lk2;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Node-parallel sweeps (few right-hand sides): one lane per (node, column).
// A workgroup takes whole tiles of at most TS - 1 nodes, lane slot i of a
// tile holding the tile's i-th node in schedule order.  Every lane issues its
// node's record and memory inputs at once; the tile's dependencies are then
// resolved in LDS, one tree level per round, so no round waits on HBM.
//
// The schedule is a post-order that takes one child's subtree before the
// other's (yfirst in the links), so a node with two children in its own tile
// finds the child taken second in the slot just before its own, and the one
// taken first before that child's subtree; a node with one such child finds
// it in the slot before its own.  Subtree sizes (in nodes of the tile) are
// therefore all the upward sweep needs, and it computes them as it goes; the
// downward sweep finds them in a first, integer-only round.
//
// Every case of k (3, 6, 9) runs the length-9 reflectors on a zero-padded
// vector: the stored tails are zero beyond k, so the results equal the
// length-k products, and the lanes of a round do not diverge on k.
// ---------------------------------------------------------------------------

// Index of value k of exchange entry (slot, column r): [slot][R][6] (the
// layout of the wide sweeps) or [slot][6][R].
template <bool WX>
__device__ __forceinline__ int64_t xidx(int slot, int k, int r, const Ctx &C) {
    return WX ? ((int64_t)slot * C.R + r) * 6 + k : ((int64_t)slot * 6 + k) * C.R + r;
}

template <typename T, bool WX>
__device__ __forceinline__ void np_fetch(int ref, T (&m)[6], const T *__restrict__ v, const T *__restrict__ xch,
                                         const Ctx &C, int r, bool act, int32_t *err) {
    if (ref >= 0) {
        if (ref >= C.N) {
            atomicOr(err, kFlagBounds);
        } else if (act) {
#pragma unroll
            for (int c = 0; c < 3; ++c) m[c] = v[velem((int64_t)3 * ref, c, r, C)];
        }
    } else if (ref != kRefStack) {
        const int slot = ref_slot(ref);
        if (slot < 0 || slot >= C.xch_cap) {
            atomicOr(err, kFlagBounds);
        } else if (act) {
#pragma unroll
            for (int c = 0; c < 6; ++c) m[c] = xch[xidx<WX>(slot, c, r, C)];
        }
    }
}

// The node's record (reflectors, weights) and its links, which the record
// carries from element kRecLinks on.
template <typename T>
__device__ __forceinline__ int4 np_record(const T *__restrict__ rec, int s, T (&g)[26]) {
    const T *p = rec + (int64_t)kRecWords * s;
    load_g(g, p);
    const int2 *lk = reinterpret_cast<const int2 *>(p + kRecLinks);
    const int2 a = lk[0], b = lk[1];
    return make_int4(a.x, a.y, b.x, b.y);
}

// Slots of the children in the node's own tile (-1: elsewhere) from the
// subtree size z2 of the slot before q: (x slot, y slot).
__device__ __forceinline__ int2 np_children(int q, int xref, int yref, int meta, int z2) {
    const bool xs = xref == kRefStack, ys = yref == kRefStack;
    int xq = -1, yq = -1;
    if (xs && ys) {
        // the child taken second sits just before the node
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

// Work item geometry shared by both directions.
template <int NB, int CW, int TS>
struct NpGeom {
    static constexpr int TPB = NB / (TS * CW);  // tiles per workgroup
    int q, c, tl, i;
    __device__ NpGeom() {
        const int tid = threadIdx.x;
        q = tid / CW;
        c = tid - q * CW;
        tl = q / TS;
        i = q - tl * TS;
    }
};

// Upward (Algorithm 2) for one tile phase.
template <typename T, int NB, int CW, int TS, bool WX>
__global__ void __launch_bounds__(NB) k_up_np(int phase, const int32_t *__restrict__ phase_tab,
                                              const int32_t *__restrict__ tile_base,
                                              const int32_t *__restrict__ tile_len, const T *__restrict__ rec,
                                              const T *__restrict__ v, T *__restrict__ out, T *__restrict__ xch,
                                              Ctx C, int32_t *err) {
    __shared__ T sv[NB * 6];
    __shared__ int ssz[NB / CW];
    const NpGeom<NB, CW, TS> G;
    constexpr int TPB = NpGeom<NB, CW, TS>::TPB;
    const int tb = phase_tab[2 * phase], te = phase_tab[2 * phase + 1];
    const int items = ((te - tb + TPB - 1) / TPB) * C.nchunks;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int grp = item / C.nchunks, chunk = item - grp * C.nchunks;
        const int t = tb + grp * TPB + G.tl;
        const int r = chunk * CW + G.c;
        int base = 0, len = 0;
        if (t < te) {
            base = tile_base[t];
            len = tile_len[t];
            if (base < 0 || len < 0 || len > TS || (int64_t)base + len > C.nsched) {
                atomicOr(err, kFlagBounds);
                len = 0;
            }
        }
        const bool valid = G.i < len;
        const bool act = valid && r < C.R;
        T g[26];
        T ma[6], mb[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) ma[k] = mb[k] = T(0);
        int4 lk = make_int4(0, 0, 0, 0);
        if (valid) {
            lk = np_record(rec, base + G.i, g);
            np_fetch<T, WX>(lk.x, ma, v, xch, C, r, act, err);
            np_fetch<T, WX>(lk.y, mb, v, xch, C, r, act, err);
        }
        const int xref = lk.x, yref = lk.y, off = lk.z, meta = lk.w;
        const int nst = (int)(xref == kRefStack) + (int)(yref == kRefStack);
        if (valid && nst > 0 && G.i == 0) {
            // a tile's first node has no node of its own tile before it
            atomicOr(err, kFlagStack);
        }
        const int q0 = G.tl * TS;  // the tile's first slot
        bool done = !valid || (nst > 0 && G.i == 0);
        __syncthreads();  // the previous item's rounds are over
        if (G.c == 0) ssz[G.q] = 0;
        for (int round = 0; round <= TS; ++round) {
            if (!__syncthreads_or(!done)) break;
            // read the subtree sizes published by earlier rounds
            int z2 = 0, z1 = 0;
            int2 ch = make_int2(-1, -1);
            bool ready = false;
            if (!done) {
                if (nst == 0) {
                    ready = true;
                } else {
                    z2 = ssz[G.q - 1];
                    if (z2 > 0) {
                        ch = np_children(G.q, xref, yref, meta, z2);
                        if (nst == 1) {
                            ready = true;
                        } else {
                            const int q1 = G.q - 1 - z2;
                            if (q1 < q0) {
                                atomicOr(err, kFlagStack);
                                done = true;
                            } else {
                                z1 = ssz[q1];
                                ready = z1 > 0;
                            }
                        }
                    }
                }
            }
            __syncthreads();
            if (ready) {
                T mx[6], my[6];
                const int cx = ch.x >= 0 ? ch.x : 0, cy = ch.y >= 0 ? ch.y : 0;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    mx[k] = ch.x >= 0 ? sv[(cx * 6 + k) * CW + G.c] : ma[k];
                    my[k] = ch.y >= 0 ? sv[(cy * 6 + k) * CW + G.c] : mb[k];
                }
                const T sx = g[kRecSx], sy = g[kRecSy];
                const bool xi = xref < 0, yi = yref < 0;
                T mp[6], sh[3], t9[9];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    mp[k] = sx * mx[k] + sy * my[k];
                    sh[k] = sy * mx[k] - sx * my[k];
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    t9[k] = xi ? mx[3 + k] : (yi ? my[3 + k] : sh[k]);
                    t9[3 + k] = (xi && yi) ? my[3 + k] : ((xi || yi) ? sh[k] : T(0));
                    t9[6 + k] = (xi && yi) ? sh[k] : T(0);
                }
                house_fwd<9>(t9, g);
#pragma unroll
                for (int k = 0; k < 3; ++k) mp[3 + k] = t9[k];
                const int dim = 3 * ((int)xi + (int)yi);
                if (dim > 0) {
                    if (off < 0 || (int64_t)off + dim > C.rows) {
                        atomicOr(err, kFlagBounds);
                    } else if (act) {
#pragma unroll
                        for (int k = 0; k < 3; ++k) out[velem(off, k, r, C)] = t9[3 + k];
                        if (dim == 6) {
#pragma unroll
                            for (int k = 0; k < 3; ++k) out[velem(off + 3, k, r, C)] = t9[6 + k];
                        }
                    }
                }
                if (meta & kMetaTileRoot) {
                    const int slot = meta >> kMetaSlotShift;
                    if (slot >= C.xch_cap) {
                        atomicOr(err, kFlagBounds);
                    } else if (act) {
#pragma unroll
                        for (int k = 0; k < 6; ++k) xch[xidx<WX>(slot, k, r, C)] = mp[k];
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 6; ++k) sv[(G.q * 6 + k) * CW + G.c] = mp[k];
                }
                if (G.c == 0) ssz[G.q] = 1 + z2 + z1;
                done = true;
            }
        }
        if (!done) atomicOr(err, kFlagStack);
    }
}

// Downward (Algorithm 3) for one tile phase.  The node's own Velocity-set
// arrives in its LDS slot from its parent (a tile root: from the exchange
// buffer, zero at a body root unless given).
template <typename T, int NB, int CW, int TS, bool WX>
__global__ void __launch_bounds__(NB) k_down_np(int phase, const int32_t *__restrict__ phase_tab,
                                                const int32_t *__restrict__ tile_base,
                                                const int32_t *__restrict__ tile_len, const T *__restrict__ rec,
                                                const T *__restrict__ w, T *__restrict__ out, T *__restrict__ xch,
                                                Ctx C, int32_t *err) {
    __shared__ T sv[NB * 6];
    __shared__ int ssz[NB / CW];
    __shared__ int sready[NB / CW];
    const NpGeom<NB, CW, TS> G;
    constexpr int TPB = NpGeom<NB, CW, TS>::TPB;
    const int tb = phase_tab[2 * phase], te = phase_tab[2 * phase + 1];
    const int items = ((te - tb + TPB - 1) / TPB) * C.nchunks;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int grp = item / C.nchunks, chunk = item - grp * C.nchunks;
        const int t = tb + grp * TPB + G.tl;
        const int r = chunk * CW + G.c;
        int base = 0, len = 0;
        if (t < te) {
            base = tile_base[t];
            len = tile_len[t];
            if (base < 0 || len < 0 || len > TS || (int64_t)base + len > C.nsched) {
                atomicOr(err, kFlagBounds);
                len = 0;
            }
        }
        const bool valid = G.i < len;
        const bool act = valid && r < C.R;
        T g[26];
        T a[6], lin[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) a[k] = lin[k] = T(0);
        int4 lk = make_int4(0, 0, 0, 0);
        if (valid) {
            lk = np_record(rec, base + G.i, g);
            const int off = lk.z;
            const int dim = 3 * (int)(lk.x < 0) + 3 * (int)(lk.y < 0);
            if (dim > 0) {
                if (off < 0 || (int64_t)off + dim > C.rows) {
                    atomicOr(err, kFlagBounds);
                } else if (act) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) a[k] = w[velem(off, k, r, C)];
                    if (dim == 6) {
#pragma unroll
                        for (int k = 0; k < 3; ++k) a[3 + k] = w[velem(off + 3, k, r, C)];
                    }
                }
            }
            if ((lk.w & kMetaTileRoot) && (!(lk.w & kMetaBodyRoot) || C.root_in)) {
                const int slot = lk.w >> kMetaSlotShift;
                if (slot >= C.xch_cap) {
                    atomicOr(err, kFlagBounds);
                } else if (act) {
#pragma unroll
                    for (int k = 0; k < 6; ++k) lin[k] = xch[xidx<WX>(slot, k, r, C)];
                }
            }
        }
        const int xref = lk.x, yref = lk.y, meta = lk.w;
        const int nst = (int)(xref == kRefStack) + (int)(yref == kRefStack);
        const int q0 = G.tl * TS;
        bool bad = valid && nst > 0 && G.i == 0;
        if (bad) atomicOr(err, kFlagStack);
        // round 0: subtree sizes, bottom up (integers only)
        bool sized = !valid || bad;
        __syncthreads();  // the previous item's rounds are over
        if (G.c == 0) {
            ssz[G.q] = (valid && nst == 0) ? 1 : 0;
            sready[G.q] = 0;
        }
        if (valid && nst == 0) sized = true;
        for (int round = 0; round <= TS; ++round) {
            if (!__syncthreads_or(!sized)) break;
            int nz = 0;
            if (!sized) {
                const int z2 = ssz[G.q - 1];
                if (z2 > 0) {
                    if (nst == 1) {
                        nz = 1 + z2;
                    } else if (G.q - 1 - z2 < q0) {
                        atomicOr(err, kFlagStack);
                        sized = true;
                        bad = true;
                    } else {
                        const int z1 = ssz[G.q - 1 - z2];
                        if (z1 > 0) nz = 1 + z2 + z1;
                    }
                }
            }
            __syncthreads();
            if (nz > 0) {
                if (G.c == 0) ssz[G.q] = nz;
                sized = true;
            }
        }
        if (!sized) {
            atomicOr(err, kFlagStack);
            bad = true;
        }
        __syncthreads();
        int2 ch = make_int2(-1, -1);
        if (valid && !bad && nst > 0) ch = np_children(G.q, xref, yref, meta, ssz[G.q - 1]);
        // rounds 1..: Velocity-sets, top down
        bool done = !valid || bad;
        for (int round = 0; round <= TS; ++round) {
            if (!__syncthreads_or(!done)) break;
            const bool ready = !done && ((meta & kMetaTileRoot) || sready[G.q] != 0);
            __syncthreads();
            if (ready) {
                T L[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) L[k] = (meta & kMetaTileRoot) ? lin[k] : sv[(G.q * 6 + k) * CW + G.c];
                const T sx = g[kRecSx], sy = g[kRecSy];
                const bool xi = xref < 0, yi = yref < 0;
                T x9[9];
#pragma unroll
                for (int k = 0; k < 3; ++k) x9[k] = L[3 + k];
#pragma unroll
                for (int k = 0; k < 6; ++k) x9[3 + k] = a[k];
                house_bwd<9>(x9, g);
                T st[3], Lx[6], Ly[6];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Lx[3 + k] = xi ? x9[k] : T(0);
                    Ly[3 + k] = (xi && yi) ? x9[3 + k] : (yi ? x9[k] : T(0));
                    st[k] = (xi && yi) ? x9[6 + k] : ((xi || yi) ? x9[3 + k] : x9[k]);
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Lx[k] = sx * L[k] + sy * st[k];
                    Ly[k] = sy * L[k] - sx * st[k];
                }
                auto emit = [&](int ref, int cq, const T (&Lc)[6]) {
                    if (ref >= 0) {
                        if (ref >= C.N) {
                            atomicOr(err, kFlagBounds);
                        } else if (act) {
#pragma unroll
                            for (int k = 0; k < 3; ++k) out[velem((int64_t)3 * ref, k, r, C)] = Lc[k];
                        }
                    } else if (ref == kRefStack) {
                        if (cq < q0 || cq >= G.q) {
                            atomicOr(err, kFlagStack);
                            return;
                        }
#pragma unroll
                        for (int k = 0; k < 6; ++k) sv[(cq * 6 + k) * CW + G.c] = Lc[k];
                        if (G.c == 0) sready[cq] = 1;
                    } else {
                        const int slot = ref_slot(ref);
                        if (slot < 0 || slot >= C.xch_cap) {
                            atomicOr(err, kFlagBounds);
                        } else if (act) {
#pragma unroll
                            for (int k = 0; k < 6; ++k) xch[xidx<WX>(slot, k, r, C)] = Lc[k];
                        }
                    }
                };
                emit(xref, ch.x, Lx);
                emit(yref, ch.y, Ly);
                done = true;
            }
        }
        if (!done) atomicOr(err, kFlagStack);
    }
}

// ---------------------------------------------------------------------------
// Wide sweeps: a lane group of 32 or 64 lanes (one right-hand side per lane)
// sweeps a run of whole tiles; a wave holds two groups of 32 or one of 64.
//
// The sweep order is fixed at build time, and so is the stack depth at every
// node: the record names the LDS slots of the two children and of the node's
// own result, so a node step has no stack pointer and no data-dependent
// branches; the case-dependent packing of the length-9 vector is done with
// selects.
//
// Latency: records are loaded PR nodes ahead and memory inputs NR - 1 nodes
// ahead.  Vector data goes through raw buffer loads and stores whose lanes
// are switched off by an out-of-range offset (loads return 0, stores are
// dropped), so every memory instruction is issued unconditionally and the
// compiler can wait for exactly the loads a node needs instead of draining
// the stores of earlier nodes.  Each buffer must stay below 2 GiB.
//
// Bead and residue vectors and node records are touched once per sweep, so
// their accesses carry the non-temporal policy (the nt bit of the buffer
// instruction's cache-policy field; a plain nontemporal load for records);
// the exchange entries, which the next phase reads back, keep the default.
// Measured on the bench workload: first-phase launches 3% shorter.
// ---------------------------------------------------------------------------

constexpr int kNT = 2;  // cache-policy operand of the streaming buffer accesses: nt

// Ring depths of the wide sweeps: records kPR nodes ahead, memory inputs
// kNR - 1 nodes ahead, in the first tile phase (1) and the later ones (L).
constexpr int kPR1 = 6, kNR1 = 3, kPRL = 6, kNRL = 3;
constexpr int kPR1d = 6, kNR1d = 3, kPRLd = 6, kNRLd = 3;

template <typename T>
__device__ __forceinline__ T bld(rsrc_t r, uint32_t vo, uint32_t so);
template <>
__device__ __forceinline__ float bld<float>(rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, kNT));
}
template <>
__device__ __forceinline__ double bld<double>(rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, kNT));
}

template <typename T>
__device__ __forceinline__ void bst(T v, rsrc_t r, uint32_t vo, uint32_t so);
template <>
__device__ __forceinline__ void bst<float>(float v, rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, vo, so, kNT);
}
template <>
__device__ __forceinline__ void bst<double>(double v, rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, kNT);
}

// ---------------------------------------------------------------------------
// Lane-per-tile sweeps of the first tile phase for few right-hand sides: a
// group of LPT lanes (one column each) walks one tile's nodes in schedule
// order (reverse order downward).  Every memory access is issued whether or
// not the node needs it, with an out-of-range offset where it does not, so
// that the compiler's wait counts are exact and no node waits for the stores
// of the nodes before it.  Three streams run ahead of the node being
// computed: its link words four nodes ahead (in FP32 with its reflectors),
// then (with two nodes of slack for the links to arrive) the vectors the
// links address, and in FP64 the reflectors, two nodes ahead.  Pending
// results sit in the fixed LDS slots the links name
// (as in the wide sweeps), plus one sink slot for the writes of absent
// values.  In the first phase every child is a bead or a node of the same
// tile, and only the tile root touches the exchange buffer.
// ---------------------------------------------------------------------------
constexpr int kLaneRing = 5;  // ring slots: links 4 nodes ahead, inputs 2
// How far ahead a lane loads a record's reflectors.  FP32: with the links,
// 4 nodes ahead, so the record's one 128-byte line is fetched once (loaded 2
// nodes after its links, the line had often left L2 on large batches, where
// each lane keeps several records in flight, and came from HBM twice).  FP64
// records span two lines, and two more nodes of FP64 reflectors would not
// fit the register budget: 2 nodes ahead.
template <typename T>
constexpr int lane_g_ahead() {
    return sizeof(T) == 4 ? 4 : 2;
}

// Buffer accesses of the lane kernels with the default cache policy: a lane
// touches parts of a line in several instructions (a record in eight loads, a
// bead's three values in three), which the non-temporal policy of the wide
// sweeps would send to memory once per instruction.
template <typename T>
__device__ __forceinline__ T bldc(rsrc_t r, uint32_t vo, uint32_t so) {
    if constexpr (sizeof(T) == 4) return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    else return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}

template <typename T>
__device__ __forceinline__ void bstc(T v, rsrc_t r, uint32_t vo, uint32_t so) {
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, vo, so, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, 0);
}

// Three or six consecutive values at byte offset vo (kOOB: switched off), for
// the lane kernels' single right-hand side: with R = 1 a bead's triple, a
// node's residue rows and an exchange entry are contiguous in either layout,
// so one wide access replaces one per value (each lane of the lane kernels
// touches its own lines, and the number of accesses bounds them).  Offsets
// stay in the vector offset, as for every store wider than 64 bits.
template <typename T>
__device__ __forceinline__ void bld3c(rsrc_t r, uint32_t vo, T (&m)[3]) {
    if constexpr (sizeof(T) == 4) {
        const u32x3 a = __builtin_amdgcn_raw_buffer_load_b96(r, vo, 0, 0);
        m[0] = __uint_as_float(a.x);
        m[1] = __uint_as_float(a.y);
        m[2] = __uint_as_float(a.z);
    } else {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, vo, 0, 0);
        const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(r, vo + 16, 0, 0);
        m[0] = __builtin_bit_cast(double, u32x2{a.x, a.y});
        m[1] = __builtin_bit_cast(double, u32x2{a.z, a.w});
        m[2] = __builtin_bit_cast(double, b);
    }
}

template <typename T>
__device__ __forceinline__ void bst3c(T m0, T m1, T m2, rsrc_t r, uint32_t vo) {
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b96(u32x3{__float_as_uint(m0), __float_as_uint(m1), __float_as_uint(m2)}, r,
                                              vo, 0, 0);
    } else {
        const u32x2 a = __builtin_bit_cast(u32x2, m0), b = __builtin_bit_cast(u32x2, m1);
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{a.x, a.y, b.x, b.y}, r, vo, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, m2), r, vo + 16, 0, 0);
    }
}

template <typename T>
__device__ __forceinline__ void bld6c(rsrc_t r, uint32_t vo, T (&m)[6]) {
    T a[3], b[3];
    bld3c<T>(r, vo, a);
    bld3c<T>(r, vo + 3 * (uint32_t)sizeof(T), b);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        m[k] = a[k];
        m[3 + k] = b[k];
    }
}

template <typename T>
__device__ __forceinline__ void bst6c(const T (&m)[6], rsrc_t r, uint32_t vo) {
    bst3c<T>(m[0], m[1], m[2], r, vo);
    bst3c<T>(m[3], m[4], m[5], r, vo + 3 * (uint32_t)sizeof(T));
}

struct LaneLk {
    int xref, yref, off, meta, slots;
};

// The link words of the record at byte offset bo (kOOB: all zero).
template <typename T>
__device__ __forceinline__ void lane_links(rsrc_t rr, uint32_t bo, LaneLk &l) {
    constexpr uint32_t L0 = kRecLinks * sizeof(T);
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(rr, bo + L0, 0, 0);
    const unsigned b = __builtin_amdgcn_raw_buffer_load_b32(rr, bo + L0 + 16, 0, 0);
    l.xref = (int)a.x;
    l.yref = (int)a.y;
    l.off = (int)a.z;
    l.meta = (int)a.w;
    l.slots = (int)b;
}

// The reflectors and weights (elements 0..25) of the record at byte offset bo.
template <typename T>
__device__ __forceinline__ void lane_g(rsrc_t rr, uint32_t bo, T (&g)[26]) {
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rr, bo + 16 * q, 0, 0);
            g[4 * q] = __uint_as_float(w.x);
            g[4 * q + 1] = __uint_as_float(w.y);
            g[4 * q + 2] = __uint_as_float(w.z);
            g[4 * q + 3] = __uint_as_float(w.w);
        }
        const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rr, bo + 96, 0, 0);
        g[24] = __uint_as_float(w.x);
        g[25] = __uint_as_float(w.y);
    } else {
#pragma unroll
        for (int q = 0; q < 13; ++q) {
            const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rr, bo + 16 * q, 0, 0);
            g[2 * q] = __hiloint2double((int)w.y, (int)w.x);
            g[2 * q + 1] = __hiloint2double((int)w.w, (int)w.z);
        }
    }
}

template <typename T>
__device__ __forceinline__ void lane_get6(const T *lds, int slot, int lane, T (&m)[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) m[k] = lds[(slot * 6 + k) * 64 + lane];
}

template <typename T>
__device__ __forceinline__ void lane_put6(T *lds, int slot, int lane, const T (&m)[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) lds[(slot * 6 + k) * 64 + lane] = m[k];
}

// Byte offset of element (row0 + k, r) of a vector, or kOOB unless en.
template <typename T>
__device__ __forceinline__ uint32_t lane_vo(bool en, int64_t row0, int k, int r, const Ctx &C) {
    return en ? (uint32_t)(velem(row0, k, r, C) * (int64_t)sizeof(T)) : kOOB;
}

// The tile of lane group tslot in work item `item`: (base, len, column r).
__device__ __forceinline__ void lane_tile(int item, int tslot, int rl, int LPT, int TPW, int tb, int te,
                                          const int32_t *__restrict__ tile_base,
                                          const int32_t *__restrict__ tile_len, const Ctx &C, int &base, int &len,
                                          int &r, int &bad) {
    const int grp = item / C.nchunks, chunk = item - grp * C.nchunks;
    const int t = tb + grp * TPW + tslot;
    r = chunk * LPT + rl;
    base = 0;
    len = 0;
    if (t < te) {
        base = tile_base[t];
        len = tile_len[t];
        if (base < 0 || len < 0 || (int64_t)base + len > C.nsched) {
            bad |= kFlagBounds;
            base = 0;
            len = 0;
        }
    }
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) v = max(v, __shfl_xor(v, sh, 64));
    return v;
}

template <typename T, int LPT>
__global__ void __launch_bounds__(64) k_up_lane(const int32_t *__restrict__ phase_tab,
                                                const int32_t *__restrict__ tile_base,
                                                const int32_t *__restrict__ tile_len, const T *__restrict__ rec,
                                                uint32_t rec_bytes, const T *__restrict__ v, T *__restrict__ out,
                                                T *__restrict__ xch, Ctx C, int32_t *err) {
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    constexpr int TPW = 64 / LPT, RD = kLaneRing, kLaneGAhead = lane_g_ahead<T>();
    constexpr uint32_t RB = kRecWords * sizeof(T);
    const int lane = threadIdx.x;
    const int tslot = lane / LPT, rl = lane % LPT;
    const int sink = C.nslot;
    const rsrc_t rr = make_rsrc(rec, rec_bytes), rv = make_rsrc(v, C.in_bytes), ro = make_rsrc(out, C.out_bytes),
                 rx = make_rsrc(xch, C.xch_bytes);
    // one right-hand side: triples, residue rows and exchange entries are
    // contiguous (one wide access each)
    const bool contig = LPT == 1 && C.R == 1;
    const int tb = phase_tab[2], te = phase_tab[3];
    const int items = ((te - tb + TPW - 1) / TPW) * C.nchunks;
    int bad = 0;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        int base, len, r;
        lane_tile(item, tslot, rl, LPT, TPW, tb, te, tile_base, tile_len, C, base, len, r, bad);
        const bool act = r < C.R;
        const int lmax = wave_max(len);
        auto bo = [&](int i) -> uint32_t { return i < len ? (uint32_t)(base + i) * RB : kOOB; };
        // the bead children's vectors of node i (links l)
        auto in_of = [&](int i, const LaneLk &l, T (&a)[3], T (&b)[3]) {
            const bool live = i < len && act;
            const bool xb = live && l.xref >= 0 && l.xref < C.N, yb = live && l.yref >= 0 && l.yref < C.N;
            if (contig) {
                bld3c<T>(rv, lane_vo<T>(xb, 3 * (int64_t)l.xref, 0, r, C), a);
                bld3c<T>(rv, lane_vo<T>(yb, 3 * (int64_t)l.yref, 0, r, C), b);
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    a[k] = bldc<T>(rv, lane_vo<T>(xb, 3 * (int64_t)l.xref, k, r, C), 0);
                    b[k] = bldc<T>(rv, lane_vo<T>(yb, 3 * (int64_t)l.yref, k, r, C), 0);
                }
            }
        };
        LaneLk lq[RD];
        T gq[RD][26], ia[RD][3], ib[RD][3];
#pragma unroll
        for (int u = 0; u < RD - 1; ++u) {
            lane_links<T>(rr, bo(u), lq[u]);
            if (u < kLaneGAhead) lane_g<T>(rr, bo(u), gq[u]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) in_of(u, lq[u], ia[u], ib[u]);
        for (int i0 = 0; i0 < lmax; i0 += RD) {
#pragma unroll
            for (int u = 0; u < RD; ++u) {
                const int i = i0 + u;
                lane_links<T>(rr, bo(i + 4), lq[(u + 4) % RD]);
                lane_g<T>(rr, bo(i + kLaneGAhead), gq[(u + kLaneGAhead) % RD]);
                in_of(i + 2, lq[(u + 2) % RD], ia[(u + 2) % RD], ib[(u + 2) % RD]);
                // node i (Eqs. 4.2-4.3)
                const LaneLk &n = lq[u];
                const T(&g)[26] = gq[u];
                const bool live = i < len;
                const bool xst = n.xref == kRefStack, yst = n.yref == kRefStack;
                const int xs = min(n.slots & 0xff, sink), ys = min((n.slots >> 8) & 0xff, sink);
                T mx[6], my[6];
                lane_get6<T>(lds, xs, lane, mx);
                lane_get6<T>(lds, ys, lane, my);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    mx[k] = xst ? mx[k] : (k < 3 ? ia[u][k] : T(0));
                    my[k] = yst ? my[k] : (k < 3 ? ib[u][k] : T(0));
                }
                const T sx = g[kRecSx], sy = g[kRecSy];
                const bool xi = n.xref < 0, yi = n.yref < 0;
                const bool both = xi && yi, any = xi || yi;
                T mp[6], tt[3], t9[9];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    mp[k] = sx * mx[k] + sy * my[k];
                    tt[k] = sy * mx[k] - sx * my[k];
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    t9[k] = xi ? mx[3 + k] : (yi ? my[3 + k] : tt[k]);
                    t9[3 + k] = both ? my[3 + k] : (any ? tt[k] : T(0));
                    t9[6 + k] = both ? tt[k] : T(0);
                }
                house_fwd<9>(t9, g);
#pragma unroll
                for (int k = 0; k < 3; ++k) mp[3 + k] = t9[k];
                const bool troot = (n.meta & kMetaTileRoot) != 0;
                const int dim = 3 * ((int)xi + (int)yi);
                const bool rok = n.off >= 0 && (int64_t)n.off + dim <= C.rows;
                const int slot = n.meta >> kMetaSlotShift;
                const bool xok = slot < C.xch_cap;
                if (live && ((dim > 0 && !rok) || (troot && !xok) || (!xst && n.xref < 0) || (!yst && n.yref < 0) ||
                             n.xref >= C.N || n.yref >= C.N))
                    bad |= kFlagBounds;
                const bool en = live && act && rok;
                const bool xen = live && act && troot && xok;
                const uint32_t xb0 = xen ? (uint32_t)(xidx<false>(slot, 0, r, C) * (int64_t)sizeof(T)) : kOOB;
                if (contig) {
                    bst3c<T>(t9[3], t9[4], t9[5], ro, lane_vo<T>(en && any, n.off, 0, r, C));
                    bst3c<T>(t9[6], t9[7], t9[8], ro, lane_vo<T>(en && both, (int64_t)n.off + 3, 0, r, C));
                    bst6c<T>(mp, rx, xb0);
                } else {
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        bstc<T>(t9[3 + k], ro, lane_vo<T>(en && any, n.off, k, r, C), 0);
                        bstc<T>(t9[6 + k], ro, lane_vo<T>(en && both, (int64_t)n.off + 3, k, r, C), 0);
                    }
                    const uint32_t xstep = (uint32_t)(C.R * sizeof(T));
#pragma unroll
                    for (int k = 0; k < 6; ++k) bstc<T>(mp[k], rx, xb0 + (xen ? k * xstep : 0), 0);
                }
                lane_put6<T>(lds, (live && !troot) ? min((n.slots >> 16) & 0xff, sink) : sink, lane, mp);
            }
        }
    }
    if (bad) atomicOr(err, bad);
}

template <typename T, int LPT>
__global__ void __launch_bounds__(64) k_down_lane(const int32_t *__restrict__ phase_tab,
                                                  const int32_t *__restrict__ tile_base,
                                                  const int32_t *__restrict__ tile_len, const T *__restrict__ rec,
                                                  uint32_t rec_bytes, const T *__restrict__ w, T *__restrict__ out,
                                                  const T *__restrict__ xch, Ctx C, int32_t *err) {
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    constexpr int TPW = 64 / LPT, RD = kLaneRing, kLaneGAhead = lane_g_ahead<T>();
    constexpr uint32_t RB = kRecWords * sizeof(T);
    const int lane = threadIdx.x;
    const int tslot = lane / LPT, rl = lane % LPT;
    const int sink = C.nslot;
    const rsrc_t rr = make_rsrc(rec, rec_bytes), rw = make_rsrc(w, C.in_bytes), ro = make_rsrc(out, C.out_bytes),
                 rx = make_rsrc(xch, C.xch_bytes);
    const bool contig = LPT == 1 && C.R == 1;  // as in k_up_lane
    const int tb = phase_tab[2], te = phase_tab[3];
    const int items = ((te - tb + TPW - 1) / TPW) * C.nchunks;
    int bad = 0;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        int base, len, r;
        lane_tile(item, tslot, rl, LPT, TPW, tb, te, tile_base, tile_len, C, base, len, r, bad);
        const bool act = r < C.R;
        const int lmax = wave_max(len);
        const int last = base + len - 1;  // node j of the sweep is schedule index last - j
        auto bo = [&](int j) -> uint32_t { return j < len ? (uint32_t)(last - j) * RB : kOOB; };
        // the node's residue coefficients and, at a tile root, its
        // Velocity-set from the exchange buffer (zero at a body root unless
        // given)
        auto in_of = [&](int j, const LaneLk &l, T (&a)[6], T (&lv)[6]) {
            const bool live = j < len && act;
            const int dim = 3 * (int)(l.xref < 0) + 3 * (int)(l.yref < 0);
            const bool rok = l.off >= 0 && (int64_t)l.off + dim <= C.rows;
            const int slot = l.meta >> kMetaSlotShift;
            const bool xin = live && (l.meta & kMetaTileRoot) && (!(l.meta & kMetaBodyRoot) || C.root_in) &&
                             slot < C.xch_cap;
            const uint32_t xb0 = xin ? (uint32_t)(xidx<false>(slot, 0, r, C) * (int64_t)sizeof(T)) : kOOB;
            if (contig) {
                T a0[3], a1[3];
                bld3c<T>(rw, lane_vo<T>(live && rok && dim >= 3, l.off, 0, r, C), a0);
                bld3c<T>(rw, lane_vo<T>(live && rok && dim == 6, (int64_t)l.off + 3, 0, r, C), a1);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    a[k] = a0[k];
                    a[3 + k] = a1[k];
                }
                bld6c<T>(rx, xb0, lv);
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    a[k] = bldc<T>(rw, lane_vo<T>(live && rok && dim >= 3, l.off, k, r, C), 0);
                    a[3 + k] = bldc<T>(rw, lane_vo<T>(live && rok && dim == 6, (int64_t)l.off + 3, k, r, C), 0);
                }
                const uint32_t xstep = (uint32_t)(C.R * sizeof(T));
#pragma unroll
                for (int k = 0; k < 6; ++k) lv[k] = bldc<T>(rx, xb0 + (xin ? k * xstep : 0), 0);
            }
        };
        LaneLk lq[RD];
        T gq[RD][26], ia[RD][6], il[RD][6];
#pragma unroll
        for (int u = 0; u < RD - 1; ++u) {
            lane_links<T>(rr, bo(u), lq[u]);
            if (u < kLaneGAhead) lane_g<T>(rr, bo(u), gq[u]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) in_of(u, lq[u], ia[u], il[u]);
        for (int j0 = 0; j0 < lmax; j0 += RD) {
#pragma unroll
            for (int u = 0; u < RD; ++u) {
                const int j = j0 + u;
                lane_links<T>(rr, bo(j + 4), lq[(u + 4) % RD]);
                lane_g<T>(rr, bo(j + kLaneGAhead), gq[(u + kLaneGAhead) % RD]);
                in_of(j + 2, lq[(u + 2) % RD], ia[(u + 2) % RD], il[(u + 2) % RD]);
                // node j (Algorithm 3)
                const LaneLk &n = lq[u];
                const T(&g)[26] = gq[u];
                const bool live = j < len;
                const bool troot = (n.meta & kMetaTileRoot) != 0;
                const int os = min((n.slots >> 16) & 0xff, sink);
                T L[6];
                lane_get6<T>(lds, os, lane, L);
#pragma unroll
                for (int k = 0; k < 6; ++k) L[k] = troot ? il[u][k] : L[k];
                const T sx = g[kRecSx], sy = g[kRecSy];
                const bool xi = n.xref < 0, yi = n.yref < 0;
                const bool both = xi && yi, any = xi || yi;
                T x9[9];
#pragma unroll
                for (int k = 0; k < 3; ++k) x9[k] = L[3 + k];
#pragma unroll
                for (int k = 0; k < 6; ++k) x9[3 + k] = ia[u][k];
                house_bwd<9>(x9, g);
                T st[3], Lx[6], Ly[6];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Lx[3 + k] = xi ? x9[k] : T(0);
                    Ly[3 + k] = both ? x9[3 + k] : (yi ? x9[k] : T(0));
                    st[k] = both ? x9[6 + k] : (any ? x9[3 + k] : x9[k]);
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Lx[k] = sx * L[k] + sy * st[k];
                    Ly[k] = sy * L[k] - sx * st[k];
                }
                const bool xst = n.xref == kRefStack, yst = n.yref == kRefStack;
                if (live && ((!xst && n.xref < 0) || (!yst && n.yref < 0) || n.xref >= C.N || n.yref >= C.N))
                    bad |= kFlagBounds;
                const bool en = live && act;
                const bool xb = en && n.xref >= 0 && n.xref < C.N, yb = en && n.yref >= 0 && n.yref < C.N;
                if (contig) {
                    bst3c<T>(Lx[0], Lx[1], Lx[2], ro, lane_vo<T>(xb, 3 * (int64_t)n.xref, 0, r, C));
                    bst3c<T>(Ly[0], Ly[1], Ly[2], ro, lane_vo<T>(yb, 3 * (int64_t)n.yref, 0, r, C));
                } else {
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        bstc<T>(Lx[k], ro, lane_vo<T>(xb, 3 * (int64_t)n.xref, k, r, C), 0);
                        bstc<T>(Ly[k], ro, lane_vo<T>(yb, 3 * (int64_t)n.yref, k, r, C), 0);
                    }
                }
                lane_put6<T>(lds, (live && xst) ? min(n.slots & 0xff, sink) : sink, lane, Lx);
                lane_put6<T>(lds, (live && yst) ? min((n.slots >> 8) & 0xff, sink) : sink, lane, Ly);
            }
        }
    }
    if (bad) atomicOr(err, bad);
}

// Cache policy of the exchange accesses: the default, or (kSC1) the bit
// that agent-scope relaxed atomics carry, which makes each access coherent
// across the L2 caches of the device's compute dies.  The fused upward sweep
// uses it, because there the entries pass between workgroups of one launch.
constexpr int kSC1 = 16;

// The six values of one exchange entry (slot, rhs) are contiguous.
template <int XP = 0>
__device__ __forceinline__ void bld6(rsrc_t r, uint32_t vo, float (&m)[6]) {
    const u32x3 a = __builtin_amdgcn_raw_buffer_load_b96(r, vo, 0, XP);
    const u32x3 b = __builtin_amdgcn_raw_buffer_load_b96(r, vo, 12, XP);
    m[0] = __uint_as_float(a.x);
    m[1] = __uint_as_float(a.y);
    m[2] = __uint_as_float(a.z);
    m[3] = __uint_as_float(b.x);
    m[4] = __uint_as_float(b.y);
    m[5] = __uint_as_float(b.z);
}
template <int XP = 0>
__device__ __forceinline__ void bld6(rsrc_t r, uint32_t vo, double (&m)[6]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, vo, 16 * k, XP);
        m[2 * k] = __builtin_bit_cast(double, u32x2{a.x, a.y});
        m[2 * k + 1] = __builtin_bit_cast(double, u32x2{a.z, a.w});
    }
}
template <int XP = 0>
__device__ __forceinline__ void bst6(rsrc_t r, uint32_t vo, const float (&m)[6]) {
    __builtin_amdgcn_raw_buffer_store_b96(u32x3{__float_as_uint(m[0]), __float_as_uint(m[1]), __float_as_uint(m[2])},
                                          r, vo, 0, XP);
    __builtin_amdgcn_raw_buffer_store_b96(u32x3{__float_as_uint(m[3]), __float_as_uint(m[4]), __float_as_uint(m[5])},
                                          r, vo, 12, XP);
}
template <int XP = 0>
__device__ __forceinline__ void bst6(rsrc_t r, uint32_t vo, const double (&m)[6]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const u32x2 a = __builtin_bit_cast(u32x2, m[2 * k]), b = __builtin_bit_cast(u32x2, m[2 * k + 1]);
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{a.x, a.y, b.x, b.y}, r, vo, 16 * k, XP);
    }
}

// lane W of each 16-lane group (ds_swizzle bit mode: and 0x10, or W)
template <int W>
__device__ __forceinline__ float bcast16(float v) {
    static_assert(W < 16, "16-lane groups");
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x10 | (W << 5)));
}

template <int W>
__device__ __forceinline__ double bcast(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffll), W << 5);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), W << 5);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// A prefetched node record, spread over the lanes of a 32-lane half.
//   float: both 16-lane rows of the half hold the record, lane l words
//          2 (l & 15) and 2 (l & 15) + 1; word w reaches all lanes of its row
//          with one DPP row broadcast (a VALU move, no LDS traffic).
//   double: lane q of the half holds word q; ds_swizzle broadcasts it.
template <typename T>
struct RecReg;

template <int W>
__device__ __forceinline__ float row_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + W, 0xf, 0xf, true));
}

// record words below kDppWords are broadcast with DPP (VALU), the rest with
// ds_swizzle (LDS), to balance the two pipes
constexpr int kDppWords = 12;

template <>
struct RecReg<float> {
    float a, b;
    __device__ __forceinline__ void load(const float *__restrict__ r, int lane) {
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        const f32x2 ab = __builtin_nontemporal_load(reinterpret_cast<const f32x2 *>(r) + (lane & 15));
        a = ab.x;
        b = ab.y;
    }
    template <int W>
    __device__ __forceinline__ float get() const {
        // word W sits in lane W / 2 of each 16-lane row, component W % 2
        if constexpr (W < kDppWords) {
            if constexpr (W & 1) return row_bcast<W / 2>(b);
            else return row_bcast<W / 2>(a);
        } else {
            if constexpr (W & 1) return bcast16<W / 2>(b);
            else return bcast16<W / 2>(a);
        }
    }
    template <int W>
    __device__ __forceinline__ int geti() const { return __float_as_int(get<W>()); }
};

template <>
struct RecReg<double> {
    double v;
    __device__ __forceinline__ void load(const double *__restrict__ r, int lane) {
        v = __builtin_nontemporal_load(r + (lane & 31));
    }
    template <int W>
    __device__ __forceinline__ double get() const { return bcast<W>(v); }
    // int32 link word i (0..5) of a double record: bytes of elements 26..28
    template <int I>
    __device__ __forceinline__ int geti() const {
        const long long b = __double_as_longlong(bcast<kRecLinks + I / 2>(v));
        return (I & 1) ? (int)(b >> 32) : (int)(b & 0xffffffffll);
    }
};

template <int W, typename T>
__device__ __forceinline__ void bcast_g(T (&g)[26], const RecReg<T> &r) {
    g[W] = r.template get<W>();
    if constexpr (W + 1 < 26) bcast_g<W + 1>(g, r);
}

// the link words of a record (elements 26.. as int32)
struct Links6 {
    int xref, yref, off, meta, slots;
};

__device__ __forceinline__ Links6 bcast_links6(const RecReg<float> &r) {
    Links6 l;
    l.xref = r.geti<26>();
    l.yref = r.geti<27>();
    l.off = r.geti<28>();
    l.meta = r.geti<29>();
    l.slots = r.geti<30>();
    return l;
}

__device__ __forceinline__ Links6 bcast_links6(const RecReg<double> &r) {
    Links6 l;
    l.xref = r.geti<0>();
    l.yref = r.geti<1>();
    l.off = r.geti<2>();
    l.meta = r.geti<3>();
    l.slots = r.geti<4>();
    return l;
}

__device__ __forceinline__ int2 bcast_refs(const RecReg<float> &r) { return make_int2(r.geti<26>(), r.geti<27>()); }

__device__ __forceinline__ int2 bcast_refs(const RecReg<double> &r) { return make_int2(r.geti<0>(), r.geti<1>()); }

// the node's body (link word 5)
__device__ __forceinline__ int bcast_body(const RecReg<float> &r) { return r.geti<31>(); }
__device__ __forceinline__ int bcast_body(const RecReg<double> &r) { return r.geti<5>(); }

// Rotation of a moved body (m x 9 row-major, the sweep's precision): the
// upward sweep takes each bead's 3-vector times Rot^T, the downward one
// gives each bead's result times Rot (transform reuse across rigid motions).
template <typename T>
__device__ __forceinline__ void load_rot(const T *__restrict__ rot, int body, int m, T (&r)[9]) {
    const T *p = rot + 9 * (int64_t)min(max(body, 0), m - 1);
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = p[i];
}

template <int RT>
__device__ __forceinline__ int rhs_count(const Ctx &C) {
    return RT ? RT : C.R;
}

// ---------------------------------------------------------------------------
// Per-lane vectors of NC adjacent right-hand sides (NC = 1 or 2): the lane
// holds columns NC * rl .. NC * rl + NC - 1 of its lane group, so one row of a
// vector is one coalesced access of NC values per lane, and the record
// broadcast, the addressing and the selects of a node are shared by the NC
// columns.
// ---------------------------------------------------------------------------
template <typename T, int NC>
__device__ __forceinline__ void bldn(rsrc_t r, uint32_t vo, uint32_t so, T (&m)[NC]) {
    if constexpr (NC == 1) {
        m[0] = bld<T>(r, vo, so);
    } else if constexpr (sizeof(T) == 4) {
        const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, kNT);
        m[0] = __uint_as_float(a.x);
        m[1] = __uint_as_float(a.y);
    } else {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, kNT);
        m[0] = __builtin_bit_cast(double, u32x2{a.x, a.y});
        m[1] = __builtin_bit_cast(double, u32x2{a.z, a.w});
    }
}

template <typename T, int NC>
__device__ __forceinline__ void bstn(const T (&m)[NC], rsrc_t r, uint32_t vo, uint32_t so) {
    if constexpr (NC == 1) {
        bst<T>(m[0], r, vo, so);
    } else if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b64(u32x2{__float_as_uint(m[0]), __float_as_uint(m[1])}, r, vo, so, kNT);
    } else {
        const u32x2 a = __builtin_bit_cast(u32x2, m[0]), b = __builtin_bit_cast(u32x2, m[1]);
        // wider than 64 bits: the offset goes into the vector offset (an SGPR
        // offset lets the next instruction overwrite the data register early)
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{a.x, a.y, b.x, b.y}, r, vo == kOOB ? kOOB : vo + so, 0, kNT);
    }
}

// Exchange entries are [slot][column][6 values]: a lane's NC entries are 6 NC
// contiguous values.
template <typename T, int NC, int XP = 0>
__device__ __forceinline__ void bld6n(rsrc_t r, uint32_t vo, T (&m)[6][NC]) {
    if constexpr (NC == 1) {
        T e[6];
        bld6<XP>(r, vo, e);
#pragma unroll
        for (int k = 0; k < 6; ++k) m[k][0] = e[k];
    } else {
        static_assert(NC == 2 && sizeof(T) == 4, "two columns per lane are float");
        // four 12-byte pieces: each column's two triples
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const u32x3 a = __builtin_amdgcn_raw_buffer_load_b96(r, vo, 24 * c + 12 * h, XP);
                m[3 * h][c] = __uint_as_float(a.x);
                m[3 * h + 1][c] = __uint_as_float(a.y);
                m[3 * h + 2][c] = __uint_as_float(a.z);
            }
    }
}

template <typename T, int NC, int XP = 0>
__device__ __forceinline__ void bst6n(rsrc_t r, uint32_t vo, const T (&m)[6][NC]) {
    if constexpr (NC == 1) {
        T e[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) e[k] = m[k][0];
        bst6<XP>(r, vo, e);
    } else {
        static_assert(NC == 2 && sizeof(T) == 4, "two columns per lane are float");
        // four 12-byte pieces: each column's two triples
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                __builtin_amdgcn_raw_buffer_store_b96(
                    u32x3{__float_as_uint(m[3 * h][c]), __float_as_uint(m[3 * h + 1][c]), __float_as_uint(m[3 * h + 2][c])},
                    r, vo, 24 * c + 12 * h, XP);
    }
}

// The three values m[S .. S + 2] of a row triple for the lane's columns.  Rows
// layout: three accesses a vector row (row bytes) apart; triples layout (one
// column per lane): the lane's three values are contiguous, one access.
template <typename T, bool TRI, int NC, int S, int K>
__device__ __forceinline__ void bld3n(rsrc_t r, uint32_t vo, uint32_t row, T (&m)[K][NC]) {
    static_assert(S + 3 <= K, "triple inside the array");
    if constexpr (!TRI) {
#pragma unroll
        for (int k = 0; k < 3; ++k) bldn<T, NC>(r, vo, k * row, m[S + k]);
    } else if constexpr (sizeof(T) == 4) {
        static_assert(NC == 1, "the triples layout holds one column per lane");
        const u32x3 a = __builtin_amdgcn_raw_buffer_load_b96(r, vo, 0, kNT);
        m[S][0] = __uint_as_float(a.x);
        m[S + 1][0] = __uint_as_float(a.y);
        m[S + 2][0] = __uint_as_float(a.z);
    } else {
        static_assert(NC == 1, "the triples layout holds one column per lane");
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, vo, 0, kNT);
        const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(r, vo, 16, kNT);
        m[S][0] = __builtin_bit_cast(double, u32x2{a.x, a.y});
        m[S + 1][0] = __builtin_bit_cast(double, u32x2{a.z, a.w});
        m[S + 2][0] = __builtin_bit_cast(double, b);
    }
}

template <typename T, bool TRI, int NC, int S, int K>
__device__ __forceinline__ void bst3n(const T (&m)[K][NC], rsrc_t r, uint32_t vo, uint32_t row) {
    static_assert(S + 3 <= K, "triple inside the array");
    if constexpr (!TRI) {
#pragma unroll
        for (int k = 0; k < 3; ++k) bstn<T, NC>(m[S + k], r, vo, k * row);
    } else if constexpr (sizeof(T) == 4) {
        static_assert(NC == 1, "the triples layout holds one column per lane");
        // zero SGPR offset: see bstn
        __builtin_amdgcn_raw_buffer_store_b96(
            u32x3{__float_as_uint(m[S][0]), __float_as_uint(m[S + 1][0]), __float_as_uint(m[S + 2][0])}, r, vo, 0, kNT);
    } else {
        static_assert(NC == 1, "the triples layout holds one column per lane");
        const u32x2 a = __builtin_bit_cast(u32x2, m[S][0]), b = __builtin_bit_cast(u32x2, m[S + 1][0]);
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{a.x, a.y, b.x, b.y}, r, vo, 0, kNT);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, m[S + 2][0]), r, vo, 16, kNT);
    }
}

// LDS slot layout: [slot][component 0..5][64 lanes][NC]
template <typename T, int NC>
__device__ __forceinline__ void lds_put6(T *lds, int slot, int lane, const T (&m)[6][NC]) {
    T *p = lds + ((slot * 6) * 64 + lane) * NC;
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) p[k * 64 * NC + c] = m[k][c];
}

template <typename T, int NC>
__device__ __forceinline__ void lds_get6(const T *lds, int slot, int lane, T (&m)[6][NC]) {
    const T *p = lds + ((slot * 6) * 64 + lane) * NC;
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) m[k][c] = p[k * 64 * NC + c];
}

// t <- G t / t <- G^T t for NC columns at once (the record words are shared)
template <typename T, int NC>
__device__ __forceinline__ void house_fwd9n(T (&t)[9][NC], const T (&g)[26]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        T u[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) u[i] = t[i][c];
        house_fwd<9>(u, g);
#pragma unroll
        for (int i = 0; i < 9; ++i) t[i][c] = u[i];
    }
}

template <typename T, int NC>
__device__ __forceinline__ void house_bwd9n(T (&t)[9][NC], const T (&g)[26]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        T u[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) u[i] = t[i][c];
        house_bwd<9>(u, g);
#pragma unroll
        for (int i = 0; i < 9; ++i) t[i][c] = u[i];
    }
}

// The buffers of one wide sweep and byte strides.
struct WBufs {
    rsrc_t in, out, xch;
    uint32_t row;  // bytes of one vector row (R values)
};

template <typename T, int RT>
__device__ __forceinline__ WBufs wide_bufs(const T *in, T *out, T *xch, const Ctx &C) {
    WBufs b;
    b.in = make_rsrc(in, C.in_bytes);
    b.out = make_rsrc(out, C.out_bytes);
    b.xch = make_rsrc(xch, C.xch_bytes);
    b.row = (uint32_t)(rhs_count<RT>(C) * sizeof(T));
    return b;
}

// Byte offsets of the lane's first column inside a row triple of a vector
// (v: r * vlane values) and inside an exchange entry (x: 6 r values).
struct LaneB {
    uint32_t v, x;
};

// Byte offset of bead ref's first row for the lane's first column: a negative
// ref (not a bead) or on = false lands past the end of the buffer.
template <typename T, int RT>
__device__ __forceinline__ uint32_t bead_off(int ref, bool on, const Ctx &C, LaneB lb) {
    const uint32_t u = on ? min((uint32_t)ref, (uint32_t)C.N) : (uint32_t)C.N;
    return u * (uint32_t)(3 * rhs_count<RT>(C) * sizeof(T)) + lb.v;
}

// Byte offset of exchange entry (slot, lane's first column), past the end when off.
template <typename T, int RT>
__device__ __forceinline__ uint32_t xch_off(int slot, bool on, const Ctx &C, LaneB lb) {
    const uint32_t sl = on ? min((uint32_t)slot, (uint32_t)C.xch_cap) : (uint32_t)C.xch_cap;
    return sl * (uint32_t)(6 * rhs_count<RT>(C) * sizeof(T)) + lb.x;
}

// Upward memory input of one child: a bead's vector (3 values; zero Info-set
// tail) or, with IW = 6, an earlier tile root's Info-set.  A stack child loads
// nothing (zeros).  IW = 3 serves the first tile phase, whose only memory
// inputs are beads.
template <typename T, int RT, int IW, int NC, bool TRI, int XP = 0>
__device__ __forceinline__ void up_input(int ref, T (&m)[IW][NC], const WBufs &B, const Ctx &C, LaneB lb) {
    if constexpr (IW == 6) {
        // later phases: beads are rare children there, so their loads go
        // under a branch (the first phase keeps them unconditional, measured
        // faster)
#pragma unroll
        for (int k = 0; k < 6; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c) m[k][c] = T(0);
        if (ref >= 0) bld3n<T, TRI, NC, 0>(B.in, bead_off<T, RT>(ref, true, C, lb), B.row, m);
    } else {
        bld3n<T, TRI, NC, 0>(B.in, bead_off<T, RT>(ref, true, C, lb), B.row, m);
    }
    if constexpr (IW == 6) {
        T e[6][NC];
        bld6n<T, NC, XP>(B.xch, xch_off<T, RT>(ref_slot(ref), ref < kRefStack, C, lb), e);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
#pragma unroll
            for (int k = 0; k < 3; ++k) m[k][c] += e[k][c];
#pragma unroll
            for (int k = 3; k < 6; ++k) m[k][c] = e[k][c];
        }
    }
}

// One upward node step (Eqs. 4.2-4.3).  A child of the same tile is read from
// its LDS slot; a bead or an earlier tile's root comes from the prefetched
// registers ax / ay.  Nothing is stored unless the node is live.
template <typename T, int RT, int IW, int NC, bool TRI, bool ROT, int XP = 0>
__device__ __forceinline__ void up_node(const T (&g)[26], const Links6 &lk, const T (&ax)[IW][NC],
                                        const T (&ay)[IW][NC], const T (&rm)[9], T *lds, int lane, const WBufs &B,
                                        const Ctx &C, LaneB lb, bool live, bool act) {
    // offsets and references were checked when the tile schedule was built;
    // an access outside a buffer would be dropped by its range check
    const int xs = min(lk.slots & 0xff, C.nslot - 1), ys = min((lk.slots >> 8) & 0xff, C.nslot - 1);
    const int os = min((lk.slots >> 16) & 0xff, C.nslot - 1);
    const bool xst = lk.xref == kRefStack, yst = lk.yref == kRefStack;
    T mx[6][NC], my[6][NC];
    lds_get6<T, NC>(lds, xs, lane, mx);
    lds_get6<T, NC>(lds, ys, lane, my);
    const T sx = g[kRecSx], sy = g[kRecSy];
    const bool xi = lk.xref < 0, yi = lk.yref < 0;
    const bool both = xi && yi, any = xi || yi;
    T mp[6][NC], t9[9][NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int k = 0; k < IW; ++k) {
            mx[k][c] = xst ? mx[k][c] : ax[k][c];
            my[k][c] = yst ? my[k][c] : ay[k][c];
        }
        if constexpr (ROT) {
            // a bead child's vector times Rot^T
            T rx[3], ry[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                rx[d] = rm[d] * ax[0][c] + rm[3 + d] * ax[1][c] + rm[6 + d] * ax[2][c];
                ry[d] = rm[d] * ay[0][c] + rm[3 + d] * ay[1][c] + rm[6 + d] * ay[2][c];
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                mx[d][c] = lk.xref >= 0 ? rx[d] : mx[d][c];
                my[d][c] = lk.yref >= 0 ? ry[d] : my[d][c];
            }
        }
        T tt[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            mp[k][c] = sx * mx[k][c] + sy * my[k][c];
            tt[k] = sy * mx[k][c] - sx * my[k][c];
        }
        // t = [M_x(4:6)?; M_y(4:6)?; tt] packed to the front, zeros behind
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            t9[k][c] = xi ? mx[3 + k][c] : (yi ? my[3 + k][c] : tt[k]);
            t9[3 + k][c] = both ? my[3 + k][c] : (any ? tt[k] : T(0));
            t9[6 + k][c] = both ? tt[k] : T(0);
        }
    }
    house_fwd9n<T, NC>(t9, g);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) mp[3 + k][c] = t9[k][c];
    const bool troot = (lk.meta & kMetaTileRoot) != 0;
    const bool en = live && act;
    // residue rows [off, off + dim), and a tile root's Info-set to the
    // exchange buffer (others stay in LDS): stores of absent values are
    // skipped rather than sent out of range, which still costs texture-unit
    // time (measured: 6% of the first-phase launch)
    const uint32_t ob = (uint32_t)lk.off * B.row + lb.v;
    if (en && any) bst3n<T, TRI, NC, 3>(t9, B.out, ob, B.row);
    if (en && both) bst3n<T, TRI, NC, 6>(t9, B.out, ob + 3 * B.row, B.row);
    if (en && troot) bst6n<T, NC, XP>(B.xch, xch_off<T, RT>(lk.meta >> kMetaSlotShift, true, C, lb), mp);
    if (live && !troot) lds_put6<T, NC>(lds, os, lane, mp);
}

// The run of lane group k of a phase: schedule range [base, base + len).
__device__ __forceinline__ void run_range(int k, int nrun, int c0, const int32_t *__restrict__ run, const Ctx &C,
                                          int &base, int &len, int &bad) {
    base = 0;
    len = 0;
    if (k < nrun) {
        base = run[c0 + k];
        len = run[c0 + k + 1] - base;
        if (base < 0 || len < 0 || (int64_t)base + len > C.nsched) {
            bad |= kFlagBounds;
            base = 0;
            len = 0;
        }
    }
}

// the longest run of the wave (wave-uniform)
template <int LPT>
__device__ __forceinline__ int wave_max_len(int len) {
    if constexpr (LPT <= 16) len = max(len, __shfl_xor(len, 16, 64));
    if constexpr (LPT <= 32) len = max(len, __shfl_xor(len, 32, 64));
    return __builtin_amdgcn_readfirstlane(len);
}

// The upward sweep of one lane group over schedule indices [base, base +
// len) (a run of whole tiles, or one tile): records PR nodes ahead, memory
// inputs NR - 1 nodes ahead; exchange accesses with cache policy XP.
template <typename T, int LPT, int RT, int PR, int NR, int IW, int NC, bool TRI, bool ROT, int XP>
__device__ __forceinline__ void up_run(int base, int len, const T *__restrict__ rec, const T *__restrict__ rot,
                                       T *lds, int lane, const WBufs &B, const Ctx &C, LaneB lb, bool act) {
    const int maxlen = wave_max_len<LPT>(len);
    const int last = max(len - 1, 0);
    const T *rp = rec + (int64_t)kRecWords * base;
    RecReg<T> RW[PR];
    T A[NR][IW][NC], Bv[NR][IW][NC];
    T RM[ROT ? NR : 1][9];
#pragma unroll
    for (int k = 0; k < PR; ++k) RW[k].load(rp + (int64_t)min(k, last) * kRecWords, lane);
#pragma unroll
    for (int k = 0; k < NR - 1; ++k) {
        const int2 ref = bcast_refs(RW[k]);
        up_input<T, RT, IW, NC, TRI, XP>(ref.x, A[k], B, C, lb);
        up_input<T, RT, IW, NC, TRI, XP>(ref.y, Bv[k], B, C, lb);
        if constexpr (ROT) load_rot(rot, bcast_body(RW[k]), C.m, RM[k]);
    }
#define HQ_UP_STEP(K)                                                                       \
    {                                                                                       \
        const int n = n0 + (K);                                                             \
        T g[26];                                                                            \
        bcast_g<0>(g, RW[K]);                                                               \
        const Links6 lk = bcast_links6(RW[K]);                                              \
        RW[K].load(rp + (int64_t)min(n + PR, last) * kRecWords, lane);                      \
        {                                                                                   \
            const int2 ref = bcast_refs(RW[((K) + NR - 1) % PR]);                           \
            up_input<T, RT, IW, NC, TRI, XP>(ref.x, A[((K) + NR - 1) % NR], B, C, lb);      \
            up_input<T, RT, IW, NC, TRI, XP>(ref.y, Bv[((K) + NR - 1) % NR], B, C, lb);     \
            if constexpr (ROT)                                                              \
                load_rot(rot, bcast_body(RW[((K) + NR - 1) % PR]), C.m, RM[((K) + NR - 1) % NR]); \
        }                                                                                   \
        up_node<T, RT, IW, NC, TRI, ROT, XP>(g, lk, A[(K) % NR], Bv[(K) % NR], RM[ROT ? (K) % NR : 0], lds, lane, \
                                             B, C, lb, n < len, act);                       \
    }
    for (int n0 = 0; n0 < maxlen; n0 += PR) {
        HQ_UP_STEP(0)
        HQ_UP_STEP(1)
        HQ_UP_STEP(2)
        if constexpr (PR >= 4) HQ_UP_STEP(3)
        if constexpr (PR >= 6) {
            HQ_UP_STEP(4)
            HQ_UP_STEP(5)
        }
        if constexpr (PR >= 12) {
            HQ_UP_STEP(6)
            HQ_UP_STEP(7)
            HQ_UP_STEP(8)
            HQ_UP_STEP(9)
            HQ_UP_STEP(10)
            HQ_UP_STEP(11)
        }
    }
#undef HQ_UP_STEP
}

template <typename T, int LPT, int RT, int PR, int NR, int IW, int NC, bool TRI, bool ROT>
__global__ void __launch_bounds__(64, (sizeof(T) * NC == 4 && NR <= 3) ? 4 : 2) k_up_wide(
    int phase, const int32_t *__restrict__ prun, const int32_t *__restrict__ run, const T *__restrict__ rec,
    const T *__restrict__ v, T *__restrict__ out, T *__restrict__ xch, const T *__restrict__ rot, Ctx C,
    int32_t *err) {
    static_assert(LPT == 16 || LPT == 32 || LPT == 64, "wide sweeps use 16, 32 or 64 lanes per run");
    static_assert(PR % NR == 0 && NR >= 2 && (PR == 3 || PR == 4 || PR == 6 || PR == 12), "ring sizes");
    static_assert(sizeof(T) == 4 || LPT >= 32, "double records are broadcast inside 32-lane halves");
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    constexpr int TPW = 64 / LPT;
    const int R = rhs_count<RT>(C);
    const int lane = threadIdx.x;
    const int tslot = lane / LPT, rl = lane % LPT;
    const int c0 = prun[kPrunStride * phase + 2], nrun = prun[kPrunStride * phase + 3];
    const int items = ((nrun + TPW - 1) / TPW) * C.nchunks;
    const WBufs B = wide_bufs<T, RT>(v, out, xch, C);
    int bad = 0;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int grp = item / C.nchunks, chunk = item - grp * C.nchunks;
        const int col = (chunk * LPT + rl) * NC;  // first column of the lane
        const int rr = min(col, R - NC);
        int base, len;
        run_range(grp * TPW + tslot, nrun, c0, run, C, base, len, bad);
        const LaneB lb{(uint32_t)(rr * (TRI ? 3 : 1) * sizeof(T)), (uint32_t)(rr * 6 * sizeof(T))};
        up_run<T, LPT, RT, PR, NR, IW, NC, TRI, ROT, 0>(base, len, rec, rot, lds, lane, B, C, lb, col < R);
    }
    if (bad) atomicOr(err, bad);
}

// ---------------------------------------------------------------------------
// The fused upward sweep: the whole of Algorithm 2 in one launch.
//
// Lane groups sweep the first tile phase's runs as above.  Every tile whose
// root has a parent belongs to a parent tile (of a later phase) that counts
// its child tiles; after a run, the group waits for its stores and takes one
// arrival per tile root of the run from that counter (a device-scope atomic).
// The group whose arrival empties a counter sweeps the parent tile itself --
// its children's Info-sets are all in the exchange buffer by then -- and
// arrives at that tile's parent in turn, so the later phases run inside the
// launch, each tile started by the last of its children to finish, and no
// group ever waits for another.  The exchange entries travel between
// workgroups of the launch, so their stores and loads carry the agent-scope
// coherence bit (kSC1), and a group's stores are complete (s_waitcnt
// vmcnt(0)) before its arrival.  The counter's last arrival restores it to
// the tile's child count for the next sweep.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// meta word of the record at schedule index s
template <typename T>
__device__ __forceinline__ int rec_meta(const T *__restrict__ rec, int s) {
    return reinterpret_cast<const int32_t *>(rec + (int64_t)kRecWords * s + kRecLinks)[3];
}

// Arrival of a finished tile at its parent tile: returns the parent tile when
// this arrival was the last one (the caller then sweeps it), else -1.
__device__ __forceinline__ int tile_arrive(int t, const int32_t *__restrict__ ptile, int32_t *tcnt,
                                           const int32_t *__restrict__ tcnt0, const Ctx &C, int &bad) {
    if ((unsigned)t >= (unsigned)C.nsched) {
        bad |= kFlagBounds;
        return -1;
    }
    const int p = ptile[t];
    if (p < 0) return -1;
    if ((unsigned)p >= (unsigned)C.nsched) {
        bad |= kFlagBounds;
        return -1;
    }
    if (__hip_atomic_fetch_add(&tcnt[p], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 1) return -1;
    __hip_atomic_store(&tcnt[p], tcnt0[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return p;
}

// value of lane src of this lane's group of LPT lanes
template <int LPT>
__device__ __forceinline__ int group_read(int v, int src, int lane) {
    return __shfl(v, (lane & ~(LPT - 1)) | src, 64);
}

template <typename T, int LPT, int RT, int NC, bool TRI, bool ROT>
__global__ void __launch_bounds__(64, 2) k_up_fused(
    const int32_t *__restrict__ prun, const int32_t *__restrict__ run, const T *__restrict__ rec,
    const T *__restrict__ v, T *__restrict__ out, T *__restrict__ xch, const T *__restrict__ rot,
    const int32_t *__restrict__ tile_base, const int32_t *__restrict__ tile_len, const int32_t *__restrict__ ptile,
    int32_t *tcnt, const int32_t *__restrict__ tcnt0, Ctx C, int32_t *err) {
    static_assert(LPT == 16 || LPT == 32 || LPT == 64, "wide sweeps use 16, 32 or 64 lanes per run");
    static_assert(sizeof(T) == 4 || LPT >= 32, "double records are broadcast inside 32-lane halves");
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    constexpr int TPW = 64 / LPT;
    const int R = rhs_count<RT>(C);
    const int lane = threadIdx.x;
    const int tslot = lane / LPT, rl = lane % LPT;
    const int c0 = prun[kPrunStride * 1 + 2], nrun = prun[kPrunStride * 1 + 3];
    const int items = ((nrun + TPW - 1) / TPW) * C.nchunks;
    const WBufs B = wide_bufs<T, RT>(v, out, xch, C);
    int bad = 0;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int grp = item / C.nchunks, chunk = item - grp * C.nchunks;
        const int col = (chunk * LPT + rl) * NC;
        const int rr = min(col, R - NC);
        const bool act = col < R;
        int base, len;
        run_range(grp * TPW + tslot, nrun, c0, run, C, base, len, bad);
        const LaneB lb{(uint32_t)(rr * (TRI ? 3 : 1) * sizeof(T)), (uint32_t)(rr * 6 * sizeof(T))};
        up_run<T, LPT, RT, kPR1, kNR1, 3, NC, TRI, ROT, kSC1>(base, len, rec, rot, lds, lane, B, C, lb, act);
        // arrivals of the run's tile roots, LPT schedule indices at a time
        // (the lanes of a group read consecutive records' meta words)
        const int maxlen = wave_max_len<LPT>(len);
        bool waited = false;
        for (int k0 = 0; k0 < maxlen; k0 += LPT) {
            int meta = 0;
            if (k0 + rl < len) meta = rec_meta(rec, base + k0 + rl);
            const bool arrives = (meta & kMetaTileRoot) && !(meta & kMetaBodyRoot);
            if (!__builtin_amdgcn_ballot_w64(arrives)) continue;
            if (!waited) {
                wait_vmem();  // this wave's exchange stores are complete
                waited = true;
            }
            int mine = arrives ? tile_arrive(meta >> kMetaSlotShift, ptile, tcnt, tcnt0, C, bad) : -1;
            // sweep the tiles this group completed, one at a time, each
            // followed up its chain of last arrivals
            uint64_t todo = __builtin_amdgcn_ballot_w64(mine >= 0) >> (tslot * LPT);
            if constexpr (LPT < 64) todo &= (1ull << LPT) - 1;
            int cur = -1;
            while (true) {
                if (cur < 0 && todo) {
                    const int src = __builtin_ctzll(todo);
                    todo &= todo - 1;
                    cur = group_read<LPT>(mine, src, lane);
                }
                if (!__builtin_amdgcn_ballot_w64(cur >= 0)) break;
                int tb = 0, tl = 0;
                if (cur >= 0) {
                    tb = tile_base[cur];
                    tl = tile_len[cur];
                    if (tb < 0 || tl < 0 || (int64_t)tb + tl > C.nsched) {
                        bad |= kFlagBounds;
                        tl = 0;
                    }
                }
                up_run<T, LPT, RT, kPRL, kNRL, 6, NC, TRI, ROT, kSC1>(tb, tl, rec, rot, lds, lane, B, C, lb, act);
                wait_vmem();
                int nxt = -1;
                if (cur >= 0 && rl == 0) nxt = tile_arrive(cur, ptile, tcnt, tcnt0, C, bad);
                cur = group_read<LPT>(nxt, 0, lane);
            }
        }
    }
    if (bad) atomicOr(err, bad);
}

// Downward memory inputs of one node: its residue coefficients w_p (dim = 0,
// 3 or 6 values) and, for a tile root below a body root, its Velocity-set from
// the exchange buffer; absent values are zeros.  Unlike the other wide-sweep
// accesses these loads are skipped, not sent out of range, when absent: the
// exchange entry is absent for all but the tile roots, and an out-of-range
// access still occupies the texture units (measured: skipping them takes 11%
// off the first phase's downward launch, while the same change to the upward
// sweep's bead loads made it slower).
template <typename T, int RT, int NC, bool TRI>
__device__ __forceinline__ void down_input(const Links6 &lk, T (&a)[6][NC], T (&b)[6][NC], const WBufs &B,
                                           const Ctx &C, LaneB lb) {
    const bool xi = lk.xref < 0, yi = lk.yref < 0;
    const uint32_t ob = (uint32_t)lk.off * B.row + lb.v;
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) a[k][c] = b[k][c] = T(0);
    if (xi || yi) bld3n<T, TRI, NC, 0>(B.in, ob, B.row, a);
    if (xi && yi) bld3n<T, TRI, NC, 3>(B.in, ob + 3 * B.row, B.row, a);
    const bool lr = (lk.meta & kMetaTileRoot) && (!(lk.meta & kMetaBodyRoot) || C.root_in);
    if (lr) bld6n<T, NC>(B.xch, xch_off<T, RT>(lk.meta >> kMetaSlotShift, true, C, lb), b);
}

// One downward node step (Theorem 4.3): L_p from its LDS slot (or the
// exchange buffer for a tile root, zero for a body root), children's
// Velocity-sets to their slots, to bead outputs, or (XC: phases after the
// first) to the exchange buffer.
template <typename T, int RT, bool XC, int NC, bool TRI, bool ROT>
__device__ __forceinline__ void down_node(const T (&g)[26], const Links6 &lk, const T (&wp)[6][NC],
                                          const T (&lroot)[6][NC], const T (&rm)[9], T *lds, int lane,
                                          const WBufs &B, const Ctx &C, LaneB lb, bool live, bool act) {
    const int xs = min(lk.slots & 0xff, C.nslot - 1), ys = min((lk.slots >> 8) & 0xff, C.nslot - 1);
    const int os = min((lk.slots >> 16) & 0xff, C.nslot - 1);
    const bool troot = (lk.meta & kMetaTileRoot) != 0;
    T L[6][NC];
    lds_get6<T, NC>(lds, os, lane, L);
    const T sx = g[kRecSx], sy = g[kRecSy];
    const bool xi = lk.xref < 0, yi = lk.yref < 0;
    const bool both = xi && yi, any = xi || yi;
    T x9[9][NC], Lx[6][NC], Ly[6][NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        // a tile root's Velocity-set comes from the exchange buffer (zeros for
        // a body root, whose entry loads as zeros)
#pragma unroll
        for (int k = 0; k < 6; ++k) L[k][c] = troot ? lroot[k][c] : L[k][c];
#pragma unroll
        for (int k = 0; k < 3; ++k) x9[k][c] = L[3 + k][c];
#pragma unroll
        for (int k = 0; k < 6; ++k) x9[3 + k][c] = wp[k][c];  // absent residue values loaded as zeros
    }
    house_bwd9n<T, NC>(x9, g);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T st = both ? x9[6 + k][c] : (any ? x9[3 + k][c] : x9[k][c]);
            Lx[3 + k][c] = x9[k][c];
            Ly[3 + k][c] = both ? x9[3 + k][c] : x9[k][c];
            Lx[k][c] = sx * L[k][c] + sy * st;
            Ly[k][c] = sy * L[k][c] - sx * st;
        }
    const bool en = live && act;
    {
        const uint32_t bx = bead_off<T, RT>(lk.xref, en, C, lb), by = bead_off<T, RT>(lk.yref, en, C, lb);
        if constexpr (ROT) {
            // a bead child's result times Rot (only the bead stores use it)
            T bxv[6][NC], byv[6][NC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    bxv[d][c] = rm[3 * d] * Lx[0][c] + rm[3 * d + 1] * Lx[1][c] + rm[3 * d + 2] * Lx[2][c];
                    byv[d][c] = rm[3 * d] * Ly[0][c] + rm[3 * d + 1] * Ly[1][c] + rm[3 * d + 2] * Ly[2][c];
                }
            bst3n<T, TRI, NC, 0>(bxv, B.out, bx, B.row);
            bst3n<T, TRI, NC, 0>(byv, B.out, by, B.row);
        } else {
            bst3n<T, TRI, NC, 0>(Lx, B.out, bx, B.row);
            bst3n<T, TRI, NC, 0>(Ly, B.out, by, B.row);
        }
    }
    if constexpr (XC) {
        bst6n<T, NC>(B.xch, xch_off<T, RT>(ref_slot(lk.xref), en && lk.xref < kRefStack, C, lb), Lx);
        bst6n<T, NC>(B.xch, xch_off<T, RT>(ref_slot(lk.yref), en && lk.yref < kRefStack, C, lb), Ly);
    }
    if (live) {
        // children of this tile go to their slots
        if (lk.xref == kRefStack) lds_put6<T, NC>(lds, xs, lane, Lx);
        if (lk.yref == kRefStack) lds_put6<T, NC>(lds, ys, lane, Ly);
    }
}

template <typename T, int LPT, int RT, int PR, int NR, bool XC, int NC, bool TRI, bool ROT>
__global__ void __launch_bounds__(64, (sizeof(T) * NC == 4 && NR <= 3) ? 4 : 2) k_down_wide(
    int phase, const int32_t *__restrict__ prun, const int32_t *__restrict__ run, const T *__restrict__ rec,
    const T *__restrict__ w, T *__restrict__ out, T *__restrict__ xch, const T *__restrict__ rot, Ctx C,
    int32_t *err) {
    static_assert(LPT == 16 || LPT == 32 || LPT == 64, "wide sweeps use 16, 32 or 64 lanes per run");
    static_assert(PR % NR == 0 && NR >= 2 && (PR == 3 || PR == 4 || PR == 6 || PR == 12), "ring sizes");
    static_assert(sizeof(T) == 4 || LPT >= 32, "double records are broadcast inside 32-lane halves");
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    constexpr int TPW = 64 / LPT;
    const int R = rhs_count<RT>(C);
    const int lane = threadIdx.x;
    const int tslot = lane / LPT, rl = lane % LPT;
    const int c0 = prun[kPrunStride * phase + 2], nrun = prun[kPrunStride * phase + 3];
    const int items = ((nrun + TPW - 1) / TPW) * C.nchunks;
    const WBufs B = wide_bufs<T, RT>(w, out, xch, C);
    int bad = 0;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int grp = item / C.nchunks, chunk = item - grp * C.nchunks;
        const int col = (chunk * LPT + rl) * NC;
        const int rr = min(col, R - NC);
        int base, len;
        run_range(grp * TPW + tslot, nrun, c0, run, C, base, len, bad);
        const bool act = col < R;
        const LaneB lb{(uint32_t)(rr * (TRI ? 3 : 1) * sizeof(T)), (uint32_t)(rr * 6 * sizeof(T))};
        const int maxlen = wave_max_len<LPT>(len);
        const int last = max(len - 1, 0);
        // node n of the sweep is schedule index base + len - 1 - n
        const T *rp = rec + (int64_t)kRecWords * (base + last);
        RecReg<T> RW[PR];
        T A[NR][6][NC], Bl[NR][6][NC];
        T RM[ROT ? NR : 1][9];
#pragma unroll
        for (int k = 0; k < PR; ++k) RW[k].load(rp - (int64_t)min(k, last) * kRecWords, lane);
#pragma unroll
        for (int k = 0; k < NR - 1; ++k) {
            down_input<T, RT, NC, TRI>(bcast_links6(RW[k]), A[k], Bl[k], B, C, lb);
            if constexpr (ROT) load_rot(rot, bcast_body(RW[k]), C.m, RM[k]);
        }
#define HQ_DOWN_STEP(K)                                                                     \
        {                                                                                   \
            const int n = n0 + (K);                                                         \
            T g[26];                                                                        \
            bcast_g<0>(g, RW[K]);                                                           \
            const Links6 lk = bcast_links6(RW[K]);                                          \
            RW[K].load(rp - (int64_t)min(n + PR, last) * kRecWords, lane);                  \
            down_input<T, RT, NC, TRI>(bcast_links6(RW[((K) + NR - 1) % PR]), A[((K) + NR - 1) % NR], \
                                       Bl[((K) + NR - 1) % NR], B, C, lb);                  \
            if constexpr (ROT)                                                              \
                load_rot(rot, bcast_body(RW[((K) + NR - 1) % PR]), C.m, RM[((K) + NR - 1) % NR]); \
            down_node<T, RT, XC, NC, TRI, ROT>(g, lk, A[(K) % NR], Bl[(K) % NR], RM[ROT ? (K) % NR : 0], lds, lane, \
                                               B, C, lb, n < len, act);                     \
        }
        for (int n0 = 0; n0 < maxlen; n0 += PR) {
            HQ_DOWN_STEP(0)
            HQ_DOWN_STEP(1)
            HQ_DOWN_STEP(2)
            if constexpr (PR >= 4) HQ_DOWN_STEP(3)
            if constexpr (PR >= 6) {
                HQ_DOWN_STEP(4)
                HQ_DOWN_STEP(5)
            }
            if constexpr (PR >= 12) {
                HQ_DOWN_STEP(6)
                HQ_DOWN_STEP(7)
                HQ_DOWN_STEP(8)
                HQ_DOWN_STEP(9)
                HQ_DOWN_STEP(10)
                HQ_DOWN_STEP(11)
            }
        }
#undef HQ_DOWN_STEP
    }
    if (bad) atomicOr(err, bad);
}

// Tiles a launch of one tile phase provisions its grid for: every tile of the
// handle in the first phase; in a later phase twice the tiles the build found
// there, plus 64 (a rebuild may move tiles between phases: the kernels stride
// over their work, so a smaller grid stays correct, only slower).  The phases
// reserved for rebuilds are normally empty, and an empty launch of thousands
// of workgroups took 4-6 us for their dispatch alone.
int64_t phase_tiles(const Plan &P, int phase) {
    return phase == 1 ? 2 * P.tiles_built + 64 : 2 * P.tiles_ph[phase] + 64;
}

// One tile phase of a wide sweep: LPT lanes per run, NC columns per lane,
// vectors in the rows or (TRI) the triples layout, bead vectors turned by
// their body's rotation (ROT).
template <typename T, int LPT, int NC, bool TRI, bool ROT>
void launch_wide(const Plan &P, int phase, int transpose, const T *rec, const T *v, T *out, T *xch, const T *rot,
                 const Ctx &C, hipStream_t s) {
    constexpr int TPW = 64 / LPT;
    const size_t lds_w = (size_t)C.nslot * 6 * 64 * NC * sizeof(T);
    // work items: groups of TPW runs (a phase has at most NI / run_nodes + 1
    // runs, or kRunTarget + 1 when its runs are shortened) x RHS chunks, one
    // per wave, so the dispatcher balances the load; waves of later phases
    // with fewer runs exit at once
    const int64_t nrun_max = std::max<int64_t>(P.NI / P.run_nodes + 2, kRunTarget + 2);
    const int64_t items = ((nrun_max + TPW - 1) / TPW) * (int64_t)C.nchunks;
    // later phases hold few runs (often none, for phases reserved for a
    // rebuild): a grid of waves_per_cu waves per CU loops over them; the
    // first phase takes one wave per item unless the handle caps its grid
    const int64_t cap = (phase == 1) ? (int64_t)P.first_wpc : (int64_t)P.waves_per_cu;
    int64_t g = (phase == 1 && cap == 0) ? items : std::min<int64_t>(items, cap * P.ncu);
    // a later phase holds one run per tile (up to kRunTarget tiles)
    if (phase > 1)
        g = std::min<int64_t>(g, std::max<int64_t>(P.ncu, ((phase_tiles(P, phase) + TPW - 1) / TPW) * C.nchunks));
    const unsigned grid = (unsigned)std::min<int64_t>(g, 1 << 20);
#define HQ_WIDE(RT, PRU1, NRU1, PRU, NRU, PRD1, NRD1, PRD, NRD)                                              \
    do {                                                                                                     \
        if (!transpose) {                                                                                    \
            if (phase == 1)                                                                                  \
                hipLaunchKernelGGL((k_up_wide<T, LPT, RT, PRU1, NRU1, 3, NC, TRI, ROT>), dim3(grid), dim3(64), lds_w, \
                                   s, phase, P.d_prun, P.d_run, rec, v, out, xch, rot, C, P.d_err);               \
            else                                                                                             \
                hipLaunchKernelGGL((k_up_wide<T, LPT, RT, PRU, NRU, 6, NC, TRI, ROT>), dim3(grid), dim3(64), lds_w,   \
                                   s, phase, P.d_prun, P.d_run, rec, v, out, xch, rot, C, P.d_err);               \
        } else {                                                                                             \
            if (phase == 1)                                                                                  \
                hipLaunchKernelGGL((k_down_wide<T, LPT, RT, PRD1, NRD1, false, NC, TRI, ROT>), dim3(grid), dim3(64),  \
                                   lds_w, s, phase, P.d_prun, P.d_run, rec, v, out, xch, rot, C, P.d_err);        \
            else                                                                                             \
                hipLaunchKernelGGL((k_down_wide<T, LPT, RT, PRD, NRD, true, NC, TRI, ROT>), dim3(grid), dim3(64),     \
                                   lds_w, s, phase, P.d_prun, P.d_run, rec, v, out, xch, rot, C, P.d_err);        \
        }                                                                                                    \
    } while (0)
    // records six nodes ahead, inputs two nodes ahead, in every phase
    // (measured: a deeper input ring for the later phases, five nodes ahead,
    // was 8% slower on their upward launches; a 12-deep record ring slower
    // still)
    if (C.R == 32) HQ_WIDE(32, kPR1, kNR1, kPRL, kNRL, kPR1d, kNR1d, kPRLd, kNRLd);
    else HQ_WIDE(0, kPR1, kNR1, kPRL, kNRL, kPR1d, kNR1d, kPRLd, kNRLd);
#undef HQ_WIDE
}

// ---------------------------------------------------------------------------
// Leaf boxes (the first tile phase of a handle with leaf_size > 1): each leaf
// of n beads applies its transform diag(-1,-1,-1,1,...,1) Q^T (six stored
// reflectors) to its 3n bead values.  Upward: [M; eps] = G f, the Info-set M
// to the leaf's exchange entry, the 3n - 6 residues to the rows from the
// leaf's first residue row.  Downward: f = G^T [L; w] with L from the
// exchange entry (zero at a body root unless given).  G lanes per leaf, one
// right-hand side per lane; the exchange entry in the layout of the sweeps
// that follow (WX: wide [slot][R][6], else [slot][6][R]).
// ---------------------------------------------------------------------------
template <typename T, int G, int SMAX, bool WX, bool UP>
__global__ void __launch_bounds__(64) k_bucket(const int32_t *__restrict__ phase_tab,
                                               const int32_t *__restrict__ tile_root,
                                               const int32_t *__restrict__ tile_base,
                                               const int32_t *__restrict__ tile_len,
                                               const int32_t *__restrict__ first, const int32_t *__restrict__ last,
                                               const int32_t *__restrict__ perm, const int32_t *__restrict__ links,
                                               const T *__restrict__ brec, int64_t bcap, const T *__restrict__ v,
                                               T *__restrict__ out, T *__restrict__ xch, Ctx C, int32_t *err) {
    constexpr int MS = 3 * SMAX, BS = 6 * MS + 8, LPW = 64 / G;
    // groups of 16 or more lanes stage their leaf's record in LDS (one
    // coalesced pass, then broadcast reads); a lane that is a leaf of its own
    // reads the record itself
    constexpr bool kStage = G >= 16;
    __shared__ T sg[kStage ? LPW : 1][kStage ? BS : 1];
    const int lane = threadIdx.x;
    const int slotw = lane / G, rl = lane % G;
    const int tb = phase_tab[2 * 1], te = phase_tab[2 * 1 + 1];
    const int ngroups = (te - tb + LPW - 1) / LPW;
    const int items = ngroups * C.nchunks;
    int bad = 0;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int grp = item / C.nchunks, chunk = item - grp * C.nchunks;
        const int t = tb + grp * LPW + slotw;
        const int r = chunk * G + rl;
        const int rc = min(r, C.R - 1);  // a column to address for lanes beyond the right-hand sides
        int f = 0, n = 0, off = 0, meta = 0;
        if (t < te) {
            const int q = tile_root[t], sr = tile_base[t] + tile_len[t] - 1;
            if (q < 0 || q >= C.nsched || sr < 0 || sr >= C.nsched || (int64_t)(t - tb) >= bcap) {
                bad |= kFlagBounds;
            } else {
                f = first[q];
                n = last[q] - f + 1;
                off = links[(int64_t)kLinkInts * sr + 2];
                meta = links[(int64_t)kLinkInts * sr + 3];
                if (n < 2 || n > SMAX || f < 0 || (int64_t)f + n > C.N || off < 0 ||
                    (int64_t)off + 3 * n - 6 > C.rows) {
                    bad |= kFlagBounds;
                    n = 0;
                }
            }
        }
        if (n == 0) f = off = 0;
        const bool act = r < C.R && n > 0;
        const int mrows = 3 * n;
        const T *g = brec + (n > 0 ? (int64_t)(t - tb) : 0) * BS;
        if constexpr (kStage) {
            __syncthreads();  // the previous item's reads of the staging rows are over
            for (int e = rl; e < BS; e += G) sg[slotw][e] = g[e];
            __syncthreads();
        }
        auto gv = [&](int e) -> T {
            if constexpr (kStage) return sg[slotw][e];
            else return g[e];
        };
        int slot = meta >> kMetaSlotShift;
        const bool xok = (meta & kMetaTileRoot) && slot < C.xch_cap;
        if (n > 0 && !xok) bad |= kFlagBounds;
        if (!xok) slot = 0;
        auto xidx = [&](int d) -> int64_t {
            return WX ? ((int64_t)slot * C.R + rc) * 6 + d : ((int64_t)slot * 6 + d) * C.R + rc;
        };
        // the record is zero beyond the leaf's 3n rows, so the reflectors run
        // over all rows; absent values load from valid addresses and are
        // replaced by zeros
        T x[MS];
        if (UP) {
#pragma unroll
            for (int k = 0; k < SMAX; ++k) {
                const bool ok = act && k < n;
                const int64_t u = perm[f + (k < n ? k : 0)];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const T val = v[velem(3 * u, d, rc, C)];
                    x[3 * k + d] = ok ? val : T(0);
                }
            }
            // x <- Q^T x = H_6 ... H_1 x
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                const T tau = gv(6 * MS + j);
                T w = x[j];
#pragma unroll
                for (int i = j + 1; i < MS; ++i) w += gv(j * MS + i) * x[i];
                w *= tau;
                x[j] -= w;
#pragma unroll
                for (int i = j + 1; i < MS; ++i) x[i] -= w * gv(j * MS + i);
            }
            if (act) {
                if (xok) {
#pragma unroll
                    for (int d = 0; d < 6; ++d) xch[xidx(d)] = (d < 3) ? -x[d] : x[d];
                }
#pragma unroll
                for (int i = 6; i < MS; ++i)
                    if (i < mrows) out[velem(off + 3 * ((i - 6) / 3), (i - 6) % 3, r, C)] = x[i];
            }
        } else {
            const bool lin = act && xok && (!(meta & kMetaBodyRoot) || C.root_in);
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const T val = xch[xidx(d)];
                x[d] = lin ? ((d < 3) ? -val : val) : T(0);
            }
#pragma unroll
            for (int i = 6; i < MS; ++i) {
                const bool ok = act && i < mrows;
                const int row = ok ? off + (i - 6) : 0;
                const T val = v[velem(row - row % 3, row % 3, rc, C)];
                x[i] = ok ? val : T(0);
            }
            // x <- Q x = H_1 ... H_6 x
#pragma unroll
            for (int j = 5; j >= 0; --j) {
                const T tau = gv(6 * MS + j);
                T w = x[j];
#pragma unroll
                for (int i = j + 1; i < MS; ++i) w += gv(j * MS + i) * x[i];
                w *= tau;
                x[j] -= w;
#pragma unroll
                for (int i = j + 1; i < MS; ++i) x[i] -= w * gv(j * MS + i);
            }
            if (act) {
#pragma unroll
                for (int k = 0; k < SMAX; ++k) {
                    if (k < n) {
                        const int64_t u = perm[f + k];
#pragma unroll
                        for (int d = 0; d < 3; ++d) out[velem(3 * u, d, r, C)] = x[3 * k + d];
                    }
                }
            }
        }
    }
    if (bad) atomicOr(err, bad);
}

template <typename T, int G, int SMAX>
void launch_bucket_g(const Plan &P, bool up, bool wide, const T *brec, const T *v, T *out, T *xch, const Ctx &C,
                     hipStream_t s) {
    constexpr int LPW = 64 / G;
    const int64_t items = ((P.bucket_cap + LPW - 1) / LPW) * (int64_t)C.nchunks;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(items, 1 << 20));
#define HQ_BK(WXV, UPV)                                                                                        \
    hipLaunchKernelGGL((k_bucket<T, G, SMAX, WXV, UPV>), dim3(grid), dim3(64), 0, s, P.d_phase, P.d_tile_root, \
                       P.d_tile_base, P.d_tile_len, P.d_first, P.d_last, P.d_perm, P.d_links, brec, P.bucket_cap,  \
                       v, out, xch, C, P.d_err)
    if (wide) {
        if (up) HQ_BK(true, true);
        else HQ_BK(true, false);
    } else {
        if (up) HQ_BK(false, true);
        else HQ_BK(false, false);
    }
#undef HQ_BK
}

template <typename T, int G>
void launch_bucket(const Plan &P, bool up, bool wide, const T *brec, const T *v, T *out, T *xch, const Ctx &C,
                   hipStream_t s) {
    // leaves of up to 8 beads take the 24-row kernel (records laid out for 8)
    if (P.leaf_smax() <= 8) launch_bucket_g<T, G, 8>(P, up, wide, brec, v, out, xch, C, s);
    else launch_bucket_g<T, G, 16>(P, up, wide, brec, v, out, xch, C, s);
}

// The fused upward sweep (one launch for every tile phase), grid as the first
// phase's wide launch.
template <typename T, int LPT, int NC, bool TRI, bool ROT>
void launch_up_fused(const Plan &P, const T *rec, const T *v, T *out, T *xch, const T *rot, const Ctx &C,
                     hipStream_t s) {
    constexpr int TPW = 64 / LPT;
    const size_t lds_w = (size_t)C.nslot * 6 * 64 * NC * sizeof(T);
    const int64_t nrun_max = std::max<int64_t>(P.NI / P.run_nodes + 2, kRunTarget + 2);
    const int64_t items = ((nrun_max + TPW - 1) / TPW) * (int64_t)C.nchunks;
    const int64_t g = (P.first_wpc == 0) ? items : std::min<int64_t>(items, (int64_t)P.first_wpc * P.ncu);
    const unsigned grid = (unsigned)std::min<int64_t>(g, 1 << 20);
    if (C.R == 32)
        hipLaunchKernelGGL((k_up_fused<T, LPT, 32, NC, TRI, ROT>), dim3(grid), dim3(64), lds_w, s, P.d_prun, P.d_run,
                           rec, v, out, xch, rot, P.d_tile_base, P.d_tile_len, P.d_ptile, P.d_tcnt, P.d_tcnt0, C,
                           P.d_err);
    else
        hipLaunchKernelGGL((k_up_fused<T, LPT, 0, NC, TRI, ROT>), dim3(grid), dim3(64), lds_w, s, P.d_prun, P.d_run,
                           rec, v, out, xch, rot, P.d_tile_base, P.d_tile_len, P.d_ptile, P.d_tcnt, P.d_tcnt0, C,
                           P.d_err);
}

template <typename T, int LPT>
void launch_narrow(const Plan &P, int phase, int transpose, const T *rec, const T *v, T *out, T *xch, const Ctx &C,
                   hipStream_t s) {
    const size_t lds = (size_t)C.dmax * 6 * 64 * sizeof(T);
    constexpr int TPW = 64 / LPT;
    // one wave per work item of the phase (tile groups x RHS chunks); waves
    // without work exit at once
    const int64_t items = ((phase_tiles(P, phase) + TPW - 1) / TPW) * (int64_t)C.nchunks;
    const unsigned grid = (unsigned)std::min<int64_t>(items, 1 << 20);
    if (!transpose)
        hipLaunchKernelGGL((k_up<T, LPT>), dim3(grid), dim3(64), lds, s, phase, P.d_phase, P.d_tile_base,
                           P.d_tile_len, P.d_links, rec, v, out, xch, C, P.d_err);
    else
        hipLaunchKernelGGL((k_down<T, LPT>), dim3(grid), dim3(64), lds, s, phase, P.d_phase, P.d_tile_base,
                           P.d_tile_len, P.d_links, rec, v, out, xch, C, P.d_err);
}

// Node-parallel sweeps of one tile phase: TS slots per tile (a power of two
// above the phase's tile size), CW columns per node.
template <typename T, int CW, int TS, bool WX>
void launch_np_ts(const Plan &P, int phase, int transpose, const T *rec, const T *v, T *out, T *xch, const Ctx &C,
                  hipStream_t s) {
    constexpr int NB = TS * CW > 256 ? TS * CW : 256;
    constexpr int TPB = NB / (TS * CW);
    // a workgroup per tile group of the phase (the largest first phase a
    // rebuild can make); later phases stride over their tiles
    const int64_t groups = (phase_tiles(P, phase) + TPB - 1) / TPB;
    const int64_t items = groups * (int64_t)C.nchunks;
    const unsigned grid = (unsigned)std::min<int64_t>(items, phase == 1 ? (1 << 20) : 4096);
    if (!transpose)
        hipLaunchKernelGGL((k_up_np<T, NB, CW, TS, WX>), dim3(grid), dim3(NB), 0, s, phase, P.d_phase, P.d_tile_base,
                           P.d_tile_len, rec, v, out, xch, C, P.d_err);
    else
        hipLaunchKernelGGL((k_down_np<T, NB, CW, TS, WX>), dim3(grid), dim3(NB), 0, s, phase, P.d_phase,
                           P.d_tile_base, P.d_tile_len, rec, v, out, xch, C, P.d_err);
}

// Slots per tile for the node-parallel sweeps of a phase (0: its tiles are
// too large for them).
int np_slots(const Plan &P, int phase) {
    const int S = phase == 1 ? P.S : P.S2;
    return S <= 16 ? 16 : S <= 32 ? 32 : S <= 64 ? 64 : 0;
}

template <typename T, int CW>
void launch_np(const Plan &P, int phase, int transpose, const T *rec, const T *v, T *out, T *xch, const Ctx &C,
               hipStream_t s) {
    switch (np_slots(P, phase)) {
    case 16: launch_np_ts<T, CW, 16, false>(P, phase, transpose, rec, v, out, xch, C, s); break;
    case 32: launch_np_ts<T, CW, 32, false>(P, phase, transpose, rec, v, out, xch, C, s); break;
    default: launch_np_ts<T, CW, 64, false>(P, phase, transpose, rec, v, out, xch, C, s); break;
    }
}

enum SweepKind { kNarrow1, kNarrow2, kNarrow4, kNarrow8, kNarrow16, kWide16, kWide32, kWide64 };

// Lane-per-tile sweep of the first tile phase (false where a buffer lies
// beyond the range of 32-bit offsets).
template <typename T, int LPT>
bool launch_lane(const Plan &P, int transpose, const T *rec, const T *v, T *out, T *xch, const Ctx &C,
                 hipStream_t s) {
    const int64_t rb = P.NI * (int64_t)kRecWords * (int64_t)sizeof(T);
    if (!C.bufs_ok || rb >= (int64_t)kOOB - (int64_t)(1 << 20)) return false;
    constexpr int TPW = 64 / LPT;
    const size_t lds = (size_t)(C.nslot + 1) * 6 * 64 * sizeof(T);
    const int64_t items = ((2 * P.tiles_built + 64 + TPW - 1) / TPW) * (int64_t)C.nchunks;
    const unsigned grid = (unsigned)std::min<int64_t>(items, 1 << 20);
    if (!transpose)
        hipLaunchKernelGGL((k_up_lane<T, LPT>), dim3(grid), dim3(64), lds, s, P.d_phase, P.d_tile_base,
                           P.d_tile_len, rec, (uint32_t)rb, v, out, xch, C, P.d_err);
    else
        hipLaunchKernelGGL((k_down_lane<T, LPT>), dim3(grid), dim3(64), lds, s, P.d_phase, P.d_tile_base,
                           P.d_tile_len, rec, (uint32_t)rb, v, out, xch, C, P.d_err);
    return true;
}

// Node-parallel launch of a later phase of a 16-column FP32 wide sweep;
// false where it does not apply.  (At 32 columns a workgroup of a whole tile
// holds 1,024 lanes that each load the node's record; on the bench workload
// that made the second phase 2.8 times slower than the wide sweep, so wider
// sweeps keep the wide kernel in every phase.)
template <typename T>
bool launch_np_wide(const Plan &P, int phase, int transpose, SweepKind kind, const T *rec, const T *v, T *out, T *xch,
                    const Ctx &C, hipStream_t s) {
    const int ts = np_slots(P, phase);
    if (ts == 0 || kind != kWide16) return false;
    if constexpr (sizeof(T) == 4) {
        if (ts == 16) launch_np_ts<T, 16, 16, true>(P, phase, transpose, rec, v, out, xch, C, s);
        else if (ts == 32) launch_np_ts<T, 16, 32, true>(P, phase, transpose, rec, v, out, xch, C, s);
        else launch_np_ts<T, 16, 64, true>(P, phase, transpose, rec, v, out, xch, C, s);
        return true;
    }
    return false;
}

// The full Q = [Q_Z; Q~] (Algorithms 2 and 3 with the root kept): every body
// root is the root of a tile, whose exchange entry holds the root's Info-set
// after the upward sweep and supplies its Velocity-set to the downward one.
// Copies between those entries and the caller's root vector (6 rows per body,
// in the call's layout): to_xch = 0 gathers Q_Z v, 1 scatters L_root.
template <typename T, bool WIDE>
__global__ void k_root_io(int64_t m, const int32_t *__restrict__ node_off, const int32_t *__restrict__ tileof,
                          T *xch, T *root, int to_xch, Ctx C, int32_t *err) {
    const int64_t total = m * 6 * C.R;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = i / (6 * C.R);
        const int rem = (int)(i - j * 6 * C.R);
        const int d = rem / C.R, r = rem - d * C.R;
        const int g = node_off[j];
        const int t = (g >= 0 && g < C.nsched) ? tileof[g] : -1;
        if (t < 0 || t >= C.xch_cap) {
            atomicOr(err, kFlagBounds);
            continue;
        }
        const int64_t xi = WIDE ? ((int64_t)t * C.R + r) * 6 + d : ((int64_t)t * 6 + d) * C.R + r;
        const int64_t ri = velem(6 * j + 3 * (d / 3), d % 3, r, C);
        if (to_xch)
            xch[xi] = root[ri];
        else
            root[ri] = xch[xi];
    }
}

template <typename T>
void launch_root_io(const Plan &P, bool wide, T *xch, T *root, int to_xch, const Ctx &C, hipStream_t s) {
    const int64_t total = P.m * 6 * (int64_t)C.R;
    const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
    if (wide)
        hipLaunchKernelGGL((k_root_io<T, true>), dim3(grid), dim3(256), 0, s, P.m, P.d_node_off, P.d_tileof, xch, root,
                           to_xch, C, P.d_err);
    else
        hipLaunchKernelGGL((k_root_io<T, false>), dim3(grid), dim3(256), 0, s, P.m, P.d_node_off, P.d_tileof, xch,
                           root, to_xch, C, P.d_err);
}

// Sweep kinds: narrow (lanes per tile 1..16, tile stack in LDS) and wide
// (runs of whole tiles, explicit slots, buffer addressing).

// fewest right-hand sides the wide sweeps take (sweep_kernel = 0)
constexpr int kWideMinR = 8;

template <typename T>
void launch_all(const Plan &P, int transpose, SweepKind kind, const T *rec, const T *v, T *out, T *xch,
                const T *rot, const Ctx &C, hipStream_t s, hipEvent_t *ev) {
    const bool tri = C.vlane == 3;
    const int nph = std::max(P.phases_built, P.phases_reserved);
    if (!transpose && P.fused_up && C.nchunks == 1 && P.leaf_s <= 1 &&
        (kind == kWide16 || kind == kWide32 || kind == kWide64)) {
        // every tile phase in one launch (the arrival counters count a
        // tile's children once, so one column chunk per sweep: up to 64
        // right-hand sides); its time is reported as the first phase's, the
        // later phases' as 0
        if (ev) (void)hipEventRecord(ev[0], s);
#define HQ_FUSED(LPT)                                                                                          \
        do {                                                                                                   \
            if (rot) {                                                                                         \
                if (tri) launch_up_fused<T, LPT, 1, true, true>(P, rec, v, out, xch, rot, C, s);               \
                else launch_up_fused<T, LPT, 1, false, true>(P, rec, v, out, xch, rot, C, s);                  \
            } else {                                                                                           \
                if (tri) launch_up_fused<T, LPT, 1, true, false>(P, rec, v, out, xch, rot, C, s);              \
                else launch_up_fused<T, LPT, 1, false, false>(P, rec, v, out, xch, rot, C, s);                 \
            }                                                                                                  \
        } while (0)
        if (kind == kWide16) {
            if constexpr (sizeof(T) == 4) HQ_FUSED(16);
        } else if (kind == kWide32) {
            HQ_FUSED(32);
        } else {
            HQ_FUSED(64);
        }
#undef HQ_FUSED
        if (ev)
            for (int k = 1; k <= nph; ++k) (void)hipEventRecord(ev[k], s);
        return;
    }
    for (int k = 0; k < nph; ++k) {
        const int phase = transpose ? (nph - k) : (k + 1);
        if (ev) (void)hipEventRecord(ev[k], s);
        if (phase == 1 && P.leaf_s > 1) {
            // the first phase holds the leaf boxes
            const T *brec = sizeof(T) == 8 ? reinterpret_cast<const T *>(P.d_brec64)
                                           : reinterpret_cast<const T *>(P.d_brec32);
            const bool wide = kind == kWide16 || kind == kWide32 || kind == kWide64;
            // one lane per leaf for a single right-hand side, else groups of
            // 16, 32 or 64 lanes (idle lanes beyond the columns)
            switch (kind) {
            case kNarrow1: launch_bucket<T, 1>(P, !transpose, wide, brec, v, out, xch, C, s); break;
            case kNarrow2:
            case kNarrow4:
            case kNarrow8:
            case kNarrow16:
            case kWide16: launch_bucket<T, 16>(P, !transpose, wide, brec, v, out, xch, C, s); break;
            case kWide32: launch_bucket<T, 32>(P, !transpose, wide, brec, v, out, xch, C, s); break;
            case kWide64: launch_bucket<T, 64>(P, !transpose, wide, brec, v, out, xch, C, s); break;
            }
            continue;
        }
        // node-parallel sweeps (up to 8 columns per pass) where the phase's
        // tiles fit them: in the later phases of 16 units or more by default,
        // in every phase on request.  (The first phase stays with the lane
        // group per tile: there every lane is busy already, and a
        // node-parallel round issues the node arithmetic across all the
        // tile's lanes, once per level; tiles of 8 units are short chains
        // for a lane group, and fill half a node-parallel tile's lanes.)
        const bool np = np_slots(P, phase) > 0 &&
                        (P.sweep_kernel == 2 || (P.sweep_kernel == 0 && phase > 1 && P.S2 >= 16));
        if (kind != kWide16 && kind != kWide32 && kind != kWide64) {
            // the first phase: lane group per tile with exact wait counts
            // (every access issued, absent ones out of range)
            const bool lane = phase == 1 && P.sweep_kernel == 0;
            if (lane) {
                bool done = false;
                switch (kind) {
                case kNarrow1: done = launch_lane<T, 1>(P, transpose, rec, v, out, xch, C, s); break;
                case kNarrow2: done = launch_lane<T, 2>(P, transpose, rec, v, out, xch, C, s); break;
                case kNarrow4: done = launch_lane<T, 4>(P, transpose, rec, v, out, xch, C, s); break;
                case kNarrow8: done = launch_lane<T, 8>(P, transpose, rec, v, out, xch, C, s); break;
                default: break;
                }
                if (done) continue;
            }
            switch (kind) {
            case kNarrow1:
                if (np) launch_np<T, 1>(P, phase, transpose, rec, v, out, xch, C, s);
                else launch_narrow<T, 1>(P, phase, transpose, rec, v, out, xch, C, s);
                break;
            case kNarrow2:
                if (np) launch_np<T, 2>(P, phase, transpose, rec, v, out, xch, C, s);
                else launch_narrow<T, 2>(P, phase, transpose, rec, v, out, xch, C, s);
                break;
            case kNarrow4:
                if (np) launch_np<T, 4>(P, phase, transpose, rec, v, out, xch, C, s);
                else launch_narrow<T, 4>(P, phase, transpose, rec, v, out, xch, C, s);
                break;
            case kNarrow8:
                if (np) launch_np<T, 8>(P, phase, transpose, rec, v, out, xch, C, s);
                else launch_narrow<T, 8>(P, phase, transpose, rec, v, out, xch, C, s);
                break;
            case kNarrow16: launch_narrow<T, 16>(P, phase, transpose, rec, v, out, xch, C, s); break;
            default: break;
            }
            continue;
        }
        // the later phases of a wide sweep, node-parallel (one lane per node
        // and column, the wide sweeps' exchange layout) where those phases
        // hold few tiles, so that the wide sweep's chains would leave the
        // device idle
        if (!rot && phase > 1 && P.sweep_kernel == 0 && P.tiles_built - P.tiles1_built <= 4 * (int64_t)P.ncu &&
            launch_np_wide(P, phase, transpose, kind, rec, v, out, xch, C, s))
            continue;
        switch (kind) {
        case kWide16:
            // 16-lane runs (four per wave) broadcast float records inside
            // 16-lane rows; double records need 32-lane halves
            if constexpr (sizeof(T) == 4) {
                if (rot) {
                    if (tri) launch_wide<T, 16, 1, true, true>(P, phase, transpose, rec, v, out, xch, rot, C, s);
                    else launch_wide<T, 16, 1, false, true>(P, phase, transpose, rec, v, out, xch, rot, C, s);
                } else {
                    if (tri) launch_wide<T, 16, 1, true, false>(P, phase, transpose, rec, v, out, xch, rot, C, s);
                    else launch_wide<T, 16, 1, false, false>(P, phase, transpose, rec, v, out, xch, rot, C, s);
                }
            }
            break;
        case kWide32:
            if (rot) {
                if (tri) launch_wide<T, 32, 1, true, true>(P, phase, transpose, rec, v, out, xch, rot, C, s);
                else launch_wide<T, 32, 1, false, true>(P, phase, transpose, rec, v, out, xch, rot, C, s);
            } else {
                if (tri) launch_wide<T, 32, 1, true, false>(P, phase, transpose, rec, v, out, xch, rot, C, s);
                else launch_wide<T, 32, 1, false, false>(P, phase, transpose, rec, v, out, xch, rot, C, s);
            }
            break;
        case kWide64:
            if (rot) {
                if (tri) launch_wide<T, 64, 1, true, true>(P, phase, transpose, rec, v, out, xch, rot, C, s);
                else launch_wide<T, 64, 1, false, true>(P, phase, transpose, rec, v, out, xch, rot, C, s);
            } else {
                if (tri) launch_wide<T, 64, 1, true, false>(P, phase, transpose, rec, v, out, xch, rot, C, s);
                else launch_wide<T, 64, 1, false, false>(P, phase, transpose, rec, v, out, xch, rot, C, s);
            }
            break;
        default: break;
        }
    }
    if (ev) (void)hipEventRecord(ev[nph], s);
}

}  // namespace

int lanes_per_tile(int64_t nrhs) {
    int l = 1;
    while (l < nrhs && l < 64) l <<= 1;
    return l;
}

// the rotation table in FP32 for the FP32 sweeps
__global__ void k_rot_to_float(int64_t n, const double *__restrict__ in, float *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

hq_status apply_device(Plan &P, const void *v, void *out, void *root, int transpose, int64_t nrhs, int prec,
                       int layout, hipStream_t s, hipEvent_t *ev, const double *rot, void *xch, size_t xch_bytes) {
    if (!xch) {
        xch = P.d_xch;
        xch_bytes = P.xch_bytes;
    }
    Ctx C;
    C.m = (int)P.m;
    C.N = P.N;
    C.rows = P.rows;
    C.nsched = P.NI;
    C.R = (int)nrhs;
    C.vlane = (layout == HQ_TRIPLES) ? 3 : 1;
    C.vcomp = (layout == HQ_TRIPLES) ? 1 : C.R;
    C.root_in = (root && transpose) ? 1 : 0;
    const size_t elem = (prec == HQ_FP64) ? sizeof(double) : sizeof(float);
    C.xch_cap = (int)std::min<int64_t>(INT32_MAX, (int64_t)(xch_bytes / (6 * elem * (size_t)nrhs)));
    // the wide sweeps address each buffer with 32-bit byte offsets below 2 GiB
    const int64_t vin = (transpose ? P.rows : 3 * P.N) * nrhs * (int64_t)elem;
    const int64_t vout = (transpose ? 3 * P.N : P.rows) * nrhs * (int64_t)elem;
    const int64_t vx = (int64_t)C.xch_cap * 6 * nrhs * (int64_t)elem;
    const int64_t lim = (int64_t)kOOB - (int64_t)(1 << 20);
    const bool wide_ok = vin < lim && vout < lim && vx < lim;
    C.bufs_ok = wide_ok ? 1 : 0;
    C.in_bytes = (uint32_t)std::min<int64_t>(vin, lim);
    C.out_bytes = (uint32_t)std::min<int64_t>(vout, lim);
    C.xch_bytes = (uint32_t)std::min<int64_t>(vx, lim);
    // Wide sweeps (a lane group per run of whole tiles, one column per lane,
    // each node record read once per group and broadcast): 32 or 64 lanes
    // per run above 16 right-hand sides; 8 to 16 of them, 16-lane runs
    // (FP32) or 32-lane runs (FP64, whose records need 32 lanes), the lanes
    // beyond the columns computing alongside without storing.  (Two columns
    // per lane measured slower: 4 runs per wave lose more to uneven run
    // lengths and to LDS-limited occupancy than they save in VALU work.)
    // Narrow sweeps (a lane group per tile, each lane reading whole records)
    // below 8 right-hand sides (measured faster at one: 0.31 against 0.39 ms
    // for both sweeps of 1,000 bodies of 200-2,000 beads, where a 16-lane run
    // idles 15 lanes; slower at 16: 0.29 against 0.21 ms on a 65,536-bead
    // body), beyond the wide sweeps' 2 GiB range, or on request.
    int lpt = lanes_per_tile(nrhs);
    SweepKind kind;
    int cols;  // right-hand sides per chunk
    if (wide_ok && (P.sweep_kernel == 3 || (P.sweep_kernel == 0 && nrhs >= kWideMinR))) {
        if (lpt >= 32) {
            kind = (lpt == 32) ? kWide32 : kWide64;
            cols = lpt;
        } else if (prec == HQ_FP32) {
            kind = kWide16;
            cols = 16;
        } else {
            kind = kWide32;
            cols = 32;
        }
    } else {
        // node-parallel sweeps take up to 8 columns per pass, the
        // lane-group-per-tile ones up to 16
        lpt = std::min(lpt, P.sweep_kernel == 1 ? 16 : 8);
        kind = lpt == 1 ? kNarrow1 : lpt == 2 ? kNarrow2 : lpt == 4 ? kNarrow4 : lpt == 8 ? kNarrow8 : kNarrow16;
        cols = lpt;
    }
    C.nchunks = (int)((nrhs + cols - 1) / cols);
    C.dmax = stack_depth(P.smax());
    C.nslot = stack_slots(P.smax());
    const bool wide = kind == kWide16 || kind == kWide32 || kind == kWide64;
    // rigid-motion rotations are fused into the wide sweeps only (not into
    // leaf boxes); the caller turns the vectors in separate passes otherwise
    if (rot && (!wide || P.leaf_s > 1)) return HQ_E_UNSUPPORTED;
    if (prec == HQ_FP64) {
        if (root && transpose) launch_root_io<double>(P, wide, (double *)xch, (double *)root, 1, C, s);
        launch_all<double>(P, transpose, kind, P.d_rec64, (const double *)v, (double *)out, (double *)xch, rot, C,
                           s, ev);
        if (root && !transpose) launch_root_io<double>(P, wide, (double *)xch, (double *)root, 0, C, s);
    } else {
        const float *rotf = nullptr;
        if (rot) {
            hipLaunchKernelGGL(k_rot_to_float, dim3(std::min<int64_t>((9 * P.m + 255) / 256, 1024)), dim3(256), 0, s,
                               9 * P.m, rot, P.d_rotf);
            rotf = P.d_rotf;
        }
        if (root && transpose) launch_root_io<float>(P, wide, (float *)xch, (float *)root, 1, C, s);
        launch_all<float>(P, transpose, kind, P.d_rec32, (const float *)v, (float *)out, (float *)xch, rotf, C, s,
                          ev);
        if (root && !transpose) launch_root_io<float>(P, wide, (float *)xch, (float *)root, 0, C, s);
    }
    HQ_HIP(hipGetLastError());
    return HQ_OK;
}

}  // namespace hq
