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
#include "hq_common.h"

#include <cstdlib>

namespace hq {

namespace {

struct Ctx {
    int64_t N, rows, nsched;
    int R, nchunks, dmax, xch_cap;
    int xslot;  // first scratch slot of the wide sweeps
};

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
            for (int c = 0; c < 3; ++c) m[c] = v[((int64_t)3 * ref + c) * C.R + r];
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
            T *o = out + (int64_t)off * C.R + r;
            o[0] = t9[3];
            o[C.R] = t9[4];
            o[2 * C.R] = t9[5];
            if (dim == 6) {
                o[3 * C.R] = t9[6];
                o[4 * C.R] = t9[7];
                o[5 * C.R] = t9[8];
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
            const T *src = w + (int64_t)off * C.R + r;
            n.a[0] = src[0];
            n.a[1] = src[C.R];
            n.a[2] = src[2 * C.R];
            if (dim == 6) {
                n.a[3] = src[3 * C.R];
                n.a[4] = src[4 * C.R];
                n.a[5] = src[5 * C.R];
            }
        }
    }
    if ((meta & kMetaTileRoot) && !(meta & kMetaBodyRoot)) {
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
            T *o = out + (int64_t)3 * ref * C.R + r;
            o[0] = L[0];
            o[C.R] = L[1];
            o[2 * C.R] = L[2];
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
    if (meta & kMetaBodyRoot) {
#pragma unroll
        for (int c = 0; c < 6; ++c) L[c] = T(0);
    } else if (meta & kMetaTileRoot) {
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
// Wide sweeps: a lane group of 32 or 64 lanes (one right-hand side per lane)
// sweeps a run of whole tiles; a wave holds two groups of 32 or one of 64.
//
// A node record is 32 elements; lane q of each 32-lane half holds element q,
// so one coalesced load fetches a whole record and ds_swizzle broadcasts
// element w inside the half when the node is processed.  The sweep order is
// fixed at build time, and so is the stack depth at every node: the record
// names the LDS slots of the two children and of the node's own result, so
// a node step has no stack pointer and no data-dependent branches; the
// case-dependent packing of the length-9 vector is done with selects.
//
// Latency: records are loaded PR nodes ahead and memory inputs NR - 1 nodes
// ahead.  Every load is issued unconditionally (a child with nothing to load
// reads a valid dummy address and the value is discarded), so the compiler
// can wait for exactly the loads a node needs instead of draining all
// outstanding ones; only stores are predicated.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ float bcast(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), W << 5));
}

template <int W>
__device__ __forceinline__ double bcast(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffll), W << 5);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), W << 5);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

template <int W, typename T>
__device__ __forceinline__ void bcast_g(T (&g)[26], T v) {
    g[W] = bcast<W>(v);
    if constexpr (W + 1 < 26) bcast_g<W + 1>(g, v);
}

// the link words of a record (elements 26.. as int32)
struct Links6 {
    int xref, yref, off, meta, slots;
};

__device__ __forceinline__ Links6 bcast_links6(float v) {
    Links6 l;
    l.xref = __float_as_int(bcast<26>(v));
    l.yref = __float_as_int(bcast<27>(v));
    l.off = __float_as_int(bcast<28>(v));
    l.meta = __float_as_int(bcast<29>(v));
    l.slots = __float_as_int(bcast<30>(v));
    return l;
}

__device__ __forceinline__ Links6 bcast_links6(double v) {
    const long long a = __double_as_longlong(bcast<26>(v)), b = __double_as_longlong(bcast<27>(v));
    const long long c = __double_as_longlong(bcast<28>(v));
    Links6 l;
    l.xref = (int)(a & 0xffffffffll);
    l.yref = (int)(a >> 32);
    l.off = (int)(b & 0xffffffffll);
    l.meta = (int)(b >> 32);
    l.slots = (int)(c & 0xffffffffll);
    return l;
}

__device__ __forceinline__ int2 bcast_refs(float v) {
    return make_int2(__float_as_int(bcast<26>(v)), __float_as_int(bcast<27>(v)));
}

__device__ __forceinline__ int2 bcast_refs(double v) {
    const long long a = __double_as_longlong(bcast<26>(v));
    return make_int2((int)(a & 0xffffffffll), (int)(a >> 32));
}

// LDS slot layout: [slot][component 0..5][64 lanes]
template <typename T>
__device__ __forceinline__ void lds_put6(T *lds, int slot, int lane, const T (&m)[6]) {
    T *p = lds + slot * 6 * 64 + lane;
#pragma unroll
    for (int c = 0; c < 6; ++c) p[c * 64] = m[c];
}

template <typename T>
__device__ __forceinline__ void lds_get6(const T *lds, int slot, int lane, T (&m)[6]) {
    const T *p = lds + slot * 6 * 64 + lane;
#pragma unroll
    for (int c = 0; c < 6; ++c) m[c] = p[c * 64];
}

template <int RT>
__device__ __forceinline__ int rhs_count(const Ctx &C) {
    return RT ? RT : C.R;
}

// Upward memory input of one child, IW values: a bead's vector (3 values,
// zero Info-set tail) or, with IW = 6, an earlier tile root's Info-set.  A
// stack child reads the dummy rows at v instead.  IW = 3 serves the first
// tile phase, whose only memory inputs are beads.
template <typename T, int RT, int IW>
__device__ __forceinline__ void up_input(int ref, T (&m)[IW], const T *__restrict__ v, const T *__restrict__ xch,
                                         const Ctx &C, int rr) {
    const int R = rhs_count<RT>(C);
    const bool isb = ref >= 0;
    const int64_t u = min((int64_t)max(ref, 0), C.N - 1);
    const T *pb = v + (3 * u) * R + rr;
    if constexpr (IW == 3) {
        const T *p = isb ? pb : v + rr;
        m[0] = p[0];
        m[1] = p[R];
        m[2] = p[2 * R];
    } else {
        const bool isx = ref < kRefStack;
        const int64_t sl = min((int64_t)max(ref_slot(ref), 0), (int64_t)C.xch_cap - 1);
        const T *px = xch + sl * 6 * R + rr;
        const T *p = isb ? pb : (isx ? px : v + rr);
        const T *q = isx ? px + 3 * R : p;
        m[0] = p[0];
        m[1] = p[R];
        m[2] = p[2 * R];
        m[3] = q[0];
        m[4] = q[R];
        m[5] = q[2 * R];
    }
}

// One upward node step (Eqs. 4.2-4.3).  A child of the same tile is read from
// its LDS slot; a bead or an earlier tile's root comes from the prefetched
// registers ax / ay.  Nothing is stored unless the node is live.
template <typename T, int RT, int IW>
__device__ __forceinline__ void up_node(const T (&g)[26], const Links6 &lk, const T (&ax)[IW], const T (&ay)[IW],
                                        T *lds, int lane, T *__restrict__ out, T *__restrict__ xch, const Ctx &C,
                                        int rr, bool live, bool act, int &bad) {
    const int R = rhs_count<RT>(C);
    const int xs = min(lk.slots & 0xff, C.xslot), ys = min((lk.slots >> 8) & 0xff, C.xslot);
    const int os = min((lk.slots >> 16) & 0xff, C.xslot);
    const bool xst = lk.xref == kRefStack, yst = lk.yref == kRefStack;
    T mx[6], my[6];
    lds_get6(lds, xs, lane, mx);
    lds_get6(lds, ys, lane, my);
#pragma unroll
    for (int c = 0; c < IW; ++c) {
        mx[c] = xst ? mx[c] : ax[c];
        my[c] = yst ? my[c] : ay[c];
    }
    const T sx = g[kRecSx], sy = g[kRecSy];
    const bool xi = lk.xref < 0, yi = lk.yref < 0;
    const bool both = xi && yi, any = xi || yi;
    T mp[6], t9[9], tt[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        mp[c] = sx * mx[c] + sy * my[c];
        tt[c] = sy * mx[c] - sx * my[c];
    }
    // t = [M_x(4:6)?; M_y(4:6)?; tt] packed to the front, zeros behind
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        t9[c] = xi ? mx[3 + c] : (yi ? my[3 + c] : tt[c]);
        t9[3 + c] = both ? my[3 + c] : (any ? tt[c] : T(0));
        t9[6 + c] = both ? tt[c] : T(0);
    }
    house_fwd<9>(t9, g);
#pragma unroll
    for (int c = 0; c < 3; ++c) mp[3 + c] = t9[c];
    const int dim = 3 * (int)xi + 3 * (int)yi;
    const int64_t off = min((int64_t)max(lk.off, 0), C.rows - dim);
    const bool troot = (lk.meta & kMetaTileRoot) != 0;
    const int64_t slot = lk.meta >> kMetaSlotShift;
    if (live) {
        if (lk.off < 0 || (int64_t)lk.off + dim > C.rows) bad |= kFlagBounds;
        if (troot && slot >= C.xch_cap) bad |= kFlagBounds;
        if (act && dim > 0) {
            T *o = out + off * R + rr;
            o[0] = t9[3];
            o[R] = t9[4];
            o[2 * R] = t9[5];
            if (dim == 6) {
                o[3 * R] = t9[6];
                o[4 * R] = t9[7];
                o[5 * R] = t9[8];
            }
        }
        if (troot) {
            if (act) {
                T *p = xch + min(slot, (int64_t)C.xch_cap - 1) * 6 * R + rr;
#pragma unroll
                for (int c = 0; c < 6; ++c) p[c * R] = mp[c];
            }
        } else {
            lds_put6(lds, os, lane, mp);
        }
    }
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

template <typename T, int LPT, int RT, int PR, int NR, int IW>
__global__ void __launch_bounds__(64, 4) k_up_wide(int phase, const int32_t *__restrict__ prun,
                                                   const int32_t *__restrict__ run, const T *__restrict__ rec,
                                                   const T *__restrict__ v, T *__restrict__ out,
                                                   T *__restrict__ xch, Ctx C, int32_t *err) {
    static_assert(LPT == 32 || LPT == 64, "wide sweeps use 32 or 64 lanes per run");
    static_assert(PR % NR == 0 && NR >= 2 && (PR == 3 || PR == 4 || PR == 6), "ring sizes");
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    constexpr int TPW = 64 / LPT;
    const int R = rhs_count<RT>(C);
    const int lane = threadIdx.x;
    const int q = lane & 31;
    const int tslot = lane / LPT, rl = lane % LPT;
    const int c0 = prun[4 * phase + 2], nrun = prun[4 * phase + 3];
    const int items = ((nrun + TPW - 1) / TPW) * C.nchunks;
    int bad = 0;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int grp = item / C.nchunks, chunk = item - grp * C.nchunks;
        const int r = chunk * LPT + rl;
        const int rr = min(r, R - 1);
        int base, len;
        run_range(grp * TPW + tslot, nrun, c0, run, C, base, len, bad);
        const bool act = r < R;
        int maxlen = len;
        if (LPT == 32) maxlen = max(maxlen, __shfl_xor(len, 32, 64));
        maxlen = __builtin_amdgcn_readfirstlane(maxlen);
        const int last = max(len - 1, 0);
        const T *rp = rec + (int64_t)kRecWords * base + q;
        T RW[PR];
        T A[NR][IW], B[NR][IW];
#pragma unroll
        for (int k = 0; k < PR; ++k) RW[k] = rp[(int64_t)min(k, last) * kRecWords];
#pragma unroll
        for (int k = 0; k < NR - 1; ++k) {
            const int2 ref = bcast_refs(RW[k]);
            up_input<T, RT, IW>(ref.x, A[k], v, xch, C, rr);
            up_input<T, RT, IW>(ref.y, B[k], v, xch, C, rr);
        }
#define HQ_UP_STEP(K)                                                                       \
        {                                                                                   \
            const int n = n0 + (K);                                                         \
            T g[26];                                                                        \
            bcast_g<0>(g, RW[K]);                                                           \
            const Links6 lk = bcast_links6(RW[K]);                                          \
            RW[K] = rp[(int64_t)min(n + PR, last) * kRecWords];                             \
            {                                                                               \
                const int2 ref = bcast_refs(RW[((K) + NR - 1) % PR]);                       \
                up_input<T, RT, IW>(ref.x, A[((K) + NR - 1) % NR], v, xch, C, rr);          \
                up_input<T, RT, IW>(ref.y, B[((K) + NR - 1) % NR], v, xch, C, rr);          \
            }                                                                               \
            up_node<T, RT, IW>(g, lk, A[(K) % NR], B[(K) % NR], lds, lane, out, xch, C, rr, n < len, act, bad); \
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
        }
#undef HQ_UP_STEP
    }
    if (bad) atomicOr(err, bad);
}

// Downward memory inputs of one node, always 12 loads: its residue
// coefficients w_p (dim = 0, 3 or 6 values) and, for a tile root below a body
// root, its Velocity-set from the exchange buffer; the rest reads dummy rows
// of the exchange buffer.
template <typename T, int RT>
__device__ __forceinline__ void down_input(const Links6 &lk, T (&a)[6], T (&b)[6], const T *__restrict__ w,
                                           const T *__restrict__ xch, const Ctx &C, int rr) {
    const int R = rhs_count<RT>(C);
    const int dim = 3 * (int)(lk.xref < 0) + 3 * (int)(lk.yref < 0);
    const int64_t off = min((int64_t)max(lk.off, 0), max(C.rows - dim, (int64_t)0));
    const T *dummy = xch + rr;
    const T *p = (dim > 0) ? w + off * R + rr : dummy;
    const T *p2 = (dim == 6) ? p + 3 * R : p;
    a[0] = p[0];
    a[1] = p[R];
    a[2] = p[2 * R];
    a[3] = p2[0];
    a[4] = p2[R];
    a[5] = p2[2 * R];
    const bool lr = (lk.meta & kMetaTileRoot) && !(lk.meta & kMetaBodyRoot);
    const int64_t sl = min((int64_t)(lk.meta >> kMetaSlotShift), (int64_t)C.xch_cap - 1);
    const T *px = lr ? xch + sl * 6 * R + rr : dummy;
#pragma unroll
    for (int c = 0; c < 6; ++c) b[c] = px[c * R];
}

// One downward node step (Theorem 4.3): L_p from its LDS slot (or the
// exchange buffer for a tile root, zero for a body root), children's
// Velocity-sets to their slots, to bead outputs, or to the exchange buffer.
template <typename T, int RT>
__device__ __forceinline__ void down_node(const T (&g)[26], const Links6 &lk, const T (&wp)[6], const T (&lroot)[6],
                                          T *lds, int lane, T *__restrict__ out, T *__restrict__ xch,
                                          const Ctx &C, int rr, bool live, bool act, int &bad) {
    const int R = rhs_count<RT>(C);
    const int xs = min(lk.slots & 0xff, C.xslot), ys = min((lk.slots >> 8) & 0xff, C.xslot);
    const int os = min((lk.slots >> 16) & 0xff, C.xslot);
    const bool troot = (lk.meta & kMetaTileRoot) != 0, broot = (lk.meta & kMetaBodyRoot) != 0;
    T L[6];
    lds_get6(lds, os, lane, L);
#pragma unroll
    for (int c = 0; c < 6; ++c) L[c] = troot ? (broot ? T(0) : lroot[c]) : L[c];
    const T sx = g[kRecSx], sy = g[kRecSy];
    const bool xi = lk.xref < 0, yi = lk.yref < 0;
    const bool both = xi && yi, any = xi || yi;
    const int dim = 3 * (int)xi + 3 * (int)yi;
    T x9[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) x9[c] = L[3 + c];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x9[3 + c] = (dim > 0) ? wp[c] : T(0);
        x9[6 + c] = (dim == 6) ? wp[3 + c] : T(0);
    }
    house_bwd<9>(x9, g);
    T st[3], Lx[6], Ly[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        st[c] = both ? x9[6 + c] : (any ? x9[3 + c] : x9[c]);
        Lx[3 + c] = x9[c];
        Ly[3 + c] = both ? x9[3 + c] : x9[c];
        Lx[c] = sx * L[c] + sy * st[c];
        Ly[c] = sy * L[c] - sx * st[c];
    }
    if (!live) return;
    // children of this tile go to their slots, others to the spare slot
    lds_put6(lds, xs, lane, Lx);
    lds_put6(lds, ys, lane, Ly);
    const int refs[2] = {lk.xref, lk.yref};
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
        const int ref = refs[ch];
        const T *Lc = ch ? Ly : Lx;
        if (ref >= 0) {
            if (ref >= C.N) bad |= kFlagBounds;
            const int64_t u = min((int64_t)ref, C.N - 1);
            if (act) {
                T *o = out + (3 * u) * R + rr;
                o[0] = Lc[0];
                o[R] = Lc[1];
                o[2 * R] = Lc[2];
            }
        } else if (ref != kRefStack) {
            if (ref_slot(ref) >= C.xch_cap) bad |= kFlagBounds;
            const int64_t sl = min((int64_t)ref_slot(ref), (int64_t)C.xch_cap - 1);
            if (act) {
                T *p = xch + sl * 6 * R + rr;
#pragma unroll
                for (int c = 0; c < 6; ++c) p[c * R] = Lc[c];
            }
        }
    }
    if (troot && !broot && (lk.meta >> kMetaSlotShift) >= C.xch_cap) bad |= kFlagBounds;
    if (dim > 0 && (lk.off < 0 || (int64_t)lk.off + dim > C.rows)) bad |= kFlagBounds;
}

template <typename T, int LPT, int RT, int PR, int NR>
__global__ void __launch_bounds__(64, 4) k_down_wide(int phase, const int32_t *__restrict__ prun,
                                                     const int32_t *__restrict__ run, const T *__restrict__ rec,
                                                     const T *__restrict__ w, T *__restrict__ out,
                                                     T *__restrict__ xch, Ctx C, int32_t *err) {
    static_assert(LPT == 32 || LPT == 64, "wide sweeps use 32 or 64 lanes per run");
    static_assert(PR % NR == 0 && NR >= 2 && (PR == 3 || PR == 4 || PR == 6), "ring sizes");
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    constexpr int TPW = 64 / LPT;
    const int R = rhs_count<RT>(C);
    const int lane = threadIdx.x;
    const int q = lane & 31;
    const int tslot = lane / LPT, rl = lane % LPT;
    const int c0 = prun[4 * phase + 2], nrun = prun[4 * phase + 3];
    const int items = ((nrun + TPW - 1) / TPW) * C.nchunks;
    int bad = 0;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int grp = item / C.nchunks, chunk = item - grp * C.nchunks;
        const int r = chunk * LPT + rl;
        const int rr = min(r, R - 1);
        int base, len;
        run_range(grp * TPW + tslot, nrun, c0, run, C, base, len, bad);
        const bool act = r < R;
        int maxlen = len;
        if (LPT == 32) maxlen = max(maxlen, __shfl_xor(len, 32, 64));
        maxlen = __builtin_amdgcn_readfirstlane(maxlen);
        const int last = max(len - 1, 0);
        // node n of the sweep is schedule index base + len - 1 - n
        const T *rp = rec + (int64_t)kRecWords * (base + last) + q;
        T RW[PR];
        T A[NR][6], B[NR][6];
#pragma unroll
        for (int k = 0; k < PR; ++k) RW[k] = rp[-(int64_t)min(k, last) * kRecWords];
#pragma unroll
        for (int k = 0; k < NR - 1; ++k) down_input<T, RT>(bcast_links6(RW[k]), A[k], B[k], w, xch, C, rr);
#define HQ_DOWN_STEP(K)                                                                     \
        {                                                                                   \
            const int n = n0 + (K);                                                         \
            T g[26];                                                                        \
            bcast_g<0>(g, RW[K]);                                                           \
            const Links6 lk = bcast_links6(RW[K]);                                          \
            RW[K] = rp[-(int64_t)min(n + PR, last) * kRecWords];                            \
            down_input<T, RT>(bcast_links6(RW[((K) + NR - 1) % PR]), A[((K) + NR - 1) % NR], \
                              B[((K) + NR - 1) % NR], w, xch, C, rr);                       \
            down_node<T, RT>(g, lk, A[(K) % NR], B[(K) % NR], lds, lane, out, xch, C, rr, n < len, act, bad); \
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
        }
#undef HQ_DOWN_STEP
    }
    if (bad) atomicOr(err, bad);
}

// ---------------------------------------------------------------------------
// Uniform sweeps: one run of whole tiles per wave, one right-hand side per
// lane (32 or 64 lanes).  The node record is wave-uniform, so it is read with
// scalar loads and the node's shape (which children are internal nodes, and
// whether they come from LDS or the exchange buffer) is a uniform branch:
// each of the four shapes runs its own Householder length (k = 3, 6 or 9)
// with no padding and no selects.
// ---------------------------------------------------------------------------
template <typename T>
struct UNode {
    T g[26];
    int xref, yref, off, meta, slots;
};

template <typename T>
__device__ __forceinline__ void uload(UNode<T> &u, const T *__restrict__ rp) {
#pragma unroll
    for (int i = 0; i < 26; ++i) u.g[i] = rp[i];
    const int32_t *li = reinterpret_cast<const int32_t *>(rp + kRecLinks);
    u.xref = li[0];
    u.yref = li[1];
    u.off = li[2];
    u.meta = li[3];
    u.slots = li[4];
}

// LDS slot layout of the uniform sweeps: [slot][component][lw lanes]
template <typename T>
__device__ __forceinline__ void ulds_put(T *lds, int slot, int lw, int lane, const T *m, int n) {
    T *p = lds + slot * 6 * lw + lane;
#pragma unroll
    for (int c = 0; c < 6; ++c)
        if (c < n) p[c * lw] = m[c];
}

template <typename T>
__device__ __forceinline__ void ulds_get(const T *lds, int slot, int lw, int lane, T (&m)[6]) {
    const T *p = lds + slot * 6 * lw + lane;
#pragma unroll
    for (int c = 0; c < 6; ++c) m[c] = p[c * lw];
}

// Upward memory inputs of a node: a bead child's vector (3 values) or an
// earlier tile root's Info-set (6 values); stack children are read later.
// One uniform base pointer and two uniform conditions keep the values in
// fixed registers.
template <typename T, int RT>
__device__ __forceinline__ void uup_fetch(int ref, T (&m)[6], const T *__restrict__ v, const T *__restrict__ xch,
                                          const Ctx &C, int rr, int &bad) {
    const int R = rhs_count<RT>(C);
    const bool isb = ref >= 0, isx = ref < kRefStack;
    if (isb && ref >= C.N) bad |= kFlagBounds;
    if (isx && ref_slot(ref) >= C.xch_cap) bad |= kFlagBounds;
    const int64_t u = min((int64_t)ref, C.N - 1);
    const int64_t sl = min((int64_t)ref_slot(ref), (int64_t)C.xch_cap - 1);
    const T *p = (isb ? v + (3 * u) * R : xch + sl * 6 * R) + rr;
    if (isb || isx) {
        m[0] = p[0];
        m[1] = p[R];
        m[2] = p[2 * R];
    }
    if (isx) {
        m[3] = p[3 * R];
        m[4] = p[4 * R];
        m[5] = p[5 * R];
    }
}

// One upward node step of shape (XI, YI) = (x is internal, y is internal).
template <typename T, int RT, bool XI, bool YI>
__device__ __forceinline__ void uup_node(const UNode<T> &u, const T (&ax)[6], const T (&ay)[6], T *lds, int lw,
                                         int lane, T *__restrict__ out, T *__restrict__ xch, const Ctx &C, int rr,
                                         bool act, int &bad) {
    constexpr int K = 3 + 3 * (int)XI + 3 * (int)YI;
    constexpr int dim = K - 3;
    const int R = rhs_count<RT>(C);
    T mx[6], my[6];
    if (u.xref == kRefStack) {
        ulds_get(lds, min(u.slots & 0xff, C.xslot), lw, lane, mx);
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) mx[c] = ax[c];
    }
    if (u.yref == kRefStack) {
        ulds_get(lds, min((u.slots >> 8) & 0xff, C.xslot), lw, lane, my);
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) my[c] = ay[c];
    }
    const T sx = u.g[kRecSx], sy = u.g[kRecSy];
    T mp[6], t[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        mp[c] = sx * mx[c] + sy * my[c];
        const T tt = sy * mx[c] - sx * my[c];
        if constexpr (XI) t[c] = mx[3 + c];
        if constexpr (YI) t[3 * (int)XI + c] = my[3 + c];
        t[dim + c] = tt;
    }
    house_fwd<K>(t, u.g);
#pragma unroll
    for (int c = 0; c < 3; ++c) mp[3 + c] = t[c];
    if constexpr (dim > 0) {
        if (u.off < 0 || (int64_t)u.off + dim > C.rows) bad |= kFlagBounds;
        const int64_t off = min((int64_t)max(u.off, 0), C.rows - dim);
        if (act) {
            T *o = out + off * R + rr;
#pragma unroll
            for (int c = 0; c < dim; ++c) o[c * R] = t[3 + c];
        }
    }
    if (u.meta & kMetaTileRoot) {
        if ((u.meta >> kMetaSlotShift) >= C.xch_cap) bad |= kFlagBounds;
        const int64_t sl = min((int64_t)(u.meta >> kMetaSlotShift), (int64_t)C.xch_cap - 1);
        if (act) {
            T *p = xch + sl * 6 * R + rr;
#pragma unroll
            for (int c = 0; c < 6; ++c) p[c * R] = mp[c];
        }
    } else {
        ulds_put(lds, min((u.slots >> 16) & 0xff, C.xslot), lw, lane, mp, 6);
    }
}

template <typename T, int RT>
__device__ __forceinline__ void uup_dispatch(const UNode<T> &u, const T (&ax)[6], const T (&ay)[6], T *lds, int lw,
                                             int lane, T *__restrict__ out, T *__restrict__ xch, const Ctx &C,
                                             int rr, bool act, int &bad) {
    const bool xi = u.xref < 0, yi = u.yref < 0;
    if (xi && yi) uup_node<T, RT, true, true>(u, ax, ay, lds, lw, lane, out, xch, C, rr, act, bad);
    else if (xi) uup_node<T, RT, true, false>(u, ax, ay, lds, lw, lane, out, xch, C, rr, act, bad);
    else if (yi) uup_node<T, RT, false, true>(u, ax, ay, lds, lw, lane, out, xch, C, rr, act, bad);
    else uup_node<T, RT, false, false>(u, ax, ay, lds, lw, lane, out, xch, C, rr, act, bad);
}

// Work item = (run, RHS chunk of 64); lanes at or above lw have no work.
struct URun {
    int base, len, chunk;
};

__device__ __forceinline__ bool urun(int item, int phase, const int32_t *__restrict__ prun,
                                     const int32_t *__restrict__ run, const Ctx &C, URun &w, int &bad) {
    const int c0 = prun[4 * phase + 2];
    const int k = item / C.nchunks;
    w.chunk = item - k * C.nchunks;
    w.base = run[c0 + k];
    w.len = run[c0 + k + 1] - w.base;
    if (w.base < 0 || w.len < 0 || (int64_t)w.base + w.len > C.nsched) {
        bad |= kFlagBounds;
        w.len = 0;
    }
    return true;
}

template <typename T, int RT>
__global__ void __launch_bounds__(64) k_up_u(int phase, const int32_t *__restrict__ prun,
                                             const int32_t *__restrict__ run, const T *__restrict__ rec,
                                             const T *__restrict__ v, T *__restrict__ out, T *__restrict__ xch,
                                             Ctx C, int lw, int32_t *err) {
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int lane = threadIdx.x;
    if (lane >= lw) return;
    const int R = rhs_count<RT>(C);
    const int items = prun[4 * phase + 3] * C.nchunks;
    int bad = 0;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        URun w;
        urun(item, phase, prun, run, C, w, bad);
        const int r = w.chunk * 64 + lane;
        const bool act = r < R;
        const int rr = min(r, R - 1);
        const T *rp = rec + (int64_t)kRecWords * w.base;
        UNode<T> u;
        T A[6], B[6];
        if (w.len > 0) {
            uload(u, rp);
            uup_fetch<T, RT>(u.xref, A, v, xch, C, rr, bad);
            uup_fetch<T, RT>(u.yref, B, v, xch, C, rr, bad);
        }
        for (int n = 0; n < w.len; ++n) {
            UNode<T> un;
            T An[6], Bn[6];
            if (n + 1 < w.len) {
                uload(un, rp + (int64_t)(n + 1) * kRecWords);
                uup_fetch<T, RT>(un.xref, An, v, xch, C, rr, bad);
                uup_fetch<T, RT>(un.yref, Bn, v, xch, C, rr, bad);
            }
            uup_dispatch<T, RT>(u, A, B, lds, lw, lane, out, xch, C, rr, act, bad);
            u = un;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                A[c] = An[c];
                B[c] = Bn[c];
            }
        }
    }
    if (bad) atomicOr(err, bad);
}

// Downward memory inputs of a node: its residue coefficients (dim values) and,
// for a tile root below a body root, its Velocity-set from the exchange buffer.
template <typename T, int RT>
__device__ __forceinline__ void udown_fetch(const UNode<T> &u, T (&a)[6], T (&b)[6], const T *__restrict__ w,
                                            const T *__restrict__ xch, const Ctx &C, int rr, int &bad) {
    const int R = rhs_count<RT>(C);
    const int dim = 3 * (int)(u.xref < 0) + 3 * (int)(u.yref < 0);
    if (dim > 0) {
        if (u.off < 0 || (int64_t)u.off + dim > C.rows) bad |= kFlagBounds;
        const int64_t off = min((int64_t)max(u.off, 0), C.rows - dim);
        const T *p = w + off * R + rr;
        a[0] = p[0];
        a[1] = p[R];
        a[2] = p[2 * R];
        if (dim == 6) {
            a[3] = p[3 * R];
            a[4] = p[4 * R];
            a[5] = p[5 * R];
        }
    }
    if ((u.meta & kMetaTileRoot) && !(u.meta & kMetaBodyRoot)) {
        if ((u.meta >> kMetaSlotShift) >= C.xch_cap) bad |= kFlagBounds;
        const int64_t sl = min((int64_t)(u.meta >> kMetaSlotShift), (int64_t)C.xch_cap - 1);
        const T *p = xch + sl * 6 * R + rr;
#pragma unroll
        for (int c = 0; c < 6; ++c) b[c] = p[c * R];
    }
}

template <typename T, int RT>
__device__ __forceinline__ void udown_emit(int ref, int slot, const T *Lc, T *lds, int lw, int lane,
                                           T *__restrict__ out, T *__restrict__ xch, const Ctx &C, int rr, bool act,
                                           int &bad) {
    const int R = rhs_count<RT>(C);
    if (ref >= 0) {
        if (ref >= C.N) bad |= kFlagBounds;
        const int64_t u = min((int64_t)ref, C.N - 1);
        if (act) {
            T *o = out + (3 * u) * R + rr;
            o[0] = Lc[0];
            o[R] = Lc[1];
            o[2 * R] = Lc[2];
        }
    } else if (ref == kRefStack) {
        ulds_put(lds, min(slot, C.xslot), lw, lane, Lc, 6);
    } else {
        if (ref_slot(ref) >= C.xch_cap) bad |= kFlagBounds;
        const int64_t sl = min((int64_t)ref_slot(ref), (int64_t)C.xch_cap - 1);
        if (act) {
            T *p = xch + sl * 6 * R + rr;
#pragma unroll
            for (int c = 0; c < 6; ++c) p[c * R] = Lc[c];
        }
    }
}

// One downward node step of shape (XI, YI) (Theorem 4.3).
template <typename T, int RT, bool XI, bool YI>
__device__ __forceinline__ void udown_node(const UNode<T> &u, const T (&wp)[6], const T (&lroot)[6], T *lds, int lw,
                                           int lane, T *__restrict__ out, T *__restrict__ xch, const Ctx &C, int rr,
                                           bool act, int &bad) {
    constexpr int K = 3 + 3 * (int)XI + 3 * (int)YI;
    constexpr int dim = K - 3;
    T L[6];
    if (u.meta & kMetaTileRoot) {
        if (u.meta & kMetaBodyRoot) {
#pragma unroll
            for (int c = 0; c < 6; ++c) L[c] = T(0);
        } else {
#pragma unroll
            for (int c = 0; c < 6; ++c) L[c] = lroot[c];
        }
    } else {
        ulds_get(lds, min((u.slots >> 16) & 0xff, C.xslot), lw, lane, L);
    }
    T x[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = L[3 + c];
#pragma unroll
    for (int c = 0; c < dim; ++c) x[3 + c] = wp[c];
    house_bwd<K>(x, u.g);
    const T sx = u.g[kRecSx], sy = u.g[kRecSy];
    T Lx[6], Ly[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T st = x[dim + c];
        if constexpr (XI) Lx[3 + c] = x[c];
        if constexpr (YI) Ly[3 + c] = x[3 * (int)XI + c];
        Lx[c] = sx * L[c] + sy * st;
        Ly[c] = sy * L[c] - sx * st;
    }
    udown_emit<T, RT>(u.xref, u.slots & 0xff, Lx, lds, lw, lane, out, xch, C, rr, act, bad);
    udown_emit<T, RT>(u.yref, (u.slots >> 8) & 0xff, Ly, lds, lw, lane, out, xch, C, rr, act, bad);
}

template <typename T, int RT>
__device__ __forceinline__ void udown_dispatch(const UNode<T> &u, const T (&wp)[6], const T (&lroot)[6], T *lds,
                                               int lw, int lane, T *__restrict__ out, T *__restrict__ xch,
                                               const Ctx &C, int rr, bool act, int &bad) {
    const bool xi = u.xref < 0, yi = u.yref < 0;
    if (xi && yi) udown_node<T, RT, true, true>(u, wp, lroot, lds, lw, lane, out, xch, C, rr, act, bad);
    else if (xi) udown_node<T, RT, true, false>(u, wp, lroot, lds, lw, lane, out, xch, C, rr, act, bad);
    else if (yi) udown_node<T, RT, false, true>(u, wp, lroot, lds, lw, lane, out, xch, C, rr, act, bad);
    else udown_node<T, RT, false, false>(u, wp, lroot, lds, lw, lane, out, xch, C, rr, act, bad);
}

template <typename T, int RT>
__global__ void __launch_bounds__(64) k_down_u(int phase, const int32_t *__restrict__ prun,
                                               const int32_t *__restrict__ run, const T *__restrict__ rec,
                                               const T *__restrict__ w, T *__restrict__ out, T *__restrict__ xch,
                                               Ctx C, int lw, int32_t *err) {
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int lane = threadIdx.x;
    if (lane >= lw) return;
    const int R = rhs_count<RT>(C);
    const int items = prun[4 * phase + 3] * C.nchunks;
    int bad = 0;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        URun ru;
        urun(item, phase, prun, run, C, ru, bad);
        const int r = ru.chunk * 64 + lane;
        const bool act = r < R;
        const int rr = min(r, R - 1);
        // node n of the sweep is schedule index base + len - 1 - n
        const T *rp = rec + (int64_t)kRecWords * (ru.base + ru.len - 1);
        UNode<T> u;
        T A[6], B[6];
        if (ru.len > 0) {
            uload(u, rp);
            udown_fetch<T, RT>(u, A, B, w, xch, C, rr, bad);
        }
        for (int n = 0; n < ru.len; ++n) {
            UNode<T> un;
            T An[6], Bn[6];
            if (n + 1 < ru.len) {
                uload(un, rp - (int64_t)(n + 1) * kRecWords);
                udown_fetch<T, RT>(un, An, Bn, w, xch, C, rr, bad);
            }
            udown_dispatch<T, RT>(u, A, B, lds, lw, lane, out, xch, C, rr, act, bad);
            u = un;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                A[c] = An[c];
                B[c] = Bn[c];
            }
        }
    }
    if (bad) atomicOr(err, bad);
}

template <typename T, int LPT>
void launch_phase(const Plan &P, int phase, int transpose, const T *rec, const T *v, T *out, T *xch, const Ctx &C,
                  hipStream_t s) {
    const size_t lds = (size_t)C.dmax * 6 * 64 * sizeof(T);
    constexpr int TPW = 64 / LPT;
    const char *genv = getenv("HQ_APPLY_GRID");
    if constexpr (LPT >= 32) {
        const size_t lds_w = (size_t)(C.xslot + 1) * 6 * 64 * sizeof(T);
        // work items: pairs of runs (a phase has at most NI / run_nodes + 1
        // runs) x RHS chunks, one per wave, so the dispatcher balances the
        // load; waves of later phases with fewer runs exit at once
        const int64_t items = ((P.NI / P.run_nodes + 2 + TPW - 1) / TPW) * (int64_t)C.nchunks;
        int64_t g = items;
        if (genv) g = std::max<int64_t>(1, atoll(genv));
        const unsigned grid = (unsigned)std::min<int64_t>(g, 1 << 20);
#define HQ_WIDE(RT, PR, NR, PR1, NR1, NRD)                                                                   \
    do {                                                                                                     \
        if (!transpose) {                                                                                    \
            if (phase == 1)                                                                                  \
                hipLaunchKernelGGL((k_up_wide<T, LPT, RT, PR1, NR1, 3>), dim3(grid), dim3(64), lds_w, s, phase, \
                                   P.d_prun, P.d_run, rec, v, out, xch, C, P.d_err);                         \
            else                                                                                             \
                hipLaunchKernelGGL((k_up_wide<T, LPT, RT, PR, NR, 6>), dim3(grid), dim3(64), lds_w, s, phase, \
                                   P.d_prun, P.d_run, rec, v, out, xch, C, P.d_err);                         \
        } else {                                                                                             \
            hipLaunchKernelGGL((k_down_wide<T, LPT, RT, 6, NRD>), dim3(grid), dim3(64), lds_w, s, phase,      \
                               P.d_prun, P.d_run, rec, v, out, xch, C, P.d_err);                             \
        }                                                                                                    \
    } while (0)
        int variant = 0;
        if (const char *e = getenv("HQ_WIDE_VARIANT")) variant = atoi(e);
        if (variant == 9) {
            // one run per wave
            const int lw = (C.R <= 32) ? 32 : 64;
            const size_t lds_u = (size_t)(C.xslot + 1) * 6 * lw * sizeof(T);
            const int64_t items_u = (P.NI / P.run_nodes + 2) * (int64_t)C.nchunks;
            const int64_t per_cu_u = std::max<int64_t>(1, std::min<int64_t>(32, (int64_t)(160 * 1024) / (int64_t)lds_u));
            int64_t gu = std::min<int64_t>(items_u, 256 * per_cu_u);
            if (genv) gu = std::max<int64_t>(1, atoll(genv));
            const unsigned grid_u = (unsigned)std::min<int64_t>(gu, 1 << 20);
            if (!transpose)
                hipLaunchKernelGGL((k_up_u<T, 0>), dim3(grid_u), dim3(64), lds_u, s, phase, P.d_prun, P.d_run,
                                   rec, v, out, xch, C, lw, P.d_err);
            else
                hipLaunchKernelGGL((k_down_u<T, 0>), dim3(grid_u), dim3(64), lds_u, s, phase, P.d_prun, P.d_run,
                                   rec, v, out, xch, C, lw, P.d_err);
            return;
        }
        if (LPT == 32 && C.R == 32) {
            switch (variant) {
            case 1: HQ_WIDE(32, 6, 2, 6, 3, 2); break;
            case 2: HQ_WIDE(32, 6, 2, 6, 6, 3); break;
            case 3: HQ_WIDE(32, 6, 2, 4, 4, 3); break;
            default: HQ_WIDE(32, 6, 2, 6, 3, 3); break;
            }
        } else {
            HQ_WIDE(0, 6, 2, 6, 3, 3);
        }
#undef HQ_WIDE
        return;
    }
    // one wave per work item of the largest phase (tile groups x RHS chunks);
    // waves without work exit at once
    int64_t items = ((2 * P.tiles_built + 64 + TPW - 1) / TPW) * (int64_t)C.nchunks;
    if (genv) items = std::max<int64_t>(1, atoll(genv));
    const unsigned grid = (unsigned)std::min<int64_t>(items, 1 << 20);
    if (!transpose)
        hipLaunchKernelGGL((k_up<T, LPT>), dim3(grid), dim3(64), lds, s, phase, P.d_phase, P.d_tile_base,
                           P.d_tile_len, P.d_links, rec, v, out, xch, C, P.d_err);
    else
        hipLaunchKernelGGL((k_down<T, LPT>), dim3(grid), dim3(64), lds, s, phase, P.d_phase, P.d_tile_base,
                           P.d_tile_len, P.d_links, rec, v, out, xch, C, P.d_err);
}

template <typename T>
void launch_all(const Plan &P, int transpose, int lpt, const T *rec, const T *v, T *out, T *xch, const Ctx &C,
                hipStream_t s) {
    const int nph = std::max(P.phases_built, P.phases_reserved);
    for (int k = 0; k < nph; ++k) {
        const int phase = transpose ? (nph - k) : (k + 1);
        switch (lpt) {
        case 1: launch_phase<T, 1>(P, phase, transpose, rec, v, out, xch, C, s); break;
        case 2: launch_phase<T, 2>(P, phase, transpose, rec, v, out, xch, C, s); break;
        case 4: launch_phase<T, 4>(P, phase, transpose, rec, v, out, xch, C, s); break;
        case 8: launch_phase<T, 8>(P, phase, transpose, rec, v, out, xch, C, s); break;
        case 16: launch_phase<T, 16>(P, phase, transpose, rec, v, out, xch, C, s); break;
        case 32: launch_phase<T, 32>(P, phase, transpose, rec, v, out, xch, C, s); break;
        default: launch_phase<T, 64>(P, phase, transpose, rec, v, out, xch, C, s); break;
        }
    }
}

}  // namespace

int lanes_per_tile(int64_t nrhs) {
    int l = 1;
    while (l < nrhs && l < 64) l <<= 1;
    return l;
}

hq_status apply_device(Plan &P, const void *v, void *out, int transpose, int64_t nrhs, int prec, hipStream_t s) {
    Ctx C;
    C.N = P.N;
    C.rows = P.rows;
    C.nsched = P.NI;
    C.R = (int)nrhs;
    int lpt = lanes_per_tile(nrhs);
    if (const char *e = getenv("HQ_LPT")) {
        const int v = atoi(e);
        if (v == 1 || v == 2 || v == 4 || v == 8 || v == 16 || v == 32 || v == 64) lpt = v;
    }
    C.nchunks = (int)((nrhs + lpt - 1) / lpt);
    C.dmax = stack_depth(P.S);
    C.xslot = scratch_slot(P.S);
    const size_t elem = (prec == HQ_FP64) ? sizeof(double) : sizeof(float);
    C.xch_cap = (int)std::min<int64_t>(INT32_MAX, (int64_t)(P.xch_bytes / (6 * elem * (size_t)nrhs)));
    if (prec == HQ_FP64)
        launch_all<double>(P, transpose, lpt, P.d_rec64, (const double *)v, (double *)out, (double *)P.d_xch, C, s);
    else
        launch_all<float>(P, transpose, lpt, P.d_rec32, (const float *)v, (float *)out, (float *)P.d_xch, C, s);
    HQ_HIP(hipGetLastError());
    return HQ_OK;
}

}  // namespace hq
