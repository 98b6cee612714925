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
    return reinterpret_cast<const int4 *>(links)[s];
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
// Wide tiles (32 or 64 lanes per tile).  A node record is 32 elements; lane q
// of each 32-lane half holds element q, so one coalesced load fetches a whole
// record for the tile, and ds_swizzle broadcasts element w inside the half
// when the node is processed.  A software pipeline keeps the records of nodes
// n+1..n+6 and the memory inputs of nodes n+1..n+2 in flight while node n is
// computed.
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

__device__ __forceinline__ int4 bcast_links(float v) {
    return make_int4(__float_as_int(bcast<26>(v)), __float_as_int(bcast<27>(v)), __float_as_int(bcast<28>(v)),
                     __float_as_int(bcast<29>(v)));
}

__device__ __forceinline__ int4 bcast_links(double v) {
    const long long a = __double_as_longlong(bcast<26>(v)), b = __double_as_longlong(bcast<27>(v));
    return make_int4((int)(a & 0xffffffffll), (int)(a >> 32), (int)(b & 0xffffffffll), (int)(b >> 32));
}


template <typename T>
__device__ __forceinline__ void child_up(int ref, T (&m)[6], const T *__restrict__ v, const T *__restrict__ xch,
                                         const Ctx &C, int r, bool act, int32_t *err) {
#pragma unroll
    for (int c = 0; c < 6; ++c) m[c] = T(0);
    fetch_child(ref, m, v, xch, C, r, act, err);
}

template <typename T, int LPT, int PR, int WPE>
__global__ void __launch_bounds__(64, WPE) k_up_wide(int phase, const int32_t *__restrict__ phase_tab,
                                                const int32_t *__restrict__ tile_base,
                                                const int32_t *__restrict__ tile_len, const T *__restrict__ rec,
                                                const T *__restrict__ v, T *__restrict__ out, T *__restrict__ xch,
                                                Ctx C, int32_t *err) {
    static_assert(LPT == 32 || LPT == 64, "wide tiles use 32 or 64 lanes");
    extern __shared__ unsigned char smem_raw[];
    T *stk = reinterpret_cast<T *>(smem_raw);
    constexpr int TPW = 64 / LPT;
    const int lane = threadIdx.x;
    const int q = lane & 31;
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
        int maxlen = len;
        if (LPT == 32) maxlen = max(maxlen, __shfl_xor(len, 32, 64));
        const T *rp = rec + (int64_t)kRecWords * base + q;
        int sp = 0;
        // records of nodes n..n+5 in RW[n % 6], memory inputs of nodes n..n+2 in A/B[n % 3]
        T RW[PR];
        T A[3][6], B[3][6];
#pragma unroll
        for (int k = 0; k < PR; ++k)
            if (k < len) RW[k] = rp[(int64_t)k * kRecWords];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (k < len) {
                const int4 lk = bcast_links(RW[k]);
                child_up(lk.x, A[k], v, xch, C, r, act, err);
                child_up(lk.y, B[k], v, xch, C, r, act, err);
            }
        }
#define HQ_UP_STEP(K)                                                                  \
        {                                                                              \
            const int n = n0 + (K);                                                    \
            if (n < len) {                                                             \
                NodeIn<T> in;                                                          \
                bcast_g<0>(in.g, RW[K]);                                               \
                in.lk = bcast_links(RW[K]);                                            \
                if (n + PR < len) RW[K] = rp[(int64_t)(n + PR) * kRecWords];             \
                if (n + 2 < len) {                                                     \
                    const int4 l2 = bcast_links(RW[((K) + 2) % PR]);                    \
                    child_up(l2.x, A[((K) + 2) % 3], v, xch, C, r, act, err);          \
                    child_up(l2.y, B[((K) + 2) % 3], v, xch, C, r, act, err);          \
                }                                                                      \
                _Pragma("unroll") for (int c = 0; c < 6; ++c) {                        \
                    in.a[c] = A[(K) % 3][c];                                           \
                    in.b[c] = B[(K) % 3][c];                                           \
                }                                                                      \
                node_up(in, stk, sp, out, xch, C, r, act, lane, err);                  \
            }                                                                          \
        }
        for (int n0 = 0; n0 < maxlen; n0 += PR) {
            HQ_UP_STEP(0)
            HQ_UP_STEP(1)
            HQ_UP_STEP(2)
            if constexpr (PR == 6) {
                HQ_UP_STEP(3)
                HQ_UP_STEP(4)
                HQ_UP_STEP(5)
            }
        }
#undef HQ_UP_STEP
    }
}

template <typename T>
__device__ __forceinline__ void inputs_down(const int4 lk, T (&a)[6], T (&b)[6], const T *__restrict__ w,
                                            const T *__restrict__ xch, const Ctx &C, int r, bool act, int32_t *err) {
    const int xref = lk.x, yref = lk.y, off = lk.z, meta = lk.w;
    const int dim = 3 * (int)(xref < 0) + 3 * (int)(yref < 0);
#pragma unroll
    for (int c = 0; c < 6; ++c) a[c] = b[c] = T(0);
    if (dim > 0) {
        if (off < 0 || (int64_t)off + dim > C.rows) {
            atomicOr(err, kFlagBounds);
        } else if (act) {
            const T *src = w + (int64_t)off * C.R + r;
            a[0] = src[0];
            a[1] = src[C.R];
            a[2] = src[2 * C.R];
            if (dim == 6) {
                a[3] = src[3 * C.R];
                a[4] = src[4 * C.R];
                a[5] = src[5 * C.R];
            }
        }
    }
    if ((meta & kMetaTileRoot) && !(meta & kMetaBodyRoot)) {
        const int slot = meta >> kMetaSlotShift;
        if (slot >= C.xch_cap) {
            atomicOr(err, kFlagBounds);
        } else if (act) {
#pragma unroll
            for (int c = 0; c < 6; ++c) b[c] = xch[((int64_t)slot * 6 + c) * C.R + r];
        }
    }
}

template <typename T, int LPT, int PR, int WPE>
__global__ void __launch_bounds__(64, WPE) k_down_wide(int phase, const int32_t *__restrict__ phase_tab,
                                                  const int32_t *__restrict__ tile_base,
                                                  const int32_t *__restrict__ tile_len, const T *__restrict__ rec,
                                                  const T *__restrict__ w, T *__restrict__ out, T *__restrict__ xch,
                                                  Ctx C, int32_t *err) {
    static_assert(LPT == 32 || LPT == 64, "wide tiles use 32 or 64 lanes");
    extern __shared__ unsigned char smem_raw[];
    T *stk = reinterpret_cast<T *>(smem_raw);
    constexpr int TPW = 64 / LPT;
    const int lane = threadIdx.x;
    const int q = lane & 31;
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
        int maxlen = len;
        if (LPT == 32) maxlen = max(maxlen, __shfl_xor(len, 32, 64));
        // node n of the sweep is schedule index base + len - 1 - n
        const T *rp = rec + (int64_t)kRecWords * (base + len - 1) + q;
        int sp = 0;
        T RW[PR];
        T A[3][6], B[3][6];
#pragma unroll
        for (int k = 0; k < PR; ++k)
            if (k < len) RW[k] = rp[-(int64_t)k * kRecWords];
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (k < len) inputs_down(bcast_links(RW[k]), A[k], B[k], w, xch, C, r, act, err);
#define HQ_DOWN_STEP(K)                                                                \
        {                                                                              \
            const int n = n0 + (K);                                                    \
            if (n < len) {                                                             \
                NodeIn<T> in;                                                          \
                bcast_g<0>(in.g, RW[K]);                                               \
                in.lk = bcast_links(RW[K]);                                            \
                if (n + PR < len) RW[K] = rp[-(int64_t)(n + PR) * kRecWords];            \
                if (n + 2 < len)                                                       \
                    inputs_down(bcast_links(RW[((K) + 2) % PR]), A[((K) + 2) % 3], B[((K) + 2) % 3], w, xch, C, r, \
                                act, err);                                             \
                _Pragma("unroll") for (int c = 0; c < 6; ++c) {                        \
                    in.a[c] = A[(K) % 3][c];                                           \
                    in.b[c] = B[(K) % 3][c];                                           \
                }                                                                      \
                node_down(in, stk, sp, out, xch, C, r, act, lane, err);                \
            }                                                                          \
        }
        for (int n0 = 0; n0 < maxlen; n0 += PR) {
            HQ_DOWN_STEP(0)
            HQ_DOWN_STEP(1)
            HQ_DOWN_STEP(2)
            if constexpr (PR == 6) {
                HQ_DOWN_STEP(3)
                HQ_DOWN_STEP(4)
                HQ_DOWN_STEP(5)
            }
        }
#undef HQ_DOWN_STEP
    }
}

template <typename T, int LPT>
void launch_phase(const Plan &P, int phase, int transpose, const T *rec, const T *v, T *out, T *xch, const Ctx &C,
                  hipStream_t s) {
    const size_t lds = (size_t)C.dmax * 6 * 64 * sizeof(T);
    // one wave per work item of the largest phase (tile groups x RHS chunks);
    // waves without work exit at once
    constexpr int TPW = 64 / LPT;
    int64_t items = ((2 * P.tiles_built + 64 + TPW - 1) / TPW) * (int64_t)C.nchunks;
    if (const char *e = getenv("HQ_APPLY_GRID")) items = std::max<int64_t>(1, atoll(e));
    const unsigned grid = (unsigned)std::min<int64_t>(items, 1 << 20);
    if constexpr (LPT >= 32) {
        {
#define HQ_WIDE_LAUNCH(PRV, WPEV)                                                                          \
            {                                                                                              \
                if (!transpose)                                                                            \
                    hipLaunchKernelGGL((k_up_wide<T, LPT, PRV, WPEV>), dim3(grid), dim3(64), lds, s, phase, \
                                       P.d_phase, P.d_tile_base, P.d_tile_len, rec, v, out, xch, C, P.d_err); \
                else                                                                                       \
                    hipLaunchKernelGGL((k_down_wide<T, LPT, PRV, WPEV>), dim3(grid), dim3(64), lds, s,      \
                                       phase, P.d_phase, P.d_tile_base, P.d_tile_len, rec, v, out, xch, C,  \
                                       P.d_err);                                                           \
            }
            // records six nodes ahead, register budget for four waves per SIMD
            // (measured best on gfx950 for 32 right-hand sides)
            HQ_WIDE_LAUNCH(6, 4)
#undef HQ_WIDE_LAUNCH
            return;
        }
    }
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
