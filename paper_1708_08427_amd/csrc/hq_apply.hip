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

// Info-set of a child that is a bead or an earlier tile's root.
template <typename T>
__device__ __forceinline__ void load_child(int ref, T (&m)[6], const T *__restrict__ v, const T *__restrict__ xch,
                                           const Ctx &C, int r, bool act, int32_t *err) {
#pragma unroll
    for (int c = 0; c < 6; ++c) m[c] = T(0);
    if (ref >= 0) {
        if (ref >= C.N) {
            atomicOr(err, kFlagBounds);
            return;
        }
        if (act) {
#pragma unroll
            for (int c = 0; c < 3; ++c) m[c] = v[((int64_t)3 * ref + c) * C.R + r];
        }
    } else {
        const int slot = ref_slot(ref);
        if (slot < 0 || slot >= C.xch_cap) {
            atomicOr(err, kFlagBounds);
            return;
        }
        if (act) {
#pragma unroll
            for (int c = 0; c < 6; ++c) m[c] = xch[((int64_t)slot * 6 + c) * C.R + r];
        }
    }
}

template <typename T, int LPT>
__global__ void __launch_bounds__(64) k_up(int phase, const int32_t *__restrict__ phase_tab,
                                           const int32_t *__restrict__ tile_base, const int32_t *__restrict__ tile_len,
                                           const T *__restrict__ rec, const T *__restrict__ v, T *__restrict__ out,
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
        int sp = 0;
        for (int i = 0; i < len; ++i) {
            const int s = base + i;
            const T *g = rec + (int64_t)kRecWords * s;
            const int32_t *lk = reinterpret_cast<const int32_t *>(g + kRecLinks);
            const int xref = lk[0], yref = lk[1], off = lk[2], meta = lk[3];
            T mx[6], my[6];
            const bool xs = xref == kRefStack, ys = yref == kRefStack;
            if (xs && ys) {
                if (meta & kMetaYFirst) {
                    pop6(stk, sp, mx, lane, err);
                    pop6(stk, sp, my, lane, err);
                } else {
                    pop6(stk, sp, my, lane, err);
                    pop6(stk, sp, mx, lane, err);
                }
            } else {
                if (xs) pop6(stk, sp, mx, lane, err);
                else load_child(xref, mx, v, xch, C, r, act, err);
                if (ys) pop6(stk, sp, my, lane, err);
                else load_child(yref, my, v, xch, C, r, act, err);
            }
            const T sx = g[kRecSx], sy = g[kRecSy];
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
                house_fwd<9>(t9, g);
                dim = 6;
            } else if (xi || yi) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    t9[c] = xi ? mx[3 + c] : my[3 + c];
                    t9[3 + c] = sy * mx[c] - sx * my[c];
                }
                house_fwd<6>(t9, g);
                dim = 3;
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) t9[c] = sy * mx[c] - sx * my[c];
                house_fwd<3>(t9, g);
                dim = 0;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) mp[3 + c] = t9[c];
            if (dim > 0) {
                if (off < 0 || (int64_t)off + dim > C.rows) {
                    atomicOr(err, kFlagBounds);
                } else if (act) {
                    for (int q = 0; q < dim; ++q) out[((int64_t)off + q) * C.R + r] = t9[3 + q];
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
            for (int c = 0; c < 3; ++c) out[((int64_t)3 * ref + c) * C.R + r] = L[c];
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

template <typename T, int LPT>
__global__ void __launch_bounds__(64) k_down(int phase, const int32_t *__restrict__ phase_tab,
                                             const int32_t *__restrict__ tile_base,
                                             const int32_t *__restrict__ tile_len, const T *__restrict__ rec,
                                             const T *__restrict__ w, T *__restrict__ out, T *__restrict__ xch, Ctx C,
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
        for (int i = len - 1; i >= 0; --i) {
            const int s = base + i;
            const T *g = rec + (int64_t)kRecWords * s;
            const int32_t *lk = reinterpret_cast<const int32_t *>(g + kRecLinks);
            const int xref = lk[0], yref = lk[1], off = lk[2], meta = lk[3];
            T L[6];
            if (meta & kMetaBodyRoot) {
#pragma unroll
                for (int c = 0; c < 6; ++c) L[c] = T(0);
            } else if (meta & kMetaTileRoot) {
                const int slot = meta >> kMetaSlotShift;
#pragma unroll
                for (int c = 0; c < 6; ++c) L[c] = T(0);
                if (slot >= C.xch_cap) {
                    atomicOr(err, kFlagBounds);
                } else if (act) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) L[c] = xch[((int64_t)slot * 6 + c) * C.R + r];
                }
            } else {
                pop6(stk, sp, L, lane, err);
            }
            const T sx = g[kRecSx], sy = g[kRecSy];
            const bool xi = xref < 0, yi = yref < 0;
            const int dim = 3 * (int)xi + 3 * (int)yi;
            T x9[9];
#pragma unroll
            for (int c = 0; c < 3; ++c) x9[c] = L[3 + c];
#pragma unroll
            for (int c = 3; c < 9; ++c) x9[c] = T(0);
            if (dim > 0) {
                if (off < 0 || (int64_t)off + dim > C.rows) {
                    atomicOr(err, kFlagBounds);
                } else if (act) {
                    if (dim == 6) {
#pragma unroll
                        for (int q = 0; q < 6; ++q) x9[3 + q] = w[((int64_t)off + q) * C.R + r];
                    } else {
#pragma unroll
                        for (int q = 0; q < 3; ++q) x9[3 + q] = w[((int64_t)off + q) * C.R + r];
                    }
                }
            }
            T st[3], Lx[6], Ly[6];
            if (xi && yi) {
                house_bwd<9>(x9, g);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Lx[3 + c] = x9[c];
                    Ly[3 + c] = x9[3 + c];
                    st[c] = x9[6 + c];
                }
            } else if (xi || yi) {
                house_bwd<6>(x9, g);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Lx[3 + c] = xi ? x9[c] : T(0);
                    Ly[3 + c] = yi ? x9[c] : T(0);
                    st[c] = x9[3 + c];
                }
            } else {
                house_bwd<3>(x9, g);
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
    }
}

template <typename T, int LPT>
void launch_phase(const Plan &P, int phase, int transpose, const T *rec, const T *v, T *out, T *xch, const Ctx &C,
                  hipStream_t s) {
    const size_t lds = (size_t)C.dmax * 6 * 64 * sizeof(T);
    const unsigned grid = 2048;
    if (!transpose)
        hipLaunchKernelGGL((k_up<T, LPT>), dim3(grid), dim3(64), lds, s, phase, P.d_phase, P.d_tile_base,
                           P.d_tile_len, rec, v, out, xch, C, P.d_err);
    else
        hipLaunchKernelGGL((k_down<T, LPT>), dim3(grid), dim3(64), lds, s, phase, P.d_phase, P.d_tile_base,
                           P.d_tile_len, rec, v, out, xch, C, P.d_err);
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
    const int lpt = lanes_per_tile(nrhs);
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
