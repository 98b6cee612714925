// Explicit Q~ (Algorithm 1) in O(n log n): the entries of a body's Q~ in the
// rows of node q and the columns of bead k are the derivatives of bead k's
// velocity with respect to q's residue coefficients in the downward sweep
// (Theorem 4.3).  One thread per bead walks from its leaf up to the body
// root carrying the 3 x 6 derivative of the bead velocity with respect to the
// current node's Velocity-set; at each ancestor one application of G per
// velocity component gives both the next derivative and the block entries:
//
//   child c of q with weights (alpha, beta) = (sx, sy) for x, (sy, -sx) for y:
//   m = beta * D(:,1:3) on s_t's slots, D(:,4:6) on c's slots (c internal)
//   u = G m;  Q~[off_q + i, bead k] = u(3 + i);  D <- [alpha D(:,1:3), u(1:3)]
//
// It is the U / Residue-vector recursion of Eqs. 3.6-3.8 read column by
// column; every node's block covers exactly its own beads.
#include "hq_common.h"

namespace hq {

namespace {

template <int K>
__device__ __forceinline__ void gather_fwd(double (&m)[9], const double *g) {
    house_fwd<K>(m, g);
}

// mode 0: dense output (row-major, leading dimension ld, caller's columns)
// mode 1: block output at blk_off[local node] (row-major dim x 3 n_q blocks,
//         columns in tree order), FP64 (prec 0) or FP32 (prec 1)
__global__ void __launch_bounds__(256) k_explicit(int body, int mode, int prec, const int32_t *bead_off,
                                                  const int32_t *node_off, const int32_t *row_off,
                                                  const int32_t *perm, const int32_t *leafpar, const int32_t *lc,
                                                  const int32_t *rc, const int32_t *par, const int32_t *first,
                                                  const int32_t *nn, const int32_t *sched, const double *rec64,
                                                  const int64_t *blk_off, double *dense, int64_t ld, void *values,
                                                  int32_t *err) {
    const int base = bead_off[body], n = bead_off[body + 1] - base;
    const int nbase = node_off[body];
    const int rbase = row_off[body];
    for (int p = base + blockIdx.x * blockDim.x + threadIdx.x; p < base + n; p += gridDim.x * blockDim.x) {
        const int u = perm[p] - base;  // caller's bead index within the body
        if (u < 0 || u >= n) {
            atomicOr(err, kFlagBounds);
            continue;
        }
        double D[3][6];
        for (int o = 0; o < 3; ++o)
            for (int c = 0; c < 6; ++c) D[o][c] = (o == c) ? 1.0 : 0.0;
        int child = -p - 1;
        int q = leafpar[p];
        for (int guard = 0; guard < 256 && q >= 0; ++guard) {
            const double *g = rec64 + (int64_t)kRecWords * sched[q];
            const int32_t *lk = reinterpret_cast<const int32_t *>(g + kRecLinks);
            const int off = lk[2] - rbase;
            const int x = lc[q], y = rc[q];
            const bool isx = (child == x);
            const bool xi = x >= 0, yi = y >= 0;
            const int dim = 3 * (int)xi + 3 * (int)yi;
            if (off < 0 || off + dim > 3 * n - 6) {
                atomicOr(err, kFlagBounds);
                break;
            }
            const double sx = g[kRecSx], sy = g[kRecSy];
            const double alpha = isx ? sx : sy, beta = isx ? sy : -sx;
            const bool ci = isx ? xi : yi;
            const int tpos = dim;                       // s_t follows the children's slots
            const int cpos = isx ? 0 : (xi ? 3 : 0);    // slot of this child's 3-vector
            for (int o = 0; o < 3; ++o) {
                double m[9];
                for (int i = 0; i < 9; ++i) m[i] = 0.0;
                for (int c = 0; c < 3; ++c) m[tpos + c] = beta * D[o][c];
                if (ci)
                    for (int c = 0; c < 3; ++c) m[cpos + c] = D[o][3 + c];
                if (dim == 6) gather_fwd<9>(m, g);
                else if (dim == 3) gather_fwd<6>(m, g);
                else gather_fwd<3>(m, g);
                for (int i = 0; i < dim; ++i) {
                    const double val = m[3 + i];
                    if (mode == 0) {
                        dense[(int64_t)(off + i) * ld + 3 * u + o] = val;
                    } else {
                        const int64_t bo = blk_off[q - nbase];
                        if (bo < 0) {
                            atomicOr(err, kFlagBounds);
                            continue;
                        }
                        const int64_t idx = bo + (int64_t)i * 3 * nn[q] + 3 * (int64_t)(p - first[q]) + o;
                        if (prec == 0) reinterpret_cast<double *>(values)[idx] = val;
                        else reinterpret_cast<float *>(values)[idx] = (float)val;
                    }
                }
                for (int c = 0; c < 3; ++c) {
                    D[o][c] *= alpha;
                    D[o][3 + c] = m[c];
                }
            }
            child = q;
            q = par[q];
        }
    }
}

__global__ void k_zero2d(double *out, int64_t rows, int64_t cols, int64_t ld) {
    const int64_t total = rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        out[(i / cols) * ld + (i % cols)] = 0.0;
}

}  // namespace

hq_status explicit_dense(Plan &P, int64_t body, double *out, int64_t ld, hipStream_t s) {
    const int64_t n = P.offsets[body + 1] - P.offsets[body];
    const int64_t rows = 3 * n - 6;
    if (rows > 0) {
        const int64_t tot = rows * 3 * n;
        const unsigned grid = (unsigned)std::min<int64_t>(65535, (tot + 255) / 256);
        hipLaunchKernelGGL(k_zero2d, dim3(grid), dim3(256), 0, s, out, rows, 3 * n, ld);
        const unsigned g2 = (unsigned)std::min<int64_t>(65535, (n + 255) / 256);
        hipLaunchKernelGGL(k_explicit, dim3(g2), dim3(256), 0, s, (int)body, 0, 0, P.d_bead_off, P.d_node_off,
                           P.d_row_off, P.d_perm, P.d_leafpar, P.d_lc, P.d_rc, P.d_par, P.d_first, P.d_nn,
                           P.d_sched, P.d_rec64, (const int64_t *)nullptr, out, ld, (void *)nullptr, P.d_err);
    }
    HQ_HIP(hipGetLastError());
    return HQ_OK;
}

hq_status explicit_blocks_launch(Plan &P, int64_t body, int prec, void *values, const int64_t *d_blk_off,
                                 hipStream_t s) {
    const int64_t n = P.offsets[body + 1] - P.offsets[body];
    const unsigned g2 = (unsigned)std::min<int64_t>(65535, (n + 255) / 256);
    hipLaunchKernelGGL(k_explicit, dim3(g2), dim3(256), 0, s, (int)body, 1, prec, P.d_bead_off, P.d_node_off,
                       P.d_row_off, P.d_perm, P.d_leafpar, P.d_lc, P.d_rc, P.d_par, P.d_first, P.d_nn, P.d_sched,
                       P.d_rec64, d_blk_off, (double *)nullptr, (int64_t)0, values, P.d_err);
    HQ_HIP(hipGetLastError());
    return HQ_OK;
}

}  // namespace hq
