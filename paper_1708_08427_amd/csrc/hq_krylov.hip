// Krylov harness for the constrained Brownian-dynamics system of Section 1:
// the constraint forces g solve 0 = Q~ D Q_Z^T F + Q~ D Q~^T g (Eq. 1.5), and
// the rigid-body velocities are V = Q_Z D (Q_Z^T F + Q~^T g) (Eq. 1.6).  D is
// the caller's mobility product (a callback); Q~ and Q_Z are applied with the
// sweeps of hq_apply_full.  Conjugate gradients on A = Q~ D Q~^T, which is
// symmetric positive definite when D is; one CG per right-hand side, run
// together, with FP64 scalars.
#include <algorithm>
#include <cmath>
#include <vector>

#include "hq_common.h"

namespace hq {
namespace {

constexpr int kKThreads = 256;

// Column (right-hand side) of element e of a vector with R columns: rows
// layout element (i, r) at i R + r; triples layout at ((i / 3) R + r) 3 + i % 3.
__device__ __forceinline__ int col_of(int64_t e, int R, int tri) {
    return (int)(tri ? (e / 3) % R : e % R);
}

// Per-column sums of a thread's partial results: the grid stride S is a
// multiple of the column period (R or 3R), so every thread stays in one
// column; a block adds its threads' partials per column in LDS (up to
// kLdsCols columns), then one atomic add per block and column.
constexpr int kLdsCols = 1024;

__device__ __forceinline__ void col_reduce(double acc, int col, int R, double *sh, double *out) {
    if (R <= kLdsCols) {
        for (int c = threadIdx.x; c < R; c += blockDim.x) sh[c] = 0.0;
        __syncthreads();
        if (acc != 0.0) atomicAdd(&sh[col], acc);
        __syncthreads();
        for (int c = threadIdx.x; c < R; c += blockDim.x)
            if (sh[c] != 0.0) atomicAdd(&out[c], sh[c]);
    } else if (acc != 0.0) {
        atomicAdd(&out[col], acc);
    }
}

// out[col] = sum_e a[e] b[e] (FP64)
template <typename T>
__global__ void __launch_bounds__(kKThreads) k_dot_cols(int64_t n, int R, int tri, int64_t S, const T *__restrict__ a,
                                                        const T *__restrict__ b, double *out) {
    __shared__ double sh[kLdsCols];
    const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (e0 < S)
        for (int64_t e = e0; e < n; e += S) acc += (double)a[e] * (double)b[e];
    col_reduce(acc, e0 < S ? col_of(e0, R, tri) : 0, R, sh, out);
}

// x += alpha p; r -= alpha Ap (per column alpha), and out[col] = ||r||^2
template <typename T>
__global__ void __launch_bounds__(kKThreads) k_cg_xr(int64_t n, int R, int tri, int64_t S,
                                                     const double *__restrict__ alpha, const T *__restrict__ p,
                                                     const T *__restrict__ Ap, T *x, T *r, double *out) {
    __shared__ double sh[kLdsCols];
    const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (e0 < S) {
        const double a = alpha[col_of(e0, R, tri)];
        for (int64_t e = e0; e < n; e += S) {
            x[e] = (T)((double)x[e] + a * (double)p[e]);
            const T rn = (T)((double)r[e] - a * (double)Ap[e]);
            r[e] = rn;
            acc += (double)rn * (double)rn;
        }
    }
    col_reduce(acc, e0 < S ? col_of(e0, R, tri) : 0, R, sh, out);
}

// p = r + beta p (per column beta)
template <typename T>
__global__ void k_cg_p(int64_t n, int R, int tri, const double *__restrict__ beta, const T *__restrict__ r, T *p) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = (T)((double)r[e] + beta[col_of(e, R, tri)] * (double)p[e]);
}

// y = -x
template <typename T>
__global__ void k_neg(int64_t n, const T *__restrict__ x, T *y) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = -x[e];
}

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kKThreads - 1) / kKThreads, 8192)); }

// Work vectors: carved from a piece of the handle's workspace (hq_build_into
// with krylov_nrhs), else allocated for the call and freed at its end.
struct Work {
    std::vector<void *> bufs;
    char *base = nullptr;
    size_t used = 0, cap = 0;
    ~Work() {
        for (void *p : bufs)
            if (p) (void)hipFree(p);
    }
    void *get(size_t bytes) {
        bytes = (std::max<size_t>(bytes, 16) + 255) / 256 * 256;
        if (base) {
            if (used + bytes > cap) return nullptr;
            void *p = base + used;
            used += bytes;
            return p;
        }
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        bufs.push_back(p);
        return p;
    }
};

template <typename T>
hq_status solve(hq_handle h, hq_dapply_fn dapply, void *user, const void *F, void *V, void *g, int64_t nrhs,
                hq_precision prec, hq_layout layout, void *dx, void *dy, hq_krylov_info *info, hq_stream stream) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hq_info q;
    HQ_TRY(hq_query(h, &q));
    const int R = (int)nrhs;
    const int tri = layout == HQ_TRIPLES ? 1 : 0;
    const int64_t nr = q.rows * nrhs;
    const int max_iter = info->max_iter > 0 ? info->max_iter : 500;
    const double rtol = info->rtol > 0 ? info->rtol : 1e-8;
    Work w;
    Plan *P = plan_of(h);
    if (!P) return HQ_E_INVALID;
    if (P->ws) {
        if (!P->d_kry || P->kry_bytes < krylov_bytes(q.rows, nrhs, sizeof(T))) {
            set_error("the handle's workspace holds no Krylov vectors for nrhs right-hand sides "
                      "(hq_options.krylov_nrhs)");
            return HQ_E_UNSUPPORTED;
        }
        w.base = (char *)P->d_kry;
        w.cap = P->kry_bytes;
    }
    T *r = (T *)w.get(nr * sizeof(T)), *p = (T *)w.get(nr * sizeof(T)), *Ap = (T *)w.get(nr * sizeof(T));
    T *zr = (T *)w.get(nr * sizeof(T));
    double *dots = (double *)w.get(2 * (size_t)R * sizeof(double)), *coef = (double *)w.get((size_t)R * sizeof(double));
    if (!r || !p || !Ap || !zr || !dots || !coef) {
        set_error("hipMalloc of the Krylov workspace");
        return HQ_E_NOMEM;
    }
    T *x = (T *)g, *u = (T *)dx, *y = (T *)dy;
    // column-fixed grid: stride S a multiple of the column period, about
    // 1024 blocks
    const int64_t per = tri ? 3 * (int64_t)R : (int64_t)R;
    const int64_t S = std::max<int64_t>(per, ((int64_t)1024 * kKThreads / per) * per);
    const unsigned gd = (unsigned)((S + kKThreads - 1) / kKThreads);
    auto dot = [&](const T *a, const T *b, double *out) -> hq_status {
        HQ_HIP(hipMemsetAsync(out, 0, (size_t)R * sizeof(double), s));
        hipLaunchKernelGGL(k_dot_cols<T>, dim3(gd), dim3(kKThreads), 0, s, nr, R, tri, S, a, b, out);
        HQ_HIP(hipGetLastError());
        return HQ_OK;
    };
    auto dprod = [&]() -> hq_status {  // y = D u
        if (dapply(u, y, nrhs, user, stream) != 0) {
            set_error("the mobility callback failed");
            return HQ_E_INVALID;
        }
        return HQ_OK;
    };
    // A p = Q~ D Q~^T p
    auto apply_A = [&](const T *in, T *out) -> hq_status {
        HQ_TRY(hq_apply_layout(h, in, u, 1, nrhs, prec, layout, stream));
        HQ_TRY(dprod());
        return hq_apply_layout(h, y, out, 0, nrhs, prec, layout, stream);
    };
    // b = -Q~ D Q_Z^T F  (Q_Z^T F: the full-Q downward sweep with zero residues)
    HQ_HIP(hipMemsetAsync(zr, 0, nr * sizeof(T), s));
    HQ_TRY(hq_apply_full(h, zr, u, const_cast<void *>(F), 1, nrhs, prec, layout, stream));
    HQ_TRY(dprod());
    HQ_TRY(hq_apply_layout(h, y, Ap, 0, nrhs, prec, layout, stream));
    hipLaunchKernelGGL(k_neg<T>, dim3(grid_of(nr)), dim3(kKThreads), 0, s, nr, Ap, r);
    HQ_HIP(hipMemsetAsync(x, 0, nr * sizeof(T), s));
    HQ_HIP(hipMemcpyAsync(p, r, nr * sizeof(T), hipMemcpyDeviceToDevice, s));
    std::vector<double> rr(R), bb(R), pap(R), c(R);
    HQ_TRY(dot(r, r, dots));
    HQ_HIP(hipMemcpyAsync(bb.data(), dots, R * sizeof(double), hipMemcpyDeviceToHost, s));
    HQ_HIP(hipStreamSynchronize(s));
    rr = bb;
    std::vector<char> active(R);
    auto converged = [&](int k) { return !(rr[k] > rtol * rtol * bb[k]); };
    int it = 0;
    for (int k = 0; k < R; ++k) active[k] = !converged(k);
    while (it < max_iter && std::any_of(active.begin(), active.end(), [](char a) { return a != 0; })) {
        HQ_TRY(apply_A(p, Ap));
        HQ_TRY(dot(p, Ap, dots));
        HQ_HIP(hipMemcpyAsync(pap.data(), dots, R * sizeof(double), hipMemcpyDeviceToHost, s));
        HQ_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < R; ++k) {
            if (active[k] && !(pap[k] > 0.0)) {
                set_error("Q~ D Q~^T is not positive definite (p^T A p <= 0): D must be symmetric positive definite");
                return HQ_E_INVALID;
            }
            c[k] = active[k] ? rr[k] / pap[k] : 0.0;
        }
        HQ_HIP(hipMemcpyAsync(coef, c.data(), R * sizeof(double), hipMemcpyHostToDevice, s));
        HQ_HIP(hipMemsetAsync(dots, 0, (size_t)R * sizeof(double), s));
        hipLaunchKernelGGL(k_cg_xr<T>, dim3(gd), dim3(kKThreads), 0, s, nr, R, tri, S, coef, p, Ap, x, r, dots);
        HQ_HIP(hipGetLastError());
        std::vector<double> rn(R);
        HQ_HIP(hipMemcpyAsync(rn.data(), dots, R * sizeof(double), hipMemcpyDeviceToHost, s));
        HQ_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < R; ++k) {
            c[k] = (active[k] && rr[k] > 0.0) ? rn[k] / rr[k] : 0.0;
            if (active[k]) rr[k] = rn[k];
            if (active[k] && converged(k)) active[k] = 0;
        }
        HQ_HIP(hipMemcpyAsync(coef, c.data(), R * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_cg_p<T>, dim3(grid_of(nr)), dim3(kKThreads), 0, s, nr, R, tri, coef, r, p);
        ++it;
    }
    // V = Q_Z D (Q_Z^T F + Q~^T g)
    HQ_TRY(hq_apply_full(h, x, u, const_cast<void *>(F), 1, nrhs, prec, layout, stream));
    HQ_TRY(dprod());
    HQ_TRY(hq_apply_full(h, y, Ap, V, 0, nrhs, prec, layout, stream));
    HQ_HIP(hipStreamSynchronize(s));
    double worst = 0.0;
    for (int k = 0; k < R; ++k) worst = std::max(worst, bb[k] > 0 ? std::sqrt(rr[k] / bb[k]) : 0.0);
    info->iters = it;
    info->max_rel_residual = worst;
    return HQ_OK;
}

}  // namespace

// four vectors of rows x nrhs and 3 nrhs FP64 scalars, each piece 256-byte aligned
size_t krylov_bytes(int64_t rows, int64_t nrhs, size_t elem) {
    auto a = [](size_t b) { return (std::max<size_t>(b, 16) + 255) / 256 * 256; };
    return 4 * a((size_t)rows * nrhs * elem) + a(2 * (size_t)nrhs * sizeof(double)) + a((size_t)nrhs * sizeof(double));
}

}  // namespace hq

using namespace hq;

extern "C" hq_status hq_constrained_solve(hq_handle h, hq_dapply_fn dapply, void *user, const void *F, void *V,
                                          void *g, int64_t nrhs, hq_precision prec, hq_layout layout, void *dx,
                                          void *dy, hq_krylov_info *info, hq_stream stream) {
    if (!dapply || !F || !V || !g || !dx || !dy || !info) {
        set_error("dapply, F, V, g, dx, dy and info must be given");
        return HQ_E_INVALID;
    }
    if (nrhs < 1 || nrhs > (1 << 20)) {
        set_error("nrhs must be in [1, 2^20]");
        return HQ_E_INVALID;
    }
    if (layout != HQ_ROWS && layout != HQ_TRIPLES) {
        set_error("layout must be HQ_ROWS or HQ_TRIPLES");
        return HQ_E_INVALID;
    }
    if (prec == HQ_FP64) return solve<double>(h, dapply, user, F, V, g, nrhs, prec, layout, dx, dy, info, stream);
    if (prec == HQ_FP32) return solve<float>(h, dapply, user, F, V, g, nrhs, prec, layout, dx, dy, info, stream);
    set_error("prec must be HQ_FP64 or HQ_FP32");
    return HQ_E_INVALID;
}
