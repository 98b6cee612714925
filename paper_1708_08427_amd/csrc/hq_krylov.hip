// Krylov harness for the constrained Brownian-dynamics system of Section 1:
// the constraint forces g solve 0 = Q~ D Q_Z^T F + Q~ D Q~^T g (Eq. 1.5), and
// the rigid-body velocities are V = Q_Z D (Q_Z^T F + Q~^T g) (Eq. 1.6).  D is
// the caller's mobility product (a callback); Q~ and Q_Z are applied with the
// sweeps of hq_apply_full.  Conjugate gradients on A = Q~ D Q~^T, which is
// symmetric positive definite when D is; one CG per right-hand side, run
// together, with FP64 scalars.
#include <algorithm>
#include <cmath>
#include <numeric>
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

// r -= alpha Ap (per column alpha), and out[col] = ||r||^2
template <typename T>
__global__ void __launch_bounds__(kKThreads) k_cg_r(int64_t n, int R, int tri, int64_t S,
                                                    const double *__restrict__ alpha, const T *__restrict__ Ap, T *r,
                                                    double *out) {
    __shared__ double sh[kLdsCols];
    const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (e0 < S) {
        const double a = alpha[col_of(e0, R, tri)];
        for (int64_t e = e0; e < n; e += S) {
            const T rn = (T)((double)r[e] - a * (double)Ap[e]);
            r[e] = rn;
            acc += (double)rn * (double)rn;
        }
    }
    col_reduce(acc, e0 < S ? col_of(e0, R, tri) : 0, R, sh, out);
}

// x += alpha p, then p = r + beta p (per column alpha, beta), in one pass
template <typename T>
__global__ void k_cg_xp(int64_t n, int R, int tri, const double *__restrict__ alpha, const double *__restrict__ beta,
                        const T *__restrict__ r, T *x, T *p) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = col_of(e, R, tri);
        const double pe = (double)p[e];
        x[e] = (T)((double)x[e] + alpha[c] * pe);
        p[e] = (T)((double)r[e] + beta[c] * pe);
    }
}

// The CG scalars of every column on the device.  State per column k:
// rr[k] = ||r||^2, bb[k] = ||b||^2, act[k] = 1 while the column iterates.
// Step 1 (after p^T A p is in pap): alpha = rr / pap for active columns
// (0 otherwise; a non-positive p^T A p of an active column is reported and
// ends that column), and the accumulator of ||r_new||^2 is cleared.
__global__ void k_cg_alpha(int R, const double *__restrict__ pap, const double *__restrict__ rr, int32_t *act,
                           double *alpha, double *rn, int32_t *bad) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < R; k += gridDim.x * blockDim.x) {
        double a = 0.0;
        if (act[k]) {
            if (pap[k] > 0.0) {
                a = rr[k] / pap[k];
            } else {
                atomicOr(bad, 1);
                act[k] = 0;
            }
        }
        alpha[k] = a;
        rn[k] = 0.0;
    }
}

// Step 2 (after ||r_new||^2 is in rn): beta = rn / rr, rr = rn, and a column
// whose relative residual reached rtol stops; iters counts the iterations of
// each column; the accumulator of the next p^T A p is cleared.
__global__ void k_cg_beta(int R, double rtol2, const double *__restrict__ rn, const double *__restrict__ bb,
                          double *rr, int32_t *act, double *beta, int32_t *iters, int32_t *nact, double *pap) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < R; k += gridDim.x * blockDim.x) {
        double b = 0.0;
        if (act[k]) {
            b = rr[k] > 0.0 ? rn[k] / rr[k] : 0.0;
            rr[k] = rn[k];
            iters[k] += 1;
            if (!(rn[k] > rtol2 * bb[k])) act[k] = 0;
        }
        beta[k] = b;
        pap[k] = 0.0;
        if (act[k]) atomicAdd(nact, 1);
    }
}

// Initial state: rr = bb = ||b||^2 (in rr), act = 1 unless already within
// rtol, iterations 0, p^T A p accumulator cleared.
__global__ void k_cg_init(int R, double rtol2, double *rr, double *bb, int32_t *act, int32_t *iters,
                          double *pap, int32_t *nact) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < R; k += gridDim.x * blockDim.x) {
        bb[k] = rr[k];
        act[k] = rr[k] > rtol2 * bb[k] ? 1 : 0;
        iters[k] = 0;
        pap[k] = 0.0;
        if (act[k]) atomicAdd(nact, 1);
    }
}

// The same three vector passes in 16-byte units (4 FP32 or 2 FP64 values),
// used when every vector is 16-byte aligned and the element count is a
// multiple of the unit: non-temporal loads and stores (each vector is
// streamed once per pass), kVUnroll units in flight per thread.  Thread t
// owns units t, t + Su, t + 2 Su, ... where the stride Su V is a multiple of
// the column period, so the V values of each of its units stay in V fixed
// columns; a block adds its partials per column in LDS, as above.
template <typename T> struct Unit16;
template <> struct Unit16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int V = 4;
};
template <> struct Unit16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int V = 2;
};
constexpr int kVUnroll = 4;

template <int V>
__device__ __forceinline__ void col_reduce_v(const double (&acc)[V], int64_t e0, bool live, int R, int tri,
                                             double *sh, double *out) {
    if (R <= kLdsCols) {
        for (int c = threadIdx.x; c < R; c += blockDim.x) sh[c] = 0.0;
        __syncthreads();
        if (live)
#pragma unroll
            for (int j = 0; j < V; ++j)
                if (acc[j] != 0.0) atomicAdd(&sh[col_of(e0 + j, R, tri)], acc[j]);
        __syncthreads();
        for (int c = threadIdx.x; c < R; c += blockDim.x)
            if (sh[c] != 0.0) atomicAdd(&out[c], sh[c]);
    } else if (live) {
#pragma unroll
        for (int j = 0; j < V; ++j)
            if (acc[j] != 0.0) atomicAdd(&out[col_of(e0 + j, R, tri)], acc[j]);
    }
}

// out[col] = sum a b over nu units
template <typename T>
__global__ void __launch_bounds__(kKThreads) k_dot_cols_v(int64_t nu, int R, int tri, int64_t Su,
                                                          const typename Unit16<T>::type *__restrict__ a,
                                                          const typename Unit16<T>::type *__restrict__ b,
                                                          double *out) {
    typedef typename Unit16<T>::type U;
    constexpr int V = Unit16<T>::V;
    __shared__ double sh[kLdsCols];
    const int64_t q0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[V] = {};
    if (q0 < Su)
        for (int64_t q = q0; q < nu; q += kVUnroll * Su) {
            U x[kVUnroll], y[kVUnroll];
#pragma unroll
            for (int u = 0; u < kVUnroll; ++u) {
                const int64_t k = q + u * Su;
                x[u] = k < nu ? __builtin_nontemporal_load(a + k) : U{};
                y[u] = k < nu ? __builtin_nontemporal_load(b + k) : U{};
            }
#pragma unroll
            for (int u = 0; u < kVUnroll; ++u)
#pragma unroll
                for (int j = 0; j < V; ++j) acc[j] += (double)x[u][j] * (double)y[u][j];
        }
    col_reduce_v<V>(acc, q0 * V, q0 < Su, R, tri, sh, out);
}

// r -= alpha Ap and out[col] = ||r||^2, over nu units
template <typename T>
__global__ void __launch_bounds__(kKThreads) k_cg_r_v(int64_t nu, int R, int tri, int64_t Su,
                                                      const double *__restrict__ alpha,
                                                      const typename Unit16<T>::type *__restrict__ Ap,
                                                      typename Unit16<T>::type *r, double *out) {
    typedef typename Unit16<T>::type U;
    constexpr int V = Unit16<T>::V;
    __shared__ double sh[kLdsCols];
    const int64_t q0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[V] = {};
    if (q0 < Su) {
        double al[V];
#pragma unroll
        for (int j = 0; j < V; ++j) al[j] = alpha[col_of(q0 * V + j, R, tri)];
        for (int64_t q = q0; q < nu; q += kVUnroll * Su) {
            U x[kVUnroll], y[kVUnroll];
#pragma unroll
            for (int u = 0; u < kVUnroll; ++u) {
                const int64_t k = q + u * Su;
                x[u] = k < nu ? __builtin_nontemporal_load(r + k) : U{};
                y[u] = k < nu ? __builtin_nontemporal_load(Ap + k) : U{};
            }
#pragma unroll
            for (int u = 0; u < kVUnroll; ++u) {
                const int64_t k = q + u * Su;
                if (k < nu) {
                    U o;
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        o[j] = (T)((double)x[u][j] - al[j] * (double)y[u][j]);
                        acc[j] += (double)o[j] * (double)o[j];
                    }
                    __builtin_nontemporal_store(o, r + k);
                }
            }
        }
    }
    col_reduce_v<V>(acc, q0 * V, q0 < Su, R, tri, sh, out);
}

// x += alpha p, then p = r + beta p, over nu units
template <typename T>
__global__ void __launch_bounds__(kKThreads) k_cg_xp_v(int64_t nu, int R, int tri, int64_t Su,
                                                       const double *__restrict__ alpha,
                                                       const double *__restrict__ beta,
                                                       const typename Unit16<T>::type *__restrict__ r,
                                                       typename Unit16<T>::type *x, typename Unit16<T>::type *p) {
    typedef typename Unit16<T>::type U;
    constexpr int V = Unit16<T>::V;
    const int64_t q0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q0 >= Su) return;
    double al[V], be[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        al[j] = alpha[col_of(q0 * V + j, R, tri)];
        be[j] = beta[col_of(q0 * V + j, R, tri)];
    }
    for (int64_t q = q0; q < nu; q += kVUnroll * Su) {
        U pv[kVUnroll], xv[kVUnroll], rv[kVUnroll];
#pragma unroll
        for (int u = 0; u < kVUnroll; ++u) {
            const int64_t k = q + u * Su;
            pv[u] = k < nu ? __builtin_nontemporal_load(p + k) : U{};
            xv[u] = k < nu ? __builtin_nontemporal_load(x + k) : U{};
            rv[u] = k < nu ? __builtin_nontemporal_load(r + k) : U{};
        }
#pragma unroll
        for (int u = 0; u < kVUnroll; ++u) {
            const int64_t k = q + u * Su;
            if (k < nu) {
                U xo, po;
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    const double pe = (double)pv[u][j];
                    xo[j] = (T)((double)xv[u][j] + al[j] * pe);
                    po[j] = (T)((double)rv[u][j] + be[j] * pe);
                }
                __builtin_nontemporal_store(xo, x + k);
                __builtin_nontemporal_store(po, p + k);
            }
        }
    }
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
    // per-column FP64 scalars: rr, bb, pap, rn, alpha, beta; int32 act, iters;
    // and two int32 counters (active columns, a bad p^T A p)
    double *sc = (double *)w.get(6 * (size_t)R * sizeof(double));
    int32_t *ic = (int32_t *)w.get((2 * (size_t)R + 2) * sizeof(int32_t));
    if (!r || !p || !Ap || !zr || !sc || !ic) {
        set_error("hipMalloc of the Krylov workspace");
        return HQ_E_NOMEM;
    }
    double *rr = sc, *bb = sc + R, *pap = sc + 2 * R, *rn = sc + 3 * R, *alpha = sc + 4 * R, *beta = sc + 5 * R;
    int32_t *act = ic, *iters = ic + R, *nact = ic + 2 * R, *bad = ic + 2 * R + 1;
    T *x = (T *)g, *u = (T *)dx, *y = (T *)dy;
    // column-fixed grid: stride S a multiple of the column period, about
    // 1024 blocks
    const int64_t per = tri ? 3 * (int64_t)R : (int64_t)R;
    const int64_t S = std::max<int64_t>(per, ((int64_t)1024 * kKThreads / per) * per);
    const unsigned gd = (unsigned)((S + kKThreads - 1) / kKThreads);
    const unsigned gs = (unsigned)std::min<int64_t>((R + kKThreads - 1) / kKThreads, 1024);
    // the 16-byte form: every vector aligned, whole units; Su V a multiple of
    // the column period and of V, one block of threads per compute unit (the
    // in-place passes stream fastest with few, deep threads: 4 units in
    // flight per thread, 5.8-7.3 TB/s on a 7.4M x 32 FP32 vector against
    // 4.6-5.2 with 1,024 blocks or more)
    typedef typename Unit16<T>::type U;
    constexpr int kV = Unit16<T>::V;
    const bool vec = nr % kV == 0 && ((uintptr_t)x | (uintptr_t)r | (uintptr_t)p | (uintptr_t)Ap) % 16 == 0;
    const int64_t pv = std::lcm(per, (int64_t)kV);
    const int64_t Sv = std::max<int64_t>(pv, ((int64_t)std::max(P->ncu, 1) * kKThreads * kV / pv) * pv);
    const int64_t nu = nr / kV, Su = Sv / kV;
    const unsigned gv = (unsigned)((Su + kKThreads - 1) / kKThreads);
    const double rtol2 = rtol * rtol;
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
    HQ_HIP(hipMemsetAsync(sc, 0, 6 * (size_t)R * sizeof(double), s));
    HQ_HIP(hipMemsetAsync(ic, 0, (2 * (size_t)R + 2) * sizeof(int32_t), s));
    if (vec)
        hipLaunchKernelGGL(k_dot_cols_v<T>, dim3(gv), dim3(kKThreads), 0, s, nu, R, tri, Su, (const U *)r,
                           (const U *)r, rr);
    else
        hipLaunchKernelGGL(k_dot_cols<T>, dim3(gd), dim3(kKThreads), 0, s, nr, R, tri, S, r, r, rr);
    hipLaunchKernelGGL(k_cg_init, dim3(gs), dim3(kKThreads), 0, s, R, rtol2, rr, bb, act, iters, pap, nact);
    HQ_HIP(hipGetLastError());
    // The iterations run without the host: the scalars stay on the device and
    // converged columns take zero steps.  The host reads the count of active
    // columns every few iterations (one synchronisation) to stop the loop.
    int it = 0, live = 1;
    int32_t hc[2] = {0, 0};
    const int check = std::max(1, std::min(info->check_every > 0 ? info->check_every : 4, 64));
    auto poll = [&]() -> hq_status {
        HQ_HIP(hipMemcpyAsync(hc, nact, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HQ_HIP(hipStreamSynchronize(s));
        live = hc[0];
        if (hc[1]) {
            set_error("Q~ D Q~^T is not positive definite (p^T A p <= 0): D must be symmetric positive definite");
            return HQ_E_INVALID;
        }
        return HQ_OK;
    };
    HQ_TRY(poll());
    while (it < max_iter && live > 0) {
        HQ_HIP(hipMemsetAsync(nact, 0, sizeof(int32_t), s));
        HQ_TRY(apply_A(p, Ap));
        if (vec)
            hipLaunchKernelGGL(k_dot_cols_v<T>, dim3(gv), dim3(kKThreads), 0, s, nu, R, tri, Su, (const U *)p,
                               (const U *)Ap, pap);
        else
            hipLaunchKernelGGL(k_dot_cols<T>, dim3(gd), dim3(kKThreads), 0, s, nr, R, tri, S, p, Ap, pap);
        hipLaunchKernelGGL(k_cg_alpha, dim3(gs), dim3(kKThreads), 0, s, R, pap, rr, act, alpha, rn, bad);
        if (vec)
            hipLaunchKernelGGL(k_cg_r_v<T>, dim3(gv), dim3(kKThreads), 0, s, nu, R, tri, Su, alpha, (const U *)Ap,
                               (U *)r, rn);
        else
            hipLaunchKernelGGL(k_cg_r<T>, dim3(gd), dim3(kKThreads), 0, s, nr, R, tri, S, alpha, Ap, r, rn);
        hipLaunchKernelGGL(k_cg_beta, dim3(gs), dim3(kKThreads), 0, s, R, rtol2, rn, bb, rr, act, beta, iters, nact,
                           pap);
        if (vec)
            hipLaunchKernelGGL(k_cg_xp_v<T>, dim3(gv), dim3(kKThreads), 0, s, nu, R, tri, Su, alpha, beta,
                               (const U *)r, (U *)x, (U *)p);
        else
            hipLaunchKernelGGL(k_cg_xp<T>, dim3(grid_of(nr)), dim3(kKThreads), 0, s, nr, R, tri, alpha, beta, r, x,
                               p);
        HQ_HIP(hipGetLastError());
        ++it;
        if (it % check == 0 || it == max_iter) HQ_TRY(poll());
    }
    // V = Q_Z D (Q_Z^T F + Q~^T g)
    HQ_TRY(hq_apply_full(h, x, u, const_cast<void *>(F), 1, nrhs, prec, layout, stream));
    HQ_TRY(dprod());
    HQ_TRY(hq_apply_full(h, y, Ap, V, 0, nrhs, prec, layout, stream));
    std::vector<double> hrr(R), hbb(R);
    std::vector<int32_t> hit(R);
    HQ_HIP(hipMemcpyAsync(hrr.data(), rr, R * sizeof(double), hipMemcpyDeviceToHost, s));
    HQ_HIP(hipMemcpyAsync(hbb.data(), bb, R * sizeof(double), hipMemcpyDeviceToHost, s));
    HQ_HIP(hipMemcpyAsync(hit.data(), iters, R * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HQ_HIP(hipStreamSynchronize(s));
    double worst = 0.0;
    int most = 0;
    for (int k = 0; k < R; ++k) {
        worst = std::max(worst, hbb[k] > 0 ? std::sqrt(hrr[k] / hbb[k]) : 0.0);
        most = std::max(most, (int)hit[k]);
    }
    info->iters = most;
    info->max_rel_residual = worst;
    return HQ_OK;
}

}  // namespace

// four vectors of rows x nrhs, 6 nrhs FP64 scalars and 2 nrhs + 2 int32
// ones, each piece 256-byte aligned
size_t krylov_bytes(int64_t rows, int64_t nrhs, size_t elem) {
    auto a = [](size_t b) { return (std::max<size_t>(b, 16) + 255) / 256 * 256; };
    return 4 * a((size_t)rows * nrhs * elem) + a(6 * (size_t)nrhs * sizeof(double)) +
           a((2 * (size_t)nrhs + 2) * sizeof(int32_t));
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
