// Device-wide prefix sums (three passes: block totals, scan of the totals,
// block scans with carry-in).  Used by the build for unit counts and for
// numbering tiles; every launch size depends only on n.  A non-null gate
// that reads 0 on the device turns all three passes into no-ops.
#include "hq_common.h"

namespace hq {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kPerBlock = kThreads * kItems;

template <typename T>
__device__ T block_exclusive(T v, T *lds, T *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < kThreads / 64; ++w) {
            T t = lds[w];
            lds[w] = run;
            run += t;
        }
        lds[kThreads / 64] = run;
    }
    __syncthreads();
    T excl = x - v + lds[wid];
    *total = lds[kThreads / 64];
    __syncthreads();
    return excl;
}

// dn: when not null, the element count is min(n, *dn), read on the device
// (launch sizes still follow n; blocks past the count do nothing).
__device__ __forceinline__ int64_t scan_count(int64_t n, const int32_t *dn) {
    return dn ? min(n, (int64_t)max(*dn, 0)) : n;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_block_sums(const T *__restrict__ in, int64_t n,
                                                         T *__restrict__ blk, const int32_t *gate,
                                                         const int32_t *dn) {
    if (gate && *gate == 0) return;
    n = scan_count(n, dn);
    if ((int64_t)blockIdx.x * kPerBlock >= n) {
        if (threadIdx.x == 0) blk[blockIdx.x] = 0;
        return;
    }
    __shared__ T lds[kThreads / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kPerBlock + (int64_t)threadIdx.x * kItems;
    T s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i)
        if (base + i < n) s += in[base + i];
    T tot;
    block_exclusive<T>(s, lds, &tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_scan_blocks(T *__restrict__ blk, int64_t nb, const int32_t *gate,
                                                          const int32_t *dn) {
    if (gate && *gate == 0) return;
    if (dn) nb = min(nb, (scan_count(nb * kPerBlock, dn) + kPerBlock - 1) / kPerBlock);
    __shared__ T lds[kThreads / 64 + 1];
    T carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
        int64_t i = b0 + threadIdx.x;
        T v = (i < nb) ? blk[i] : T(0);
        T tot;
        T e = block_exclusive<T>(v, lds, &tot);
        if (i < nb) blk[i] = e + carry;
        carry += tot;
    }
}

template <typename T, bool kInclusive>
__global__ void __launch_bounds__(kThreads) k_scan_apply(const T *__restrict__ in, T *__restrict__ out,
                                                         int64_t n, const T *__restrict__ blk,
                                                         const int32_t *gate, const int32_t *dn) {
    if (gate && *gate == 0) return;
    n = scan_count(n, dn);
    if ((int64_t)blockIdx.x * kPerBlock >= n) return;
    __shared__ T lds[kThreads / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kPerBlock + (int64_t)threadIdx.x * kItems;
    T v[kItems];
    T s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : T(0);
        s += v[i];
    }
    T tot;
    T run = block_exclusive<T>(s, lds, &tot) + blk[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        if (kInclusive) run += v[i];
        if (base + i < n) out[base + i] = run;
        if (!kInclusive) run += v[i];
    }
}

template <typename T, bool kInclusive>
hq_status scan_impl(Plan &P, const T *in, T *out, int64_t n, hipStream_t s, const int32_t *gate,
                    const int32_t *dn = nullptr) {
    if (n <= 0) return HQ_OK;
    const int64_t nb = (n + kPerBlock - 1) / kPerBlock;
    if (nb > P.scan_blk_cap) {
        set_error("scan larger than the reserved scratch");
        return HQ_E_UNSUPPORTED;
    }
    T *blk = reinterpret_cast<T *>(P.d_scan_blk);
    hipLaunchKernelGGL((k_block_sums<T>), dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, blk, gate, dn);
    hipLaunchKernelGGL((k_scan_blocks<T>), dim3(1), dim3(kThreads), 0, s, blk, nb, gate, dn);
    hipLaunchKernelGGL((k_scan_apply<T, kInclusive>), dim3((unsigned)nb), dim3(kThreads), 0, s, in, out, n,
                       (const T *)blk, gate, dn);
    HQ_HIP(hipGetLastError());
    return HQ_OK;
}

}  // namespace

int64_t scan_blocks_needed(int64_t n) { return (n + kPerBlock - 1) / kPerBlock; }

hq_status scan_i32_inclusive(Plan &P, const int32_t *in, int32_t *out, int64_t n, hipStream_t s,
                             const int32_t *gate) {
    return scan_impl<int32_t, true>(P, in, out, n, s, gate);
}

hq_status scan_i64_exclusive(Plan &P, const long long *in, long long *out, int64_t n, hipStream_t s,
                             const int32_t *gate, const int32_t *dn) {
    return scan_impl<long long, false>(P, in, out, n, s, gate, dn);
}

}  // namespace hq
