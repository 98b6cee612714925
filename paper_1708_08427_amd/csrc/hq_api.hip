// The C ABI of include/hq.h: argument checks, the plan behind a handle, device
// buffers, and the launch sequences of hq_build.hip / hq_apply.hip /
// hq_explicit.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "hq_common.h"

namespace hq {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

Plan *plan_of(hq_handle h) {
    Plan *P = reinterpret_cast<Plan *>(h);
    if (!P || P->magic != kPlanMagic) {
        set_error("invalid or destroyed handle");
        return nullptr;
    }
    return P;
}

// Workspace pieces start on 256-byte boundaries.
constexpr size_t kWsAlign = 256;

hq_status plan_alloc(Plan &P, void **p, size_t bytes) {
    *p = nullptr;
    bytes = std::max<size_t>(bytes, 1);
    if (P.sizing || P.ws) {
        const size_t b = (bytes + kWsAlign - 1) / kWsAlign * kWsAlign;
        if (P.ws) {
            if (P.ws_used + b > P.ws_bytes) {
                set_error("the workspace is too small (hq_workspace_bytes gives the size)");
                return HQ_E_INVALID;
            }
            *p = P.ws + P.ws_used;
        }
        P.ws_used += b;
        return HQ_OK;
    }
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
        return HQ_E_NOMEM;
    }
    P.allocs.push_back(q);
    *p = q;
    return HQ_OK;
}

namespace {

template <typename T>
hq_status dalloc(Plan &P, T **p, int64_t count) {
    void *q = nullptr;
    HQ_TRY(plan_alloc(P, &q, (size_t)std::max<int64_t>(count, 1) * sizeof(T)));
    *p = reinterpret_cast<T *>(q);
    return HQ_OK;
}

template <typename T>
hq_status upload(Plan &P, T **dst, const std::vector<T> &src) {
    HQ_TRY(dalloc(P, dst, (int64_t)src.size()));
    if (!P.sizing && !src.empty())
        HQ_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return HQ_OK;
}

void free_plan(Plan *P) {
    if (!P) return;
    // teardown: work queued on the handle's stream may still read its memory
    // (errors of earlier work were reported by the calls that queued it)
    if (!P->sizing) (void)hipStreamSynchronize(P->stream);
    for (void *p : P->allocs) (void)hipFree(p);
    if (P->d_xch && !P->ws) (void)hipFree(P->d_xch);
    P->magic = 0;
    delete P;
}

Plan *get_plan(hq_handle h) { return plan_of(h); }

int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

hq_status create_plan(Plan &P, const int64_t *off, int64_t m, const hq_options *opt) {
    P.m = m;
    P.offsets.assign(off, off + m + 1);
    P.N = off[m];
    P.NI = P.N - m;
    P.row_off.assign(m + 1, 0);
    for (int64_t j = 0; j < m; ++j) {
        const int64_t n = off[j + 1] - off[j];
        P.row_off[j + 1] = P.row_off[j] + 3 * n - 6;
        P.max_n = (int)std::max<int64_t>(P.max_n, n);
    }
    P.rows = P.row_off[m];
    P.S = (opt && opt->tile_units) ? opt->tile_units : 32;
    P.S2 = (opt && opt->later_tile_units) ? opt->later_tile_units : P.S;
    if (opt && opt->leaf_size > 1) {
        // the first tile phase holds the leaf boxes; tile_units sizes the rest
        P.leaf_s = opt->leaf_size;
        P.S = P.leaf_s;
    }
    if (opt && opt->run_nodes) P.run_nodes = opt->run_nodes;
    if (opt && opt->waves_per_cu) P.waves_per_cu = opt->waves_per_cu;
    if (opt) P.first_wpc = opt->first_waves_per_cu;
    if (opt) P.sweep_kernel = opt->sweep_kernel;
    if (opt) P.fused_up = opt->fused_upward;
    P.keep_node_data = opt && opt->keep_node_data != 0;
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            P.ncu = ncu;
    }
    P.store = (opt && opt->store) ? opt->store : 3;
    P.dense_max_n = (opt && opt->explicit_dense_max_n) ? opt->explicit_dense_max_n : 4096;
    P.phases_reserved = (opt && opt->max_phases) ? opt->max_phases : 0;

    const int64_t N = P.N, NI = P.NI;
    std::vector<int32_t> bead_off(m + 1), node_off(m + 1), row_off(m + 1);
    for (int64_t j = 0; j <= m; ++j) {
        bead_off[j] = (int32_t)off[j];
        node_off[j] = (int32_t)(off[j] - j);
        row_off[j] = (int32_t)P.row_off[j];
    }
    HQ_TRY(upload(P, &P.d_bead_off, bead_off));
    HQ_TRY(upload(P, &P.d_node_off, node_off));
    HQ_TRY(dalloc(P, &P.d_rotf, 9 * m));
    HQ_TRY(upload(P, &P.d_row_off, row_off));

    // chunk table for the per-bead kernels
    std::vector<int32_t> chunks;
    constexpr int64_t kChunk = 2048;
    for (int64_t j = 0; j < m; ++j)
        for (int64_t b = off[j]; b < off[j + 1]; b += kChunk) {
            chunks.push_back((int32_t)j);
            chunks.push_back((int32_t)b);
            chunks.push_back((int32_t)std::min(off[j + 1], b + kChunk));
        }
    P.nchunks = (int)(chunks.size() / 3);
    HQ_TRY(upload(P, &P.d_chunks, chunks));

    // sort plan: bodies up to kSortChunk beads sorted by one block each
    // (longest first, so the longest sorts start earliest), larger ones as
    // block-sorted chunks followed by merge passes
    struct Seg {
        int32_t start, len, body;  // body stored as ~body for a chunk of a large body
    };
    std::vector<Seg> small;
    std::vector<int32_t> large;
    std::vector<int64_t> large_prefix;
    int64_t lsum = 0;
    for (int64_t j = 0; j < m; ++j) {
        const int64_t n = off[j + 1] - off[j];
        if (n <= kSortChunk) {
            small.push_back({(int32_t)off[j], (int32_t)n, (int32_t)j});
        } else {
            large.push_back((int32_t)j);
            large_prefix.push_back(lsum);
            lsum += n;
            int passes = 0;
            for (int64_t L = kSortChunk; L < n; L *= 2) ++passes;
            P.large_passes = std::max(P.large_passes, passes);
            for (int64_t b = 0; b < n; b += kSortChunk) {
                small.push_back({(int32_t)(off[j] + b), (int32_t)std::min<int64_t>(kSortChunk, n - b), ~(int32_t)j});
            }
        }
    }
    std::stable_sort(small.begin(), small.end(), [](const Seg &a, const Seg &b) { return a.len > b.len; });
    std::vector<int32_t> segs;
    for (const auto &e : small) {
        segs.push_back(e.start);
        segs.push_back(e.len);
        segs.push_back(e.body);
    }
    P.sort_segs.nseg = (int)small.size();
    if (P.sort_segs.nseg) HQ_TRY(upload(P, &P.sort_segs.d_seg, segs));
    P.nlarge = (int)large.size();
    P.large_elems = lsum;
    if (P.nlarge) {
        HQ_TRY(upload(P, &P.d_large, large));
        HQ_TRY(upload(P, &P.d_large_prefix, large_prefix));
    }

    // body level
    HQ_TRY(dalloc(P, &P.d_bmin, 3 * m));
    HQ_TRY(dalloc(P, &P.d_bmax, 3 * m));
    HQ_TRY(dalloc(P, &P.d_lo, 3 * m));
    HQ_TRY(dalloc(P, &P.d_h, m));
    HQ_TRY(dalloc(P, &P.d_cen, 3 * m));
    HQ_TRY(dalloc(P, &P.d_kappa, m));
    HQ_TRY(dalloc(P, &P.d_bflags, m));
    // bead level
    HQ_TRY(dalloc(P, &P.d_keyA, N));
    HQ_TRY(dalloc(P, &P.d_valA, N));
    if (P.nlarge) {
        HQ_TRY(dalloc(P, &P.d_keyB, N));
        HQ_TRY(dalloc(P, &P.d_valB, N));
    }
    HQ_TRY(dalloc(P, &P.d_scode, N));
    HQ_TRY(dalloc(P, &P.d_perm, N));
    HQ_TRY(dalloc(P, &P.d_leafpar, N));
    HQ_TRY(dalloc(P, &P.d_mark, N));
    HQ_TRY(dalloc(P, &P.d_msum, N));
    // node level
    HQ_TRY(dalloc(P, &P.d_lc, NI));
    HQ_TRY(dalloc(P, &P.d_rc, NI));
    HQ_TRY(dalloc(P, &P.d_par, NI));
    HQ_TRY(dalloc(P, &P.d_first, NI));
    HQ_TRY(dalloc(P, &P.d_last, NI));
    HQ_TRY(dalloc(P, &P.d_nbody, NI));
    HQ_TRY(dalloc(P, &P.d_cov, NI));
    HQ_TRY(dalloc(P, &P.d_units, NI));
    HQ_TRY(dalloc(P, &P.d_tileof, NI));
    HQ_TRY(dalloc(P, &P.d_sched, NI));
    HQ_TRY(dalloc(P, &P.d_yfirst, NI));
    HQ_TRY(dalloc(P, &P.d_slot, NI));
    HQ_TRY(dalloc(P, &P.d_aw, NI));
    HQ_TRY(dalloc(P, &P.d_lw, NI));
    HQ_TRY(dalloc(P, &P.d_trval, NI));
    HQ_TRY(dalloc(P, &P.d_trscan, NI));
    HQ_TRY(dalloc(P, &P.d_rem, NI));
    HQ_TRY(dalloc(P, &P.d_tord, NI));
    HQ_TRY(dalloc(P, &P.d_lhist, (int64_t)P.S * 256));
    HQ_TRY(dalloc(P, &P.d_lincl, (int64_t)P.S * 256));
    HQ_TRY(dalloc(P, &P.d_nn, NI));
    HQ_TRY(dalloc(P, &P.d_ncen, 3 * NI));
    HQ_TRY(dalloc(P, &P.d_T22, 6 * NI));
    HQ_TRY(dalloc(P, &P.d_tile_root, NI));
    HQ_TRY(dalloc(P, &P.d_tile_base, NI));
    HQ_TRY(dalloc(P, &P.d_tile_len, NI));
    HQ_TRY(dalloc(P, &P.d_sched_node, NI));
    HQ_TRY(dalloc(P, &P.d_ptile, NI));
    HQ_TRY(dalloc(P, &P.d_tcnt, NI));
    HQ_TRY(dalloc(P, &P.d_tcnt0, NI));
    HQ_TRY(dalloc(P, &P.d_links, (int64_t)kLinkInts * NI));
    if (P.store & 2) HQ_TRY(dalloc(P, &P.d_rec32, (int64_t)kRecWords * NI));
    if (P.store & 1) HQ_TRY(dalloc(P, &P.d_rec64, (int64_t)kRecWords * NI));
    HQ_TRY(dalloc(P, &P.d_phase, 2 * kMaxPhases));
    HQ_TRY(dalloc(P, &P.d_prun, kPrunStride * kMaxPhases));
    // a phase of n nodes uses ceil(n / tp) + 1 entries, with tp = run_nodes or
    // fewer than kRunTarget + 1 runs
    P.run_cap = NI / P.run_nodes + (int64_t)kMaxPhases * (kRunTarget + 3) + 4;
    HQ_TRY(dalloc(P, &P.d_run, P.run_cap));
    HQ_TRY(dalloc(P, &P.d_cnt, kCntNum));
    HQ_TRY(dalloc(P, &P.d_err, 1));
    if (!P.sizing) HQ_HIP(hipMemset(P.d_err, 0, sizeof(int32_t)));
    P.scan_blk_cap = scan_blocks_needed(std::max(std::max(N, NI), (int64_t)P.S * 256)) + 8;
    HQ_TRY(dalloc(P, &P.d_scan_blk, P.scan_blk_cap));
    return HQ_OK;
}

// Elements of the largest precision a handle keeps.
size_t store_elem(const Plan &P) { return (P.store & 1) ? sizeof(double) : sizeof(float); }

// The rest of a workspace handle's memory, which a library-allocated handle
// sizes after its first build or on demand: the tile-root table and the
// sweeps' exchange entries for (max_tiles or, without it, every internal
// node: tiles are disjoint and hold at least one) tiles plus 64, the
// exchange entries for max_nrhs right-hand sides, the explicit-block offsets
// of the largest body, and the Krylov solve's vectors for krylov_nrhs
// right-hand sides.
hq_status reserve_workspace_extras(Plan &P, const hq_options *opt) {
    const int64_t tiles = ((opt && opt->max_tiles > 0) ? (int64_t)opt->max_tiles : P.NI) + 64;
    HQ_TRY(dalloc(P, &P.d_troot, tiles * kGenWords));
    P.troot_cap = tiles;
    const int64_t nrhs = (opt && opt->max_nrhs > 0) ? opt->max_nrhs : 32;
    P.xch_bytes = (size_t)tiles * 6 * (size_t)nrhs * store_elem(P);
    HQ_TRY(plan_alloc(P, &P.d_xch, P.xch_bytes));
    HQ_TRY(dalloc(P, &P.d_blk, P.max_n));
    if (P.leaf_s > 1) {
        // leaf boxes hold two or more beads each
        P.bucket_cap = P.N / 2 + 64;
        const int64_t vals = P.bucket_cap * (int64_t)bucket_stride(P.leaf_smax());
        if (P.store & 1) HQ_TRY(dalloc(P, &P.d_brec64, vals));
        if (P.store & 2) HQ_TRY(dalloc(P, &P.d_brec32, vals));
    }
    if (opt && opt->krylov_nrhs > 0) {
        P.kry_bytes = krylov_bytes(P.rows, opt->krylov_nrhs, store_elem(P));
        HQ_TRY(plan_alloc(P, &P.d_kry, P.kry_bytes));
    }
    return HQ_OK;
}

hq_status ensure_xch(Plan &P, int64_t nrhs, hq_precision prec, hipStream_t s) {
    const size_t elem = (prec == HQ_FP64) ? sizeof(double) : sizeof(float);
    if (P.ws) {
        // the workspace holds entries for troot_cap tiles
        if (P.xch_bytes < (size_t)P.troot_cap * 6 * (size_t)nrhs * elem) {
            set_error("nrhs beyond the workspace's exchange entries (hq_options.max_nrhs)");
            return HQ_E_UNSUPPORTED;
        }
        return HQ_OK;
    }
    const int64_t cap_tiles = 2 * P.tiles_built + 64;
    const size_t need = (size_t)cap_tiles * 6 * (size_t)nrhs * elem;
    if (P.xch_bytes >= need) return HQ_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
        set_error("exchange buffer too small during stream capture: call hq_reserve first");
        return HQ_E_INVALID;
    }
    // the old buffer may still be in use by work queued on this stream
    HQ_HIP(hipStreamSynchronize(s));
    if (P.d_xch) {
        (void)hipFree(P.d_xch);
        P.d_xch = nullptr;
        P.xch_bytes = 0;
    }
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, need);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc of the exchange buffer: ") + hipGetErrorString(e));
        return HQ_E_NOMEM;
    }
    P.d_xch = q;
    P.xch_bytes = need;
    return HQ_OK;
}

// Argument checks of hq_apply and its variants.
hq_status check_apply(const Plan &P, const void *v, const void *out, const void *root, int transpose, int64_t nrhs,
                      hq_precision prec, hq_layout layout) {
    if (!v || !out) {
        set_error("v or out is NULL");
        return HQ_E_INVALID;
    }
    if (v == out || root == v || root == out) {
        set_error("v, out and root must not overlap");
        return HQ_E_INVALID;
    }
    if (transpose != 0 && transpose != 1) {
        set_error("transpose must be 0 or 1");
        return HQ_E_INVALID;
    }
    if (nrhs < 1 || nrhs > (1 << 20)) {
        set_error("nrhs must be in [1, 2^20]");
        return HQ_E_INVALID;
    }
    if (prec != HQ_FP64 && prec != HQ_FP32) {
        set_error("prec must be HQ_FP64 or HQ_FP32");
        return HQ_E_INVALID;
    }
    if ((prec == HQ_FP64 && !(P.store & 1)) || (prec == HQ_FP32 && !(P.store & 2))) {
        set_error("transforms of this precision were not kept (hq_options.store)");
        return HQ_E_INVALID;
    }
    if (layout != HQ_ROWS && layout != HQ_TRIPLES) {
        set_error("layout must be HQ_ROWS or HQ_TRIPLES");
        return HQ_E_INVALID;
    }
    if ((3 * P.N) * nrhs > (int64_t(1) << 40)) {
        set_error("vector too large");
        return HQ_E_UNSUPPORTED;
    }
    return HQ_OK;
}

// Argument checks and launch of hq_apply (ev: optional per-phase events).
hq_status hq_apply_checked(Plan &P, const void *v, void *out, void *root, int transpose, int64_t nrhs,
                           hq_precision prec, hq_layout layout, hipStream_t s, hipEvent_t *ev) {
    HQ_TRY(check_apply(P, v, out, root, transpose, nrhs, prec, layout));
    HQ_TRY(ensure_xch(P, nrhs, prec, s));
    return apply_device(P, v, out, root, transpose, nrhs, prec, layout, s, ev);
}

// ---------------------------------------------------------------------------
// The exchange buffer of hq_apply_noalloc: one static array per device, so
// that the call allocates nothing.  In host code the name `scratch` is only a
// stand-in for the symbol; its device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is
// handed to kernels.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hq_status scratch_address(void **out) {
    int dev = 0;
    HQ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the static exchange table");
        return HQ_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress of the static exchange buffer: ") + hipGetErrorString(e));
            return HQ_E_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HQ_OK;
}

}  // namespace
}  // namespace hq

using namespace hq;

extern "C" {

hq_status hq_apply_noalloc(hq_handle h, const void *v, void *out, int transpose, int64_t nrhs, hq_precision prec,
                           hq_layout layout, hq_stream stream) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    HQ_TRY(check_apply(*P, v, out, nullptr, transpose, nrhs, prec, layout));
    // one exchange entry (6 nrhs values) per tile, with the same margin of 64
    // entries as the handle's own buffer for trees rebuilt with more tiles
    const size_t elem = (prec == HQ_FP64) ? sizeof(double) : sizeof(float);
    const double need = (double)(P->tiles_built + 64) * 6.0 * (double)nrhs * (double)elem;
    if (need > (double)kScratchBytes) {
        set_error("hq_apply_noalloc: the exchange buffer needs " + std::to_string((long long)need) +
                  " bytes (tiles x 6 x nrhs values), above the static limit of " + std::to_string(kScratchBytes) +
                  "; use hq_apply_layout");
        return HQ_E_UNSUPPORTED;
    }
    void *xch = nullptr;
    HQ_TRY(scratch_address(&xch));
    return apply_device(*P, v, out, nullptr, transpose, nrhs, prec, layout, reinterpret_cast<hipStream_t>(stream),
                        nullptr, nullptr, xch, kScratchBytes);
}

const char *hq_last_error(void) { return g_last_error.c_str(); }

const char *hq_status_string(hq_status s) {
    switch (s) {
    case HQ_OK: return "HQ_OK";
    case HQ_E_INVALID: return "HQ_E_INVALID";
    case HQ_E_DEGENERATE: return "HQ_E_DEGENERATE";
    case HQ_E_NOMEM: return "HQ_E_NOMEM";
    case HQ_E_DEVICE: return "HQ_E_DEVICE";
    case HQ_E_UNSUPPORTED: return "HQ_E_UNSUPPORTED";
    }
    return "unknown status";
}

}  // extern "C"

namespace hq {
namespace {

// Argument checks shared by hq_build, hq_build_into and hq_workspace_bytes.
hq_status check_build_args(const int64_t *body_offsets, int64_t m, const hq_options *opt) {
    if (!body_offsets) {
        set_error("body_offsets is NULL");
        return HQ_E_INVALID;
    }
    if (m < 1 || m > (1 << 26)) {
        set_error("m must be in [1, 2^26]");
        return HQ_E_INVALID;
    }
    if (body_offsets[0] != 0) {
        set_error("body_offsets[0] must be 0");
        return HQ_E_INVALID;
    }
    for (int64_t j = 0; j < m; ++j) {
        if (body_offsets[j + 1] - body_offsets[j] < 2) {
            set_error("body " + std::to_string(j) + " has fewer than 2 beads (offsets must increase by >= 2)");
            return HQ_E_INVALID;
        }
    }
    if (body_offsets[m] > (int64_t(1) << 28)) {
        set_error("more than 2^28 beads");
        return HQ_E_UNSUPPORTED;
    }
    if (opt) {
        if (opt->later_tile_units != 0 && (opt->later_tile_units < 2 || opt->later_tile_units > kMaxTileUnits)) {
            set_error("later_tile_units must be 0 or in [2, 1024]");
            return HQ_E_INVALID;
        }
        if (opt->tile_units != 0 && (opt->tile_units < 2 || opt->tile_units > kMaxTileUnits)) {
            set_error("tile_units must be 0 or in [2, 1024]");
            return HQ_E_INVALID;
        }
        if (opt->store < 0 || opt->store > 3) {
            set_error("store must be 0..3");
            return HQ_E_INVALID;
        }
        if (opt->max_phases < 0 || opt->max_phases >= kMaxPhases) {
            set_error("max_phases must be in [0, 63]");
            return HQ_E_INVALID;
        }
        if (opt->explicit_dense_max_n < 0) {
            set_error("explicit_dense_max_n must be >= 0");
            return HQ_E_INVALID;
        }
        if (opt->run_nodes != 0 && (opt->run_nodes < 8 || opt->run_nodes > 4096)) {
            set_error("run_nodes must be 0 or in [8, 4096]");
            return HQ_E_INVALID;
        }
        if (opt->keep_node_data != 0 && opt->keep_node_data != 1) {
            set_error("keep_node_data must be 0 or 1");
            return HQ_E_INVALID;
        }
        if (opt->first_waves_per_cu < 0 || opt->first_waves_per_cu > 64) {
            set_error("first_waves_per_cu must be 0 or in [1, 64]");
            return HQ_E_INVALID;
        }
        if (opt->waves_per_cu != 0 && (opt->waves_per_cu < 1 || opt->waves_per_cu > 64)) {
            set_error("waves_per_cu must be 0 or in [1, 64]");
            return HQ_E_INVALID;
        }
        if (opt->leaf_size < 0 || opt->leaf_size > kMaxLeaf) {
            set_error("leaf_size must be in [0, 16]");
            return HQ_E_INVALID;
        }
        if (opt->fused_upward < 0 || opt->fused_upward > 1) {
            set_error("fused_upward must be 0 (one launch per tile phase) or 1 (one upward launch)");
            return HQ_E_INVALID;
        }
        if (opt->sweep_kernel < 0 || opt->sweep_kernel > 3) {
            set_error("sweep_kernel must be 0 (automatic), 1 (a lane group per tile), 2 (node-parallel sweeps) "
                      "or 3 (wide sweeps in every phase)");
            return HQ_E_INVALID;
        }
        if (opt->max_nrhs < 0 || opt->max_nrhs > (1 << 20) || opt->max_tiles < 0 || opt->krylov_nrhs < 0 ||
            opt->krylov_nrhs > (1 << 20)) {
            set_error("max_nrhs, max_tiles and krylov_nrhs must be >= 0 (nrhs <= 2^20)");
            return HQ_E_INVALID;
        }
    }
    return HQ_OK;
}

// Device bytes of a workspace handle (the plan, then the pieces a
// library-allocated handle sizes later).
hq_status workspace_size(const int64_t *off, int64_t m, const hq_options *opt, size_t *bytes) {
    Plan P;
    P.sizing = true;
    HQ_TRY(create_plan(P, off, m, opt));
    HQ_TRY(reserve_workspace_extras(P, opt));
    *bytes = P.ws_used;
    return HQ_OK;
}

// hq_build (ws = nullptr: the handle allocates its memory) and hq_build_into.
hq_status build_handle(const double *positions, const int64_t *body_offsets, int64_t m, const hq_options *opt,
                       void *ws, size_t ws_bytes, hipStream_t s, hq_handle *out) {
    if (!out) {
        set_error("out is NULL");
        return HQ_E_INVALID;
    }
    *out = nullptr;
    if (!positions) {
        set_error("positions is NULL");
        return HQ_E_INVALID;
    }
    HQ_TRY(check_build_args(body_offsets, m, opt));
    if (ws) {
        size_t need = 0;
        HQ_TRY(workspace_size(body_offsets, m, opt, &need));
        if (ws_bytes < need) {
            set_error("the workspace holds " + std::to_string(ws_bytes) + " bytes, the handle needs " +
                      std::to_string(need) + " (hq_workspace_bytes)");
            return HQ_E_INVALID;
        }
        if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
            set_error("the workspace must be 256-byte aligned");
            return HQ_E_INVALID;
        }
    }
    Plan *P = new (std::nothrow) Plan;
    if (!P) {
        set_error("host allocation failed");
        return HQ_E_NOMEM;
    }
    P->magic = kPlanMagic;
    P->stream = s;
    P->ws = reinterpret_cast<char *>(ws);
    P->ws_bytes = ws_bytes;
    hq_status st = create_plan(*P, body_offsets, m, opt);
    if (st == HQ_OK && ws) st = reserve_workspace_extras(*P, opt);
    if (st == HQ_OK) st = build_device(*P, positions, s, true);
    if (st == HQ_OK) {
        if (P->phases_reserved == 0) P->phases_reserved = std::min(kMaxPhases - 1, P->phases_built + 2);
        P->phases_reserved = std::max(P->phases_reserved, P->phases_built);
        hipError_t e = hipStreamSynchronize(s);
        int32_t err = 0;
        if (e == hipSuccess) e = hipMemcpy(&err, P->d_err, sizeof err, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            set_error(std::string("hq_build: ") + hipGetErrorString(e));
            st = HQ_E_DEVICE;
        } else if (err & kFlagNonFinite) {
            set_error("non-finite bead position");
            st = HQ_E_INVALID;
        } else if (err) {
            set_error("device flags raised during the build: " + std::to_string(err));
            st = HQ_E_DEVICE;
        }
    }
    if (st != HQ_OK) {
        free_plan(P);
        return st;
    }
    *out = reinterpret_cast<hq_handle>(P);
    return HQ_OK;
}

}  // namespace
}  // namespace hq

extern "C" {

hq_status hq_build(const double *positions, const int64_t *body_offsets, int64_t m, const hq_options *opt,
                   hq_stream stream, hq_handle *out) {
    return build_handle(positions, body_offsets, m, opt, nullptr, 0, reinterpret_cast<hipStream_t>(stream), out);
}

hq_status hq_workspace_bytes(const int64_t *body_offsets, int64_t m, const hq_options *opt, size_t *bytes) {
    if (!bytes) {
        set_error("bytes is NULL");
        return HQ_E_INVALID;
    }
    *bytes = 0;
    HQ_TRY(check_build_args(body_offsets, m, opt));
    return workspace_size(body_offsets, m, opt, bytes);
}

hq_status hq_build_into(const double *positions, const int64_t *body_offsets, int64_t m, const hq_options *opt,
                        void *workspace, size_t bytes, hq_stream stream, hq_handle *out) {
    if (!workspace) {
        if (out) *out = nullptr;
        set_error("workspace is NULL");
        return HQ_E_INVALID;
    }
    return build_handle(positions, body_offsets, m, opt, workspace, bytes, reinterpret_cast<hipStream_t>(stream),
                        out);
}

hq_status hq_autotune(const double *positions, const int64_t *body_offsets, int64_t m, int64_t nrhs,
                      hq_precision prec, hq_layout layout, int include_rebuild, const hq_options *base, hq_stream stream,
                      hq_options *best, double *best_ms) {
    if (!best) {
        set_error("best is NULL");
        return HQ_E_INVALID;
    }
    if (nrhs < 1 || nrhs > (1 << 20) || (prec != HQ_FP64 && prec != HQ_FP32)) {
        set_error("nrhs must be in [1, 2^20] and prec HQ_FP64 or HQ_FP32");
        return HQ_E_INVALID;
    }
    if (layout != HQ_ROWS && layout != HQ_TRIPLES) {
        set_error("layout must be HQ_ROWS or HQ_TRIPLES");
        return HQ_E_INVALID;
    }
    if (!body_offsets || m < 1) {
        set_error("body_offsets is NULL or m < 1");
        return HQ_E_INVALID;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hq_options opt = base ? *base : hq_options{};
    opt.store = (prec == HQ_FP64) ? 1 : 2;
    const int64_t N = body_offsets[m];
    int64_t rows = 0;
    for (int64_t j = 0; j < m; ++j) rows += 3 * (body_offsets[j + 1] - body_offsets[j]) - 6;
    const size_t elem = (prec == HQ_FP64) ? sizeof(double) : sizeof(float);
    const size_t vbytes = (size_t)std::max<int64_t>(3 * N, std::max<int64_t>(rows, 1)) * (size_t)nrhs * elem;
    void *va = nullptr, *vb = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hq_status st = HQ_OK;
    auto fail = [&](hq_status code, const std::string &msg) {
        set_error(msg);
        st = code;
    };
    if (hipMalloc(&va, vbytes) != hipSuccess || hipMalloc(&vb, vbytes) != hipSuccess) {
        fail(HQ_E_NOMEM, "hipMalloc of the autotune vectors");
    } else if (hipMemsetAsync(va, 0, vbytes, s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
               hipEventCreate(&e1) != hipSuccess) {
        fail(HQ_E_DEVICE, "autotune setup");
    }
    const int s_cand[] = {16, 32, 64}, r_cand[] = {32, 48, 64}, w_cand[] = {8, 16, 32};
    const int s2_cand[] = {4, 8, 16};
    double best_t = 1e300;
    hq_options chosen = opt;
    // one trial build, timed at every waves_per_cu candidate
    auto trial = [&](const hq_options &o) {
        {
            hq_handle h = nullptr;
            hq_status bs = hq_build(positions, body_offsets, m, &o, stream, &h);
            if (bs != HQ_OK) {
                st = bs;
                return;
            }
            Plan *P = get_plan(h);
            for (int wi = 0; wi < 3 && st == HQ_OK; ++wi) {
                P->waves_per_cu = w_cand[wi];
                double ts[5];
                for (int rep = 0; rep < 7 && st == HQ_OK; ++rep) {
                    if (hipEventRecord(e0, s) != hipSuccess) fail(HQ_E_DEVICE, "hipEventRecord");
                    hq_status a = HQ_OK;
                    if (include_rebuild) a = hq_rebuild(h, positions, stream);
                    if (a == HQ_OK) a = hq_apply_layout(h, va, vb, 0, nrhs, prec, layout, stream);
                    if (a == HQ_OK) a = hq_apply_layout(h, vb, va, 1, nrhs, prec, layout, stream);
                    if (a != HQ_OK) {
                        st = a;
                        break;
                    }
                    float ms = 0.f;
                    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                        fail(HQ_E_DEVICE, "autotune timing");
                        break;
                    }
                    if (rep >= 2) ts[rep - 2] = ms;
                }
                if (st != HQ_OK) break;
                std::sort(ts, ts + 5);
                if (ts[2] < best_t) {
                    best_t = ts[2];
                    chosen = o;
                    chosen.waves_per_cu = w_cand[wi];
                }
            }
            int32_t flags = 0;
            if (st == HQ_OK && hipMemcpy(&flags, P->d_err, sizeof flags, hipMemcpyDeviceToHost) == hipSuccess && flags)
                fail(HQ_E_DEVICE, "device flags raised during autotuning: " + std::to_string(flags));
            hq_destroy(h);
        }
    };
    // stage 1: first-phase tile size and run length, later phases with the
    // same tile size
    for (int si = 0; si < 3 && st == HQ_OK; ++si)
        for (int ri = 0; ri < 3 && st == HQ_OK; ++ri) {
            hq_options o = opt;
            o.tile_units = s_cand[si];
            o.run_nodes = r_cand[ri];
            o.later_tile_units = 0;
            trial(o);
        }
    // stage 2: smaller tiles for the later phases under the chosen first phase
    const hq_options first = chosen;
    for (int k = 0; k < 3 && st == HQ_OK; ++k) {
        if (s2_cand[k] >= first.tile_units) continue;
        hq_options o = first;
        o.later_tile_units = s2_cand[k];
        trial(o);
    }
    // stage 3: leaf boxes of 4, 8 or 16 beads under the chosen tiles (their
    // tile_units then sizes the tiles above the leaves), unless the caller
    // fixed the leaf size
    if (!(base && base->leaf_size)) {
        const hq_options second = chosen;
        const int leaf_cand[] = {4, 8, 16};
        for (int k = 0; k < 3 && st == HQ_OK; ++k) {
            hq_options o = second;
            o.leaf_size = leaf_cand[k];
            o.later_tile_units = 0;
            trial(o);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (va) (void)hipFree(va);
    if (vb) (void)hipFree(vb);
    if (st != HQ_OK) return st;
    chosen.store = base ? base->store : 0;
    *best = chosen;
    if (best_ms) *best_ms = best_t;
    return HQ_OK;
}

hq_status hq_rebuild(hq_handle h, const double *positions, hq_stream stream) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (!positions) {
        set_error("positions is NULL");
        return HQ_E_INVALID;
    }
    return build_device(*P, positions, reinterpret_cast<hipStream_t>(stream), false);
}

hq_status hq_reserve(hq_handle h, int64_t nrhs, hq_precision prec) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (nrhs < 1 || (prec != HQ_FP64 && prec != HQ_FP32)) {
        set_error("nrhs must be >= 1 and prec HQ_FP64 or HQ_FP32");
        return HQ_E_INVALID;
    }
    HQ_TRY(ensure_xch(*P, nrhs, prec, P->stream));
    HQ_HIP(hipStreamSynchronize(P->stream));
    return HQ_OK;
}

hq_status hq_apply_timed(hq_handle h, const void *v, void *out, int transpose, int64_t nrhs, hq_precision prec,
                         hq_layout layout, hq_stream stream, float *phase_ms, int32_t max_phases, int32_t *nphases) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (!phase_ms || !nphases || max_phases < 1) {
        set_error("phase_ms and nphases must be given, max_phases >= 1");
        return HQ_E_INVALID;
    }
    const int nph = std::max(P->phases_built, P->phases_reserved);
    if (nph > max_phases) {
        set_error("max_phases is below the handle's tile phases (" + std::to_string(nph) + ")");
        return HQ_E_INVALID;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::vector<hipEvent_t> ev(nph + 1, nullptr);
    hq_status st = HQ_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            set_error("hipEventCreate");
            st = HQ_E_DEVICE;
        }
    if (st == HQ_OK) st = hq_apply_checked(*P, v, out, nullptr, transpose, nrhs, prec, layout, s, ev.data());
    if (st == HQ_OK && hipEventSynchronize(ev[nph]) != hipSuccess) {
        set_error("hipEventSynchronize");
        st = HQ_E_DEVICE;
    }
    for (int k = 0; st == HQ_OK && k < nph; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) {
            set_error("hipEventElapsedTime");
            st = HQ_E_DEVICE;
            break;
        }
        const int phase = transpose ? (nph - k) : (k + 1);  // launch k sweeps this phase
        phase_ms[phase - 1] = ms;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (st == HQ_OK) *nphases = nph;
    return st;
}

hq_status hq_node_phase(hq_handle h, int32_t *phase) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (!phase) {
        set_error("phase is NULL");
        return HQ_E_INVALID;
    }
    HQ_HIP(hipStreamSynchronize(P->stream));
    HQ_HIP(hipMemcpy(phase, P->d_cov, P->NI * sizeof(int32_t), hipMemcpyDeviceToHost));
    return HQ_OK;
}

hq_status hq_apply(hq_handle h, const void *v, void *out, int transpose, int64_t nrhs, hq_precision prec,
                   hq_stream stream) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    return hq_apply_checked(*P, v, out, nullptr, transpose, nrhs, prec, HQ_ROWS,
                            reinterpret_cast<hipStream_t>(stream), nullptr);
}

hq_status hq_apply_layout(hq_handle h, const void *v, void *out, int transpose, int64_t nrhs, hq_precision prec,
                          hq_layout layout, hq_stream stream) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    return hq_apply_checked(*P, v, out, nullptr, transpose, nrhs, prec, layout,
                            reinterpret_cast<hipStream_t>(stream), nullptr);
}

hq_status hq_apply_rotated(hq_handle h, const double *rot, const void *v, void *out, void *work, int transpose,
                           int64_t nrhs, hq_precision prec, hq_layout layout, hq_stream stream) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (!rot) {
        set_error("rot is NULL");
        return HQ_E_INVALID;
    }
    if (!transpose && (!work || work == v || work == out)) {
        set_error("the upward product needs a work vector distinct from v and out");
        return HQ_E_INVALID;
    }
    HQ_TRY(check_apply(*P, v, out, nullptr, transpose, nrhs, prec, layout));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // wide sweeps: the rotations are fused into their bead loads and stores
    HQ_TRY(ensure_xch(*P, nrhs, prec, s));
    const hq_status fused = apply_device(*P, v, out, nullptr, transpose, nrhs, prec, layout, s, nullptr, rot);
    if (fused != HQ_E_UNSUPPORTED) return fused;
    // narrow sweeps: separate rotation passes
    if (!transpose) {
        // Q~(moved) v = Q~ (blockdiag(Rot^T) v)
        HQ_TRY(rotate_vectors(*P, rot, v, work, nrhs, prec, layout, 1, s));
        return hq_apply_checked(*P, work, out, nullptr, 0, nrhs, prec, layout, s, nullptr);
    }
    // Q~(moved)^T w = blockdiag(Rot) (Q~^T w)
    HQ_TRY(hq_apply_checked(*P, v, out, nullptr, 1, nrhs, prec, layout, s, nullptr));
    return rotate_vectors(*P, rot, out, out, nrhs, prec, layout, 0, s);
}

hq_status hq_apply_full(hq_handle h, const void *v, void *out, void *root, int transpose, int64_t nrhs,
                        hq_precision prec, hq_layout layout, hq_stream stream) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (!root) {
        set_error("root is NULL");
        return HQ_E_INVALID;
    }
    return hq_apply_checked(*P, v, out, root, transpose, nrhs, prec, layout, reinterpret_cast<hipStream_t>(stream),
                            nullptr);
}

hq_status hq_explicit(hq_handle h, int64_t body, double *out, int64_t ld, hq_stream stream) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (body < 0 || body >= P->m) {
        set_error("body out of range");
        return HQ_E_INVALID;
    }
    const int64_t n = P->offsets[body + 1] - P->offsets[body];
    if (n == 2) return HQ_OK;  // Q~ has no rows
    if (!out) {
        set_error("out is NULL");
        return HQ_E_INVALID;
    }
    if (n > P->dense_max_n) {
        set_error("body larger than explicit_dense_max_n");
        return HQ_E_UNSUPPORTED;
    }
    if (P->leaf_s > 1) {
        set_error("explicit Q~ is not available for leaf boxes of more than one bead (hq_options.leaf_size)");
        return HQ_E_UNSUPPORTED;
    }
    if (ld < 3 * n) {
        set_error("ld must be >= 3 n_j");
        return HQ_E_INVALID;
    }
    if (!(P->store & 1)) {
        set_error("explicit Q~ needs the FP64 transforms (hq_options.store)");
        return HQ_E_INVALID;
    }
    return explicit_dense(*P, body, out, ld, reinterpret_cast<hipStream_t>(stream));
}

namespace {

struct BodyNodes {
    std::vector<int32_t> lc, rc, nn, first, sched;
};

hq_status read_body_nodes(Plan &P, int64_t body, BodyNodes &B, int64_t &nb, int64_t &nin) {
    nb = P.offsets[body];
    const int64_t n = P.offsets[body + 1] - nb;
    nin = n - 1;
    const int64_t g0 = nb - body;
    HQ_HIP(hipStreamSynchronize(P.stream));
    B.lc.resize(nin);
    B.rc.resize(nin);
    B.nn.resize(nin);
    B.first.resize(nin);
    B.sched.resize(nin);
    HQ_HIP(hipMemcpy(B.lc.data(), P.d_lc + g0, nin * 4, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(B.rc.data(), P.d_rc + g0, nin * 4, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(B.nn.data(), P.d_nn + g0, nin * 4, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(B.first.data(), P.d_first + g0, nin * 4, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(B.sched.data(), P.d_sched + g0, nin * 4, hipMemcpyDeviceToHost));
    return HQ_OK;
}

}  // namespace

hq_status hq_explicit_blocks_size(hq_handle h, int64_t body, int64_t *nblocks, int64_t *nvalues) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (P->leaf_s > 1) {
        set_error("explicit Q~ is not available for leaf boxes of more than one bead (hq_options.leaf_size)");
        return HQ_E_UNSUPPORTED;
    }
    if (!nblocks || !nvalues || body < 0 || body >= P->m) {
        set_error("NULL output or body out of range");
        return HQ_E_INVALID;
    }
    BodyNodes B;
    int64_t nb, nin;
    HQ_TRY(read_body_nodes(*P, body, B, nb, nin));
    int64_t cnt = 0, vals = 0;
    for (int64_t q = 0; q < nin; ++q) {
        const int dim = 3 * (B.lc[q] >= 0) + 3 * (B.rc[q] >= 0);
        if (dim == 0) continue;
        ++cnt;
        vals += (int64_t)dim * 3 * B.nn[q];
    }
    *nblocks = cnt;
    *nvalues = vals;
    return HQ_OK;
}

hq_status hq_explicit_blocks(hq_handle h, int64_t body, hq_precision prec, void *values, int64_t *val_off,
                             int64_t *row_off, int64_t *bead_first, int32_t *rows, int32_t *cols, hq_stream stream) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (P->leaf_s > 1) {
        set_error("explicit Q~ is not available for leaf boxes of more than one bead (hq_options.leaf_size)");
        return HQ_E_UNSUPPORTED;
    }
    if (!values || !val_off || !row_off || !bead_first || !rows || !cols || body < 0 || body >= P->m ||
        (prec != HQ_FP64 && prec != HQ_FP32)) {
        set_error("NULL argument, bad precision or body out of range");
        return HQ_E_INVALID;
    }
    if (!(P->store & 1)) {
        set_error("explicit Q~ needs the FP64 transforms (hq_options.store)");
        return HQ_E_INVALID;
    }
    BodyNodes B;
    int64_t nb, nin;
    HQ_TRY(read_body_nodes(*P, body, B, nb, nin));
    std::vector<int32_t> links((size_t)kLinkInts * P->NI);
    HQ_HIP(hipMemcpy(links.data(), P->d_links, links.size() * 4, hipMemcpyDeviceToHost));
    std::vector<int64_t> blk_off(nin, -1);
    int64_t b = 0, acc = 0;
    val_off[0] = 0;
    for (int64_t q = 0; q < nin; ++q) {
        const int dim = 3 * (B.lc[q] >= 0) + 3 * (B.rc[q] >= 0);
        if (dim == 0) continue;
        blk_off[q] = acc;
        row_off[b] = links[kLinkInts * (size_t)B.sched[q] + 2] - P->row_off[body];
        bead_first[b] = B.first[q] - nb;
        rows[b] = dim;
        cols[b] = 3 * B.nn[q];
        acc += (int64_t)dim * 3 * B.nn[q];
        ++b;
        val_off[b] = acc;
    }
    int64_t *d_blk = P->d_blk;  // the workspace's piece, else allocated for the call
    if (!d_blk) HQ_HIP(hipMalloc(&d_blk, std::max<int64_t>(1, nin) * sizeof(int64_t)));
    hipError_t e = hipMemcpy(d_blk, blk_off.data(), nin * sizeof(int64_t), hipMemcpyHostToDevice);
    hq_status st = HQ_OK;
    if (e != hipSuccess) {
        set_error(hipGetErrorString(e));
        st = HQ_E_DEVICE;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (st == HQ_OK) st = explicit_blocks_launch(*P, body, prec == HQ_FP64 ? 0 : 1, values, d_blk, s);
    const hipError_t se = hipStreamSynchronize(s);
    if (d_blk != P->d_blk) (void)hipFree(d_blk);
    if (st == HQ_OK && se != hipSuccess) {
        set_error(std::string("hq_explicit_blocks: ") + hipGetErrorString(se));
        st = HQ_E_DEVICE;
    }
    return st;
}

hq_status hq_sorted_beads(hq_handle h, int64_t body, int64_t *bead_index) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (!bead_index || body < 0 || body >= P->m) {
        set_error("NULL output or body out of range");
        return HQ_E_INVALID;
    }
    const int64_t b0 = P->offsets[body], n = P->offsets[body + 1] - b0;
    std::vector<int32_t> tmp(n);
    HQ_HIP(hipStreamSynchronize(P->stream));
    HQ_HIP(hipMemcpy(tmp.data(), P->d_perm + b0, n * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) bead_index[i] = tmp[i] - b0;
    return HQ_OK;
}

hq_status hq_rigid_update(hq_handle h, double *positions, const double *rot, const double *trans, hq_stream stream) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (!positions || !rot || !trans) {
        set_error("NULL argument");
        return HQ_E_INVALID;
    }
    return rigid_update(*P, positions, rot, trans, reinterpret_cast<hipStream_t>(stream));
}

hq_status hq_rigid_motion(hq_handle h, const double *positions, double *out, const double *rot, const double *trans,
                          const double *centers, hq_stream stream) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (!positions || !out || !rot || !trans || !centers) {
        set_error("NULL argument");
        return HQ_E_INVALID;
    }
    return rigid_motion(*P, positions, out, rot, trans, centers, reinterpret_cast<hipStream_t>(stream));
}

hq_status hq_query(hq_handle h, hq_info *info) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if (!info) {
        set_error("info is NULL");
        return HQ_E_INVALID;
    }
    HQ_HIP(hipStreamSynchronize(P->stream));
    int32_t err = 0, cnt[kCntNum];
    HQ_HIP(hipMemcpy(&err, P->d_err, sizeof err, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(cnt, P->d_cnt, sizeof cnt, hipMemcpyDeviceToHost));
    std::vector<unsigned long long> kap(P->m);
    std::vector<int32_t> fl(P->m);
    HQ_HIP(hipMemcpy(kap.data(), P->d_kappa, P->m * 8, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(fl.data(), P->d_bflags, P->m * 4, hipMemcpyDeviceToHost));
    std::memset(info, 0, sizeof *info);
    info->N = P->N;
    info->m = P->m;
    info->rows = P->rows;
    info->internal_nodes = P->NI;
    info->tiles = cnt[kCntTiles];
    info->phases = cnt[kCntPhases];
    info->device_flags = err;
    info->tile_units = P->S;
    info->store = P->store;
    double mk = 0.0;
    for (int64_t j = 0; j < P->m; ++j) {
        double d;
        std::memcpy(&d, &kap[j], 8);
        mk = std::max(mk, d);
        if (fl[j] & HQ_BODY_ILLCOND) ++info->ill_conditioned_bodies;
        if (fl[j] & HQ_BODY_DEGENERATE) ++info->degenerate_bodies;
    }
    info->max_kappa = mk;
    return HQ_OK;
}

hq_status hq_body_info(hq_handle h, int32_t *flags, double *kappa) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    HQ_HIP(hipStreamSynchronize(P->stream));
    if (flags) HQ_HIP(hipMemcpy(flags, P->d_bflags, P->m * 4, hipMemcpyDeviceToHost));
    if (kappa) HQ_HIP(hipMemcpy(kappa, P->d_kappa, P->m * 8, hipMemcpyDeviceToHost));
    return HQ_OK;
}

hq_status hq_node_data(hq_handle h, int32_t *first, int32_t *last, int32_t *xchild, int32_t *ychild, int32_t *body,
                       int32_t *nbeads, double *centroid, double *T22, double *G, int32_t *k, int32_t *row) {
    Plan *P = get_plan(h);
    if (!P) return HQ_E_INVALID;
    if ((centroid || T22 || G) && P->leaf_s > 1) {
        set_error("per-node centroids, T22 and G are not kept inside leaf boxes (hq_options.leaf_size)");
        return HQ_E_UNSUPPORTED;
    }
    if ((centroid || T22) && !P->node_data_fresh) {
        set_error("centroids and T22 after hq_rebuild need hq_options.keep_node_data = 1");
        return HQ_E_INVALID;
    }
    const int64_t NI = P->NI;
    HQ_HIP(hipStreamSynchronize(P->stream));
    std::vector<int32_t> lc(NI), rc(NI), nbody(NI), fst(NI), lst(NI), nn(NI), sched(NI);
    HQ_HIP(hipMemcpy(lc.data(), P->d_lc, NI * 4, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(rc.data(), P->d_rc, NI * 4, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(nbody.data(), P->d_nbody, NI * 4, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(fst.data(), P->d_first, NI * 4, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(lst.data(), P->d_last, NI * 4, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(nn.data(), P->d_nn, NI * 4, hipMemcpyDeviceToHost));
    HQ_HIP(hipMemcpy(sched.data(), P->d_sched, NI * 4, hipMemcpyDeviceToHost));
    std::vector<double> cen, t22, rec;
    if (centroid) {
        cen.resize(3 * NI);
        HQ_HIP(hipMemcpy(cen.data(), P->d_ncen, 3 * NI * 8, hipMemcpyDeviceToHost));
    }
    if (T22) {
        t22.resize(6 * NI);
        HQ_HIP(hipMemcpy(t22.data(), P->d_T22, 6 * NI * 8, hipMemcpyDeviceToHost));
    }
    std::vector<int32_t> links;
    if (G || row) {
        links.resize((size_t)kLinkInts * NI);
        HQ_HIP(hipMemcpy(links.data(), P->d_links, links.size() * 4, hipMemcpyDeviceToHost));
    }
    if (G) {
        if (!(P->store & 1)) {
            set_error("G needs the FP64 transforms");
            return HQ_E_INVALID;
        }
        rec.resize((size_t)kRecWords * NI);
        HQ_HIP(hipMemcpy(rec.data(), P->d_rec64, rec.size() * 8, hipMemcpyDeviceToHost));
    }
    for (int64_t g = 0; g < NI; ++g) {
        const int j = nbody[g];
        const int64_t b0 = P->offsets[j], g0 = b0 - j;
        auto loc = [&](int c) -> int32_t {
            if (c >= 0) return (int32_t)(c - g0);
            return (int32_t)(-((-(c + 1)) - b0) - 1);
        };
        if (first) first[g] = (int32_t)(fst[g] - b0);
        if (last) last[g] = (int32_t)(lst[g] - b0);
        if (xchild) xchild[g] = loc(lc[g]);
        if (ychild) ychild[g] = loc(rc[g]);
        if (body) body[g] = j;
        if (nbeads) nbeads[g] = nn[g];
        const int kk = 3 + 3 * (lc[g] >= 0) + 3 * (rc[g] >= 0);
        if (k) k[g] = kk;
        if (centroid)
            for (int d = 0; d < 3; ++d) centroid[3 * g + d] = cen[3 * (size_t)sched[g] + d];
        if (T22) {
            const double *t = &t22[6 * (size_t)sched[g]];
            double M[9] = {t[0], 0, 0, t[1], t[2], 0, t[3], t[4], t[5]};
            std::memcpy(T22 + 9 * g, M, sizeof M);
        }
        if (row) row[g] = links[kLinkInts * (size_t)sched[g] + 2] - (int32_t)P->row_off[j];
        if (G) {
            const double *r = &rec[(size_t)kRecWords * sched[g]];
            double *Gg = G + 81 * g;
            for (int i = 0; i < 81; ++i) Gg[i] = 0.0;
            for (int col = 0; col < kk; ++col) {
                double t[9] = {0};
                t[col] = 1.0;
                for (int jj = 0; jj < 3; ++jj) {
                    const double *tl = r + tail_off(jj);
                    double w = t[jj];
                    for (int i = jj + 1; i < kk; ++i) w += tl[i - jj - 1] * t[i];
                    w *= r[kRecTau + jj];
                    t[jj] -= w;
                    for (int i = jj + 1; i < kk; ++i) t[i] -= w * tl[i - jj - 1];
                }
                for (int i = 0; i < kk; ++i) Gg[9 * i + col] = t[i];
            }
        }
    }
    return HQ_OK;
}

hq_status hq_capture_begin(hq_stream stream) {
    HQ_HIP(hipStreamBeginCapture(reinterpret_cast<hipStream_t>(stream), hipStreamCaptureModeRelaxed));
    return HQ_OK;
}

hq_status hq_capture_end(hq_stream stream, void **graph_exec) {
    if (!graph_exec) {
        set_error("graph_exec is NULL");
        return HQ_E_INVALID;
    }
    hipGraph_t g = nullptr;
    HQ_HIP(hipStreamEndCapture(reinterpret_cast<hipStream_t>(stream), &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        return HQ_E_DEVICE;
    }
    *graph_exec = reinterpret_cast<void *>(ex);
    return HQ_OK;
}

hq_status hq_graph_launch(void *graph_exec, hq_stream stream) {
    if (!graph_exec) {
        set_error("graph_exec is NULL");
        return HQ_E_INVALID;
    }
    HQ_HIP(hipGraphLaunch(reinterpret_cast<hipGraphExec_t>(graph_exec), reinterpret_cast<hipStream_t>(stream)));
    return HQ_OK;
}

void hq_graph_destroy(void *graph_exec) {
    if (graph_exec) (void)hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(graph_exec));
}

void hq_destroy(hq_handle h) {
    Plan *P = reinterpret_cast<Plan *>(h);
    if (!P || P->magic != kPlanMagic) return;
    free_plan(P);
}

}  // extern "C"
