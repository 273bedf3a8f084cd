// lg_sssp: single-source shortest paths over a weighted graph (SSSP of
// section "Considered Algorithms", a delta-stepping traversal), reading the
// weight stored right after each ID (subsection "Accessing an Edge Weight").
//
// Distances are uint64 (UINT64_MAX: not reached).  A bitmap marks vertices
// whose distance dropped since their edges were last relaxed.  Each step of
// bucket k (distances below hi = (k+1) delta):
//   collect  marked vertices with a distance below hi leave the bitmap and
//            join the frontier queue with their list start, ID width,
//            degree and distance (a count pass per 64-vertex word, a scan,
//            a write pass); the smallest distance among the marked vertices
//            left behind is kept for choosing the next bucket
//   relax    the frontier's edges, flattened by an exclusive scan of the
//            degrees, 64 consecutive edges per wave step: nd = dist(u) + w;
//            an atomic minimum on dist(v), and v is marked when it lowered it
// An empty frontier moves to the bucket of the smallest marked distance;
// none marked ends the search.  Every vertex relaxed from a distance d
// reaches the final distances of the paths through it, so the result is the
// exact distances whatever delta and the order of the atomics.
#include <algorithm>

#include <mutex>

#include "lg_device.hpp"

namespace lg {

// ---------------------------------------------------------------------------
// Weighted entries (subsections "Logarithmization of Edge Weights" and
// "Accessing an Edge Weight"): packed, each entry is the ID at its width w
// followed by the weight at omega bits; plain, the CSR plus a weight array.
// ---------------------------------------------------------------------------

// start: first bit (packed) or first index (plain); w: ID width
struct WInfo {
    uint64_t start;
    uint32_t deg;
    uint32_t w;
};

template <int IDM, int OFM>
struct WPackedAcc {
    PackedAcc<IDM, OFM> base;
    uint32_t omega;

    __device__ __forceinline__ WInfo info(uint32_t v) const {
        uint64_t o0, o1;
        base.offsets(v, o0, o1);
        WInfo r;
        if constexpr (IDM == kIdsGlobal) {
            r.w = base.pv.s;
            r.start = o0 * (uint64_t)(r.w + omega);
            r.deg = (uint32_t)(o1 - o0);
        } else {
            r.w = base.width(v);
            r.start = o0;
            r.deg = o1 > o0 ? (uint32_t)((o1 - o0) / (uint64_t)(r.w + omega)) : 0u;
        }
        return r;
    }
    __device__ __forceinline__ void entry(uint64_t start, uint32_t w, uint64_t i, uint32_t &id, uint32_t &wt) const {
        const uint64_t b = start + i * (uint64_t)(w + omega);
        id = base.get(b, width_mask(w));
        wt = base.get(b + w, width_mask(omega));
    }
};

template <bool OFF64>
struct WPlainAcc {
    PlainAcc<OFF64> base;
    const uint32_t *wt;

    __device__ __forceinline__ WInfo info(uint32_t v) const {
        const VInfo vi = base.info(v);
        return WInfo{vi.start, vi.deg, 32u};
    }
    __device__ __forceinline__ void entry(uint64_t start, uint32_t, uint64_t i, uint32_t &id, uint32_t &w) const {
        id = base.pv.col[start + i];
        w = wt[start + i];
    }
};

template <class Fn>
lg_status dispatch_wacc(const lg_graph *g, Fn &&fn) {
    if (!g->weighted) {
        set_error("the graph has no edge weights (build it with lg_encode_weighted)");
        return LG_ERR_UNSUPPORTED;
    }
    if (g->layout == LG_LAYOUT_PLAIN) {
        const uint32_t *wt = g->pwt.as<uint32_t>();
        if (g->poff64) return fn(WPlainAcc<true>{PlainAcc<true>{g->plain_view()}, wt});
        return fn(WPlainAcc<false>{PlainAcc<false>{g->plain_view()}, wt});
    }
    const PackedView pv = g->packed_view();
    const uint32_t om = g->omega;
    if (g->id_mode == LG_IDS_GLOBAL) {
        if (g->offset_mode == LG_OFFS_PACKED) return fn(WPackedAcc<kIdsGlobal, kOffsPacked>{{pv}, om});
        return fn(WPackedAcc<kIdsGlobal, kOffsEF>{{pv}, om});
    }
    if (g->offset_mode == LG_OFFS_PACKED) return fn(WPackedAcc<kIdsLocal, kOffsPacked>{{pv}, om});
    return fn(WPackedAcc<kIdsLocal, kOffsEF>{{pv}, om});
}

constexpr uint64_t kInfDist = ~0ull;

struct SsspWork {
    DevBuf upd;                         // bitmap, one bit per vertex
    DevBuf qv, qw, qdeg;                // frontier: vertex, ID width, degree
    DevBuf qstart, qdist, qoff;         // list start, distance, exclusive scan of qdeg
    DevBuf ctr;                         // [0] frontier size, [1] smallest distance left marked
    DevBuf tmask, wcnt, woff;           // per bitmap word: vertices taken, their count, queue position
    DevBuf dl;                          // label-space distances (relabeled graphs)
    DevBuf scan_tmp;
    uint64_t *host = nullptr;           // pinned readback slots
    SsspWork() = default;
    SsspWork(const SsspWork &) = delete;
    SsspWork &operator=(const SsspWork &) = delete;
    ~SsspWork() {
        if (host) (void)hipHostFree(host);
    }
    uint64_t bytes() const {
        return upd.bytes + qv.bytes + qw.bytes + qdeg.bytes + qstart.bytes + qdist.bytes + qoff.bytes + ctr.bytes +
               tmask.bytes + wcnt.bytes + woff.bytes + dl.bytes + scan_tmp.bytes;
    }
};

uint64_t sssp_bytes(const lg_graph *g) { return g->sssp ? g->sssp->bytes() : 0; }

lg_status sssp_free(lg_graph *g) {
    delete g->sssp;
    g->sssp = nullptr;
    return LG_OK;
}

// The root arrives as its original ID and is mapped to its label (inv,
// when relabeled) here.
__global__ void sssp_init_kernel(uint32_t n, uint64_t words, uint32_t root_id, const uint32_t *__restrict__ inv,
                                 uint64_t *__restrict__ dist, uint64_t *__restrict__ upd) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t total = n > words ? n : words;
    const uint32_t root = inv ? inv[root_id] : root_id;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        if (i < n) dist[i] = i == root ? 0ull : kInfDist;
        if (i < words) upd[i] = i == (root >> 6) ? 1ull << (root & 63) : 0ull;
    }
}

// ctr[0] = 0 (frontier size), ctr[1] = no marked distance left
__global__ void sssp_ctr_kernel(unsigned long long *__restrict__ ctr) {
    if (threadIdx.x == 0) {
        ctr[0] = 0ull;
        ctr[1] = kInfDist;
    }
}

// The frontier is compacted without a shared counter (one atomic add per
// wave on a single address serializes the whole pass): a count pass takes
// each word's marked vertices below the bound out of the bitmap and counts
// them, an exclusive scan over the words gives every word its queue
// position, and a write pass fills the queue.  Every marked vertex has edges
// (it was reached over one) but the root, which may have none: it is then
// alone in the first frontier, which holds no edges.
constexpr int kCollectThreads = 256;
constexpr uint32_t kCollectBlocks = 4096;

__global__ __launch_bounds__(kCollectThreads) void sssp_count_kernel(
    uint32_t n, uint64_t words, uint64_t hi, const uint64_t *__restrict__ dist, uint64_t *__restrict__ upd,
    uint64_t *__restrict__ tmask, uint32_t *__restrict__ cnt, unsigned long long *__restrict__ ctr) {
    __shared__ unsigned long long s_left[kCollectThreads / kWave];
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    uint64_t left = kInfDist;  // the smallest distance staying marked
    for (uint64_t q = wave; q < words; q += nwaves) {
        const uint64_t bits = upd[q];
        uint64_t take_m = 0;
        if (bits) {  // same for every lane
            const uint64_t v = q * 64 + lane;
            const bool set = ((bits >> lane) & 1ull) && v < n;
            const uint64_t d = set ? dist[v] : kInfDist;
            const bool take = set && d < hi;
            take_m = __ballot(take);
            if (set && !take && d < left) left = d;
            if (lane == 0 && take_m) upd[q] = bits & ~take_m;
        }
        if (lane == 0) {
            tmask[q] = take_m;
            cnt[q] = (uint32_t)__popcll(take_m);
        }
    }
#pragma unroll
    for (int s = kWave / 2; s > 0; s >>= 1) {
        const uint64_t o = __shfl_xor(left, s, kWave);
        left = o < left ? o : left;
    }
    if (lane == 0) s_left[threadIdx.x / kWave] = left;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = s_left[0];
        for (int i = 1; i < kCollectThreads / kWave; ++i) m = s_left[i] < m ? s_left[i] : m;
        if (m != kInfDist) atomicMin(&ctr[1], m);
    }
}

template <class Acc>
__global__ __launch_bounds__(kCollectThreads) void sssp_write_kernel(
    Acc acc, uint32_t n, uint64_t words, const uint64_t *__restrict__ dist, const uint64_t *__restrict__ tmask,
    const uint64_t *__restrict__ woff, uint32_t *__restrict__ qv, uint64_t *__restrict__ qstart, uint32_t *__restrict__ qw,
    uint32_t *__restrict__ qdeg, uint64_t *__restrict__ qdist, unsigned long long *__restrict__ ctr) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr[0] = woff[words];  // frontier size
    for (uint64_t q = wave; q < words; q += nwaves) {
        const uint64_t m = tmask[q];
        if (!m) continue;  // same for every lane
        if ((m >> lane) & 1ull) {
            const uint64_t v = q * 64 + lane;
            const WInfo vi = acc.info((uint32_t)v);
            const uint64_t pos = woff[q] + popc_below(m);
            qv[pos] = (uint32_t)v;
            qstart[pos] = vi.start;
            qw[pos] = vi.w;
            qdeg[pos] = vi.deg;
            qdist[pos] = dist[v];
        }
    }
}

// Edge t of the frontier belongs to slot s with qoff[s] <= t < qoff[s + 1];
// every slot holds at least one edge.  Each wave takes a contiguous range
// of edges, 64 per step, and finds its first slot by one binary search.  In
// a step starting at edge t0 in slot s0, lane j loads the boundary
// qoff[s0 + 1 + j]; the boundaries inside (t0, t0 + 64) form a bit mask
// (a wave sum of distinct bits), so the slot of edge t0 + i is s0 plus the
// number of mask bits at or below i, and the next step's slot is s0 plus
// the number of boundaries at or below t0 + 64.  No lane runs a search per
// edge.
template <class Acc>
__global__ void sssp_relax_kernel(Acc acc, uint32_t n, const uint64_t *__restrict__ count_p,
                                  const uint64_t *__restrict__ qoff, const uint32_t *__restrict__ qv,
                                  const uint64_t *__restrict__ qstart,
                                  const uint32_t *__restrict__ qw, const uint64_t *__restrict__ qdist,
                                  unsigned long long *__restrict__ dist, unsigned long long *__restrict__ upd) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    const uint64_t count = *count_p;
    const uint64_t E = qoff[count];
    const uint64_t per = ((E + nwaves - 1) / nwaves + kWave - 1) / kWave * kWave;
    const uint64_t tb = wave * per;
    if (tb >= E) return;  // same for every lane
    const uint64_t te = tb + per < E ? tb + per : E;
    uint64_t s0 = 0, hi = count;  // qoff[s0] <= tb < qoff[hi]
    while (hi - s0 > 1) {
        const uint64_t mid = s0 + (hi - s0) / 2;
        if (qoff[mid] <= tb) s0 = mid;
        else hi = mid;
    }
    const uint64_t below = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);  // bits 0..lane
    for (uint64_t t0 = tb; t0 < te; t0 += kWave) {
        const uint64_t j = s0 + 1 + lane;
        const uint64_t b = j <= count ? qoff[j] : ~0ull;  // > t0
        const uint64_t o = b - t0;
        const uint64_t M = wave_sum(o < kWave ? 1ull << o : 0ull);
        const uint64_t adv = (uint64_t)__popcll(__ballot(o <= kWave));
        const uint64_t t = t0 + lane;
        // a frontier vertex whose distance dropped again since it was
        // collected is marked again and relaxes next step from the lower
        // distance: its edges are skipped now
        const uint64_t a = s0 + (uint64_t)__popcll(M & below);
        if (t < te && dist[qv[a]] >= qdist[a]) {
            uint32_t id, w;
            acc.entry(qstart[a], qw[a], t - qoff[a], id, w);
            if (id < n) {  // only a corrupt stream fails this
                const unsigned long long nd = qdist[a] + (unsigned long long)w;
                if (nd < dist[id]) {
                    const unsigned long long old = atomicMin(&dist[id], nd);
                    if (nd < old) atomicOr(&upd[id >> 6], 1ull << (id & 63));
                }
            }
        }
        s0 += adv;
    }
}

// distances in original IDs: dist[o] = dist of label inv[o]
__global__ void sssp_unpermute_kernel(uint32_t n, const uint32_t *__restrict__ inv, const uint64_t *__restrict__ dl,
                                      uint64_t *__restrict__ dist) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += stride) dist[o] = dl[inv[o]];
}

}  // namespace lg

static lg_status lg_sssp_impl(const lg_graph *gc, uint32_t root, uint32_t delta, uint64_t *dist, hipStream_t stream) {
    using namespace lg;
    lg_graph *g = const_cast<lg_graph *>(gc);
    if (!g || !dist) { set_error("lg_sssp: NULL argument"); return LG_ERR_INVALID; }
    if (root >= g->n) { set_error("lg_sssp: root %u >= n", root); return LG_ERR_INVALID; }
    if (!g->weighted) {
        set_error("lg_sssp: the graph has no edge weights (build it with lg_encode_weighted)");
        return LG_ERR_UNSUPPORTED;
    }
    // default bucket width: the weight range 2^omega (one edge of the
    // heaviest weight spans about one bucket; 256 for 8-bit weights, the
    // best of a sweep on weights in [1, 255])
    const uint64_t D = delta ? delta : (1ull << g->omega);
    const uint32_t n = g->n;
    const uint64_t words = ((uint64_t)n + 63) / 64;
    // one workspace per graph: calls on the same graph run one at a time, and
    // each waits for its own last kernel before letting the next one in
    std::lock_guard<std::mutex> hold(g->sssp_mu);
    if (!g->sssp) {
        g->sssp = new (std::nothrow) SsspWork();
        if (!g->sssp) { set_error("lg_sssp: host allocation failed"); return LG_ERR_OOM; }
    }
    SsspWork &W = *g->sssp;
    if (!W.host) {
        if (hipHostMalloc((void **)&W.host, 4 * sizeof(uint64_t)) != hipSuccess) {
            W.host = nullptr;
            set_error("lg_sssp: pinned host allocation failed");
            return LG_ERR_OOM;
        }
    }
    LG_TRY(W.upd.ensure(words * 8));
    LG_TRY(W.tmask.ensure(words * 8));
    LG_TRY(W.wcnt.ensure(words * 4));
    LG_TRY(W.woff.ensure((words + 1) * 8));
    LG_TRY(W.qv.ensure((uint64_t)n * 4));
    LG_TRY(W.qw.ensure((uint64_t)n * 4));
    LG_TRY(W.qdeg.ensure((uint64_t)n * 4));
    LG_TRY(W.qstart.ensure((uint64_t)n * 8));
    LG_TRY(W.qdist.ensure((uint64_t)n * 8));
    LG_TRY(W.qoff.ensure(((uint64_t)n + 1) * 8));
    LG_TRY(W.ctr.ensure(16));
    // a relabeled graph runs in label space, then maps back
    const bool rel = g->relabel != LG_RELABEL_NONE;
    uint64_t *const dist_out = dist;
    if (rel) {
        LG_TRY(W.dl.ensure((uint64_t)n * 8));
        dist = W.dl.as<uint64_t>();
    }
    LG_LAUNCH(sssp_init_kernel, grid_for(std::max<uint64_t>(n, words), 256, 1u << 16), 256, 0, stream, n, words, root,
              rel ? (const uint32_t *)g->inv.as<uint32_t>() : (const uint32_t *)nullptr, dist, W.upd.as<uint64_t>());
    LG_CHECK_LAUNCH();
    return dispatch_wacc(g, [&](auto acc) -> lg_status {
        using Acc = decltype(acc);
        int cus = 0;
        LG_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
        const uint32_t collect_grid = grid_for(words * kWave, kCollectThreads, kCollectBlocks);
        const uint32_t relax_grid = (uint32_t)std::max(1, cus) * 8;
        uint64_t hi = D;
        // every step either relaxes a non-empty frontier (each entry of it
        // lowered a distance) or moves to a later bucket: bounded for
        // non-negative weights; the cap only guards against a corrupt graph
        const uint64_t cap = 64ull * n + 1024;
        for (uint64_t step = 0;; ++step) {
            if (step > cap) {
                set_error("lg_sssp: no convergence after %llu steps", (unsigned long long)step);
                return LG_ERR_DEVICE;
            }
            LG_LAUNCH(sssp_ctr_kernel, 1, 64, 0, stream, W.ctr.as<unsigned long long>());
            LG_CHECK_LAUNCH();
            LG_LAUNCH(sssp_count_kernel, collect_grid, kCollectThreads, 0, stream, n, words, hi,
                      (const uint64_t *)dist, W.upd.as<uint64_t>(), W.tmask.as<uint64_t>(), W.wcnt.as<uint32_t>(),
                      W.ctr.as<unsigned long long>());
            LG_CHECK_LAUNCH();
            LG_TRY(exclusive_scan_u32(W.wcnt.as<uint32_t>(), W.woff.as<uint64_t>(), words, W.scan_tmp, stream));
            LG_LAUNCH(sssp_write_kernel<Acc>, collect_grid, kCollectThreads, 0, stream, acc, n, words,
                      (const uint64_t *)dist, (const uint64_t *)W.tmask.as<uint64_t>(),
                      (const uint64_t *)W.woff.as<uint64_t>(), W.qv.as<uint32_t>(), W.qstart.as<uint64_t>(), W.qw.as<uint32_t>(),
                      W.qdeg.as<uint32_t>(), W.qdist.as<uint64_t>(), W.ctr.as<unsigned long long>());
            LG_CHECK_LAUNCH();
            LG_CHECK_HIP(hipMemcpyAsync(W.host, W.ctr.p, 16, hipMemcpyDeviceToHost, stream));
            LG_CHECK_HIP(hipStreamSynchronize(stream));
            const uint64_t count = W.host[0], left = W.host[1];
            if (count == 0) {
                if (left == kInfDist) break;
                const uint64_t k = left / D;
                hi = k + 1 > kInfDist / D ? kInfDist : (k + 1) * D;
                continue;
            }
            LG_TRY(exclusive_scan_u32(W.qdeg.as<uint32_t>(), W.qoff.as<uint64_t>(), count, W.scan_tmp, stream));
            LG_LAUNCH(sssp_relax_kernel<Acc>, relax_grid, 256, 0, stream, acc, n,
                      (const uint64_t *)W.ctr.as<uint64_t>(), (const uint64_t *)W.qoff.as<uint64_t>(),
                      (const uint32_t *)W.qv.as<uint32_t>(), (const uint64_t *)W.qstart.as<uint64_t>(), (const uint32_t *)W.qw.as<uint32_t>(),
                      (const uint64_t *)W.qdist.as<uint64_t>(), (unsigned long long *)dist,
                      W.upd.as<unsigned long long>());
            LG_CHECK_LAUNCH();
        }
        if (rel) {
            LG_LAUNCH(sssp_unpermute_kernel, grid_for(n, 256, 1u << 16), 256, 0, stream, n, g->inv.as<uint32_t>(),
                      (const uint64_t *)dist, dist_out);
            LG_CHECK_LAUNCH();
            LG_CHECK_HIP(hipStreamSynchronize(stream));
        }
        return LG_OK;
    });
}

extern "C" lg_status lg_sssp(const lg_graph *gc, uint32_t root, uint32_t delta, uint64_t *dist, hipStream_t stream) {
    LG_TRY(lg_sssp_impl(gc, root, delta, dist, stream));
    return lg::mark_use(const_cast<lg_graph *>(gc), stream);
}
