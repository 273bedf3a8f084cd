// lg_pagerank: pull PageRank without atomics on global memory (PR of
// section "Considered Algorithms"), FP32 storage, decoding every list inside
// the pull kernels.
//
//   PR_0 = 1/n
//   PR_{t+1}(v) = (1-a)/n + a (sum_{u in N_v} PR_t(u)/d_u + D_t/n)
//
// An iteration reads contrib_t[u] = PR_t(u)/d_u and writes contrib_{t+1};
// the final one also writes the scores.  All vertices without edges hold the
// same value b_t = (1-a)/n + a D_t/n, so the dangling mass follows
// D_{t+1} = z b_t (z = number of such vertices) and is passed to the kernels
// as a scalar instead of being reduced over the graph.
//
// Work split, bounded work per wave whatever the degree distribution (the
// tables are built once per graph, see lg_heavy.hip):
//   lists longer than pr_split are cut into segments of seg_size edges; one
//     wave sums one segment and stores the sum in that segment's slot
//   all other vertices come in units (consecutive vertices of one 64-aligned
//     block, about pr_unit_edges edges in total); the wave's lanes walk the
//     unit's edges 64 at a time, so consecutive lanes decode consecutive
//     packed elements (coalesced), and a lane's running sum is flushed to its
//     vertex's LDS accumulator when the owner changes; the wave then
//     finalizes the unit's vertices
//   a second, small kernel adds up every segmented vertex's slots, in
//     segment order, and finalizes it
// Each workgroup first copies the contributions of the smallest labels into
// LDS.  Waves then take segments, then units, by static interleaving and
// never wait for each other; every sum is taken in an order fixed by the
// data, so results repeat bit for bit.
#include <algorithm>

#include "lg_device.hpp"
#include "lg_varint.hpp"

namespace lg {

constexpr int kPrThreads = 512;
constexpr int kPrWaves = kPrThreads / kWave;
constexpr int kBatch = 4;           // independent edges in flight per lane
constexpr uint32_t kPrHot = 16384;  // contributions each workgroup keeps in LDS (64 KiB)

struct PrWork {
    DevBuf ca, cb;  // contrib ping-pong
};

uint64_t pr_bytes(const lg_graph *g) {
    if (!g->pr) return 0;
    const PrWork *w = g->pr;
    return w->ca.bytes + w->cb.bytes;
}

lg_status pr_free(lg_graph *g) {
    delete g->pr;
    g->pr = nullptr;
    return LG_OK;
}

// contrib_0 = PR_0 / d in both ping-pong buffers (zero for vertices without
// edges, which the iterations then leave alone when a whole word of them)
template <class Acc>
__global__ void pr_init_kernel(Acc acc, uint32_t n, double inv_n, float *__restrict__ contrib,
                               float *__restrict__ contrib2) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v0 = (uint64_t)blockIdx.x * blockDim.x; v0 < n; v0 += stride) {
        const uint64_t w0 = v0 + (threadIdx.x & ~(uint64_t)(kWave - 1));
        const uint64_t v = w0 + lane_id();
        uint32_t deg;
        if constexpr (IsGapAcc<Acc>::value) deg = v < n ? acc.info((uint32_t)v).deg : 0u;
        else deg = wave_info(acc, w0, n).deg;
        if (v < n) {
            const float c = deg ? (float)(inv_n / (double)deg) : 0.0f;
            contrib[v] = c;
            contrib2[v] = c;
        }
    }
}

// Lanes of one wave exchange data through its own LDS rows: keep the
// compiler from moving LDS accesses across this point (a wave's LDS
// operations complete in order).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One launch per iteration: every wave of the grid takes segments
// (grid-stride), then units (grid-stride).
template <class Acc>
__global__ __launch_bounds__(kPrThreads) void pr_iter_kernel(
    Acc acc, uint32_t n, uint32_t split, const float *__restrict__ cin, float *__restrict__ cout, float base,
    float alpha, uint32_t seg_size, uint64_t n_seg, const uint32_t *__restrict__ seg_map,
    const uint64_t *__restrict__ seg_off, const uint64_t *__restrict__ hstart, const uint32_t *__restrict__ hdeg,
    const uint32_t *__restrict__ hw, float *__restrict__ seg_part, uint64_t n_units,
    const uint32_t *__restrict__ units, const uint64_t *__restrict__ iso, float *__restrict__ scores,
    const uint32_t *__restrict__ perm) {
    __shared__ float s_hot[kPrHot];
    __shared__ uint32_t s_excl[kPrWaves][kWave + 1];
    __shared__ uint64_t s_start[kPrWaves][kWave];
    __shared__ uint32_t s_w[kPrWaves][kWave];
    __shared__ float s_acc[kPrWaves][kWave];
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    // A divergent 4-byte gather from global memory costs a whole cache-line
    // fill of the vector L1; from LDS it costs a bank access.  The smallest
    // labels are the highest-degree vertices after the degree-descending
    // relabel (the sources of about a quarter of all gathers at Kronecker
    // scale 24), so their contributions are read from an LDS copy.
    const uint32_t hot = kPrHot < n ? kPrHot : n;
    for (uint32_t i = threadIdx.x; i < hot; i += kPrThreads) s_hot[i] = cin[i];
    __syncthreads();
    auto gather = [&](uint32_t u) -> float { return u < hot ? s_hot[u] : cin[u]; };
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = (uint64_t)gridDim.x * kPrWaves;
    for (uint64_t k = wave; k < n_seg; k += nwaves) {
        const uint32_t h = seg_map[k];
        const uint64_t e0 = (k - seg_off[h]) * seg_size;
        const uint64_t d = hdeg[h];
        const uint64_t e1 = e0 + seg_size < d ? e0 + seg_size : d;
        const uint32_t w = hw[h];
        const uint64_t start = hstart[h];
        const uint32_t st = Acc::step(w), mk = Acc::mask(w);
        float sum = 0.0f;
        for (uint64_t e = e0 + lane; e < e1; e += kWave * kBatch) {
            uint32_t u[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const uint64_t eb = e + (uint64_t)b * kWave;
                u[b] = eb < e1 ? acc.get(start + eb * st, mk) : 0xFFFFFFFFu;
            }
            float x[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) x[b] = u[b] != 0xFFFFFFFFu ? gather(u[b]) : 0.0f;
#pragma unroll
            for (int b = 0; b < kBatch; ++b) sum += x[b];
        }
        sum = wave_sum(sum);
        if (lane == 0) seg_part[k] = sum;
    }
    for (uint64_t k = wave; k < n_units; k += nwaves) {
        const uint32_t vb = units[k], ve = units[k + 1];
        const uint64_t w0 = vb & ~(uint64_t)(kWave - 1);
        const uint64_t v = w0 + lane;
        const bool mine = v >= vb && v < ve;
        // a block of vertices without edges: contrib stays 0, only scores change
        const bool all_iso = iso[w0 / kWave] == ~0ull;
        EFSamples smp{0, 0};
        if constexpr (Acc::kPacked && Acc::kEF) smp = ef_samples(acc.pv.ef, w0, n + 1);
        if (all_iso && !scores) continue;
        const VInfo vi = all_iso ? VInfo{0, 0, 0} : wave_info(acc, w0, n, &smp);
        const bool segmented = vi.deg > split;
        const uint32_t d = (mine && !segmented) ? vi.deg : 0u;
        const uint32_t incl = wave_incl_scan(d);
        const uint32_t total = __shfl(incl, kWave - 1, kWave);
        s_excl[wv][lane] = incl - d;
        if (lane == kWave - 1) s_excl[wv][kWave] = total;
        s_start[wv][lane] = vi.start;
        s_w[wv][lane] = vi.w;
        s_acc[wv][lane] = 0.0f;
        wave_lds_sync();
        uint32_t j = 0, owner = 0xFFFFFFFFu;
        float part = 0.0f;
        for (uint32_t e = lane; e < total; e += kWave * kBatch) {
            uint32_t u[kBatch], own[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const uint32_t eb = e + (uint32_t)b * kWave;
                own[b] = 0xFFFFFFFFu;
                u[b] = 0;
                if (eb < total) {
                    while (s_excl[wv][j + 1] <= eb) ++j;
                    const uint32_t w = s_w[wv][j];
                    u[b] = acc.get(s_start[wv][j] + (uint64_t)(eb - s_excl[wv][j]) * Acc::step(w), Acc::mask(w));
                    own[b] = j;
                }
            }
            float x[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) x[b] = own[b] != 0xFFFFFFFFu ? gather(u[b]) : 0.0f;
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                if (own[b] == 0xFFFFFFFFu) continue;
                if (own[b] != owner) {
                    if (owner != 0xFFFFFFFFu) atomicAdd(&s_acc[wv][owner], part);
                    owner = own[b];
                    part = 0.0f;
                }
                part += x[b];
            }
        }
        if (owner != 0xFFFFFFFFu) atomicAdd(&s_acc[wv][owner], part);
        wave_lds_sync();
        if (mine && !segmented) {
            const float pr = base + alpha * s_acc[wv][lane];
            if (!all_iso) cout[v] = vi.deg ? pr / (float)vi.deg : 0.0f;
            if (scores) scores[perm ? perm[v] : v] = pr;
        }
        wave_lds_sync();
    }
}

// The same iteration over gap-encoded lists (first element, then the
// differences between neighbours, section "Fixed-Size Gap Encoding"): every
// 64 consecutive entries a wave decodes, a wave prefix sum turns into
// neighbour IDs.  A segment's prefix starts from the value of the entry before
// it (seg_base, built with the tables); in a unit the prefix restarts at each
// list's first entry and otherwise carries the last value of the previous 64
// entries.
template <class Acc>
__global__ __launch_bounds__(kPrThreads) void pr_iter_gap_kernel(
    Acc acc, uint32_t n, uint32_t split, const float *__restrict__ cin, float *__restrict__ cout, float base,
    float alpha, uint32_t seg_size, uint64_t n_seg, const uint32_t *__restrict__ seg_map,
    const uint64_t *__restrict__ seg_off, const uint64_t *__restrict__ hstart, const uint32_t *__restrict__ hdeg,
    const uint32_t *__restrict__ hw, const uint32_t *__restrict__ hg, const uint32_t *__restrict__ seg_base,
    float *__restrict__ seg_part, uint64_t n_units, const uint32_t *__restrict__ units,
    const uint64_t *__restrict__ iso, float *__restrict__ scores, const uint32_t *__restrict__ perm) {
    __shared__ float s_hot[kPrHot];
    __shared__ uint32_t s_excl[kPrWaves][kWave + 1];
    __shared__ uint64_t s_start[kPrWaves][kWave];
    __shared__ uint32_t s_w[kPrWaves][kWave];
    __shared__ uint32_t s_g[kPrWaves][kWave];
    __shared__ float s_acc[kPrWaves][kWave];
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t hot = kPrHot < n ? kPrHot : n;
    for (uint32_t i = threadIdx.x; i < hot; i += kPrThreads) s_hot[i] = cin[i];
    __syncthreads();
    const uint32_t last = n - 1;
    // a decoded ID outside [0, n) only comes from a corrupt stream; clamp it
    // so that the gather stays inside the buffer
    auto gather = [&](uint32_t u) -> float {
        u = u < n ? u : last;
        return u < hot ? s_hot[u] : cin[u];
    };
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = (uint64_t)gridDim.x * kPrWaves;
    for (uint64_t k = wave; k < n_seg; k += nwaves) {
        const uint32_t h = seg_map[k];
        const uint64_t e0 = (k - seg_off[h]) * seg_size;
        const uint64_t d = hdeg[h];
        const uint64_t e1 = e0 + seg_size < d ? e0 + seg_size : d;
        const GapInfo gi{hstart[h], (uint32_t)d, hw[h], hg[h]};
        uint32_t carry = seg_base[k];
        float sum = 0.0f;
        for (uint64_t e = e0 + lane; e < e1 + lane; e += kWave * kBatch) {
            uint32_t x[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const uint64_t eb = e + (uint64_t)b * kWave;
                x[b] = eb < e1 ? acc.get(Acc::entry_bit(gi, eb), eb == 0 ? gi.w : gi.g) : 0u;
            }
            uint32_t u[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                u[b] = carry + wave_incl_scan(x[b]);
                carry = __shfl(u[b], kWave - 1, kWave);
            }
            float y[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) y[b] = e + (uint64_t)b * kWave < e1 ? gather(u[b]) : 0.0f;
#pragma unroll
            for (int b = 0; b < kBatch; ++b) sum += y[b];
        }
        sum = wave_sum(sum);
        if (lane == 0) seg_part[k] = sum;
    }
    for (uint64_t k = wave; k < n_units; k += nwaves) {
        const uint32_t vb = units[k], ve = units[k + 1];
        const uint64_t w0 = vb & ~(uint64_t)(kWave - 1);
        const uint64_t v = w0 + lane;
        const bool mine = v >= vb && v < ve;
        const bool all_iso = iso[w0 / kWave] == ~0ull;
        if (all_iso && !scores) continue;
        // the block's 65 offsets decoded by the whole wave (one select with
        // Elias-Fano offsets, not one per lane)
        GapInfo gi{0, 0, 0, 0};
        if (!all_iso) {  // same for every lane
            uint64_t o0, o1;
            wave_offsets(acc.base, w0, n, o0, o1);
            if (v < n && o1 > o0) {
                gi.start = o0;
                gi.w = acc.base.width((uint32_t)v);
                gi.g = acc.gap_width((uint32_t)v);
                gi.deg = gi.g == 0 ? 1u : 1u + exact_div_width(o1 - o0 - gi.w, gi.g);
            }
        }
        const bool segmented = gi.deg > split;
        const uint32_t d = (mine && !segmented) ? gi.deg : 0u;
        const uint32_t incl = wave_incl_scan(d);
        const uint32_t total = __shfl(incl, kWave - 1, kWave);
        s_excl[wv][lane] = incl - d;
        if (lane == kWave - 1) s_excl[wv][kWave] = total;
        s_start[wv][lane] = gi.start;
        s_w[wv][lane] = gi.w;
        s_g[wv][lane] = gi.g;
        s_acc[wv][lane] = 0.0f;
        wave_lds_sync();
        uint32_t j = 0, owner = 0xFFFFFFFFu, carry = 0;
        float part = 0.0f;
        // every lane runs the same number of passes: the scans need all lanes
        for (uint32_t e0 = 0; e0 < total; e0 += kWave * kBatch) {
            uint32_t x[kBatch], own[kBatch], head[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const uint32_t eb = e0 + lane + (uint32_t)b * kWave;
                own[b] = 0xFFFFFFFFu;
                x[b] = 0;
                head[b] = 0xFFFFFFFFu;  // lane of this list's first entry in the same 64, if any
                if (eb < total) {
                    while (s_excl[wv][j + 1] <= eb) ++j;
                    const uint32_t i = eb - s_excl[wv][j];
                    const GapInfo gj{s_start[wv][j], 0u, s_w[wv][j], s_g[wv][j]};
                    x[b] = acc.get(Acc::entry_bit(gj, i), i == 0 ? gj.w : gj.g);
                    own[b] = j;
                    const uint32_t c0 = e0 + (uint32_t)b * kWave;  // first position of these 64
                    if (s_excl[wv][j] >= c0) head[b] = s_excl[wv][j] - c0;
                }
            }
            uint32_t u[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const uint32_t p = wave_incl_scan(x[b]);
                // prefix up to the lane before the list's first entry
                const uint32_t hb = head[b] != 0xFFFFFFFFu && head[b] > 0 ? head[b] - 1 : 0u;
                const uint32_t before = __shfl(p, (int)hb, kWave);
                u[b] = head[b] == 0xFFFFFFFFu ? carry + p : (head[b] > 0 ? p - before : p);
                carry = __shfl(u[b], kWave - 1, kWave);
            }
            float y[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) y[b] = own[b] != 0xFFFFFFFFu ? gather(u[b]) : 0.0f;
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                if (own[b] == 0xFFFFFFFFu) continue;
                if (own[b] != owner) {
                    if (owner != 0xFFFFFFFFu) atomicAdd(&s_acc[wv][owner], part);
                    owner = own[b];
                    part = 0.0f;
                }
                part += y[b];
            }
        }
        if (owner != 0xFFFFFFFFu) atomicAdd(&s_acc[wv][owner], part);
        wave_lds_sync();
        if (mine && !segmented) {
            const float pr = base + alpha * s_acc[wv][lane];
            if (!all_iso) cout[v] = gi.deg ? pr / (float)gi.deg : 0.0f;
            if (scores) scores[perm ? perm[v] : v] = pr;
        }
        wave_lds_sync();
    }
}

// Segmented vertices: the sum of their segments' slots, in segment order.
__global__ void pr_segmented_kernel(uint32_t n_heavy, const uint32_t *__restrict__ heavy,
                                    const uint64_t *__restrict__ seg_off, const uint32_t *__restrict__ hdeg,
                                    const float *__restrict__ seg_part, float base, float alpha,
                                    float *__restrict__ cout, float *__restrict__ scores,
                                    const uint32_t *__restrict__ perm) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n_heavy; h += stride) {
        const uint64_t s0 = seg_off[h], s1 = seg_off[h + 1];
        if (s0 == s1) continue;
        float sum = 0.0f;
        for (uint64_t k = s0; k < s1; ++k) sum += seg_part[k];
        const uint32_t v = heavy[h];
        const float pr = base + alpha * sum;
        cout[v] = pr / (float)hdeg[h];
        if (scores) scores[perm ? perm[v] : v] = pr;
    }
}

__global__ void pr_fill_kernel(uint32_t n, float value, float *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) out[v] = value;
}

}  // namespace lg

static lg_status lg_pagerank_impl(const lg_graph *gc, float damping, uint32_t iters, float *scores,
                                 hipStream_t stream) {
    using namespace lg;
    lg_graph *g = const_cast<lg_graph *>(gc);
    if (!g || !scores) { set_error("lg_pagerank: NULL argument"); return LG_ERR_INVALID; }
    if (!(damping >= 0.0f && damping <= 1.0f)) { set_error("lg_pagerank: damping outside [0, 1]"); return LG_ERR_INVALID; }
    const uint32_t n = g->n;
    const double nd = (double)n;
    if (iters == 0) {
        LG_LAUNCH(pr_fill_kernel, grid_for(n, 256, 1u << 16), 256, 0, stream, n, (float)(1.0 / nd), scores);
        LG_CHECK_LAUNCH();
        return LG_OK;
    }
    if (g->layout == LG_LAYOUT_PACKED && (g->id_mode == LG_IDS_VARINT_FULL || g->id_mode == LG_IDS_VARINT_DIFF))
        return pagerank_varint(g, damping, iters, scores, stream);
    // contributions without locality (large unrelabeled graphs): streamed
    // through destination bins instead of gathered
    if (pb_applies(g)) return pagerank_pb(g, damping, iters, scores, stream);
    if (!g->pr) {
        g->pr = new (std::nothrow) PrWork();
        if (!g->pr) { set_error("lg_pagerank: host allocation failed"); return LG_ERR_OOM; }
    }
    if (g->pr->ca.bytes < (uint64_t)n * 4) LG_TRY(g->pr->ca.scratch((uint64_t)n * 4, stream));
    if (g->pr->cb.bytes < (uint64_t)n * 4) LG_TRY(g->pr->cb.scratch((uint64_t)n * 4, stream));
    LG_TRY(ensure_heavy_segments(g, stream));
    const uint32_t *perm = g->relabel != LG_RELABEL_NONE ? g->perm.as<uint32_t>() : nullptr;
    const double a = damping;
    const double z = g->isolated;
    return dispatch_acc_all(g, [&](auto acc) -> lg_status {
        using Acc = decltype(acc);
        constexpr bool kGap = IsGapAcc<Acc>::value;
        PrWork &w = *g->pr;
        float *cin = w.ca.as<float>(), *cout = w.cb.as<float>();
        LG_LAUNCH(pr_init_kernel<Acc>, grid_for(n, 256, 1u << 16), 256, 0, stream, acc, n, 1.0 / nd, cin, cout);
        LG_CHECK_LAUNCH();
        double D = z / nd;  // D_0: rank on vertices without edges
        // persistent grid: as many workgroups as fit on the device at once,
        // fewer when there is little work
        int cus = 0, per_cu = 0;
        LG_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
        if constexpr (kGap)
            LG_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pr_iter_gap_kernel<Acc>, kPrThreads, 0));
        else
            LG_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pr_iter_kernel<Acc>, kPrThreads, 0));
        const uint64_t want = (g->n_units + g->n_seg + kPrWaves - 1) / kPrWaves;
        const uint32_t blocks =
            (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)std::max(cus, 1) * std::max(per_cu, 1), want));
        for (uint32_t t = 0; t < iters; ++t) {
            const double b = (1.0 - a) / nd + a * D / nd;
            const bool last = t + 1 == iters;
            float *sc = last ? scores : (float *)nullptr;
            const uint32_t *pm = last ? perm : (const uint32_t *)nullptr;
            if constexpr (kGap) {
                LG_LAUNCH(pr_iter_gap_kernel<Acc>, blocks, kPrThreads, 0, stream, acc, n, g->pr_split,
                          (const float *)cin, cout, (float)b, (float)a, g->seg_size, g->n_seg,
                          (const uint32_t *)g->seg_map.p, (const uint64_t *)g->seg_off.p,
                          (const uint64_t *)g->hstart.p, (const uint32_t *)g->hdeg.p, (const uint32_t *)g->hw.p,
                          (const uint32_t *)g->hg.p, (const uint32_t *)g->seg_base.p, g->seg_part.as<float>(),
                          g->n_units, (const uint32_t *)g->units.p, g->iso.as<uint64_t>(), sc, pm);
            } else {
                LG_LAUNCH(pr_iter_kernel<Acc>, blocks, kPrThreads, 0, stream, acc, n, g->pr_split,
                          (const float *)cin, cout, (float)b, (float)a, g->seg_size, g->n_seg,
                          (const uint32_t *)g->seg_map.p, (const uint64_t *)g->seg_off.p,
                          (const uint64_t *)g->hstart.p, (const uint32_t *)g->hdeg.p, (const uint32_t *)g->hw.p,
                          g->seg_part.as<float>(), g->n_units, (const uint32_t *)g->units.p, g->iso.as<uint64_t>(),
                          sc, pm);
            }
            LG_CHECK_LAUNCH();
            if (g->n_seg) {
                LG_LAUNCH(pr_segmented_kernel, grid_for(g->n_heavy, 256, 4096), 256, 0, stream, g->n_heavy,
                          (const uint32_t *)g->heavy.p, (const uint64_t *)g->seg_off.p, (const uint32_t *)g->hdeg.p,
                          (const float *)g->seg_part.p, (float)b, (float)a, cout, sc, pm);
                LG_CHECK_LAUNCH();
            }
            D = z * b;
            float *tmp = cin; cin = cout; cout = tmp;
        }
        return LG_OK;
    });
}

extern "C" lg_status lg_pagerank(const lg_graph *gc, float damping, uint32_t iters, float *scores,
                                 hipStream_t stream) {
    LG_TRY(lg_pagerank_impl(gc, damping, iters, scores, stream));
    return lg::mark_use(const_cast<lg_graph *>(gc), stream);
}
