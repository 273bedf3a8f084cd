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
// Work split (bounded work per wave, whatever the degree distribution), in
// one kernel per iteration (pr_iter_kernel):
//   heavy vertices (degree > threshold) are cut into segments of seg_size edges;
//     one wave sums one segment and adds it, in fixed point, to its vertex's
//     64-bit accumulator; the last segment to arrive finalizes the vertex
//   light vertices are taken 64 consecutive vertices per wave; the wave's
//     lanes walk the chunk's (at most 64 * threshold) edges 64 at a time, so
//     consecutive lanes decode consecutive packed elements (coalesced), and a
//     lane's running sum is flushed to its vertex's LDS accumulator when the
//     owner changes
// All summation orders are fixed by the data: results repeat bit for bit.
#include "lg_device.hpp"

namespace lg {

constexpr int kPrThreads = 256;
constexpr int kPrWaves = kPrThreads / kWave;
constexpr int kBatch = 4;            // independent edges in flight per lane

struct PrWork {
    DevBuf ca, cb;                   // contrib ping-pong
    DevBuf acc;                      // per heavy vertex: arrivals | fixed-point sum
};

uint64_t pr_bytes(const lg_graph *g) {
    if (!g->pr) return 0;
    const PrWork *w = g->pr;
    return w->ca.bytes + w->cb.bytes + w->acc.bytes;
}

lg_status pr_free(lg_graph *g) {
    delete g->pr;
    g->pr = nullptr;
    return LG_OK;
}

template <class Acc>
__global__ void pr_init_kernel(Acc acc, uint32_t n, double inv_n, float *__restrict__ contrib) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v0 = (uint64_t)blockIdx.x * blockDim.x; v0 < n; v0 += stride) {
        const uint64_t w0 = v0 + (threadIdx.x & ~(uint64_t)(kWave - 1));
        const VInfo vi = wave_info(acc, w0, n);
        const uint64_t v = w0 + lane_id();
        if (v < n) contrib[v] = vi.deg ? (float)(inv_n / (double)vi.deg) : 0.0f;
    }
}

// One launch per iteration, two kinds of blocks running side by side:
//   blocks [0, heavy_blocks): a wave per heavy segment sums its contributions
//     and adds them to its vertex's accumulator; the arrival that completes a
//     vertex finalizes it
//   the other blocks: 64 consecutive vertices per wave, lanes walk the
//     light lists edge-parallel, flushing running sums to LDS accumulators
//     when the owner changes, then finalize every light vertex
template <class Acc>
__global__ __launch_bounds__(kPrThreads) void pr_iter_kernel(
    Acc acc, uint32_t n, uint32_t threshold, const float *__restrict__ cin, float *__restrict__ cout, float base,
    float alpha, uint32_t heavy_blocks, uint32_t seg_size, const uint32_t *__restrict__ heavy, uint64_t n_seg,
    const uint32_t *__restrict__ seg_map, const uint64_t *__restrict__ seg_off, const uint64_t *__restrict__ hstart,
    const uint32_t *__restrict__ hdeg, const uint32_t *__restrict__ hw, unsigned long long *__restrict__ hsum,
    float *__restrict__ scores, const uint32_t *__restrict__ perm) {
    __shared__ uint32_t s_excl[kPrWaves][kWave + 1];
    __shared__ uint64_t s_start[kPrWaves][kWave];
    __shared__ uint32_t s_w[kPrWaves][kWave];
    __shared__ float s_acc[kPrWaves][kWave];
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    if (blockIdx.x < heavy_blocks) {
        const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
        const uint64_t nwaves = (uint64_t)heavy_blocks * (kPrThreads / kWave);
        for (uint64_t k = wave; k < n_seg; k += nwaves) {
            const uint32_t h = seg_map[k];
            const uint64_t s0 = seg_off[h], s1 = seg_off[h + 1];
            const uint64_t e0 = (k - s0) * seg_size;
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
                for (int b = 0; b < kBatch; ++b) x[b] = u[b] != 0xFFFFFFFFu ? cin[u[b]] : 0.0f;
#pragma unroll
                for (int b = 0; b < kBatch; ++b) sum += x[b];
            }
            sum = wave_sum(sum);
            if (lane == 0) {
                // One integer atomic carries both the segment's sum, as a
                // fixed-point value with 2^-46 resolution in the low 48 bits
                // (a vertex's total is at most 1), and an arrival count in the
                // high 16 bits (at most 65535 segments per vertex).  Integer
                // addition does not depend on arrival order, and the last
                // arrival reads the total from the atomic's own result: no
                // fence, no cross-XCD data reads.
                const uint64_t fixed = (uint64_t)__double2ll_rn((double)sum * 0x1p46);
                const unsigned long long add = (1ull << 48) | fixed;
                const unsigned long long now = atomicAdd(&hsum[h], add) + add;
                if ((now >> 48) == s1 - s0) {
                    const double hs = (double)(now & ((1ull << 48) - 1)) * 0x1p-46;
                    const uint32_t v = heavy[h];
                    const float pr = base + alpha * (float)hs;
                    cout[v] = pr / (float)d;
                    if (scores) scores[perm ? perm[v] : v] = pr;
                    hsum[h] = 0ull;  // ready for the next launch
                }
            }
        }
        return;
    }
    const uint64_t nchunks = ((uint64_t)n + kPrThreads - 1) / kPrThreads;
    const uint32_t lblocks = gridDim.x - heavy_blocks;
    for (uint64_t c = blockIdx.x - heavy_blocks; c < nchunks; c += lblocks) {
        const uint64_t w0 = c * kPrThreads + (uint64_t)wv * kWave;
        const uint64_t v = w0 + lane;
        const VInfo vi = wave_info(acc, w0, n);
        const bool is_heavy = vi.deg > threshold;
        const uint32_t d = is_heavy ? 0u : vi.deg;  // heavy lists are summed by segments
        const uint32_t incl = wave_incl_scan(d);
        const uint32_t total = __shfl(incl, kWave - 1, kWave);
        s_excl[wv][lane] = incl - d;
        if (lane == kWave - 1) s_excl[wv][kWave] = total;
        s_start[wv][lane] = vi.start;
        s_w[wv][lane] = vi.w;
        s_acc[wv][lane] = 0.0f;
        __syncthreads();
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
            for (int b = 0; b < kBatch; ++b) x[b] = own[b] != 0xFFFFFFFFu ? cin[u[b]] : 0.0f;
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
        __syncthreads();
        if (v < n && !is_heavy) {
            const float pr = base + alpha * s_acc[wv][lane];
            cout[v] = vi.deg ? pr / (float)vi.deg : 0.0f;
            if (scores) scores[perm ? perm[v] : v] = pr;
        }
        __syncthreads();
    }
}

__global__ void pr_fill_kernel(uint32_t n, float value, float *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) out[v] = value;
}

}  // namespace lg

extern "C" lg_status lg_pagerank(const lg_graph *gc, float damping, uint32_t iters, float *scores,
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
    if (!g->pr) {
        g->pr = new (std::nothrow) PrWork();
        if (!g->pr) { set_error("lg_pagerank: host allocation failed"); return LG_ERR_OOM; }
    }
    LG_TRY(g->pr->ca.ensure((uint64_t)n * 4));
    LG_TRY(g->pr->cb.ensure((uint64_t)n * 4));
    LG_TRY(ensure_heavy_segments(g, stream));
    LG_TRY(g->pr->acc.ensure((uint64_t)(g->n_heavy ? g->n_heavy : 1) * 8));
    LG_TRY(fill_u64(g->pr->acc.as<uint64_t>(), 0, g->n_heavy ? g->n_heavy : 1, stream));
    const uint32_t *perm = g->relabel == LG_RELABEL_DEGREE ? g->perm.as<uint32_t>() : nullptr;
    const double a = damping;
    const double z = g->isolated;
    return dispatch_acc(g, [&](auto acc) -> lg_status {
        using Acc = decltype(acc);
        PrWork &w = *g->pr;
        float *cin = w.ca.as<float>(), *cout = w.cb.as<float>();
        LG_LAUNCH(pr_init_kernel<Acc>, grid_for(n, 256, 1u << 16), 256, 0, stream, acc, n, 1.0 / nd, cin);
        LG_CHECK_LAUNCH();
        double D = z / nd;  // D_0: rank on vertices without edges
        // heavy blocks: enough waves for the segments, capped; light blocks: one
        // per 256-vertex chunk, capped (both loops are grid-stride)
        const uint32_t heavy_blocks = g->n_seg ? grid_for(g->n_seg, kPrThreads / kWave, 8192) : 0;
        const uint32_t light_blocks = grid_for(n, kPrThreads, 8192);
        for (uint32_t t = 0; t < iters; ++t) {
            const double b = (1.0 - a) / nd + a * D / nd;
            const bool last = t + 1 == iters;
            LG_LAUNCH(pr_iter_kernel<Acc>, heavy_blocks + light_blocks, kPrThreads, 0, stream, acc, n,
                      g->heavy_threshold, (const float *)cin, cout, (float)b, (float)a, heavy_blocks, g->seg_size,
                      (const uint32_t *)g->heavy.p, g->n_seg, (const uint32_t *)g->seg_map.p,
                      (const uint64_t *)g->seg_off.p, (const uint64_t *)g->hstart.p, (const uint32_t *)g->hdeg.p,
                      (const uint32_t *)g->hw.p, w.acc.as<unsigned long long>(),
                      last ? scores : (float *)nullptr, last ? perm : (const uint32_t *)nullptr);
            LG_CHECK_LAUNCH();
            D = z * b;
            float *tmp = cin; cin = cout; cout = tmp;
        }
        return LG_OK;
    });
}
