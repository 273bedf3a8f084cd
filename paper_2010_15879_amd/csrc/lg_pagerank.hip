// lg_pagerank: pull PageRank without atomics on global memory (PR of
// section "Considered Algorithms"), FP32 storage, decoding every list inside
// the pull kernel.
//
//   PR_0 = 1/n
//   PR_{t+1}(v) = (1-a)/n + a (sum_{u in N_v} PR_t(u)/d_u + D_t/n)
//
// Each iteration is one kernel.  It reads contrib_t[u] = PR_t(u)/d_u and
// writes contrib_{t+1}[v]; the final iteration also writes the scores.  All
// vertices without edges hold the same value, b_t = (1-a)/n + a D_t/n, so the
// dangling mass follows D_{t+1} = z b_t (z = number of such vertices) and is
// passed to the kernel as a scalar instead of being reduced over the graph.
//
// Work split: a wave owns 64 consecutive vertices.  It scans their degrees,
// then its lanes walk the chunk's edges 64 at a time (consecutive lanes read
// consecutive packed elements, so the stream is coalesced).  A lane keeps a
// running sum while its edges belong to one vertex and adds it to that
// vertex's LDS accumulator when the owner changes; the accumulation order is
// fixed by the data, so results are reproducible run to run.
#include "lg_device.hpp"

namespace lg {

struct PrWork {
    DevBuf ca, cb;  // contrib ping-pong
};

uint64_t pr_bytes(const lg_graph *g) { return g->pr ? g->pr->ca.bytes + g->pr->cb.bytes : 0; }

lg_status pr_free(lg_graph *g) {
    delete g->pr;
    g->pr = nullptr;
    return LG_OK;
}

constexpr int kPrThreads = 256;
constexpr int kPrWaves = kPrThreads / kWave;

template <class Acc>
__global__ void pr_init_kernel(Acc acc, uint32_t n, double inv_n, float *__restrict__ contrib) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint32_t d = acc.info((uint32_t)v).deg;
        contrib[v] = d ? (float)(inv_n / (double)d) : 0.0f;
    }
}

template <class Acc>
__global__ __launch_bounds__(kPrThreads) void pr_pull_kernel(Acc acc, uint32_t n, const float *__restrict__ cin,
                                                             float *__restrict__ cout, float base, float alpha,
                                                             float *__restrict__ scores,
                                                             const uint32_t *__restrict__ perm) {
    __shared__ uint64_t s_excl[kPrWaves][kWave + 1];
    __shared__ uint64_t s_start[kPrWaves][kWave];
    __shared__ uint32_t s_w[kPrWaves][kWave];
    __shared__ float s_acc[kPrWaves][kWave];
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t nchunks = ((uint64_t)n + kPrThreads - 1) / kPrThreads;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t v = c * kPrThreads + threadIdx.x;
        VInfo vi{0, 0, 0};
        if (v < n) vi = acc.info((uint32_t)v);
        const uint64_t d = vi.deg;
        const uint64_t incl = wave_incl_scan(d);
        const uint64_t total = __shfl(incl, kWave - 1, kWave);
        s_excl[wv][lane] = incl - d;
        if (lane == kWave - 1) s_excl[wv][kWave] = total;
        s_start[wv][lane] = vi.start;
        s_w[wv][lane] = vi.w;
        s_acc[wv][lane] = 0.0f;
        __syncthreads();
        if (total) {
            uint32_t j = 0;
            uint64_t nb = 0;  // first edge index past owner j
            uint64_t pos = 0, adv = 0;
            uint32_t mk = 0;
            float part = 0.0f;
            uint32_t owner = 0xFFFFFFFFu;
            for (uint64_t e = lane; e < total; e += kWave) {
                if (e >= nb || owner == 0xFFFFFFFFu) {
                    while (s_excl[wv][j + 1] <= e) ++j;
                    if (owner != 0xFFFFFFFFu) atomicAdd(&s_acc[wv][owner], part);
                    owner = j;
                    part = 0.0f;
                    nb = s_excl[wv][j + 1];
                    const uint32_t w = s_w[wv][j];
                    pos = s_start[wv][j] + (e - s_excl[wv][j]) * Acc::step(w);
                    adv = (uint64_t)kWave * Acc::step(w);
                    mk = Acc::mask(w);
                }
                const uint32_t u = acc.get(pos, mk);
                part += cin[u];
                pos += adv;
            }
            if (owner != 0xFFFFFFFFu) atomicAdd(&s_acc[wv][owner], part);
        }
        __syncthreads();
        if (v < n) {
            const float pr = base + alpha * s_acc[wv][lane];
            cout[v] = d ? pr / (float)d : 0.0f;
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
    const uint32_t *perm = g->relabel == LG_RELABEL_DEGREE ? g->perm.as<uint32_t>() : nullptr;
    const double a = damping;
    const double z = g->isolated;
    return dispatch_acc(g, [&](auto acc) -> lg_status {
        using Acc = decltype(acc);
        float *cin = g->pr->ca.as<float>(), *cout = g->pr->cb.as<float>();
        LG_LAUNCH(pr_init_kernel<Acc>, grid_for(n, 256, 1u << 16), 256, 0, stream, acc, n, 1.0 / nd, cin);
        LG_CHECK_LAUNCH();
        double D = z / nd;  // D_0: rank on vertices without edges
        const uint32_t grid = grid_for(n, kPrThreads, 1u << 20);
        for (uint32_t t = 0; t < iters; ++t) {
            const double b = (1.0 - a) / nd + a * D / nd;
            const bool last = t + 1 == iters;
            LG_LAUNCH(pr_pull_kernel<Acc>, grid, kPrThreads, 0, stream, acc, n, (const float *)cin, cout, (float)b,
                      (float)a, last ? scores : (float *)nullptr, last ? perm : (const uint32_t *)nullptr);
            LG_CHECK_LAUNCH();
            D = z * b;
            float *tmp = cin; cin = cout; cout = tmp;
        }
        return LG_OK;
    });
}
