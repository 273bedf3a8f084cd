// PageRank over Varint lists (subsection "Incorporating Degree-Minimizing
// (DM)"; PR of section "Considered Algorithms", pull without atomics, FP32):
// the iteration of lg_pagerank with in-order list reads.
//
//   d_v: counted once per graph (the bytes with the top bit clear in each
//        list, a wave per vertex)
//   a list of at most 64 values (not a heavy vertex): a lane per vertex,
//        reading it from 8-byte windows
//   a heavy list of at most vseg_split bytes: a wave each, 64 bytes per step,
//        a lane holding a value's last byte gathers that neighbor's
//        contribution (DMd: the label is a wave prefix sum of differences)
//   a longer list: a wave per 4 KiB chunk of the graph's chunk tables (the
//        values ending in the chunk, DMd from the chunk's stored label) writes
//        a partial sum; a second kernel adds each list's partial sums in
//        chunk order
// Every sum has an order fixed by the data, so results repeat bit for bit.
#include <algorithm>

#include "lg_device.hpp"
#include "lg_varint.hpp"

namespace lg {

template <class Acc>
__global__ void vpr_degree_kernel(Acc acc, uint32_t n, uint32_t *__restrict__ deg) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t v = wave; v < n; v += nwaves) {
        uint64_t b0, b1;
        acc.offsets((uint32_t)v, b0, b1);
        uint32_t cnt = 0;
        for (uint64_t q = (b0 >> 3) + lane; q * 8 < b1; q += kWave) {
            const uint64_t p = q * 8;
            const uint64_t lo = p < b0 ? b0 - p : 0;
            const uint64_t hi = p + 8 > b1 ? p + 8 - b1 : 0;
            uint64_t keep = ~0ull << (8 * lo);
            if (hi) keep &= ~0ull >> (8 * hi);
            cnt += (uint32_t)__popcll(~acc.word(p) & 0x8080808080808080ull & keep);
        }
        cnt = wave_sum(cnt);
        if (lane == 0) deg[v] = cnt;
    }
}

__global__ void vpr_init_kernel(uint32_t n, const uint32_t *__restrict__ deg, double inv_n, float *__restrict__ ca,
                                float *__restrict__ cb) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const float c = deg[v] ? (float)(inv_n / (double)deg[v]) : 0.0f;
        ca[v] = c;
        cb[v] = c;
    }
}

// the sum of the contributions of the values ending in bytes [c0, c1)
template <class Acc>
__device__ __forceinline__ float vpr_range_sum(const Acc &acc, uint32_t n, const float *__restrict__ cin,
                                               uint64_t c0, uint64_t c1, uint32_t prevb, uint32_t carry) {
    float sum = 0.0f;
    for (uint64_t p0 = c0; p0 < c1; p0 += kWave) {
        uint32_t x;
        const bool end = varint_step(acc, p0, c1, prevb, x);
        uint32_t label = x;
        if constexpr (Acc::kDifferences) {
            const uint32_t sc = wave_incl_scan(end ? x : 0u);
            label = carry + sc;
            carry += __shfl(sc, kWave - 1, kWave);
        }
        // a stored label is < n; the clamp keeps the gather in bounds
        if (end) sum += cin[label < n ? label : n - 1];
    }
    return wave_sum(sum);
}

// Lists of at most lane_max values (the heavy-vertex threshold: at most five
// bytes each), a lane per vertex over 64-vertex words (offsets decoded by the
// whole wave): each lane reads its list from 8-byte windows (two aligned
// words and a funnel shift; the pad word keeps the second in bounds) and
// sums the contributions in list order.

template <class Acc>
__global__ void vpr_lane_kernel(Acc acc, uint32_t n, uint32_t lane_max, const uint32_t *__restrict__ deg,
                                const float *__restrict__ cin,
                                float *__restrict__ cout, float base, float alpha, float *__restrict__ scores,
                                const uint32_t *__restrict__ perm) {
    const uint32_t lane = lane_id();
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t q = wave; q < words; q += nwaves) {
        uint64_t b0, b1;
        wave_offsets(acc.base, q * 64, n, b0, b1);
        const uint64_t v = q * 64 + lane;
        if (v >= n || deg[v] > lane_max) continue;
        if (b1 == b0 && !scores) continue;  // no edges: contribution stays 0
        float sum = 0.0f;
        uint32_t label = 0, accv = 0, shift = 0, count = 0;
        for (uint64_t pos = b0; pos < b1;) {
            const uint64_t k = pos >> 3;
            const uint32_t sh = (uint32_t)(pos & 7) * 8;
            const uint64_t w0 = acc.word(k * 8), w1 = acc.word(k * 8 + 8);
            const uint64_t win = sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0;
            const uint32_t avail = b1 - pos < 8 ? (uint32_t)(b1 - pos) : 8u;
            for (uint32_t j = 0; j < avail; ++j) {
                const uint32_t b = (uint32_t)(win >> (8 * j)) & 255u;
                accv |= (b & 127u) << shift;
                shift += 7;
                if (!(b & 128u)) {
                    label = Acc::kDifferences && count ? label + accv : accv;
                    ++count;
                    accv = 0;
                    shift = 0;
                    sum += cin[label < n ? label : n - 1];
                }
            }
            pos += avail;
        }
        const float pr = base + alpha * sum;
        const uint32_t d = deg[v];
        cout[v] = d ? pr / (float)d : 0.0f;
        if (scores) scores[perm ? perm[v] : v] = pr;
    }
}

// The heavy lists that are not chunked, a wave each, from their stored
// byte ranges
template <class Acc>
__global__ void vpr_list_kernel(Acc acc, uint32_t n, uint32_t n_heavy, const uint32_t *__restrict__ heavy,
                                const uint64_t *__restrict__ hb0, const uint64_t *__restrict__ hb1,
                                const uint64_t *__restrict__ seg_off, const uint32_t *__restrict__ deg,
                                const float *__restrict__ cin, float *__restrict__ cout, float base, float alpha,
                                float *__restrict__ scores, const uint32_t *__restrict__ perm) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t h = wave; h < n_heavy; h += nwaves) {
        if (seg_off[h + 1] > seg_off[h]) continue;  // chunked: vpr_chunk_kernel
        const uint32_t v = heavy[h];
        const float sum = vpr_range_sum(acc, n, cin, hb0[h], hb1[h], 0u, 0u);
        if (lane == 0) {
            const float pr = base + alpha * sum;
            cout[v] = pr / (float)deg[v];
            if (scores) scores[perm ? perm[v] : v] = pr;
        }
    }
}

template <class Acc>
__global__ void vpr_chunk_kernel(Acc acc, uint32_t n, uint64_t n_seg, uint32_t chunk,
                                 const uint32_t *__restrict__ seg_map, const uint64_t *__restrict__ seg_off,
                                 const uint64_t *__restrict__ hb0, const uint64_t *__restrict__ hb1,
                                 const uint32_t *__restrict__ seg_base, const float *__restrict__ cin,
                                 float *__restrict__ part) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t k = wave; k < n_seg; k += nwaves) {
        const uint32_t h = seg_map[k];
        const uint64_t b0 = hb0[h], b1 = hb1[h];
        const uint64_t c0 = b0 + (k - seg_off[h]) * chunk;
        const uint64_t c1 = c0 + chunk < b1 ? c0 + chunk : b1;
        const float sum = vpr_range_sum(acc, n, cin, c0, c1, varint_chunk_prevb(acc, b0, c0), seg_base[k]);
        if (lane == 0) part[k] = sum;
    }
}

__global__ void vpr_heavy_kernel(uint32_t n_heavy, const uint32_t *__restrict__ heavy,
                                 const uint64_t *__restrict__ seg_off, const uint32_t *__restrict__ deg,
                                 const float *__restrict__ part, float base, float alpha, float *__restrict__ cout,
                                 float *__restrict__ scores, const uint32_t *__restrict__ perm) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n_heavy; h += stride) {
        const uint64_t s0 = seg_off[h], s1 = seg_off[h + 1];
        if (s0 == s1) continue;
        float sum = 0.0f;
        for (uint64_t k = s0; k < s1; ++k) sum += part[k];
        const uint32_t v = heavy[h];
        const float pr = base + alpha * sum;
        cout[v] = pr / (float)deg[v];
        if (scores) scores[perm ? perm[v] : v] = pr;
    }
}

lg_status pagerank_varint(lg_graph *g, float damping, uint32_t iters, float *scores, hipStream_t s) {
    const uint32_t n = g->n;
    const double nd = (double)n;
    LG_TRY(g->vca.ensure((uint64_t)n * 4));
    LG_TRY(g->vcb.ensure((uint64_t)n * 4));
    LG_TRY(g->vpart.ensure((g->n_vseg ? g->n_vseg : 1) * 4));
    const uint32_t *perm = g->relabel != LG_RELABEL_NONE ? g->perm.as<uint32_t>() : nullptr;
    const double a = damping;
    const double z = g->isolated;
    return dispatch_acc_dec(g, [&](auto acc) -> lg_status {
        using Acc = decltype(acc);
        if constexpr (IsVarintAcc<Acc>::value) {
            const uint32_t vgrid = grid_for((uint64_t)n * kWave, 256, 1u << 16);
            if (!g->vdeg.p) {
                LG_TRY(g->vdeg.ensure((uint64_t)n * 4));
                LG_LAUNCH(vpr_degree_kernel<Acc>, vgrid, 256, 0, s, acc, n, g->vdeg.as<uint32_t>());
                LG_CHECK_LAUNCH();
            }
            float *cin = g->vca.as<float>(), *cout = g->vcb.as<float>();
            LG_LAUNCH(vpr_init_kernel, grid_for(n, 256, 1u << 16), 256, 0, s, n, g->vdeg.as<uint32_t>(), 1.0 / nd,
                      cin, cout);
            LG_CHECK_LAUNCH();
            double D = z / nd;
            for (uint32_t t = 0; t < iters; ++t) {
                const double b = (1.0 - a) / nd + a * D / nd;
                const bool last = t + 1 == iters;
                float *sc = last ? scores : (float *)nullptr;
                const uint32_t *pm = last ? perm : (const uint32_t *)nullptr;
                if (g->n_vseg) {
                    LG_LAUNCH(vpr_chunk_kernel<Acc>, grid_for(g->n_vseg * kWave, 256, 1u << 16), 256, 0, s, acc, n,
                              g->n_vseg, g->vseg_bytes, g->vseg_map.as<uint32_t>(), g->vseg_off.as<uint64_t>(),
                              g->vhb0.as<uint64_t>(), g->vhb1.as<uint64_t>(), g->vseg_base.as<uint32_t>(),
                              (const float *)cin, g->vpart.as<float>());
                    LG_CHECK_LAUNCH();
                }
                LG_LAUNCH(vpr_lane_kernel<Acc>, grid_for(((uint64_t)n + 63) / 64 * kWave, 256, 1u << 16), 256, 0,
                          s, acc, n, g->heavy_threshold, g->vdeg.as<uint32_t>(), (const float *)cin, cout, (float)b,
                          (float)a, sc, pm);
                LG_CHECK_LAUNCH();
                if (g->n_heavy) {
                    LG_LAUNCH(vpr_list_kernel<Acc>, grid_for((uint64_t)g->n_heavy * kWave, 256, 1u << 16), 256, 0, s,
                              acc, n, g->n_heavy, g->heavy.as<uint32_t>(), g->vhb0.as<uint64_t>(),
                              g->vhb1.as<uint64_t>(), g->vseg_off.as<uint64_t>(), g->vdeg.as<uint32_t>(),
                              (const float *)cin, cout, (float)b, (float)a, sc, pm);
                    LG_CHECK_LAUNCH();
                }
                if (g->n_vseg) {
                    LG_LAUNCH(vpr_heavy_kernel, grid_for(g->n_heavy, 256, 4096), 256, 0, s, g->n_heavy,
                              g->heavy.as<uint32_t>(), g->vseg_off.as<uint64_t>(), g->vdeg.as<uint32_t>(),
                              (const float *)g->vpart.as<float>(), (float)b, (float)a, cout, sc, pm);
                    LG_CHECK_LAUNCH();
                }
                D = z * b;
                std::swap(cin, cout);
            }
            return LG_OK;
        }
        return LG_ERR_UNSUPPORTED;
    });
}

}  // namespace lg
