// PageRank work tables (built once per graph, at the first lg_pagerank):
//   * every heavy vertex (degree above the traversal threshold) gets its
//     (first bit, degree, width) cached;
//   * lists longer than pr_split are cut into segments of seg_size edges,
//     one wave per segment, so that no wave walks a hub's list alone;
//   * all other vertices are grouped into units: consecutive vertices of one
//     64-aligned block whose first edges fall into the same window of
//     pr_unit_edges edges of that block.  A unit then holds at most 64
//     vertices and at most pr_unit_edges + pr_split edges, and a wave takes
//     one unit at a time, so waves get comparable work whatever the degree
//     distribution, without giving a wave to a list of a hundred edges.
#include "lg_device.hpp"

namespace lg {

template <class Acc>
__global__ void heavy_info_kernel(Acc acc, const uint32_t *__restrict__ heavy, uint32_t n_heavy,
                                  uint64_t *__restrict__ hstart, uint32_t *__restrict__ hdeg,
                                  uint32_t *__restrict__ hw, uint32_t *__restrict__ hg, uint32_t split,
                                  uint32_t seg_size, uint32_t *__restrict__ segcnt) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n_heavy; h += stride) {
        const auto vi = acc.info(heavy[h]);
        hstart[h] = vi.start;
        hdeg[h] = vi.deg;
        hw[h] = vi.w;
        if constexpr (IsGapAcc<Acc>::value) hg[h] = vi.g;
        segcnt[h] = vi.deg > split ? (vi.deg + seg_size - 1) / seg_size : 0u;
    }
}

// Gap lists: the sum of segment k's entries (the first element counts for
// entry 0, a difference for every other), one wave per segment.
template <class Acc>
__global__ void gap_seg_sum_kernel(Acc acc, uint64_t n_seg, uint32_t seg_size, const uint32_t *__restrict__ seg_map,
                                   const uint64_t *__restrict__ seg_off, const uint64_t *__restrict__ hstart,
                                   const uint32_t *__restrict__ hdeg, const uint32_t *__restrict__ hw,
                                   const uint32_t *__restrict__ hg, uint32_t *__restrict__ seg_sum) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t k = wave; k < n_seg; k += nwaves) {
        const uint32_t h = seg_map[k];
        const uint64_t e0 = (k - seg_off[h]) * seg_size;
        const uint64_t e1 = e0 + seg_size < hdeg[h] ? e0 + seg_size : hdeg[h];
        const GapInfo gi{hstart[h], hdeg[h], hw[h], hg[h]};
        uint32_t sum = 0;
        for (uint64_t e = e0 + lane; e < e1; e += kWave)
            sum += acc.get(Acc::entry_bit(gi, e), e == 0 ? gi.w : gi.g);
        sum = wave_sum(sum);
        if (lane == 0) seg_sum[k] = sum;
    }
}

// seg_base[k] = the sums of the segments of the same list before k
__global__ void gap_seg_base_kernel(uint64_t n_seg, const uint32_t *__restrict__ seg_map,
                                    const uint64_t *__restrict__ seg_off, const uint64_t *__restrict__ scan,
                                    uint32_t *__restrict__ seg_base) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_seg; k += stride)
        seg_base[k] = (uint32_t)(scan[k] - scan[seg_off[seg_map[k]]]);
}

__global__ void heavy_sum_kernel(uint32_t n_heavy, const uint32_t *__restrict__ hdeg, const uint32_t *__restrict__ hw,
                                 unsigned long long *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long e = 0, b = 0;
    for (uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n_heavy; h += stride) {
        e += hdeg[h];
        b += (unsigned long long)hdeg[h] * hw[h];
    }
    e = block_sum_u64(e);
    b = block_sum_u64(b);
    if (threadIdx.x == 0) {
        atomicAdd(&out[0], e);
        atomicAdd(&out[1], b);
    }
}

__global__ void heavy_seg_map_kernel(uint32_t n_heavy, const uint64_t *__restrict__ seg_off,
                                     uint32_t *__restrict__ seg_map) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n_heavy; h += stride)
        for (uint64_t k = seg_off[h]; k < seg_off[h + 1]; ++k) seg_map[k] = (uint32_t)h;
}

// Unit starts of block q (vertices 64q .. 64q+63): the block's first vertex,
// and every vertex whose first unit edge lies in a later window of `budget`
// edges than its predecessor's.  Pass 1 counts them, pass 2 writes them.
template <class Acc, bool kWrite>
__global__ void pr_units_kernel(Acc acc, uint32_t n, uint32_t split, uint32_t budget,
                                uint32_t *__restrict__ cnt, const uint64_t *__restrict__ off,
                                uint32_t *__restrict__ units) {
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    const uint32_t lane = lane_id();
    for (uint64_t q = wave; q < words; q += nwaves) {
        const uint64_t v = q * 64 + lane;
        uint32_t deg;
        if constexpr (IsGapAcc<Acc>::value) deg = v < n ? acc.info((uint32_t)v).deg : 0u;
        else deg = wave_info(acc, q * 64, n).deg;
        const uint32_t d = (v < n && deg <= split) ? deg : 0u;
        const uint32_t excl = wave_incl_scan(d) - d;
        const uint32_t prev = __shfl_up(excl, 1, kWave);
        const bool start = v < n && (lane == 0 || excl / budget != prev / budget);
        const uint64_t m = __ballot(start);
        if (!kWrite) {
            if (lane == 0) cnt[q] = (uint32_t)__popcll(m);
        } else if (start) {
            units[off[q] + popc_below(m)] = (uint32_t)v;
        }
    }
}

lg_status ensure_heavy_segments(lg_graph *g, hipStream_t s) {
    if (g->segs_built) return LG_OK;
    const uint32_t nh = g->n_heavy;
    const uint32_t n = g->n;
    g->seg_size = 4096;
    while (((uint64_t)g->max_degree + g->seg_size - 1) / g->seg_size > 65535) g->seg_size *= 2;
    g->pr_split = 4096;
    g->pr_unit_edges = 8192;
    LG_TRY(g->hstart.scratch((uint64_t)(nh ? nh : 1) * 8, s));
    LG_TRY(g->hdeg.scratch((uint64_t)(nh ? nh : 1) * 4, s));
    LG_TRY(g->hw.scratch((uint64_t)(nh ? nh : 1) * 4, s));
    const bool gap = g->id_mode == LG_IDS_LOCAL_GAP;
    if (gap) LG_TRY(g->hg.scratch((uint64_t)(nh ? nh : 1) * 4, s));
    LG_TRY(g->seg_off.scratch(((uint64_t)nh + 1) * 8, s));
    g->n_seg = 0;
    DevBuf tmp;
    LG_TRY(tmp.scratch(8, s));
    if (nh) {
        DevBuf segcnt;
        LG_TRY(segcnt.scratch((uint64_t)nh * 4, s));
        LG_TRY(dispatch_acc_all(g, [&](auto acc) -> lg_status {
            using Acc = decltype(acc);
            LG_LAUNCH(heavy_info_kernel<Acc>, grid_for(nh, 256, 1u << 16), 256, 0, s, acc, g->heavy.as<uint32_t>(),
                      nh, g->hstart.as<uint64_t>(), g->hdeg.as<uint32_t>(), g->hw.as<uint32_t>(),
                      gap ? g->hg.as<uint32_t>() : (uint32_t *)nullptr, g->pr_split, g->seg_size,
                      segcnt.as<uint32_t>());
            LG_CHECK_LAUNCH();
            return LG_OK;
        }));
        LG_TRY(exclusive_scan_u32(segcnt.as<uint32_t>(), g->seg_off.as<uint64_t>(), nh, tmp, s));
        DevBuf sums;
        LG_TRY(sums.scratch(16, s));
        LG_TRY(fill_u64(sums.as<uint64_t>(), 0, 2, s));
        LG_LAUNCH(heavy_sum_kernel, grid_for(nh, 256, 1024), 256, 0, s, nh, g->hdeg.as<uint32_t>(),
                  g->hw.as<uint32_t>(), sums.as<unsigned long long>());
        LG_CHECK_LAUNCH();
        uint64_t hs[2];
        LG_CHECK_HIP(hipMemcpyAsync(hs, sums.p, 16, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
        g->heavy_edges = hs[0];
        g->heavy_bits = hs[1];
        LG_CHECK_HIP(hipMemcpyAsync(&g->n_seg, g->seg_off.as<uint64_t>() + nh, 8, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
    } else {
        LG_TRY(fill_u64(g->seg_off.as<uint64_t>(), 0, 1, s));
    }
    LG_TRY(g->seg_map.scratch((g->n_seg ? g->n_seg : 1) * 4, s));
    LG_TRY(g->seg_part.scratch((g->n_seg ? g->n_seg : 1) * 4, s));
    if (g->n_seg) {
        LG_LAUNCH(heavy_seg_map_kernel, grid_for(nh, 256, 1u << 16), 256, 0, s, nh, g->seg_off.as<uint64_t>(),
                  g->seg_map.as<uint32_t>());
        LG_CHECK_LAUNCH();
    }
    if (gap) {
        LG_TRY(g->seg_base.scratch((g->n_seg ? g->n_seg : 1) * 4, s));
        if (g->n_seg) {
            DevBuf ssum, sscan;
            LG_TRY(ssum.scratch(g->n_seg * 4, s));
            LG_TRY(sscan.scratch((g->n_seg + 1) * 8, s));
            LG_TRY(dispatch_acc_all(g, [&](auto acc) -> lg_status {
                using Acc = decltype(acc);
                if constexpr (IsGapAcc<Acc>::value) {
                    LG_LAUNCH(gap_seg_sum_kernel<Acc>, grid_for(g->n_seg * kWave, 256, 1u << 16), 256, 0, s, acc,
                              g->n_seg, g->seg_size, g->seg_map.as<uint32_t>(), g->seg_off.as<uint64_t>(),
                              g->hstart.as<uint64_t>(), g->hdeg.as<uint32_t>(), g->hw.as<uint32_t>(),
                              g->hg.as<uint32_t>(), ssum.as<uint32_t>());
                    LG_CHECK_LAUNCH();
                    return LG_OK;
                }
                return LG_ERR_UNSUPPORTED;
            }));
            LG_TRY(exclusive_scan_u32(ssum.as<uint32_t>(), sscan.as<uint64_t>(), g->n_seg, tmp, s));
            LG_LAUNCH(gap_seg_base_kernel, grid_for(g->n_seg, 256, 1u << 16), 256, 0, s, g->n_seg,
                      g->seg_map.as<uint32_t>(), g->seg_off.as<uint64_t>(), sscan.as<uint64_t>(),
                      g->seg_base.as<uint32_t>());
            LG_CHECK_LAUNCH();
            LG_CHECK_HIP(hipStreamSynchronize(s));
        }
    }
    // units
    const uint64_t words = ((uint64_t)n + 63) / 64;
    DevBuf cnt, uoff;
    LG_TRY(cnt.scratch(words * 4, s));
    LG_TRY(uoff.scratch((words + 1) * 8, s));
    const uint32_t ugrid = grid_for(words * kWave, 256, 1u << 16);
    LG_TRY(dispatch_acc_all(g, [&](auto acc) -> lg_status {
        using Acc = decltype(acc);
        LG_LAUNCH((pr_units_kernel<Acc, false>), ugrid, 256, 0, s, acc, n, g->pr_split, g->pr_unit_edges,
                  cnt.as<uint32_t>(), (const uint64_t *)nullptr, (uint32_t *)nullptr);
        LG_CHECK_LAUNCH();
        LG_TRY(exclusive_scan_u32(cnt.as<uint32_t>(), uoff.as<uint64_t>(), words, tmp, s));
        LG_CHECK_HIP(hipMemcpyAsync(&g->n_units, uoff.as<uint64_t>() + words, 8, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
        LG_TRY(g->units.scratch((g->n_units + 1) * 4, s));
        LG_LAUNCH((pr_units_kernel<Acc, true>), ugrid, 256, 0, s, acc, n, g->pr_split, g->pr_unit_edges,
                  (uint32_t *)nullptr, (const uint64_t *)uoff.as<uint64_t>(), g->units.as<uint32_t>());
        LG_CHECK_LAUNCH();
        return LG_OK;
    }));
    LG_TRY(fill_u32(g->units.as<uint32_t>() + g->n_units, n, 1, s));  // sentinel
    LG_CHECK_HIP(hipStreamSynchronize(s));
    g->segs_built = true;
    return LG_OK;
}

}  // namespace lg
