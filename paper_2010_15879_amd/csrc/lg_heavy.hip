// Heavy-vertex segment table shared by the bottom-up BFS step and the
// PageRank pull: every vertex of degree above the threshold gets its
// (first bit, degree, width) cached and its list cut into segments of
// seg_size edges, so that one wave handles one segment and no wave walks a
// hub's whole list alone.
#include "lg_device.hpp"

namespace lg {

template <class Acc>
__global__ void heavy_info_kernel(Acc acc, const uint32_t *__restrict__ heavy, uint32_t n_heavy,
                                  uint64_t *__restrict__ hstart, uint32_t *__restrict__ hdeg,
                                  uint32_t *__restrict__ hw, uint32_t seg_size, uint32_t *__restrict__ segcnt) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n_heavy; h += stride) {
        const VInfo vi = acc.info(heavy[h]);
        hstart[h] = vi.start;
        hdeg[h] = vi.deg;
        hw[h] = vi.w;
        segcnt[h] = (vi.deg + seg_size - 1) / seg_size;
    }
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

lg_status ensure_heavy_segments(lg_graph *g, hipStream_t s) {
    if (g->segs_built) return LG_OK;
    const uint32_t nh = g->n_heavy;
    g->seg_size = 1024;
    while (((uint64_t)g->max_degree + g->seg_size - 1) / g->seg_size > 65535) g->seg_size *= 2;
    LG_TRY(g->hstart.alloc((uint64_t)(nh ? nh : 1) * 8));
    LG_TRY(g->hdeg.alloc((uint64_t)(nh ? nh : 1) * 4));
    LG_TRY(g->hw.alloc((uint64_t)(nh ? nh : 1) * 4));
    LG_TRY(g->seg_off.alloc(((uint64_t)nh + 1) * 8));
    g->n_seg = 0;
    if (nh) {
        DevBuf segcnt, tmp;
        LG_TRY(segcnt.alloc((uint64_t)nh * 4));
        LG_TRY(dispatch_acc(g, [&](auto acc) -> lg_status {
            using Acc = decltype(acc);
            LG_LAUNCH(heavy_info_kernel<Acc>, grid_for(nh, 256, 1u << 16), 256, 0, s, acc, g->heavy.as<uint32_t>(),
                      nh, g->hstart.as<uint64_t>(), g->hdeg.as<uint32_t>(), g->hw.as<uint32_t>(), g->seg_size,
                      segcnt.as<uint32_t>());
            LG_CHECK_LAUNCH();
            return LG_OK;
        }));
        LG_TRY(exclusive_scan_u32(segcnt.as<uint32_t>(), g->seg_off.as<uint64_t>(), nh, tmp, s));
        DevBuf sums;
        LG_TRY(sums.alloc(16));
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
    LG_TRY(g->seg_map.alloc((g->n_seg ? g->n_seg : 1) * 4));
    if (nh) {
        LG_LAUNCH(heavy_seg_map_kernel, grid_for(nh, 256, 1u << 16), 256, 0, s, nh, g->seg_off.as<uint64_t>(),
                  g->seg_map.as<uint32_t>());
        LG_CHECK_LAUNCH();
    }
    LG_CHECK_HIP(hipStreamSynchronize(s));
    g->segs_built = true;
    return LG_OK;
}

}  // namespace lg
