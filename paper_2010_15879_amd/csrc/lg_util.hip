// Device utilities of liblg: fills, exclusive prefix sums and a stable LSD
// radix sort of key/value pairs (used by the degree relabeling and the
// sorted neighbor decode).
#include "lg_device.hpp"

namespace lg {

// ---------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------

template <class T>
__global__ void fill_kernel(T *__restrict__ p, T value, uint64_t count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

lg_status fill_u32(uint32_t *p, uint32_t value, uint64_t count, hipStream_t s) {
    if (!count) return LG_OK;
    LG_LAUNCH(fill_kernel<uint32_t>, grid_for(count, 256 * 8, 1u << 16), 256, 0, s, p, value, count);
    LG_CHECK_LAUNCH();
    return LG_OK;
}

lg_status fill_u64(uint64_t *p, uint64_t value, uint64_t count, hipStream_t s) {
    if (!count) return LG_OK;
    LG_LAUNCH(fill_kernel<uint64_t>, grid_for(count, 256 * 8, 1u << 16), 256, 0, s, p, value, count);
    LG_CHECK_LAUNCH();
    return LG_OK;
}

// ---------------------------------------------------------------------------
// exclusive scan: reduce tiles -> scan tile sums (recursively) -> scan tiles
// ---------------------------------------------------------------------------

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr uint64_t kScanTile = (uint64_t)kScanThreads * kScanItems;

// block-wide exclusive scan of one value per thread; returns the block total
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t x, uint64_t &excl) {
    __shared__ uint64_t wave_tot[kScanThreads / kWave];
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const uint64_t incl = wave_incl_scan(x);
    if (lane == kWave - 1) wave_tot[wv] = incl;
    __syncthreads();
    uint64_t base = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        if (w < (int)wv) base += wave_tot[w];
        total += wave_tot[w];
    }
    __syncthreads();
    excl = base + incl - x;
    return total;
}

template <class T>
__global__ void scan_reduce_kernel(const T *__restrict__ in, uint64_t count, uint64_t *__restrict__ sums) {
    const uint64_t t0 = (uint64_t)blockIdx.x * kScanTile;
    uint64_t acc = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const uint64_t i = t0 + (uint64_t)r * kScanThreads + threadIdx.x;
        if (i < count) acc += (uint64_t)in[i];
    }
    uint64_t excl;
    const uint64_t total = block_excl_scan(acc, excl);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Each thread scans kScanItems consecutive inputs; offsets[b] is the
// exclusive prefix of the tile (NULL: 0).  The block owning the last item
// also writes out[count].
template <class T>
__global__ void scan_tile_kernel(const T *__restrict__ in, uint64_t count, const uint64_t *__restrict__ offsets,
                                 uint64_t *__restrict__ out) {
    const uint64_t t0 = (uint64_t)blockIdx.x * kScanTile;
    const uint64_t i0 = t0 + (uint64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t acc = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        v[r] = (i0 + r < count) ? (uint64_t)in[i0 + r] : 0ull;
        acc += v[r];
    }
    uint64_t excl;
    const uint64_t total = block_excl_scan(acc, excl);
    const uint64_t base = (offsets ? offsets[blockIdx.x] : 0ull);
    uint64_t run = base + excl;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        if (i0 + r < count) out[i0 + r] = run;
        run += v[r];
    }
    if (t0 + kScanTile >= count && threadIdx.x == 0) out[count] = base + total;
}

template <class T>
static lg_status scan_level(const T *in, uint64_t *out, uint64_t count, uint64_t *tmp, hipStream_t s) {
    if (count <= kScanTile) {
        LG_LAUNCH((scan_tile_kernel<T>), 1, kScanThreads, 0, s, in, count, (const uint64_t *)nullptr, out);
        LG_CHECK_LAUNCH();
        return LG_OK;
    }
    const uint64_t nb = (count + kScanTile - 1) / kScanTile;
    uint64_t *sums = tmp;
    uint64_t *sums_scan = tmp + nb;
    LG_LAUNCH((scan_reduce_kernel<T>), (uint32_t)nb, kScanThreads, 0, s, in, count, sums);
    LG_CHECK_LAUNCH();
    LG_TRY(scan_level<uint64_t>(sums, sums_scan, nb, tmp + 2 * nb + 1, s));
    LG_LAUNCH((scan_tile_kernel<T>), (uint32_t)nb, kScanThreads, 0, s, in, count,
              (const uint64_t *)sums_scan, out);
    LG_CHECK_LAUNCH();
    return LG_OK;
}

static uint64_t scan_tmp_words(uint64_t count) {
    uint64_t words = 0;
    while (count > kScanTile) {
        const uint64_t nb = (count + kScanTile - 1) / kScanTile;
        words += 2 * nb + 1;
        count = nb;
    }
    return words + 1;
}

uint64_t scan_tmp_bytes(uint64_t count) { return count ? scan_tmp_words(count) * sizeof(uint64_t) : 0; }

lg_status exclusive_scan_u32(const uint32_t *in, uint64_t *out, uint64_t count, DevBuf &tmp, hipStream_t s) {
    if (count == 0) return fill_u64(out, 0, 1, s);
    LG_TRY(tmp.ensure(scan_tmp_words(count) * sizeof(uint64_t)));
    return scan_level<uint32_t>(in, out, count, tmp.as<uint64_t>(), s);
}

lg_status exclusive_scan_u64(const uint64_t *in, uint64_t *out, uint64_t count, DevBuf &tmp, hipStream_t s) {
    if (count == 0) return fill_u64(out, 0, 1, s);
    LG_TRY(tmp.ensure(scan_tmp_words(count) * sizeof(uint64_t)));
    return scan_level<uint64_t>(in, out, count, tmp.as<uint64_t>(), s);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (key, value) pairs, 8-bit digits
// ---------------------------------------------------------------------------

constexpr int kSortThreads = 512;
constexpr int kSortRounds = 16;
constexpr uint64_t kSortTile = (uint64_t)kSortThreads * kSortRounds;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr uint32_t kXcds = 8;  // accelerator complex dies; each has its own L2
static_assert(kSortTile < (1u << 16), "per-tile digit counts are kept in 16 bits");

// Tile of block b.  Blocks go to the dies in turn (block b to die b mod 8).
// A digit's run in tile j ends where the same digit's run of tile j + 1
// begins, in the same cache line; when neighbouring tiles run on different
// dies, each die's L2 writes such a line back half-filled.  Giving every die
// one contiguous range of tiles keeps both halves in one L2 (25 % less sort
// time on 5.2e8 pairs).
__device__ __forceinline__ uint32_t sort_tile_of(uint32_t b, uint32_t ntiles) {
    const uint32_t q = ntiles / kXcds, r = ntiles % kXcds, x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// Per-tile digit counts.  kVec: 16-byte loads (keys 16-byte aligned), all
// issued before the first count; every wave counts into its own histogram.
template <class K, bool kVec>
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const K *__restrict__ keys, uint64_t count,
                                                                  uint32_t shift, uint32_t ntiles,
                                                                  uint32_t *__restrict__ counts) {
    __shared__ uint32_t hist[kSortWaves][256];
    for (uint32_t i = threadIdx.x; i < kSortWaves * 256; i += kSortThreads) (&hist[0][0])[i] = 0;
    __syncthreads();
    const uint32_t tile = sort_tile_of(blockIdx.x, ntiles);
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t t0 = (uint64_t)tile * kSortTile;
    constexpr int kPer = kVec ? (int)(16 / sizeof(K)) : 1;  // consecutive keys per load
    constexpr int kLoads = kSortRounds / kPer;
    K kr[kSortRounds];
#pragma unroll
    for (int l = 0; l < kLoads; ++l) {
        const uint64_t i = t0 + ((uint64_t)l * kSortThreads + threadIdx.x) * kPer;
        if (kVec && i + kPer <= count) {
            const uint4 x = *reinterpret_cast<const uint4 *>(keys + i);
            __builtin_memcpy(&kr[l * kPer], &x, 16);
        } else {
#pragma unroll
            for (int j = 0; j < kPer; ++j) kr[l * kPer + j] = i + j < count ? keys[i + j] : (K)0;
        }
    }
#pragma unroll
    for (int l = 0; l < kLoads; ++l) {
        const uint64_t i = t0 + ((uint64_t)l * kSortThreads + threadIdx.x) * kPer;
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            if (i + j < count) atomicAdd(&hist[wv][(uint32_t)(kr[l * kPer + j] >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 256) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) c += hist[w][threadIdx.x];
        counts[(uint64_t)threadIdx.x * ntiles + tile] = c;
    }
}

// A tile is eight contiguous sub-tiles of 1,024 keys, one per wave.  A wave
// ranks its keys 64 at a time: lanes with equal digits are found with eight
// ballots, and a wave-private LDS counter per digit carries the running count
// from one group of 64 to the next, so every key gets its rank among equal
// digits of its sub-tile in input order without waiting for the other waves.
// One prefix over the waves' counts then gives every key its place in the
// tile (stability), keys are placed in LDS in digit order, and written out so
// that consecutive threads store consecutive addresses of one digit's run.
template <class K>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const K *__restrict__ keys, const uint32_t *__restrict__ vals, uint64_t count, uint32_t shift, uint32_t ntiles,
    const uint32_t *__restrict__ counts, const uint64_t *__restrict__ offsets, K *__restrict__ keys_out,
    uint32_t *__restrict__ vals_out) {
    constexpr int kPer = kSortRounds;  // keys per lane (sub-tile = kWave * kPer keys)
    __shared__ K s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    __shared__ uint32_t s_start[256];
    __shared__ uint64_t s_gbase[256];
    __shared__ uint32_t s_wtot[kSortWaves];
    __shared__ uint16_t wave_cnt[kSortWaves][256];  // counts within a tile (< 2^16)
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = sort_tile_of(blockIdx.x, ntiles);
    // tile-local start of every digit (threads 0..255, one digit each):
    // exclusive scan of this tile's histogram
    const uint32_t c = tid < 256 ? counts[(uint64_t)tid * ntiles + tile] : 0u;
    const uint32_t incl = wave_incl_scan(c);
    if (lane == kWave - 1) s_wtot[wv] = incl;
    for (uint32_t i = tid; i < kSortWaves * 256; i += kSortThreads) (&wave_cnt[0][0])[i] = 0;
    __syncthreads();
    if (tid < 256) {
        uint32_t before = 0;
        for (uint32_t w = 0; w < wv; ++w) before += s_wtot[w];
        s_start[tid] = before + incl - c;
        s_gbase[tid] = offsets[(uint64_t)tid * ntiles + tile] - (before + incl - c);
    }
    // this wave's sub-tile, all loads in flight before the first use
    const uint64_t w0 = (uint64_t)tile * kSortTile + (uint64_t)wv * kWave * kPer;
    K kr[kPer];
    uint32_t vr[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const uint64_t i = w0 + (uint64_t)r * kWave + lane;
        kr[r] = i < count ? keys[i] : (K)0;
        vr[r] = i < count ? vals[i] : 0u;
    }
    uint32_t rank[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const bool valid = w0 + (uint64_t)r * kWave + lane < count;
        const uint32_t digit = (uint32_t)(kr[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((digit >> b) & 1u);
            peers &= ((digit >> b) & 1u) ? m : ~m;
        }
        const uint32_t below = popc_below(peers);
        const uint32_t run = valid ? wave_cnt[wv][digit] : 0u;
        rank[r] = run + below;
        // the group's first lane advances the digit's running count; the wave
        // reads every count of this group before any lane writes
        __builtin_amdgcn_wave_barrier();
        if (valid && below == 0) wave_cnt[wv][digit] = (uint16_t)(run + (uint32_t)__popcll(peers));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
    if (tid < 256) {  // per digit: exclusive prefix of the waves' counts
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            const uint32_t cw = wave_cnt[w][tid];
            wave_cnt[w][tid] = (uint16_t)run;
            run += cw;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        if (w0 + (uint64_t)r * kWave + lane < count) {
            const uint32_t digit = (uint32_t)(kr[r] >> shift) & 255u;
            const uint32_t idx = s_start[digit] + wave_cnt[wv][digit] + rank[r];
            s_key[idx] = kr[r];
            s_val[idx] = vr[r];
        }
    }
    __syncthreads();
    const uint64_t t0 = (uint64_t)tile * kSortTile;
    const uint64_t tile_n = count - t0 < kSortTile ? count - t0 : kSortTile;
    for (uint32_t idx = tid; idx < tile_n; idx += kSortThreads) {
        const K key = s_key[idx];
        const uint64_t dst = s_gbase[(uint32_t)(key >> shift) & 255u] + idx;
        keys_out[dst] = key;
        vals_out[dst] = s_val[idx];
    }
}

uint64_t radix_sort_tmp_bytes(uint64_t count) {
    if (count <= 1) return 0;
    const uint64_t ncount = (count + kSortTile - 1) / kSortTile * 256;
    return ((ncount * 4 + 7) & ~7ull) + (ncount + 1) * 8 + scan_tmp_words(ncount) * 8;
}

template <class K>
static lg_status radix_sort_impl(K *keys, uint32_t *vals, K *keys_alt, uint32_t *vals_alt, uint64_t count,
                                 uint32_t bits, DevBuf &tmp, hipStream_t s, int *in_alt) {
    if (in_alt) *in_alt = 0;
    if (count <= 1 || bits == 0) return LG_OK;
    const uint64_t ntiles = (count + kSortTile - 1) / kSortTile;
    if (ntiles * 256 >= (1ull << 32)) {
        set_error("radix sort: %llu items is too many", (unsigned long long)count);
        return LG_ERR_UNSUPPORTED;
    }
    const uint64_t ncount = ntiles * 256;
    // layout of tmp: counts (u32, ncount) | offsets (u64, ncount + 1) | scan scratch
    LG_TRY(tmp.ensure(radix_sort_tmp_bytes(count)));
    uint32_t *counts = tmp.as<uint32_t>();
    uint64_t *offs = reinterpret_cast<uint64_t *>(tmp.as<char>() + ((ncount * 4 + 7) & ~7ull));
    uint64_t *scratch = offs + ncount + 1;
    K *src_k = keys, *dst_k = keys_alt;
    uint32_t *src_v = vals, *dst_v = vals_alt;
    int passes = 0;
    for (uint32_t shift = 0; shift < bits; shift += 8, ++passes) {
        if (((uintptr_t)src_k & 15u) == 0)
            LG_LAUNCH((radix_hist_kernel<K, true>), (uint32_t)ntiles, kSortThreads, 0, s, src_k, count, shift,
                      (uint32_t)ntiles, counts);
        else
            LG_LAUNCH((radix_hist_kernel<K, false>), (uint32_t)ntiles, kSortThreads, 0, s, src_k, count, shift,
                      (uint32_t)ntiles, counts);
        LG_CHECK_LAUNCH();
        LG_TRY(scan_level<uint32_t>(counts, offs, ncount, scratch, s));
        LG_LAUNCH(radix_scatter_kernel<K>, (uint32_t)ntiles, kSortThreads, 0, s, src_k, src_v, count, shift,
                  (uint32_t)ntiles, (const uint32_t *)counts, (const uint64_t *)offs, dst_k, dst_v);
        LG_CHECK_LAUNCH();
        K *tk = src_k; src_k = dst_k; dst_k = tk;
        uint32_t *tv = src_v; src_v = dst_v; dst_v = tv;
    }
    if (passes & 1) {
        if (in_alt) {
            *in_alt = 1;
            return LG_OK;
        }
        LG_CHECK_HIP(hipMemcpyAsync(keys, keys_alt, count * sizeof(K), hipMemcpyDeviceToDevice, s));
        LG_CHECK_HIP(hipMemcpyAsync(vals, vals_alt, count * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    return LG_OK;
}

lg_status radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt, uint64_t count,
                           uint32_t bits, DevBuf &tmp, hipStream_t s, int *in_alt) {
    return radix_sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, count, bits, tmp, s, in_alt);
}

lg_status radix_sort_pairs64(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, uint64_t count,
                             uint32_t bits, DevBuf &tmp, hipStream_t s, int *in_alt) {
    return radix_sort_impl<uint64_t>(keys, vals, keys_alt, vals_alt, count, bits, tmp, s, in_alt);
}

}  // namespace lg
