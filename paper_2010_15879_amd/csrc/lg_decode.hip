// lg_decode_neighbors: N_v for a batch of vertices (getNeighbors of the
// library listing in section "High-Performance Library"): the offset lookup,
// d_v = O[v+1] - O[v] (subsection "Accessing a Degree") and the element
// extraction of subsection "Accessing An Edge", one wave per requested
// vertex so that consecutive lanes decode consecutive elements; gap and
// Varint lists are decoded in order, 64 entries or bytes per wave step.
#include <mutex>

#include "lg_device.hpp"

namespace lg {

__global__ void dec_map_kernel(uint32_t n, const uint32_t *__restrict__ vin, uint32_t k,
                               const uint32_t *__restrict__ inv, uint32_t *__restrict__ labels,
                               uint32_t *__restrict__ bad) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride) {
        const uint32_t v = vin[i];
        if (v >= n) { atomicOr(bad, 1u); labels[i] = 0; continue; }
        labels[i] = inv ? inv[v] : v;
    }
}

template <class Acc>
__global__ void dec_degree_kernel(Acc acc, const uint32_t *__restrict__ labels, uint32_t k,
                                  uint32_t *__restrict__ deg) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride)
        deg[i] = acc.info(labels[i]).deg;
}

// Varint lists: d_v is the number of bytes with the top bit clear in the
// list's byte range; one wave per vertex counts them 8 bytes per lane.
template <class Acc>
__global__ void dec_varint_degree_kernel(Acc acc, const uint32_t *__restrict__ labels, uint32_t k,
                                         uint32_t *__restrict__ deg) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t i = wave; i < k; i += nwaves) {
        uint64_t b0, b1;
        acc.offsets(labels[i], b0, b1);
        uint32_t cnt = 0;
        for (uint64_t q = (b0 >> 3) + lane; q * 8 < b1; q += kWave) {
            const uint64_t p = q * 8;
            const uint64_t lo = p < b0 ? b0 - p : 0;         // bytes below the list
            const uint64_t hi = p + 8 > b1 ? p + 8 - b1 : 0;  // bytes above it
            uint64_t keep = ~0ull << (8 * lo);
            if (hi) keep &= ~0ull >> (8 * hi);
            cnt += (uint32_t)__popcll(~acc.word(p) & 0x8080808080808080ull & keep);
        }
        cnt = wave_sum(cnt);
        if (lane == 0) deg[i] = cnt;
    }
}

// kSorted: emit ((i << 32) | original ID) keys for the segmented sort
template <class Acc, bool kSorted>
__global__ void dec_lists_kernel(Acc acc, uint32_t n, const uint32_t *__restrict__ labels, uint32_t k,
                                 const uint64_t *__restrict__ out_off, const uint32_t *__restrict__ perm,
                                 uint32_t *__restrict__ out_ids, uint64_t *__restrict__ keys) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    if constexpr (IsGapAcc<Acc>::value) {
        // gap lists: element j is the first element plus the differences
        // 1..j; 64 at a time, a wave prefix sum plus the running total of the
        // steps before (lanes past the end read the first element and drop it)
        for (uint64_t i = wave; i < k; i += nwaves) {
            const GapInfo gi = acc.info(labels[i]);
            const uint64_t o = out_off[i];
            uint32_t carry = 0;
            for (uint64_t j0 = 0; j0 < gi.deg; j0 += kWave) {
                const uint64_t j = j0 + lane;
                const bool valid = j < gi.deg;
                const uint64_t jj = valid ? j : 0;
                const uint32_t x = acc.get(Acc::entry_bit(gi, jj), jj ? gi.g : gi.w);
                const uint32_t val = wave_incl_scan(valid ? x : 0u) + carry;
                carry = __shfl(val, kWave - 1, kWave);
                if (valid) {
                    // a stored label is < n; the clamp keeps the lookup in
                    // bounds whatever the stream holds
                    const uint32_t u = perm ? perm[val < n ? val : n - 1] : val;
                    if (kSorted) keys[o + j] = (i << 32) | u;
                    else out_ids[o + j] = u;
                }
            }
        }
    } else if constexpr (IsVarintAcc<Acc>::value) {
        // Varint lists: 64 bytes per step, one per lane.  A lane holding a
        // value's last byte (top bit clear) assembles the value from its own
        // byte and the continuation bytes right before it (at most four, the
        // ones before the step's first lane come from the previous step);
        // the value's index in the list is the number of last bytes before
        // it.  DMd adds a wave prefix sum of the differences to the running
        // label.
        for (uint64_t i = wave; i < k; i += nwaves) {
            uint64_t b0, b1;
            acc.offsets(labels[i], b0, b1);
            const uint64_t o = out_off[i];
            uint64_t done = 0;
            uint32_t carry = 0;
            uint32_t prevb = 0;  // a value's last byte: stops the look-back at the list's start
            for (uint64_t p0 = b0; p0 < b1; p0 += kWave) {
                const uint64_t p = p0 + lane;
                const bool in = p < b1;
                const uint32_t b = in ? acc.byte(p) : 128u;
                const bool end = in && !(b & 128u);
                uint32_t val = b & 127u;
                bool open = true;
#pragma unroll
                for (int t = 1; t <= 4; ++t) {
                    const int src = (int)lane - t;
                    const uint32_t cur = __shfl(b, src & (kWave - 1), kWave);
                    const uint32_t old = __shfl(prevb, src & (kWave - 1), kWave);
                    const uint32_t bt = src >= 0 ? cur : old;
                    open = open && (bt & 128u);
                    if (open) val = (val << 7) | (bt & 127u);
                }
                const uint64_t ends = __ballot(end);
                uint32_t label = val;
                if constexpr (Acc::kDifferences) {
                    const uint32_t sc = wave_incl_scan(end ? val : 0u);
                    label = carry + sc;
                    carry += __shfl(sc, kWave - 1, kWave);
                }
                if (end) {
                    const uint64_t j = done + popc_below(ends);
                    // a stored label is < n; the clamp keeps the lookup in
                    // bounds whatever the stream holds
                    const uint32_t u = perm ? perm[label < n ? label : n - 1] : label;
                    if (kSorted) keys[o + j] = (i << 32) | u;
                    else out_ids[o + j] = u;
                }
                done += (uint64_t)__popcll(ends);
                prevb = b;
            }
        }
    } else {
        for (uint64_t i = wave; i < k; i += nwaves) {
            const VInfo vi = acc.info(labels[i]);
            const uint64_t o = out_off[i];
            const uint32_t st = Acc::step(vi.w), mk = Acc::mask(vi.w);
            for (uint64_t j = lane; j < vi.deg; j += kWave) {
                uint32_t u = acc.get(vi.start + j * st, mk);
                if (perm) u = perm[u];
                if (kSorted) keys[o + j] = (i << 32) | u;
                else out_ids[o + j] = u;
            }
        }
    }
}

__global__ void dec_unkey_kernel(uint64_t total, const uint64_t *__restrict__ keys, uint32_t *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += stride)
        out[j] = (uint32_t)keys[j];
}

DecodeWork::~DecodeWork() {
    if (host && host_owned) (void)hipHostFree(host);
}

uint64_t DecodeWork::bytes() const {
    return head.bytes + scan_tmp.bytes + keys.bytes + keys2.bytes + vals.bytes + vals2.bytes + sort_tmp.bytes;
}

lg_status decode_run(lg_graph *g, DecodeWork &w, const uint32_t *vertices, uint32_t k, uint64_t *out_off,
                     uint32_t *out_ids, uint64_t cap, uint32_t flags, hipStream_t stream, uint64_t *total_out) {
    if (total_out) *total_out = 0;
    if (k == 0) return fill_u64(out_off, 0, 1, stream);
    if (!w.host) {
        if (hipHostMalloc((void **)&w.host, 4 * sizeof(uint64_t)) != hipSuccess) {
            w.host = nullptr;
            set_error("lg_decode_neighbors: pinned host allocation failed");
            return LG_ERR_OOM;
        }
    }
    const bool rel = g->relabel != LG_RELABEL_NONE;
    const uint32_t *inv = (rel && flags != LG_DECODE_RAW) ? g->inv.as<uint32_t>() : nullptr;
    const uint32_t *perm = (rel && flags != LG_DECODE_RAW) ? g->perm.as<uint32_t>() : nullptr;
    const bool sorted = rel && flags == LG_DECODE_SORTED;

    // head: labels (k) | degrees (k) | flag
    LG_TRY(w.head.ensure(((uint64_t)k * 8 + 8 + 7) & ~7ull));
    uint32_t *labels = w.head.as<uint32_t>();
    uint32_t *deg = labels + k;
    uint32_t *bad = deg + k;
    LG_TRY(fill_u32(bad, 0, 1, stream));
    LG_LAUNCH(dec_map_kernel, grid_for(k, 256, 1u << 16), 256, 0, stream, g->n, vertices, k, inv, labels, bad);
    LG_CHECK_LAUNCH();
    return dispatch_acc_decode(g, [&](auto acc) -> lg_status {
        using Acc = decltype(acc);
        if constexpr (IsVarintAcc<Acc>::value)
            LG_LAUNCH(dec_varint_degree_kernel<Acc>, grid_for((uint64_t)k * kWave, 256, 1u << 16), 256, 0, stream,
                      acc, labels, k, deg);
        else
            LG_LAUNCH(dec_degree_kernel<Acc>, grid_for(k, 256, 1u << 16), 256, 0, stream, acc, labels, k, deg);
        LG_CHECK_LAUNCH();
        LG_TRY(exclusive_scan_u32(deg, out_off, k, w.scan_tmp, stream));
        LG_CHECK_HIP(hipMemcpyAsync(w.host, out_off + k, 8, hipMemcpyDeviceToHost, stream));
        LG_CHECK_HIP(hipMemcpyAsync(w.host + 1, bad, 4, hipMemcpyDeviceToHost, stream));
        LG_CHECK_HIP(hipStreamSynchronize(stream));
        if (*reinterpret_cast<uint32_t *>(w.host + 1)) {
            set_error("lg_decode_neighbors: vertex id >= n");
            return LG_ERR_INVALID;
        }
        const uint64_t total = w.host[0];
        if (total_out) *total_out = total;
        if (!out_ids || total > cap) {
            set_error("lg_decode_neighbors: %llu ids do not fit in capacity %llu", (unsigned long long)total,
                      (unsigned long long)cap);
            return LG_ERR_CAPACITY;
        }
        if (total == 0) return LG_OK;
        const uint32_t grid = grid_for((uint64_t)k * kWave, 256, 1u << 16);
        if (!sorted) {
            LG_LAUNCH((dec_lists_kernel<Acc, false>), grid, 256, 0, stream, acc, g->n, labels, k,
                      (const uint64_t *)out_off, perm, out_ids, (uint64_t *)nullptr);
            LG_CHECK_LAUNCH();
            return LG_OK;
        }
        LG_TRY(w.keys.ensure(total * 8));
        LG_TRY(w.keys2.ensure(total * 8));
        LG_TRY(w.vals.ensure(total * 4));
        LG_TRY(w.vals2.ensure(total * 4));
        LG_LAUNCH((dec_lists_kernel<Acc, true>), grid, 256, 0, stream, acc, g->n, labels, k,
                  (const uint64_t *)out_off, perm, out_ids, w.keys.as<uint64_t>());
        LG_CHECK_LAUNCH();
        const uint32_t bits = 32 + bitlen_u64(k - 1);
        LG_TRY(radix_sort_pairs64(w.keys.as<uint64_t>(), w.vals.as<uint32_t>(), w.keys2.as<uint64_t>(),
                                  w.vals2.as<uint32_t>(), total, bits, w.sort_tmp, stream));
        LG_LAUNCH(dec_unkey_kernel, grid_for(total, 256, 1u << 16), 256, 0, stream, total, w.keys.as<uint64_t>(),
                  out_ids);
        LG_CHECK_LAUNCH();
        return LG_OK;
    });
}

}  // namespace lg

static lg_status lg_decode_neighbors_impl(const lg_graph *gc, const uint32_t *vertices, uint32_t k,
                                         uint64_t *out_off, uint32_t *out_ids, uint64_t cap, uint32_t flags,
                                         hipStream_t stream) {
    using namespace lg;
    lg_graph *g = const_cast<lg_graph *>(gc);
    if (!g || !out_off || (k && !vertices)) { set_error("lg_decode_neighbors: NULL argument"); return LG_ERR_INVALID; }
    if (flags > LG_DECODE_RAW) { set_error("lg_decode_neighbors: unknown flags"); return LG_ERR_INVALID; }
    if (!g->dec) {
        g->dec = new (std::nothrow) DecodeWork();
        if (!g->dec) { set_error("lg_decode_neighbors: host allocation failed"); return LG_ERR_OOM; }
    }
    const lg_status st = decode_run(g, *g->dec, vertices, k, out_off, out_ids, cap, flags, stream, nullptr);
    if (st == LG_OK) LG_CHECK_HIP(hipStreamSynchronize(stream));
    return st;
}

extern "C" lg_status lg_decode_neighbors(const lg_graph *gc, const uint32_t *vertices, uint32_t k,
                                         uint64_t *out_off, uint32_t *out_ids, uint64_t cap, uint32_t flags,
                                         hipStream_t stream) {
    const lg_status st = lg_decode_neighbors_impl(gc, vertices, k, out_off, out_ids, cap, flags, stream);
    if (gc && (st == LG_OK || st == LG_ERR_CAPACITY)) LG_TRY(lg::mark_use(const_cast<lg_graph *>(gc), stream));
    return st;
}

// ---------------------------------------------------------------------------
// lg_decode_neighbors_noalloc: the same decode, its temporaries in a fixed
// device array instead of buffers allocated for the graph
// ---------------------------------------------------------------------------

// One copy per GPU, loaded with the library's code object.  In host code this
// name is a stand-in, not a device address: the address on each device comes
// from hipGetSymbolAddress and is the only one passed to kernels.
static __device__ __align__(256) unsigned char scratch[LG_NOALLOC_SCRATCH_BYTES];

namespace lg {
namespace {

constexpr int kNoallocDevices = 64;

struct NoallocDevice {
    std::mutex mu;        // calls on one GPU share its array: one at a time
    void *ptr = nullptr;  // device address of `scratch` on this GPU (set once)
};
NoallocDevice g_noalloc[kNoallocDevices];

inline uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// byte offsets of the temporaries inside the array, for the largest request
struct NoallocLayout {
    uint64_t head, scan, keys, keys2, vals, vals2, sort, end;
};
NoallocLayout noalloc_layout() {
    NoallocLayout L{};
    uint64_t o = 0;
    L.head = o;  o += align256((uint64_t)LG_NOALLOC_MAX_VERTICES * 8 + 8);  // labels | degrees | flag
    L.scan = o;  o += align256(scan_tmp_bytes(LG_NOALLOC_MAX_VERTICES));
    L.keys = o;  o += align256((uint64_t)LG_NOALLOC_MAX_SORTED_IDS * 8);
    L.keys2 = o; o += align256((uint64_t)LG_NOALLOC_MAX_SORTED_IDS * 8);
    L.vals = o;  o += align256((uint64_t)LG_NOALLOC_MAX_SORTED_IDS * 4);
    L.vals2 = o; o += align256((uint64_t)LG_NOALLOC_MAX_SORTED_IDS * 4);
    L.sort = o;  o += align256(radix_sort_tmp_bytes(LG_NOALLOC_MAX_SORTED_IDS));
    L.end = o;
    return L;
}

}  // namespace
}  // namespace lg

extern "C" lg_status lg_decode_neighbors_noalloc(const lg_graph *gc, const uint32_t *vertices, uint32_t k,
                                                 uint64_t *out_off, uint32_t *out_ids, uint64_t cap,
                                                 uint32_t flags, hipStream_t stream) {
    using namespace lg;
    lg_graph *g = const_cast<lg_graph *>(gc);
    if (!g || !out_off || (k && !vertices)) {
        set_error("lg_decode_neighbors_noalloc: NULL argument");
        return LG_ERR_INVALID;
    }
    if (flags > LG_DECODE_RAW) { set_error("lg_decode_neighbors_noalloc: unknown flags"); return LG_ERR_INVALID; }
    if (k > LG_NOALLOC_MAX_VERTICES) {
        set_error("lg_decode_neighbors_noalloc: %u vertices exceed the limit of %u (LG_NOALLOC_MAX_VERTICES)", k,
                  (unsigned)LG_NOALLOC_MAX_VERTICES);
        return LG_ERR_UNSUPPORTED;
    }
    int dev = 0;
    LG_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoallocDevices) {
        set_error("lg_decode_neighbors_noalloc: device %d beyond the %d supported", dev, kNoallocDevices);
        return LG_ERR_UNSUPPORTED;
    }
    const NoallocLayout L = noalloc_layout();
    if (L.end > sizeof(scratch)) {
        set_error("lg_decode_neighbors_noalloc: temporaries need %llu bytes, the array holds %llu",
                  (unsigned long long)L.end, (unsigned long long)sizeof(scratch));
        return LG_ERR_UNSUPPORTED;
    }
    NoallocDevice &D = g_noalloc[dev];
    std::lock_guard<std::mutex> hold(D.mu);
    if (!D.ptr) {
        // once per GPU, with that GPU current: this GPU's copy of the array
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("lg_decode_neighbors_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
            return LG_ERR_DEVICE;
        }
        D.ptr = p;
    }
    char *base = static_cast<char *>(D.ptr);
    DecodeWork w;
    w.head.borrow(base + L.head, L.scan - L.head);
    w.scan_tmp.borrow(base + L.scan, L.keys - L.scan);
    w.keys.borrow(base + L.keys, L.keys2 - L.keys);
    w.keys2.borrow(base + L.keys2, L.vals - L.keys2);
    w.vals.borrow(base + L.vals, L.vals2 - L.vals);
    w.vals2.borrow(base + L.vals2, L.sort - L.vals2);
    w.sort_tmp.borrow(base + L.sort, L.end - L.sort);
    uint64_t slots[4] = {0, 0, 0, 0};  // readback into host memory the caller's thread owns
    w.host = slots;
    w.host_owned = false;
    uint64_t total = 0;
    const lg_status st = decode_run(g, w, vertices, k, out_off, out_ids, cap, flags, stream, &total);
    w.host = nullptr;
    // the next call may reuse the array only after this one's kernels ran
    const hipError_t se = hipStreamSynchronize(stream);
    if (st == LG_ERR_UNSUPPORTED && total > LG_NOALLOC_MAX_SORTED_IDS) {
        // the only temporaries whose size depends on the result: the sort keys
        set_error("lg_decode_neighbors_noalloc: sorting %llu ids exceeds the limit of %u "
                  "(LG_NOALLOC_MAX_SORTED_IDS)", (unsigned long long)total, (unsigned)LG_NOALLOC_MAX_SORTED_IDS);
        return st;
    }
    if (st != LG_OK && st != LG_ERR_CAPACITY) return st;
    if (se != hipSuccess) {
        set_error("lg_decode_neighbors_noalloc: hipStreamSynchronize failed: %s", hipGetErrorString(se));
        return LG_ERR_DEVICE;
    }
    LG_TRY(mark_use(g, stream));
    return st;
}
