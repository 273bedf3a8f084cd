// Wave-level helpers of the in-order list readers: Varint steps (subsection
// "Incorporating Degree-Minimizing (DM)": base-128 values, lowest group
// first, the top bit set on every byte of a value but its last) and the
// wave-cooperative offset decode shared with the gap-list kernels.
#pragma once

#include "lg_device.hpp"

namespace lg {

// One step of 64 bytes [p0, p0 + 64) of a list ending at b1: whether this
// lane holds a value's last byte, and the value (a label, or for DMd a
// difference to be summed by the caller).  prevb is this lane's byte of the
// previous step (0 before the list: a value's end).
template <class Acc>
__device__ __forceinline__ bool varint_step(const Acc &acc, uint64_t p0, uint64_t b1, uint32_t &prevb,
                                            uint32_t &val) {
    const uint32_t lane = lane_id();
    const uint64_t p = p0 + lane;
    const bool in = p < b1;
    const uint32_t b = in ? acc.byte(p) : 128u;
    const bool end = in && !(b & 128u);
    uint32_t v = b & 127u;
    bool open = true;
#pragma unroll
    for (int t = 1; t <= 4; ++t) {
        const int src = (int)lane - t;
        const uint32_t cur = __shfl(b, src & (kWave - 1), kWave);
        const uint32_t old = __shfl(prevb, src & (kWave - 1), kWave);
        const uint32_t bt = src >= 0 ? cur : old;
        open = open && (bt & 128u);
        if (open) v = (v << 7) | (bt & 127u);
    }
    prevb = b;
    val = v;
    return end;
}

// The look-back bytes for a step starting at chunk start c0 inside the list
// [b0, b1): the last four lanes hold the four bytes before c0 (0 before the
// list: a value's end), as varint_step reads them from the previous step.
template <class Acc>
__device__ __forceinline__ uint32_t varint_chunk_prevb(const Acc &acc, uint64_t b0, uint64_t c0) {
    const uint32_t lane = lane_id();
    if (lane < kWave - 4 || c0 < b0 + (kWave - lane)) return 0u;
    return acc.byte(c0 - (kWave - lane));
}

// The two offset values bracketing the list of v0 + lane, decoded by the
// whole wave for a 64-aligned v0 (with Elias-Fano offsets one select per
// wave instead of one per lane); every lane of the wave must call it.
// Base: the local-ID packed accessor under a gap or Varint accessor.
template <class Base>
__device__ __forceinline__ void wave_offsets(const Base &acc, uint64_t v0, uint32_t n, uint64_t &o0, uint64_t &o1) {
    const uint32_t lane = lane_id();
    const uint64_t v = v0 + lane;
    const uint64_t vv = v < n ? v : n;
    const uint64_t ve = v0 + kWave < n ? v0 + kWave : n;
    uint64_t end;
    if constexpr (Base::kEF) {
        const EFView &e = acc.pv.ef;
        const uint64_t lo0 = e.l ? extract64(e.L, vv * e.l, e.l) : 0ull;
        const uint64_t lo_end = (e.l && v0 + kWave <= n) ? extract64(e.L, ve * e.l, e.l) : 0ull;
        uint64_t pos, pos_end;
        ef_wave_select(e, v0, n + 1, ef_samples(e, v0, n + 1), pos, pos_end);
        if (v > n) pos = 0;
        o0 = v <= n ? (((pos - vv) << e.l) | lo0) : 0ull;
        if (v0 + kWave <= n) end = ((pos_end - ve) << e.l) | lo_end;
        else end = __shfl(o0, (uint32_t)(n - v0), kWave);
    } else {
        o0 = acc.offset_value((uint32_t)vv);
        end = acc.offset_value((uint32_t)ve);
    }
    o1 = __shfl_down(o0, 1, kWave);
    if (lane == kWave - 1) o1 = end;
}

// The sampled direction estimate of the in-order traversals: degrees (gap)
// or list bytes (Varint) of kDirSample frontier vertices at evenly spaced
// queue positions, a partial sum per block.
}  // namespace lg
