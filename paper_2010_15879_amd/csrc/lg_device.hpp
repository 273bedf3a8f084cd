// Device-side building blocks of liblg: bit-field extraction from packed
// streams, Elias-Fano select, per-vertex accessors for every layout, and
// wave64 primitives for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lg_internal.hpp"

namespace lg {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// wave64 primitives
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of `mask` at lanes below this one
__device__ __forceinline__ uint32_t popc_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <class T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T y = __shfl_up(x, d, kWave);
        if (lane >= (uint32_t)d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x |= __shfl_xor(x, d, kWave);
    return x;
}

template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// ---------------------------------------------------------------------------
// bit-field extraction
// ---------------------------------------------------------------------------

// A packed list element of width <= 32: the two 32-bit words holding stream
// bits [bit, bit + 32) are joined with one funnel shift (v_alignbit_b32) and
// masked.  The zero pad word at the end of every stream keeps A32[k + 1] in
// bounds.
__device__ __forceinline__ uint32_t extract32(const uint32_t *__restrict__ A32, uint64_t bit,
                                              uint32_t mask) {
    const uint64_t k = bit >> 5;
    const uint32_t lo = A32[k];
    const uint32_t hi = A32[k + 1];
    return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)bit & 31u) & mask;
}

__device__ __forceinline__ uint32_t width_mask(uint32_t w) {
    return w >= 32 ? 0xFFFFFFFFu : ((1u << w) - 1u);
}

// A fixed-width field of up to 64 bits from a stream of 64-bit words.
__device__ __forceinline__ uint64_t extract64(const uint64_t *__restrict__ S, uint64_t bit, uint32_t w) {
    if (w == 0) return 0;
    const uint64_t k = bit >> 6;
    const uint32_t sh = (uint32_t)bit & 63u;
    uint64_t v = S[k] >> sh;
    if (sh + w > 64) v |= S[k + 1] << (64 - sh);
    return w >= 64 ? v : (v & ((1ull << w) - 1ull));
}

// ---------------------------------------------------------------------------
// Elias-Fano select over the upper bit vector H
// ---------------------------------------------------------------------------

// Position of the r-th set bit (0-based) of x; x must hold more than r ones.
__device__ __forceinline__ uint32_t select_in_word(uint64_t x, uint32_t r) {
    uint32_t pos = 0;
    uint32_t w = (uint32_t)x;
    uint32_t c = __popc(w);
    if (r >= c) { r -= c; pos = 32; w = (uint32_t)(x >> 32); }
    c = __popc(w & 0xFFFFu);
    if (r >= c) { r -= c; pos += 16; w >>= 16; }
    c = __popc(w & 0xFFu);
    if (r >= c) { r -= c; pos += 8; w >>= 8; }
    c = __popc(w & 0xFu);
    if (r >= c) { r -= c; pos += 4; w >>= 4; }
    c = __popc(w & 0x3u);
    if (r >= c) { r -= c; pos += 2; w >>= 2; }
    c = w & 1u;
    if (r >= c) pos += 1;
    return pos;
}

// select1(k): the sample table gives the position of one number 64*floor(k/64);
// the rank directory is searched between that superblock and the next
// sample's, then at most eight words are scanned with popcount.  The
// directory matters where H is sparse (between the offsets of long lists
// lie thousands of zero words).
__device__ __forceinline__ uint64_t ef_select1(const EFView &e, uint32_t k) {
    const uint32_t j = k >> 6;
    const uint32_t p = e.sel[j];
    if ((k & 63u) == 0) return p;
    uint32_t lo = p >> 9;
    uint32_t hi = (j + 1 < e.n_sel) ? (e.sel[j + 1] >> 9) : (e.n_sb - 1);
    while (lo < hi) {  // largest superblock b with rank_sb[b] <= k
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (e.rank_sb[mid] <= k) lo = mid; else hi = mid - 1;
    }
    uint32_t r = e.rank_sb[lo];
    uint64_t wi = (uint64_t)lo * 8;
    for (;;) {
        const uint64_t x = e.H[wi];
        const uint32_t c = (uint32_t)__popcll(x);
        if (r + c > k) return wi * 64 + select_in_word(x, k - r);
        r += c;
        ++wi;
    }
}

// The same select for random vertices (top-down frontiers, tables): one
// number k is the (k mod 64)-th one after the sample's position p; the four
// words from p are loaded at once and searched in registers, which settles
// dense stretches of H in one round trip after the sample; a longer gap goes
// through the rank directory.
__device__ __forceinline__ uint64_t ef_select1_wide(const EFView &e, uint32_t k) {
    const uint64_t p = e.sel[k >> 6];
    uint32_t need = k & 63u;
    if (need == 0) return p;
    --need;  // index among the ones after p
    const uint64_t w0 = p >> 6;
    const uint32_t sh = (uint32_t)(p & 63u);
    uint64_t x[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) x[t] = w0 + t < e.n_hw ? e.H[w0 + t] : 0ull;
    x[0] = sh == 63 ? 0ull : (x[0] & (~0ull << (sh + 1)));
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const uint32_t c = (uint32_t)__popcll(x[t]);
        if (need < c) return (w0 + t) * 64 + select_in_word(x[t], need);
        need -= c;
    }
    return ef_select1(e, k);
}

// position of the first set bit of H after position p (one must exist)
__device__ __forceinline__ uint64_t ef_next_one(const EFView &e, uint64_t p) {
    uint64_t wi = p >> 6;
    const uint32_t sh = (uint32_t)(p & 63);
    uint64_t x = sh == 63 ? 0ull : (e.H[wi] & (~0ull << (sh + 1)));
    while (!x) x = e.H[++wi];
    return wi * 64 + (uint64_t)(__ffsll((long long)x) - 1);
}

__device__ __forceinline__ uint64_t ef_get(const EFView &e, uint32_t v) {
    const uint64_t pos = ef_select1(e, v);
    const uint64_t low = e.l ? extract64(e.L, (uint64_t)v * e.l, e.l) : 0ull;
    return ((pos - v) << e.l) | low;
}

// ---------------------------------------------------------------------------
// select over the interleaved bit vector (bvIL)
// ---------------------------------------------------------------------------

// select1(k): a binary search over the blocks' leading counts for the block
// holding the k-th one (the last block whose count of earlier ones is at most
// k; the k-th one sits at position >= k, so no block before k / 512), then a
// popcount scan of at most eight data words.  k must be below the number of
// ones.
__device__ __forceinline__ uint64_t il_select1(const ILView &e, uint64_t k) {
    uint64_t lo = k >> 9, hi = e.blocks - 1;
    if (lo > hi) lo = hi;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (e.W[9 * mid] <= k) lo = mid; else hi = mid - 1;
    }
    uint64_t r = k - e.W[9 * lo];
    const uint64_t *d = e.W + 9 * lo + 1;
    uint32_t t = 0;
    for (; t < 7; ++t) {
        const uint64_t c = (uint64_t)__popcll(d[t]);
        if (r < c) break;
        r -= c;
    }
    return lo * 512 + (uint64_t)t * 64 + select_in_word(d[t], (uint32_t)r);
}

// position of the first one after position p, skipping the count words
// between blocks (one must exist)
__device__ __forceinline__ uint64_t il_next_one(const ILView &e, uint64_t p) {
    const uint64_t q = p + 1;
    uint64_t j = q >> 9;
    uint32_t t = (uint32_t)(q >> 6) & 7u;
    const uint32_t sh = (uint32_t)q & 63u;
    uint64_t x = e.W[9 * j + 1 + t] & (~0ull << sh);
    while (!x) {
        if (++t == 8) { t = 0; ++j; }
        x = e.W[9 * j + 1 + t];
    }
    return j * 512 + (uint64_t)t * 64 + (uint64_t)(__ffsll((long long)x) - 1);
}

// exact quotient of a multiple of w (1 <= w <= 32) by w, below 2^51
static __device__ __constant__ double c_inv_width[33] = {
    0.0, 1.0, 1.0 / 2, 1.0 / 3, 1.0 / 4, 1.0 / 5, 1.0 / 6, 1.0 / 7, 1.0 / 8, 1.0 / 9, 1.0 / 10,
    1.0 / 11, 1.0 / 12, 1.0 / 13, 1.0 / 14, 1.0 / 15, 1.0 / 16, 1.0 / 17, 1.0 / 18, 1.0 / 19,
    1.0 / 20, 1.0 / 21, 1.0 / 22, 1.0 / 23, 1.0 / 24, 1.0 / 25, 1.0 / 26, 1.0 / 27, 1.0 / 28,
    1.0 / 29, 1.0 / 30, 1.0 / 31, 1.0 / 32};

__device__ __forceinline__ uint32_t exact_div_width(uint64_t x, uint32_t w) {
    return (uint32_t)((double)x * c_inv_width[w] + 0.5);
}

// ---------------------------------------------------------------------------
// per-vertex accessors
// ---------------------------------------------------------------------------

// start: first bit of the list (packed) or first element index (plain);
// deg: list length; w: element width (packed) or 32 (plain).
struct VInfo {
    uint64_t start;
    uint32_t deg;
    uint32_t w;
};

enum : int { kIdsGlobal = 0, kIdsLocal = 1 };
enum : int { kOffsPacked = 0, kOffsEF = 1, kOffsIL = 2 };

template <int IDM, int OFM>
struct PackedAcc {
    PackedView pv;
    static constexpr bool kPacked = true;
    static constexpr bool kEF = OFM == kOffsEF;

    __device__ __forceinline__ uint64_t offset_value(uint32_t v) const {
        if constexpr (OFM == kOffsPacked) return extract64(pv.po.O, (uint64_t)v * pv.po.w, pv.po.w);
        else if constexpr (OFM == kOffsIL) return il_select1(pv.il, v) - v;
        else return ef_get(pv.ef, v);
    }
    __device__ __forceinline__ uint32_t width(uint32_t v) const {
        if constexpr (IDM == kIdsGlobal) return pv.s;
        else return (uint32_t)extract64(pv.W, (uint64_t)v * pv.F, pv.F);
    }
    // info from the two offset values bracketing the list of v
    __device__ __forceinline__ VInfo make(uint32_t v, uint64_t o0, uint64_t o1) const {
        VInfo r;
        if constexpr (IDM == kIdsGlobal) {
            r.start = o0 * pv.s;
            r.deg = (uint32_t)(o1 - o0);
            r.w = pv.s;
        } else {
            r.w = width(v);
            r.start = o0;
            r.deg = r.w ? exact_div_width(o1 - o0, r.w) : 0u;
        }
        return r;
    }
    // make() with the width already loaded (ignored in global mode)
    __device__ __forceinline__ VInfo make_w(uint32_t v, uint64_t o0, uint64_t o1, uint32_t w) const {
        VInfo r;
        if constexpr (IDM == kIdsGlobal) {
            (void)w;
            r.start = o0 * pv.s;
            r.deg = (uint32_t)(o1 - o0);
            r.w = pv.s;
        } else {
            r.w = w;
            r.start = o0;
            r.deg = r.w ? exact_div_width(o1 - o0, r.w) : 0u;
        }
        return r;
    }
    // the two offset values bracketing the list of v
    __device__ __forceinline__ void offsets(uint32_t v, uint64_t &o0, uint64_t &o1) const {
        if constexpr (OFM == kOffsPacked) {
            o0 = offset_value(v);
            o1 = offset_value(v + 1);
        } else if constexpr (OFM == kOffsIL) {
            // x_{v+1}'s one is the next one after x_v's
            const uint64_t p0 = il_select1(pv.il, v);
            o0 = p0 - v;
            o1 = il_next_one(pv.il, p0) - v - 1;
        } else {
            // x_{v+1}'s upper bit is the next one of H after x_v's
            const EFView &e = pv.ef;
            const uint64_t p0 = ef_select1_wide(e, v);
            const uint64_t p1 = ef_next_one(e, p0);
            const uint64_t lo0 = e.l ? extract64(e.L, (uint64_t)v * e.l, e.l) : 0ull;
            const uint64_t lo1 = e.l ? extract64(e.L, (uint64_t)(v + 1) * e.l, e.l) : 0ull;
            o0 = ((p0 - v) << e.l) | lo0;
            o1 = ((p1 - v - 1) << e.l) | lo1;
        }
    }
    __device__ __forceinline__ VInfo info(uint32_t v) const {
        uint64_t o0, o1;
        offsets(v, o0, o1);
        return make(v, o0, o1);
    }
    // element at position `pos` (a bit position)
    __device__ __forceinline__ uint32_t get(uint64_t pos, uint32_t mask) const {
        return extract32(pv.A32, pos, mask);
    }
    __device__ __forceinline__ static uint32_t step(uint32_t w) { return w; }
    __device__ __forceinline__ static uint32_t mask(uint32_t w) { return width_mask(w); }
};

template <bool OFF64>
struct PlainAcc {
    PlainView pv;
    static constexpr bool kPacked = false;
    static constexpr bool kEF = false;

    __device__ __forceinline__ uint64_t offset_value(uint32_t v) const {
        if constexpr (OFF64) return static_cast<const uint64_t *>(pv.off)[v];
        else return static_cast<const uint32_t *>(pv.off)[v];
    }
    __device__ __forceinline__ VInfo make(uint32_t, uint64_t o0, uint64_t o1) const {
        VInfo r;
        r.start = o0;
        r.deg = (uint32_t)(o1 - o0);
        r.w = 32;
        return r;
    }
    __device__ __forceinline__ VInfo info(uint32_t v) const {
        return make(v, offset_value(v), offset_value(v + 1));
    }
    __device__ __forceinline__ uint32_t get(uint64_t pos, uint32_t) const { return pv.col[pos]; }
    __device__ __forceinline__ static uint32_t step(uint32_t) { return 1; }
    __device__ __forceinline__ static uint32_t mask(uint32_t) { return 0xFFFFFFFFu; }
};

// Fixed-size gap encoding (subsection "Adding Fixed-Size Gap Encoding",
// local approach): the list of v is its first element at w_v bits, then its
// d_v - 1 differences at g_v bits.  The offsets are bit starts, as in the
// local approach, so d_v follows from the list's bit length l:
// 0 when l = 0, 1 when g_v = 0, else 1 + (l - w_v) / g_v.  Entries are read
// in order only (a running sum); the traversal kernels, which read entries
// at any position, do not take this accessor.
struct GapInfo {
    uint64_t start;
    uint32_t deg;
    uint32_t w;  // width of the first element
    uint32_t g;  // width of every difference
};

template <int OFM>
struct GapAcc {
    PackedAcc<kIdsLocal, OFM> base;  // offsets, width table and stream

    __device__ __forceinline__ uint32_t gap_width(uint32_t v) const {
        return (uint32_t)extract64(base.pv.G, (uint64_t)v * base.pv.F, base.pv.F);
    }
    __device__ __forceinline__ GapInfo info(uint32_t v) const {
        uint64_t o0, o1;
        base.offsets(v, o0, o1);
        GapInfo r;
        r.start = o0;
        r.w = base.width(v);
        r.g = gap_width(v);
        const uint64_t l = o1 - o0;
        r.deg = l == 0 ? 0u : (r.g == 0 ? 1u : 1u + exact_div_width(l - r.w, r.g));
        return r;
    }
    // bit position and width of entry i of a list (first element, then
    // differences)
    __device__ __forceinline__ static uint64_t entry_bit(const GapInfo &gi, uint64_t i) {
        return i == 0 ? gi.start : gi.start + gi.w + (i - 1) * gi.g;
    }
    __device__ __forceinline__ uint32_t get(uint64_t bit, uint32_t w) const { return base.get(bit, width_mask(w)); }
};

// Varint lists (subsection "Incorporating Degree-Minimizing (DM)"): a
// byte stream of base-128 values, lowest group first, the top bit set on
// every byte of a value but its last; the offsets are byte starts.  kDiff:
// the first value is a label and each further one the difference to the
// previous label (DMd); otherwise every value is a label (DMf).
template <int OFM, bool kDiff>
struct VarintAcc {
    static constexpr bool kDifferences = kDiff;
    PackedAcc<kIdsLocal, OFM> base;  // offsets and stream

    __device__ __forceinline__ void offsets(uint32_t v, uint64_t &b0, uint64_t &b1) const {
        base.offsets(v, b0, b1);
    }
    __device__ __forceinline__ uint32_t byte(uint64_t p) const {
        return reinterpret_cast<const uint8_t *>(base.pv.A32)[p];
    }
    // 8 stream bytes from the 8-aligned position p (the stream ends in a zero
    // pad word, so any word that holds a stream byte is readable)
    __device__ __forceinline__ uint64_t word(uint64_t p) const {
        return reinterpret_cast<const uint64_t *>(base.pv.A32)[p >> 3];
    }
};

// Upper-bit positions of ones number v0 + lane and v0 + 64 (broadcast) for a
// 64-aligned v0: sel[v0/64] is select1(v0) and sel[v0/64 + 1] is select1(v0 +
// 64), so the 65 ones lie in the H words between those two positions.  When
// they span at most 64 words, lane i loads word i, a wave prefix of the
// popcounts tells every lane which word holds its one, and an in-word select
// finishes; otherwise each lane runs a full select.
// The two samples sel[v0/64] and sel[v0/64 + 1] (0 when v0 + 64 >= count),
// loaded ahead by callers that can issue them early.
struct EFSamples {
    uint64_t p0, p1;
};

__device__ __forceinline__ EFSamples ef_samples(const EFView &e, uint64_t v0, uint32_t count) {
    const uint32_t q = (uint32_t)(v0 >> 6);
    return EFSamples{e.sel[q], v0 + kWave < count ? e.sel[q + 1] : 0ull};
}

__device__ __forceinline__ void ef_wave_select(const EFView &e, uint64_t v0, uint32_t count, EFSamples smp,
                                               uint64_t &pos, uint64_t &pos_end) {
    const uint32_t lane = lane_id();
    const uint64_t p0 = smp.p0;
    // one number v0 + 64 exists iff v0 + 64 < count
    const bool have_end = v0 + kWave < count;
    const uint64_t p1 = smp.p1;
    const uint64_t w0 = p0 >> 6;
    const uint64_t w1 = have_end ? (p1 >> 6) : w0 + kWave;  // unknown end: let the fallback decide
    if (have_end && w1 - w0 < (uint64_t)kWave) {
        const uint32_t nw = (uint32_t)(w1 - w0 + 1);
        uint64_t x = lane < nw ? e.H[w0 + lane] : 0ull;
        if (lane == 0) x &= ~0ull << (p0 & 63);
        const uint32_t c = (uint32_t)__popcll(x);
        const uint32_t incl = wave_incl_scan(c);
        // lane t wants one number t of the window (t = 0..63): the word i with
        // excl(i) <= t < incl(i), i.e. the count of words whose inclusive
        // prefix is <= t.  Fixed power-of-two steps keep every shuffle
        // wave-uniform; the window holds at least 65 ones, so lo < nw.
        uint32_t lo = 0;
#pragma unroll
        for (uint32_t step = kWave / 2; step > 0; step >>= 1) {
            const uint32_t probe = lo + step - 1;  // at most 62
            const uint32_t val = __shfl(incl, probe, kWave);
            if (probe < nw && val <= lane) lo += step;
        }
        const uint64_t xi = __shfl(x, lo, kWave);
        const uint32_t ei = __shfl(incl, lo, kWave) - __shfl(c, lo, kWave);
        pos = (w0 + lo) * 64 + select_in_word(xi, lane - ei);
        pos_end = p1;
        return;
    }
    const uint64_t v = v0 + lane;
    pos = v < count ? ef_select1(e, (uint32_t)v) : 0;
    pos_end = (v0 + kWave < count) ? ef_select1(e, (uint32_t)(v0 + kWave)) : 0;
}

// VInfo of vertex v0 + lane for the 64 lanes of a wave (v0 a multiple of
// 64): every lane decodes one offset value and takes the next one from its
// neighbor lane, so a sweep over consecutive vertices decodes each offset
// once.  Lanes past n get an empty list.  With Elias-Fano offsets the low
// bits and widths do not depend on the select, so they are loaded first and
// overlap it; `smp` carries select samples a caller loaded ahead.
template <class Acc>
__device__ __forceinline__ VInfo wave_info(const Acc &acc, uint64_t v0, uint32_t n, const EFSamples *smp = nullptr) {
    const uint32_t lane = lane_id();
    const uint64_t v = v0 + lane;
    if (v0 >= n) return VInfo{0, 0, 0};  // wave-uniform: a block past the last vertex
    uint64_t o0, end;
    if constexpr (Acc::kPacked && Acc::kEF) {
        const EFView &e = acc.pv.ef;
        const uint64_t vv = v < n ? v : n;
        const uint64_t ve = v0 + kWave < n ? v0 + kWave : n;
        const uint64_t lo0 = e.l ? extract64(e.L, vv * e.l, e.l) : 0ull;
        const uint64_t lo_end = (e.l && v0 + kWave <= n) ? extract64(e.L, ve * e.l, e.l) : 0ull;
        const uint32_t wv = v < n ? acc.width((uint32_t)v) : 0u;
        uint64_t pos, pos_end;
        ef_wave_select(e, v0, n + 1, smp ? *smp : ef_samples(e, v0, n + 1), pos, pos_end);
        if (v > n) pos = 0;
        o0 = v <= n ? (((pos - vv) << e.l) | lo0) : 0ull;
        // the end value: one number ve; when ve = n it is one number n itself
        if (v0 + kWave <= n) {
            end = ((pos_end - ve) << e.l) | lo_end;
        } else {
            end = __shfl(o0, (uint32_t)(n - v0), kWave);
        }
        uint64_t o1 = __shfl_down(o0, 1, kWave);
        if (lane == kWave - 1) o1 = end;
        if (v >= n) return VInfo{0, 0, 0};
        return acc.make_w((uint32_t)v, o0, o1, wv);
    } else {
        (void)smp;
        o0 = acc.offset_value((uint32_t)(v < n ? v : n));
        end = acc.offset_value((uint32_t)(v0 + kWave < n ? v0 + kWave : n));
        uint64_t o1 = __shfl_down(o0, 1, kWave);
        if (lane == kWave - 1) o1 = end;
        if (v >= n) return VInfo{0, 0, 0};
        return acc.make((uint32_t)v, o0, o1);
    }
}

// Sum of one value per thread over a block of up to 1024 threads (result
// valid in thread 0).  Every thread of the block must call it.
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long x) {
    __shared__ unsigned long long s_part[16];
    x = wave_sum(x);
    const uint32_t wv = threadIdx.x / kWave;
    if (lane_id() == 0) s_part[wv] = x;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (uint32_t w = 0; w < (blockDim.x + kWave - 1) / kWave; ++w) t += s_part[w];
    __syncthreads();
    return t;
}

// index of v in the ascending heavy list (v must be in it)
__device__ __forceinline__ uint32_t heavy_index(const uint32_t *__restrict__ heavy, uint32_t n_heavy, uint32_t v) {
    uint32_t lo = 0, hi = n_heavy - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (heavy[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Call `fn(acc)` with the accessor matching the graph's layout.
template <class Fn>
lg_status dispatch_acc(const lg_graph *g, Fn &&fn) {
    if (g->layout == LG_LAYOUT_PLAIN) {
        if (g->poff64) return fn(PlainAcc<true>{g->plain_view()});
        return fn(PlainAcc<false>{g->plain_view()});
    }
    if (g->weighted) {
        set_error("packed weighted lists (ID then weight per entry) are read by lg_sssp only");
        return LG_ERR_UNSUPPORTED;
    }
    if (g->id_mode == LG_IDS_LOCAL_GAP) {
        set_error("gap-encoded lists are read in order only: this operation is not available for them "
                  "(lg_decode_neighbors, lg_bfs and lg_pagerank are)");
        return LG_ERR_UNSUPPORTED;
    }
    if (g->id_mode == LG_IDS_VARINT_FULL || g->id_mode == LG_IDS_VARINT_DIFF) {
        set_error("Varint lists are read in order only: this operation is not available for them "
                  "(lg_decode_neighbors, lg_bfs and lg_pagerank are)");
        return LG_ERR_UNSUPPORTED;
    }
    if (g->offset_mode == LG_OFFS_INTERLEAVED_BV) {
        set_error("interleaved bit-vector offsets (bvIL) are read by lg_decode_neighbors only");
        return LG_ERR_UNSUPPORTED;
    }
    // the plain bit vector (LG_OFFS_PLAIN_BV) is read as Elias-Fano without low bits
    const PackedView pv = g->packed_view();
    if (g->id_mode == LG_IDS_GLOBAL) {
        if (g->offset_mode == LG_OFFS_PACKED) return fn(PackedAcc<kIdsGlobal, kOffsPacked>{pv});
        return fn(PackedAcc<kIdsGlobal, kOffsEF>{pv});
    }
    if (g->offset_mode == LG_OFFS_PACKED) return fn(PackedAcc<kIdsLocal, kOffsPacked>{pv});
    return fn(PackedAcc<kIdsLocal, kOffsEF>{pv});
}

template <class Acc>
struct IsGapAcc {
    static constexpr bool value = false;
};
template <int OFM>
struct IsGapAcc<GapAcc<OFM>> {
    static constexpr bool value = true;
};

// dispatch_acc plus the gap accessors, for the paths that read gap lists in
// order (the neighbor decode and PageRank)
template <class Fn>
lg_status dispatch_acc_all(const lg_graph *g, Fn &&fn) {
    if (g->layout == LG_LAYOUT_PACKED && g->id_mode == LG_IDS_LOCAL_GAP) {
        const PackedView pv = g->packed_view();
        if (g->offset_mode == LG_OFFS_PACKED) return fn(GapAcc<kOffsPacked>{PackedAcc<kIdsLocal, kOffsPacked>{pv}});
        return fn(GapAcc<kOffsEF>{PackedAcc<kIdsLocal, kOffsEF>{pv}});
    }
    return dispatch_acc(g, fn);
}

template <class Acc>
struct IsVarintAcc {
    static constexpr bool value = false;
};
template <int OFM, bool kDiff>
struct IsVarintAcc<VarintAcc<OFM, kDiff>> {
    static constexpr bool value = true;
};

// dispatch_acc_all plus the Varint accessors (the neighbor decode)
template <class Fn>
lg_status dispatch_acc_dec(const lg_graph *g, Fn &&fn) {
    if (g->layout == LG_LAYOUT_PACKED && (g->id_mode == LG_IDS_VARINT_FULL || g->id_mode == LG_IDS_VARINT_DIFF)) {
        const PackedView pv = g->packed_view();
        const bool diff = g->id_mode == LG_IDS_VARINT_DIFF;
        if (g->offset_mode == LG_OFFS_PACKED) {
            const PackedAcc<kIdsLocal, kOffsPacked> b{pv};
            return diff ? fn(VarintAcc<kOffsPacked, true>{b}) : fn(VarintAcc<kOffsPacked, false>{b});
        }
        const PackedAcc<kIdsLocal, kOffsEF> b{pv};
        return diff ? fn(VarintAcc<kOffsEF, true>{b}) : fn(VarintAcc<kOffsEF, false>{b});
    }
    return dispatch_acc_all(g, fn);
}

// dispatch_acc_dec plus the interleaved bit-vector offsets (bvIL), which
// only the neighbor decode reads
template <class Fn>
lg_status dispatch_acc_decode(const lg_graph *g, Fn &&fn) {
    if (g->layout == LG_LAYOUT_PACKED && g->offset_mode == LG_OFFS_INTERLEAVED_BV) {
        const PackedView pv = g->packed_view();
        if (g->id_mode == LG_IDS_GLOBAL) return fn(PackedAcc<kIdsGlobal, kOffsIL>{pv});
        return fn(PackedAcc<kIdsLocal, kOffsIL>{pv});
    }
    return dispatch_acc_dec(g, fn);
}

}  // namespace lg
