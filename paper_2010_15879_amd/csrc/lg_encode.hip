// lg_encode: build the logarithmized representation on the GPU.
//
// Steps (each a kernel or a short sequence of kernels on the caller's
// stream):
//   validate      canonical undirected adjacency array (sorted lists, IDs < n,
//                 no self-loops, symmetric)
//   relabel       degree-minimizing permutation (section "Incorporating
//                 Degree-Minimizing (DM)"): stable radix sort of vertices by
//                 degree; or the greedy heuristic of subsection "Adding
//                 Integer Linear Programming"; then the relabeled lists via
//                 one stable radix sort of (original target, new source)
//                 pairs by target
//   widths        global s or local w_v ("Logarithmization of Vertex IDs")
//   scan          bit starts P_v = exclusive prefix of d_v * w_v
//   pack          fixed widths: each thread assembles one 64-bit output word;
//                 local widths: a walk over the lists, words gathered in LDS
//   offsets       packed offsets ("Logarithmization of Single Offsets") or an
//                 Elias-Fano sequence with a rank/select directory ("Succinct
//                 Bit Vectors in Log(Graph)")
#include <cstring>
#include <utility>

#include "lg_device.hpp"

namespace lg {

enum : uint32_t {
    kBadOffsets = 1u,
    kBadId = 2u,
    kSelfLoop = 4u,
    kUnsorted = 8u,
    kAsymmetric = 16u,
};

// ---------------------------------------------------------------------------
// validation and degree statistics
// ---------------------------------------------------------------------------

// Offsets: non-decreasing, off[0] = 0, off[n] = m (one thread per vertex).
__global__ void validate_offsets_kernel(uint32_t n, uint64_t m, const uint64_t *__restrict__ off,
                                        uint32_t *__restrict__ status) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint64_t o0 = off[v], o1 = off[v + 1];
        bad |= o1 < o0 || o1 > m || (v == 0 && o0 != 0) || (v + 1 == n && o1 != m);
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(status, kBadOffsets);
}

// ---------------------------------------------------------------------------
// edge walks over 64-row blocks
// ---------------------------------------------------------------------------
//
// The lists of rows 64q .. 64q+63 are one contiguous range of entries.  It is
// cut into pieces of at most kWalkChunk entries; a piece is one work item, so
// that a hub's list is shared by many waves and a block of short lists is one
// wave's work.  Item k belongs to block map[k] and is its piece k - coff[q].

constexpr uint64_t kWalkChunk = 8192;

__global__ void walk_count_kernel(uint32_t n, const uint64_t *__restrict__ off, uint32_t *__restrict__ cnt) {
    const uint64_t blocks = ((uint64_t)n + 63) / 64;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < blocks; q += stride) {
        const uint64_t e0 = off[q * 64], e1 = off[q * 64 + 64 <= n ? q * 64 + 64 : n];
        const uint64_t pieces = (e1 - e0 + kWalkChunk - 1) / kWalkChunk;
        cnt[q] = (uint32_t)(pieces ? pieces : 1);
    }
}

__global__ void walk_map_kernel(uint64_t blocks, const uint64_t *__restrict__ coff, uint32_t *__restrict__ map) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < blocks; q += stride)
        for (uint64_t k = coff[q]; k < coff[q + 1]; ++k) map[k] = (uint32_t)q;
}

// Lanes of one wave exchange data through its own LDS rows: keep the
// compiler from moving LDS accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work item k of a walk over the rows of `off`: s_rs gets the block's 65 row
// starts.  Entries e = base + lane are taken in steps of 64, with j the row
// of e within the block and valid = e lies in the piece.  Four steps at a
// time, every lane calls x = load(e, j, valid) for each step, then
// use(e, j, valid, x) for each step.  load reads in bounds whatever valid is
// and does not branch on it, so the four steps' loads are in flight
// together; every lane makes the same calls (shuffles inside use are safe).
template <class Load, class Use>
__device__ __forceinline__ void walk_item(uint32_t n, const uint64_t *__restrict__ off,
                                          const uint32_t *__restrict__ map, const uint64_t *__restrict__ coff,
                                          uint64_t k, uint64_t *s_rs, Load &&load, Use &&use) {
    const uint32_t lane = lane_id();
    const uint64_t q = map[k];
    const uint64_t v0 = q * 64;
    const uint64_t o = off[v0 + lane <= n ? v0 + lane : n];
    const uint64_t E1 = off[v0 + 64 <= n ? v0 + 64 : n];
    s_rs[lane] = o;
    if (lane == 0) s_rs[64] = E1;
    wave_lds_sync();
    const uint64_t eb = __shfl(o, 0, kWave) + (k - coff[q]) * kWalkChunk;
    const uint64_t ee = eb + kWalkChunk < E1 ? eb + kWalkChunk : E1;
    if (eb < ee) {
        // row of eb: the largest j with s_rs[j] <= eb (empty rows share starts)
        uint32_t j = 0;
#pragma unroll
        for (uint32_t step = 32; step > 0; step >>= 1)
            if (s_rs[j + step] <= eb) j += step;
        constexpr int kSteps = 4;
        for (uint64_t base = eb; base < ee; base += kSteps * kWave) {
            uint64_t e[kSteps];
            uint32_t row[kSteps];
            bool valid[kSteps];
#pragma unroll
            for (int r = 0; r < kSteps; ++r) {  // rows from LDS only
                e[r] = base + (uint64_t)r * kWave + lane;
                valid[r] = e[r] < ee;
                if (valid[r])
                    while (s_rs[j + 1] <= e[r]) ++j;
                row[r] = j;
            }
            decltype(load(e[0], row[0], valid[0])) x[kSteps];
#pragma unroll
            for (int r = 0; r < kSteps; ++r) x[r] = load(e[r], row[r], valid[r]);
#pragma unroll
            for (int r = 0; r < kSteps; ++r) use(e[r], row[r], valid[r], x[r]);
        }
    }
    wave_lds_sync();
}

// IDs < n, no self-loop, strictly increasing lists.
// Also low[v], the entries of row v below v (the symmetry check's split of
// each row): in a sorted row without v the first entry above v sits at
// position low[v], and a row whose last entry is below v has low[v] = its
// degree; one store per row (empty rows keep the zero low starts with).
__global__ void validate_edges_kernel(uint32_t n, const uint64_t *__restrict__ off, const uint32_t *__restrict__ col,
                                      uint64_t items, const uint32_t *__restrict__ map,
                                      const uint64_t *__restrict__ coff, uint32_t *__restrict__ status,
                                      uint32_t *__restrict__ low) {
    __shared__ uint64_t s_rs[4][kWave + 1];
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    uint32_t flags = 0;
    for (uint64_t k = wave; k < items; k += nwaves) {
        const uint64_t v0 = (uint64_t)map[k] * 64;
        // the entry and, for lane 0, the one before it (other lanes get theirs
        // from the lane below)
        auto load = [&](uint64_t e, uint32_t, bool valid) {
            const uint64_t i = valid ? e : 0;
            const uint64_t ip = lane_id() == 0 && valid && e > 0 ? e - 1 : i;
            return make_uint2(col[i], col[ip]);
        };
        walk_item(n, off, map, coff, k, s_rs[wv], load, [&](uint64_t e, uint32_t j, bool valid, uint2 x) {
            const uint32_t u = x.x;
            uint32_t prev = __shfl_up(u, 1, kWave);
            if (!valid) return;
            if (lane_id() == 0) prev = x.y;
            const uint32_t v = (uint32_t)(v0 + j);
            const uint64_t rs = s_rs[wv][j], re = s_rs[wv][j + 1];
            if (u >= n) flags |= kBadId;
            if (u == v) flags |= kSelfLoop;
            if (e > rs && prev >= u) flags |= kUnsorted;
            if (u > v && (e == rs || prev < v)) low[v] = (uint32_t)(e - rs);  // the row's first entry above v
            else if (u < v && e + 1 == re) low[v] = (uint32_t)(re - rs);     // all of the row is below v
        });
    }
    if (__ballot(flags != 0)) {
        flags = wave_or(flags);
        if (lane_id() == 0) atomicOr(status, flags);
    }
}

// Symmetry, exactly, from the entries below the diagonal.  Row v's entries
// smaller than v come first in its sorted list: low[v] of them.  Taken in
// row order and transposed, (v, u) -> (u, v), then sorted stably by u, they
// list for every u the rows v > u that hold u, ascending.  The graph is
// symmetric iff that sequence is, entry for entry, the entries above the
// diagonal in row order: row u's entries larger than u.  Both halves hold
// lowoff[n] entries (checked first), and the upper entry at stream position
// e of row u has index e - lowoff[u + 1] among the upper entries.

// the rows' lowoff values for block q (65 of them, clamped at n) into s_lo
__device__ __forceinline__ void sym_block_lowoff(uint32_t n, const uint32_t *__restrict__ map, uint64_t k,
                                                 const uint64_t *__restrict__ lowoff, uint64_t *s_lo) {
    const uint32_t lane = lane_id();
    const uint64_t v0 = (uint64_t)map[k] * 64;
    s_lo[lane] = lowoff[v0 + lane <= n ? v0 + lane : n];
    if (lane == 0) s_lo[64] = lowoff[v0 + 64 <= n ? v0 + 64 : n];
    // walk_item's opening wave sync orders these writes before its uses
}

__global__ void sym_emit_kernel(uint32_t n, const uint64_t *__restrict__ off, const uint32_t *__restrict__ col,
                                uint64_t items, const uint32_t *__restrict__ map, const uint64_t *__restrict__ coff,
                                const uint64_t *__restrict__ lowoff, uint32_t *__restrict__ key,
                                uint32_t *__restrict__ val) {
    __shared__ uint64_t s_rs[4][kWave + 1];
    __shared__ uint64_t s_lo[4][kWave + 1];
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t k = wave; k < items; k += nwaves) {
        const uint32_t v0 = map[k] * 64u;
        sym_block_lowoff(n, map, k, lowoff, s_lo[wv]);
        walk_item(
            n, off, map, coff, k, s_rs[wv], [&](uint64_t e, uint32_t, bool valid) { return col[valid ? e : 0]; },
            [&](uint64_t e, uint32_t j, bool valid, uint32_t u) {
                if (!valid || u >= v0 + j) return;  // the row's entries below the diagonal only
                const uint64_t pos = s_lo[wv][j] + (e - s_rs[wv][j]);
                key[pos] = u;
                val[pos] = v0 + j;
            });
    }
}

__global__ void sym_check_kernel(uint32_t n, const uint64_t *__restrict__ off, const uint32_t *__restrict__ col,
                                 uint64_t items, const uint32_t *__restrict__ map, const uint64_t *__restrict__ coff,
                                 const uint64_t *__restrict__ lowoff, uint64_t half,
                                 const uint32_t *__restrict__ key, const uint32_t *__restrict__ val,
                                 uint32_t *__restrict__ status) {
    __shared__ uint64_t s_rs[4][kWave + 1];
    __shared__ uint64_t s_lo[4][kWave + 1];
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    bool bad = false;
    for (uint64_t k = wave; k < items; k += nwaves) {
        const uint32_t v0 = map[k] * 64u;
        sym_block_lowoff(n, map, k, lowoff, s_lo[wv]);
        // every entry's would-be index among the upper entries (meaningful for
        // upper entries only; others read index 0)
        auto upper_index = [&](uint64_t e, uint32_t j) -> uint64_t {
            const uint64_t lo1 = s_lo[wv][j + 1];
            return e >= lo1 && e - lo1 < half ? e - lo1 : 0;
        };
        auto load = [&](uint64_t e, uint32_t j, bool valid) {
            const uint64_t i = valid ? upper_index(e, j) : 0;
            return make_uint3(key[i], val[i], col[valid ? e : 0]);
        };
        walk_item(n, off, map, coff, k, s_rs[wv], load, [&](uint64_t e, uint32_t j, bool valid, uint3 x) {
            if (!valid || x.z <= v0 + j) return;  // the row's entries above the diagonal only
            const uint64_t lo1 = s_lo[wv][j + 1];
            bad |= e < lo1 || e - lo1 >= half || x.x != v0 + j || x.y != x.z;
        });
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(status, kAsymmetric);
}

// deg[v] (uint32), plus the maximum degree and the number of isolated vertices
__global__ void degree_kernel(uint32_t n, const uint64_t *__restrict__ off, uint32_t *__restrict__ deg,
                              uint32_t *__restrict__ stats) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t mx = 0, iso = 0;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint32_t d = (uint32_t)(off[v + 1] - off[v]);
        deg[v] = d;
        mx = d > mx ? d : mx;
        iso += d == 0;
    }
#pragma unroll
    for (int k = kWave / 2; k > 0; k >>= 1) {
        const uint32_t o = __shfl_xor(mx, k, kWave);
        mx = o > mx ? o : mx;
    }
    iso = wave_sum(iso);
    __shared__ uint32_t s_mx[4], s_iso[4];  // blockDim = 256: four waves
    const uint32_t wv = threadIdx.x / kWave;
    if (lane_id() == 0) { s_mx[wv] = mx; s_iso[wv] = iso; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) { mx = s_mx[w] > mx ? s_mx[w] : mx; iso += s_iso[w]; }
        atomicMax(&stats[0], mx);
        if (iso) atomicAdd(&stats[1], iso);
    }
}

// ---------------------------------------------------------------------------
// degree-minimizing relabeling
// ---------------------------------------------------------------------------

// sort key: (n - 1) - d_v, so an ascending stable sort orders by degree
// descending and keeps equal degrees in ID order
__global__ void dm_keys_kernel(uint32_t n, const uint32_t *__restrict__ deg, uint32_t *__restrict__ keys,
                               uint32_t *__restrict__ vals) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        keys[v] = (n - 1) - deg[v];
        vals[v] = (uint32_t)v;
    }
}

__global__ void dm_inverse_kernel(uint32_t n, const uint32_t *__restrict__ perm, const uint32_t *__restrict__ deg,
                                  uint32_t *__restrict__ inv, uint32_t *__restrict__ deg_new) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
        const uint32_t v = perm[x];
        inv[v] = (uint32_t)x;
        deg_new[x] = deg[v];
    }
}

// The relabeled lists without a gather per entry.  Rows are taken in new
// order x, and every entry w of the list of perm[x] is emitted as the pair
// (w, x): original target, new source.  A stable sort by w groups, for each
// original vertex w, the new labels x of the vertices whose lists hold w, in
// increasing order; by symmetry that group is the relabeled list of w, which
// becomes row inv[w] (one lookup per row, not per entry).
__global__ void dm_emit_kernel(uint32_t n, const uint32_t *__restrict__ perm, const uint64_t *__restrict__ off,
                               const uint32_t *__restrict__ col, const uint64_t *__restrict__ off_new, uint64_t items,
                               const uint32_t *__restrict__ map, const uint64_t *__restrict__ coff,
                               uint32_t *__restrict__ key, uint32_t *__restrict__ val) {
    __shared__ uint64_t s_rs[4][kWave + 1];
    __shared__ uint64_t s_src[4][kWave];
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t k = wave; k < items; k += nwaves) {
        // new rows x = 64q + lane take the list of perm[x]: its first entry in col
        const uint32_t x0 = map[k] * 64u;
        s_src[wv][lane] = x0 + lane < n ? off[perm[x0 + lane]] : 0ull;
        auto load = [&](uint64_t e, uint32_t j, bool valid) {
            return col[valid ? s_src[wv][j] + (e - s_rs[wv][j]) : 0];
        };
        walk_item(n, off_new, map, coff, k, s_rs[wv], load, [&](uint64_t e, uint32_t j, bool valid, uint32_t w) {
            if (!valid) return;
            key[e] = w;
            val[e] = x0 + j;
        });
    }
}

// After the sort, the group of original vertex w sits at [off[w], off[w+1])
// (its degree is unchanged); new row y = inv[w], i.e. w = perm[y], copies it.
__global__ void dm_place_kernel(uint32_t n, const uint32_t *__restrict__ perm, const uint64_t *__restrict__ off,
                                const uint32_t *__restrict__ grouped, const uint64_t *__restrict__ off_new,
                                uint64_t items, const uint32_t *__restrict__ map, const uint64_t *__restrict__ coff,
                                uint32_t *__restrict__ col_new) {
    __shared__ uint64_t s_rs[4][kWave + 1];
    __shared__ uint64_t s_src[4][kWave];
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t k = wave; k < items; k += nwaves) {
        const uint32_t y0 = map[k] * 64u;
        s_src[wv][lane] = y0 + lane < n ? off[perm[y0 + lane]] : 0ull;
        auto load = [&](uint64_t e, uint32_t j, bool valid) {
            return grouped[valid ? s_src[wv][j] + (e - s_rs[wv][j]) : 0];
        };
        walk_item(n, off_new, map, coff, k, s_rs[wv], load, [&](uint64_t e, uint32_t, bool valid, uint32_t x) {
            if (valid) col_new[e] = x;
        });
    }
}

// Greedy relabeling (subsection "Adding Integer Linear Programming", its
// listing of a greedy heuristic): vertices taken by increasing degree (ties
// by ID) hand the next label to each neighbor, in list order, that has none
// yet; edgeless vertices take the last labels in ID order.  The label order
// of a vertex x is that of its first hand-out: the smallest rank r(u) of a
// neighbor u in the processing order, then x's position in the list of u.
// So the sequential loop becomes: ranks by a sort on degree; per x the
// minimum rank over its own list (lists are symmetric); x's position in that
// neighbor's list by binary search; a stable sort of the vertices by
// (rank, position).

// sort key d_v (an ascending stable sort orders by degree, ties by ID)
__global__ void greedy_order_keys_kernel(uint32_t n, const uint32_t *__restrict__ deg, uint32_t *__restrict__ keys,
                                         uint32_t *__restrict__ vals) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        keys[v] = deg[v];
        vals[v] = (uint32_t)v;
    }
}

// rank[order[r]] = r
__global__ void greedy_rank_kernel(uint32_t n, const uint32_t *__restrict__ order, uint32_t *__restrict__ rank) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) rank[order[r]] = (uint32_t)r;
}

// rmin[x] = min over u in N_x of rank[u] (rmin starts at ~0): a walk over
// the lists, a per-row minimum in LDS, one global atomic per row and piece
__global__ void greedy_min_kernel(uint32_t n, const uint64_t *__restrict__ off, const uint32_t *__restrict__ col,
                                  const uint32_t *__restrict__ rank, uint64_t items, const uint32_t *__restrict__ map,
                                  const uint64_t *__restrict__ coff, uint32_t *__restrict__ rmin) {
    __shared__ uint64_t s_rs[4][kWave + 1];
    __shared__ uint32_t s_min[4][kWave];
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t k = wave; k < items; k += nwaves) {
        const uint64_t v0 = (uint64_t)map[k] * 64;
        s_min[wv][lane] = 0xFFFFFFFFu;
        walk_item(
            n, off, map, coff, k, s_rs[wv], [&](uint64_t e, uint32_t, bool valid) { return col[valid ? e : 0]; },
            [&](uint64_t, uint32_t j, bool valid, uint32_t u) {
                if (valid) atomicMin(&s_min[wv][j], rank[u]);
            });
        // walk_item ends with a wave LDS sync: every lane's minimum is in
        if (v0 + lane < n && s_min[wv][lane] != 0xFFFFFFFFu) atomicMin(&rmin[v0 + lane], s_min[wv][lane]);
        wave_lds_sync();
    }
}

// key[x] = rmin[x] << jbits | (position of x in the list of order[rmin[x]]),
// n << jbits for a vertex without edges; val[x] = x.  The lists are
// symmetric and strictly increasing, so x is found.
__global__ void greedy_key_kernel(uint32_t n, const uint64_t *__restrict__ off, const uint32_t *__restrict__ col,
                                  const uint32_t *__restrict__ order, const uint32_t *__restrict__ rmin,
                                  uint32_t jbits, uint64_t *__restrict__ key, uint32_t *__restrict__ val) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
        const uint32_t r = rmin[x];
        uint64_t k = (uint64_t)n << jbits;
        if (r != 0xFFFFFFFFu) {
            const uint32_t u = order[r];
            uint64_t lo = off[u], hi = off[u + 1];
            const uint64_t base = lo;
            while (lo < hi) {
                const uint64_t mid = lo + ((hi - lo) >> 1);
                if (col[mid] < (uint32_t)x) lo = mid + 1; else hi = mid;
            }
            k = ((uint64_t)r << jbits) | (lo - base);
        }
        key[x] = k;
        val[x] = (uint32_t)x;
    }
}

// ---------------------------------------------------------------------------
// widths and bit lengths
// ---------------------------------------------------------------------------

// w_v = max(1, bl(max N_v)) for a non-empty list (its last element, lists
// being sorted), 0 otherwise; len[v] = d_v * w_v.
__global__ void local_width_kernel(uint32_t n, const uint64_t *__restrict__ off, const uint32_t *__restrict__ col,
                                   uint8_t *__restrict__ w, uint64_t *__restrict__ len) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint64_t o0 = off[v], o1 = off[v + 1];
        uint32_t wv = 0;
        if (o1 > o0) {
            const uint32_t mx = col[o1 - 1];
            wv = mx ? 32u - (uint32_t)__clz(mx) : 1u;
        }
        w[v] = (uint8_t)wv;
        len[v] = (o1 - o0) * wv;
    }
}

// floor(x / d) for x < 2^53 and a small d, via a double reciprocal and an
// exact correction
__device__ __forceinline__ uint64_t div_small(uint64_t x, uint64_t d, double inv_d) {
    uint64_t q = (uint64_t)((double)x * inv_d);
    while (q * d > x) --q;
    while ((q + 1) * d <= x) ++q;
    return q;
}

// ---------------------------------------------------------------------------
// packing: one thread per output word
// ---------------------------------------------------------------------------

struct SrcU32 {
    const uint32_t *p;
    __device__ __forceinline__ uint64_t operator()(uint64_t j) const { return p[j]; }
};
struct SrcU8 {
    const uint8_t *p;
    __device__ __forceinline__ uint64_t operator()(uint64_t j) const { return p[j]; }
};
struct SrcU64Mask {
    const uint64_t *p;
    uint64_t mask;
    __device__ __forceinline__ uint64_t operator()(uint64_t j) const { return p[j] & mask; }
};

// Value j of a sequence of `count` values occupies bits [j*w, j*w + w).
// Word k gathers the values overlapping bits [64k, 64k + 64): the value j0
// holding bit 64k and those after it, at most ceil(63 / w) + 1 of them.
// With kMax >= that bound the loads go out together (indices clamped into
// the sequence, values past the word or the sequence dropped); kMax = 0 is
// the loop for narrow widths.
template <int kMax, class Src>
__device__ __forceinline__ uint64_t pack_word(Src src, uint64_t count, uint32_t w, uint64_t b0, uint64_t j0) {
    uint64_t word = 0;
    if constexpr (kMax > 0) {
        uint64_t x[kMax];
#pragma unroll
        for (int t = 0; t < kMax; ++t) x[t] = src(j0 + t < count ? j0 + t : count - 1);
#pragma unroll
        for (int t = 0; t < kMax; ++t) {
            const uint64_t j = j0 + t, b = j * w;
            if (j < count && b < b0 + 64) word |= (b >= b0) ? (x[t] << (b - b0)) : (x[t] >> (b0 - b));
        }
    } else {
        for (uint64_t j = j0; j < count; ++j) {
            const uint64_t b = j * w;
            if (b >= b0 + 64) break;
            const uint64_t x = src(j);
            word |= (b >= b0) ? (x << (b - b0)) : (x >> (b0 - b));
        }
    }
    return word;
}

template <class Src>
__global__ void pack_fixed_kernel(Src src, uint64_t count, uint32_t w, double inv_w, uint64_t words,
                                  uint64_t *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t total_bits = count * w;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += stride) {
        const uint64_t b0 = k * 64;
        uint64_t word = 0;
        if (w && b0 < total_bits) {
            const uint64_t j0 = div_small(b0, w, inv_w);
            if (w >= 22) word = pack_word<4>(src, count, w, b0, j0);        // ceil(63/22) + 1 = 4
            else if (w >= 16) word = pack_word<5>(src, count, w, b0, j0);   // ceil(63/16) + 1 = 5
            else if (w >= 11) word = pack_word<7>(src, count, w, b0, j0);   // ceil(63/11) + 1 = 7
            else if (w >= 8) word = pack_word<9>(src, count, w, b0, j0);    // ceil(63/8) + 1 = 9
            else word = pack_word<0>(src, count, w, b0, j0);
        }
        out[k] = word;
    }
}

// Local widths: entry i of list v occupies stream bits [P_v + i w_v, + w_v).
// Walked like the validation passes: a wave takes a piece of consecutive
// entries, 64 per step (four steps' loads issued together).  The lanes of a
// step cover adjacent bit ranges; their parts are ORed into words in the
// wave's LDS, every word completed inside the piece is stored once, and the
// word a step leaves open is carried into the next step.  The first word of
// a piece and the word left open at its end may hold bits of the
// neighbouring pieces: those two are ORed into the (zeroed) stream
// atomically.
constexpr int kPackBuf = 34;  // words one step can touch: 64 x 32 bits, misaligned, plus the carry

// kGap: fixed-size gap encoding -- entry 0 of a list at w_v bits, entry i > 0
// is its difference from entry i - 1, at g_v bits (gwid).
template <bool kGap>
__global__ void pack_walk_kernel(uint32_t n, const uint64_t *__restrict__ off, const uint32_t *__restrict__ col,
                                 const uint8_t *__restrict__ wid, const uint8_t *__restrict__ gwid,
                                 const uint64_t *__restrict__ P, uint64_t items, const uint32_t *__restrict__ map,
                                 const uint64_t *__restrict__ coff, unsigned long long *__restrict__ out) {
    __shared__ uint64_t s_rs[4][kWave + 1];
    __shared__ uint64_t s_p[4][kWave];
    __shared__ uint32_t s_w[4][kWave];
    __shared__ uint32_t s_g[4][kWave];
    __shared__ unsigned long long s_buf[4][kPackBuf];
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    // bit position and width of entry i of row r of this wave's block
    auto place = [&](uint32_t r, uint64_t i, uint64_t &bit, uint32_t &width) {
        if (kGap) {
            bit = s_p[wv][r] + (i == 0 ? 0ull : s_w[wv][r] + (i - 1) * s_g[wv][r]);
            width = i == 0 ? s_w[wv][r] : s_g[wv][r];
        } else {
            bit = s_p[wv][r] + i * s_w[wv][r];
            width = s_w[wv][r];
        }
    };
    for (uint64_t k = wave; k < items; k += nwaves) {
        const uint64_t q = map[k];
        const uint64_t v0 = q * 64;
        const uint64_t o = off[v0 + lane <= n ? v0 + lane : n];
        const uint64_t E1 = off[v0 + 64 <= n ? v0 + 64 : n];
        s_rs[wv][lane] = o;
        if (lane == 0) s_rs[wv][64] = E1;
        s_p[wv][lane] = v0 + lane < n ? P[v0 + lane] : 0ull;
        s_w[wv][lane] = v0 + lane < n ? wid[v0 + lane] : 0u;
        s_g[wv][lane] = kGap && v0 + lane < n ? gwid[v0 + lane] : 0u;
        wave_lds_sync();
        const uint64_t eb = __shfl(o, 0, kWave) + (k - coff[q]) * kWalkChunk;
        const uint64_t ee = eb + kWalkChunk < E1 ? eb + kWalkChunk : E1;
        if (eb < ee) {
            uint32_t j = 0;
#pragma unroll
            for (uint32_t step = 32; step > 0; step >>= 1)
                if (s_rs[wv][j + step] <= eb) j += step;
            uint64_t fb;
            uint32_t fw;
            place(j, eb - s_rs[wv][j], fb, fw);
            const uint64_t first_word = fb >> 6;
            bool open = false;  // a word of the previous step is still being filled
            unsigned long long carry = 0;
            uint64_t carry_word = 0;
            constexpr int kSteps = 4;
            for (uint64_t base = eb; base < ee; base += kSteps * kWave) {
                uint64_t e[kSteps];
                uint32_t row[kSteps];
                bool valid[kSteps];
                uint32_t x[kSteps], xp[kSteps];
#pragma unroll
                for (int r = 0; r < kSteps; ++r) {
                    e[r] = base + (uint64_t)r * kWave + lane;
                    valid[r] = e[r] < ee;
                    if (valid[r])
                        while (s_rs[wv][j + 1] <= e[r]) ++j;
                    row[r] = j;
                }
#pragma unroll
                for (int r = 0; r < kSteps; ++r) {
                    x[r] = col[valid[r] ? e[r] : 0];
                    // the entry before (same row when it is not the row's first)
                    xp[r] = kGap ? col[valid[r] && e[r] > 0 ? e[r] - 1 : 0] : 0u;
                }
#pragma unroll
                for (int r = 0; r < kSteps; ++r) {
                    const uint64_t sb = base + (uint64_t)r * kWave;
                    if (sb >= ee) break;  // same for every lane
                    uint64_t b = 0;
                    uint32_t ww = 0;
                    uint32_t val = 0;
                    if (valid[r]) {
                        const uint64_t i = e[r] - s_rs[wv][row[r]];
                        place(row[r], i, b, ww);
                        val = (kGap && i > 0) ? x[r] - xp[r] : x[r];
                    }
                    const uint32_t last = (uint32_t)(ee - sb < kWave ? ee - sb : kWave) - 1;
                    const uint64_t b_first = __shfl(b, 0, kWave);
                    const uint64_t b_end = __shfl(b + ww, last, kWave);
                    const uint64_t kw0 = b_first >> 6;
                    const uint32_t nw = (uint32_t)(((b_end - 1) >> 6) - kw0) + 1;
                    // an open word of the previous step is this step's first word
                    if (lane < kPackBuf) s_buf[wv][lane] = (lane == 0 && open) ? carry : 0ull;
                    wave_lds_sync();
                    if (valid[r]) {
                        const uint32_t sh = (uint32_t)(b & 63);
                        const uint32_t idx = (uint32_t)((b >> 6) - kw0);
                        atomicOr(&s_buf[wv][idx], (unsigned long long)val << sh);
                        if (sh + ww > 64) atomicOr(&s_buf[wv][idx + 1], (unsigned long long)val >> (64 - sh));
                    }
                    wave_lds_sync();
                    open = (b_end & 63) != 0;
                    const uint32_t done = open ? nw - 1 : nw;
                    if (lane < done) {
                        const uint64_t word = kw0 + lane;
                        if (word == first_word) atomicOr(&out[word], s_buf[wv][lane]);
                        else out[word] = s_buf[wv][lane];
                    }
                    carry = s_buf[wv][nw - 1];
                    carry_word = kw0 + nw - 1;
                    wave_lds_sync();
                }
            }
            if (open && lane == 0) atomicOr(&out[carry_word], carry);
        }
        wave_lds_sync();
    }
}

// g_v = bl(largest difference of consecutive entries of list v): a walk over
// the lists, per-row maxima in LDS, one global atomic per row and piece
// (gmax starts at 0)
__global__ void gap_max_kernel(uint32_t n, const uint64_t *__restrict__ off, const uint32_t *__restrict__ col,
                               uint64_t items, const uint32_t *__restrict__ map, const uint64_t *__restrict__ coff,
                               uint32_t *__restrict__ gmax) {
    __shared__ uint64_t s_rs[4][kWave + 1];
    __shared__ uint32_t s_max[4][kWave];
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t k = wave; k < items; k += nwaves) {
        const uint64_t v0 = (uint64_t)map[k] * 64;
        s_max[wv][lane] = 0;
        auto load = [&](uint64_t e, uint32_t, bool valid) {
            return make_uint2(col[valid ? e : 0], col[valid && e > 0 ? e - 1 : 0]);
        };
        walk_item(n, off, map, coff, k, s_rs[wv], load, [&](uint64_t e, uint32_t j, bool valid, uint2 x) {
            if (valid && e > s_rs[wv][j]) atomicMax(&s_max[wv][j], x.x - x.y);
        });
        if (v0 + lane < n && s_max[wv][lane]) atomicMax(&gmax[v0 + lane], s_max[wv][lane]);
        wave_lds_sync();
    }
}

// gap widths g_v = bl(gmax_v) and list bit lengths w_v + (d_v - 1) g_v (0 when
// the list is empty)
__global__ void gap_len_kernel(uint32_t n, const uint64_t *__restrict__ off, const uint8_t *__restrict__ w8,
                               const uint32_t *__restrict__ gmax, uint8_t *__restrict__ g8,
                               uint64_t *__restrict__ len) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint64_t d = off[v + 1] - off[v];
        const uint32_t gm = gmax[v];
        const uint32_t g = gm ? 32u - (uint32_t)__clz(gm) : 0u;
        g8[v] = (uint8_t)g;
        len[v] = d ? (uint64_t)w8[v] + (d - 1) * (uint64_t)g : 0ull;
    }
}

// ---------------------------------------------------------------------------
// Weighted entries (subsections "Logarithmization of Edge Weights" and
// "Accessing an Edge Weight"): the ID, then the weight at omega bits.
// ---------------------------------------------------------------------------

// a grid-stride maximum, one atomic per block (launched with a bounded grid:
// atomics on one address serialize)
__global__ __launch_bounds__(256) void max_u32_kernel(uint64_t count, const uint32_t *__restrict__ x,
                                                      uint32_t *__restrict__ out) {
    __shared__ uint32_t s_max[256 / kWave];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t mx = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        mx = x[i] > mx ? x[i] : mx;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const uint32_t o = __shfl_xor(mx, d, kWave);
        mx = o > mx ? o : mx;
    }
    if (lane_id() == 0) s_max[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256 / kWave; ++i) mx = s_max[i] > mx ? s_max[i] : mx;
        if (mx) atomicMax(out, mx);
    }
}

// The weight of every relabeled entry: new entry e of row r stands for the
// original edge (perm[r], perm[c]); a binary search of perm[c] in the
// original (ascending) list of perm[r] finds its weight.
__global__ void relabel_weights_kernel(uint32_t n, uint64_t m, const uint64_t *__restrict__ off_new,
                                       const uint32_t *__restrict__ col_new, const uint32_t *__restrict__ perm,
                                       const uint64_t *__restrict__ off, const uint32_t *__restrict__ col,
                                       const uint32_t *__restrict__ wt, uint32_t *__restrict__ out,
                                       uint32_t *__restrict__ miss) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        uint32_t lo = 0, hi = n;  // off_new[lo] <= e < off_new[hi]
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (off_new[mid] <= e) lo = mid;
            else hi = mid;
        }
        const uint32_t u = perm[lo], x = perm[col_new[e]];
        const uint64_t end = off[u + 1];
        uint64_t a = off[u], b = end;
        while (a < b) {
            const uint64_t mid = a + (b - a) / 2;
            if (col[mid] < x) a = mid + 1;
            else b = mid;
        }
        // Row lo of the relabeled lists is the original list of u renamed, so
        // its entry e stands for the original edge (u, x), which the search
        // finds; a miss means the arrays were corrupted and fails the encode.
        if (a < end && col[a] == x) {
            out[e] = wt[a];
        } else {
            out[e] = 0u;
            atomicOr(miss, 1u);
        }
    }
}

// list bit lengths d_v (w_v + omega), local IDs
__global__ void weighted_len_kernel(uint32_t n, const uint64_t *__restrict__ off, const uint8_t *__restrict__ w8,
                                    uint32_t omega, uint64_t *__restrict__ len) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        len[v] = (off[v + 1] - off[v]) * (uint64_t)(w8[v] + omega);
}

// Entry e at bit e (s + omega) (global IDs) or P_v + (e - off_v)(w_v + omega)
// (local IDs, the row found by a binary search of the offsets); an entry
// spans at most two words, ORed into the zeroed stream.
template <bool kLocal>
__global__ void pack_weighted_kernel(uint32_t n, uint64_t m, const uint64_t *__restrict__ off,
                                     const uint32_t *__restrict__ col, const uint32_t *__restrict__ wt,
                                     const uint8_t *__restrict__ wid, const uint64_t *__restrict__ P, uint32_t s,
                                     uint32_t omega, unsigned long long *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        uint64_t bit;
        uint32_t w;
        if constexpr (kLocal) {
            uint32_t lo = 0, hi = n;  // off[lo] <= e < off[hi]
            while (hi - lo > 1) {
                const uint32_t mid = lo + (hi - lo) / 2;
                if (off[mid] <= e) lo = mid;
                else hi = mid;
            }
            w = wid[lo];
            bit = P[lo] + (e - off[lo]) * (uint64_t)(w + omega);
        } else {
            w = s;
            bit = e * (uint64_t)(s + omega);
        }
        const uint64_t val = (uint64_t)col[e] | ((uint64_t)wt[e] << w);
        const uint32_t sh = (uint32_t)(bit & 63);
        const uint64_t k = bit >> 6;
        atomicOr(&out[k], (unsigned long long)(val << sh));
        if (sh + w + omega > 64) atomicOr(&out[k + 1], (unsigned long long)(val >> (64 - sh)));
    }
}

// ---------------------------------------------------------------------------
// Varint lists (subsection "Incorporating Degree-Minimizing (DM)"): every
// label (DMf) or the first label and then the differences (DMd), each in
// base-128 bytes, lowest group first, the top bit set on every byte of a
// value but its last.  One byte length per edge, an exclusive scan gives
// every value's byte position, and each lane writes its value's bytes.
// ---------------------------------------------------------------------------

// head[e] = 1 where a non-empty row starts
__global__ void varint_head_kernel(uint32_t n, const uint64_t *__restrict__ off, uint8_t *__restrict__ head) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        if (off[v + 1] > off[v]) head[off[v]] = 1;
}

template <bool kDiff>
__device__ __forceinline__ uint32_t varint_value(const uint32_t *__restrict__ col,
                                                 const uint8_t *__restrict__ head, uint64_t e) {
    if (!kDiff || e == 0 || head[e]) return col[e];
    return col[e] - col[e - 1];
}

__device__ __forceinline__ uint32_t varint_bytes(uint32_t x) {
    return x < (1u << 7) ? 1u : x < (1u << 14) ? 2u : x < (1u << 21) ? 3u : x < (1u << 28) ? 4u : 5u;
}

template <bool kDiff>
__global__ void varint_len_kernel(uint64_t m, const uint32_t *__restrict__ col, const uint8_t *__restrict__ head,
                                  uint32_t *__restrict__ len) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride)
        len[e] = varint_bytes(varint_value<kDiff>(col, head, e));
}

// byte start of every list: the position of its first value (count n + 1;
// pos holds m + 1 entries, the last the stream length)
__global__ void varint_starts_kernel(uint32_t n, const uint64_t *__restrict__ off, const uint64_t *__restrict__ pos,
                                     uint64_t *__restrict__ P) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) P[v] = pos[off[v]];
}

template <bool kDiff>
__global__ void varint_write_kernel(uint64_t m, const uint32_t *__restrict__ col, const uint8_t *__restrict__ head,
                                    const uint64_t *__restrict__ pos, uint8_t *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        uint32_t x = varint_value<kDiff>(col, head, e);
        uint64_t p = pos[e];
        for (;;) {
            const uint32_t low = x & 127u;
            x >>= 7;
            out[p++] = (uint8_t)(x ? (low | 128u) : low);
            if (!x) break;
        }
    }
}

// ---------------------------------------------------------------------------
// Elias-Fano upper bits and directory
// ---------------------------------------------------------------------------

// Bit (x_v >> l) + v of H for every v.  The positions increase with v, so
// the lanes of a wave that set bits of one word are adjacent: a segmented OR
// across the lanes gathers each word's bits, and the word's first lane ORs
// them in (a few atomics per wave instead of one per vertex).
__global__ void ef_high_kernel(uint64_t count, const uint64_t *__restrict__ x, uint32_t l,
                               unsigned long long *__restrict__ H) {
    const uint32_t lane = lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; base < count; base += stride) {
        const uint64_t v = base + lane;
        const bool valid = v < count;
        const uint64_t y = valid ? (x[v] >> l) + v : 0ull;
        const uint64_t word = valid ? y >> 6 : ~0ull;
        unsigned long long bits = valid ? 1ull << (y & 63) : 0ull;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const unsigned long long ob = __shfl_down(bits, d, kWave);
            const uint64_t ow = __shfl_down(word, d, kWave);
            if (lane + d < kWave && ow == word) bits |= ob;
        }
        const uint64_t prev = __shfl_up(word, 1, kWave);
        if (valid && (lane == 0 || prev != word)) atomicOr(&H[word], bits);
    }
}

__global__ void ef_superblock_count_kernel(uint64_t nsb, uint64_t hwords, const uint64_t *__restrict__ H,
                                           uint32_t *__restrict__ cnt) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nsb; b += stride) {
        uint32_t c = 0;
        for (uint64_t k = 8 * b; k < 8 * b + 8 && k < hwords; ++k) c += (uint32_t)__popcll(H[k]);
        cnt[b] = c;
    }
}

__global__ void u64_to_u32_kernel(uint64_t count, const uint64_t *__restrict__ in, uint32_t *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        out[i] = (uint32_t)in[i];
}

__global__ void ef_select_kernel(uint64_t nsel, const uint64_t *__restrict__ x, uint32_t l,
                                 uint32_t *__restrict__ sel) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nsel; j += stride)
        sel[j] = (uint32_t)((x[64 * j] >> l) + 64 * j);
}

__global__ void offsets_to_u32_kernel(uint64_t count, const uint64_t *__restrict__ in, uint32_t *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        out[i] = (uint32_t)in[i];
}

// ---------------------------------------------------------------------------
// heavy vertices: degree above the threshold, listed in ascending order
// ---------------------------------------------------------------------------

__global__ void heavy_flag_kernel(uint32_t n, const uint64_t *__restrict__ off, uint32_t threshold,
                                  uint32_t *__restrict__ flag) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        flag[v] = (off[v + 1] - off[v]) > threshold ? 1u : 0u;
}

// bit v of word v/64: vertex v has no edges, or v >= n (padding)
__global__ void isolated_bitmap_kernel(uint32_t n, const uint64_t *__restrict__ off, uint64_t *__restrict__ iso) {
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    const uint32_t lane = lane_id();
    for (uint64_t q = wave; q < words; q += nwaves) {
        const uint64_t v = q * 64 + lane;
        const bool empty = v >= n || off[v + 1] == off[v];
        const uint64_t m = __ballot(empty);
        if (lane == 0) iso[q] = m;
    }
}

__global__ void heavy_scatter_kernel(uint32_t n, const uint32_t *__restrict__ flag, const uint64_t *__restrict__ pos,
                                     uint32_t *__restrict__ heavy) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        if (flag[v]) heavy[pos[v]] = (uint32_t)v;
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------

static inline uint32_t grid1(uint64_t count) { return grid_for(count, 256, 1u << 20); }

template <class Src>
static lg_status pack_fixed(Src src, uint64_t count, uint32_t w, DevBuf &dst, uint64_t &words, hipStream_t s) {
    words = (count * w + 63) / 64 + 1;
    LG_TRY(dst.scratch(words * 8, s));
    LG_LAUNCH(pack_fixed_kernel<Src>, grid1(words), 256, 0, s, src, count, w, w ? 1.0 / (double)w : 0.0, words,
              dst.as<uint64_t>());
    LG_CHECK_LAUNCH();
    return LG_OK;
}

// offsets structure over the values x[0..n] (element offsets or bit starts)
// bvIL words: block j at [9j, 9j + 9) = ones before it (the exclusive scan of
// the per-block counts), then the block's eight words of the plain vector;
// the last word is the total
__global__ void il_interleave_kernel(uint64_t blocks, const uint64_t *__restrict__ H, uint64_t hwords,
                                     const uint64_t *__restrict__ before, uint64_t *__restrict__ out) {
    const uint64_t total = 9 * blocks + 1;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const uint64_t j = i / 9, r = i - 9 * j;
        if (r == 0) {
            out[i] = before[j];  // j == blocks: the total
        } else {
            const uint64_t k = 8 * j + r - 1;
            out[i] = k < hwords ? H[k] : 0ull;
        }
    }
}

// Interleaved bit vector (bvIL): the plain vector (one at x_v + v) is built
// in a temporary, counted per 512-bit block, scanned, and laid out with the
// counts in front of the blocks.
static lg_status build_interleaved_bv(lg_graph *g, const uint64_t *x, uint64_t universe, DevBuf &tmp, hipStream_t s) {
    const uint64_t count = (uint64_t)g->n + 1;
    g->hbits = universe + count;
    const uint64_t hwords = (g->hbits + 63) / 64;
    DevBuf H, cnt, before;
    LG_TRY(H.scratch((hwords + 1) * 8, s));
    LG_TRY(fill_u64(H.as<uint64_t>(), 0, hwords + 1, s));
    LG_LAUNCH(ef_high_kernel, grid1(count), 256, 0, s, count, x, 0u, H.as<unsigned long long>());
    LG_CHECK_LAUNCH();
    const uint64_t blocks = (g->hbits + 511) / 512;
    LG_TRY(cnt.scratch(blocks * 4, s));
    LG_TRY(before.scratch((blocks + 1) * 8, s));
    LG_LAUNCH(ef_superblock_count_kernel, grid1(blocks), 256, 0, s, blocks, hwords, H.as<uint64_t>(),
              cnt.as<uint32_t>());
    LG_CHECK_LAUNCH();
    LG_TRY(exclusive_scan_u32(cnt.as<uint32_t>(), before.as<uint64_t>(), blocks, tmp, s));
    g->il_blocks = blocks;
    g->IL_words = 9 * blocks + 1;
    LG_TRY(g->IL.scratch(g->IL_words * 8, s));
    LG_LAUNCH(il_interleave_kernel, grid1(g->IL_words), 256, 0, s, blocks, H.as<uint64_t>(), hwords,
              before.as<uint64_t>(), g->IL.as<uint64_t>());
    LG_CHECK_LAUNCH();
    // the temporaries are read before this function returns and frees them
    LG_CHECK_HIP(hipStreamSynchronize(s));
    return LG_OK;
}

static lg_status build_offsets(lg_graph *g, const uint64_t *x, uint64_t universe, DevBuf &tmp, hipStream_t s) {
    const uint64_t count = (uint64_t)g->n + 1;
    g->universe = universe;
    if (g->offset_mode == LG_OFFS_PACKED) {
        g->wO = bitlen_u64(universe);  // 0 when every offset is 0 (no edges)
        return pack_fixed(SrcU64Mask{x, ~0ull}, count, g->wO, g->O, g->O_words, s);
    }
    if (g->offset_mode == LG_OFFS_INTERLEAVED_BV) return build_interleaved_bv(g, x, universe, tmp, s);
    // Elias-Fano: l = floor(log2(universe / count)) when universe >= count.
    // The plain bit vector (bvPL) is the same vector and directory without
    // low bits: its one for list v sits at x_v + v.
    const uint32_t l =
        (g->offset_mode == LG_OFFS_SUCCINCT && universe >= count) ? bitlen_u64(universe / count) - 1 : 0;
    g->ef_l = l;
    g->hbits = (universe >> l) + count;
    if (g->hbits >= (1ull << 32)) {
        set_error("%s offsets: bit vector of %llu bits exceeds 2^32",
                  g->offset_mode == LG_OFFS_SUCCINCT ? "succinct" : "plain bit-vector", (unsigned long long)g->hbits);
        return LG_ERR_UNSUPPORTED;
    }
    const uint64_t lowmask = l ? ((1ull << l) - 1) : 0ull;
    if (g->offset_mode == LG_OFFS_SUCCINCT)  // bvPL keeps no low bits
        LG_TRY(pack_fixed(SrcU64Mask{x, lowmask}, count, l, g->L, g->L_words, s));
    g->H_words = (g->hbits + 63) / 64 + 1;
    LG_TRY(g->H.scratch(g->H_words * 8, s));
    LG_TRY(fill_u64(g->H.as<uint64_t>(), 0, g->H_words, s));
    LG_LAUNCH(ef_high_kernel, grid1(count), 256, 0, s, count, x, l, g->H.as<unsigned long long>());
    LG_CHECK_LAUNCH();
    const uint64_t nsb = (g->hbits + 511) / 512;
    g->n_rank = nsb + 1;
    DevBuf cnt, scanned;
    LG_TRY(cnt.scratch(nsb * 4, s));
    LG_TRY(scanned.scratch((nsb + 1) * 8, s));
    LG_LAUNCH(ef_superblock_count_kernel, grid1(nsb), 256, 0, s, nsb, g->H_words, g->H.as<uint64_t>(),
              cnt.as<uint32_t>());
    LG_CHECK_LAUNCH();
    LG_TRY(exclusive_scan_u32(cnt.as<uint32_t>(), scanned.as<uint64_t>(), nsb, tmp, s));
    LG_TRY(g->rank_sb.scratch(g->n_rank * 4, s));
    LG_LAUNCH(u64_to_u32_kernel, grid1(g->n_rank), 256, 0, s, g->n_rank, scanned.as<uint64_t>(),
              g->rank_sb.as<uint32_t>());
    LG_CHECK_LAUNCH();
    g->n_sel = (count + 63) / 64;
    LG_TRY(g->sel.scratch(g->n_sel * 4, s));
    LG_LAUNCH(ef_select_kernel, grid1(g->n_sel), 256, 0, s, g->n_sel, x, l, g->sel.as<uint32_t>());
    LG_CHECK_LAUNCH();
    // the kernels above read cnt/scanned before this function returns and
    // frees them: wait for the stream
    LG_CHECK_HIP(hipStreamSynchronize(s));
    return LG_OK;
}

// Work items of an edge walk over the rows of `off` (see walk_item).
struct WalkTable {
    DevBuf cnt, coff, map;
    uint64_t items = 0;
    uint32_t grid = 1;
};

static lg_status walk_table(uint32_t n, const uint64_t *off, WalkTable &t, DevBuf &tmp, hipStream_t s) {
    const uint64_t blocks = ((uint64_t)n + 63) / 64;
    LG_TRY(t.cnt.scratch(blocks * 4, s));
    LG_TRY(t.coff.scratch((blocks + 1) * 8, s));
    LG_LAUNCH(walk_count_kernel, grid_for(blocks, 256, 1u << 16), 256, 0, s, n, off, t.cnt.as<uint32_t>());
    LG_CHECK_LAUNCH();
    LG_TRY(exclusive_scan_u32(t.cnt.as<uint32_t>(), t.coff.as<uint64_t>(), blocks, tmp, s));
    LG_CHECK_HIP(hipMemcpyAsync(&t.items, t.coff.as<uint64_t>() + blocks, 8, hipMemcpyDeviceToHost, s));
    LG_CHECK_HIP(hipStreamSynchronize(s));
    LG_TRY(t.map.scratch(t.items * 4, s));
    LG_LAUNCH(walk_map_kernel, grid_for(blocks, 256, 1u << 16), 256, 0, s, blocks, t.coff.as<uint64_t>(),
              t.map.as<uint32_t>());
    LG_CHECK_LAUNCH();
    t.grid = grid_for(t.items * kWave, 256, 16384);
    return LG_OK;
}

// perm (new label -> vertex) of the greedy relabeling; `walk` walks the
// input lists, `deg` holds the degrees
static lg_status greedy_permutation(uint32_t n, const uint64_t *off, const uint32_t *col, const DevBuf &deg,
                                    uint32_t max_degree, const WalkTable &walk, uint32_t *perm, DevBuf &tmp,
                                    hipStream_t s) {
    DevBuf k1, v1, k2, v2, rank, rmin, key, key2, val2;
    // processing order: degree ascending, ties by ID (stable sort)
    LG_TRY(k1.scratch((uint64_t)n * 4, s));
    LG_TRY(v1.scratch((uint64_t)n * 4, s));
    LG_TRY(k2.scratch((uint64_t)n * 4, s));
    LG_TRY(v2.scratch((uint64_t)n * 4, s));
    LG_LAUNCH(greedy_order_keys_kernel, grid1(n), 256, 0, s, n, deg.as<uint32_t>(), k1.as<uint32_t>(),
              v1.as<uint32_t>());
    LG_CHECK_LAUNCH();
    int alt = 0;
    LG_TRY(radix_sort_pairs(k1.as<uint32_t>(), v1.as<uint32_t>(), k2.as<uint32_t>(), v2.as<uint32_t>(), n,
                            std::max<uint32_t>(bitlen_u64(max_degree), 1u), tmp, s, &alt));
    const uint32_t *order = (alt ? v2 : v1).as<uint32_t>();
    LG_TRY(rank.scratch((uint64_t)n * 4, s));
    LG_LAUNCH(greedy_rank_kernel, grid1(n), 256, 0, s, n, order, rank.as<uint32_t>());
    LG_CHECK_LAUNCH();
    LG_TRY(rmin.scratch((uint64_t)n * 4, s));
    LG_TRY(fill_u32(rmin.as<uint32_t>(), 0xFFFFFFFFu, n, s));
    LG_LAUNCH(greedy_min_kernel, walk.grid, 256, 0, s, n, off, col, rank.as<uint32_t>(), walk.items,
              walk.map.as<uint32_t>(), walk.coff.as<uint64_t>(), rmin.as<uint32_t>());
    LG_CHECK_LAUNCH();
    // keys: rank below n (bitlen(n) bits) over a position below max_degree
    const uint32_t jbits = std::max<uint32_t>(bitlen_u64(max_degree ? max_degree - 1 : 0), 1u);
    LG_TRY(key.scratch((uint64_t)n * 8, s));
    LG_TRY(key2.scratch((uint64_t)n * 8, s));
    LG_TRY(val2.scratch((uint64_t)n * 4, s));
    LG_LAUNCH(greedy_key_kernel, grid1(n), 256, 0, s, n, off, col, order, rmin.as<uint32_t>(), jbits,
              key.as<uint64_t>(), perm);
    LG_CHECK_LAUNCH();
    LG_TRY(radix_sort_pairs64(key.as<uint64_t>(), perm, key2.as<uint64_t>(), val2.as<uint32_t>(), n,
                              bitlen_u64(n) + jbits, tmp, s));
    LG_CHECK_HIP(hipStreamSynchronize(s));
    return LG_OK;
}

static lg_status encode_impl(uint32_t n, uint64_t m, const uint64_t *row_offsets, const uint32_t *col,
                             const uint32_t *weights, const lg_encode_opts &o, hipStream_t s, lg_graph *g) {
    DevBuf tmp, status, deg, stats;
    DevBuf wt_new;  // relabeled weights
    LG_CHECK_HIP(hipGetDevice(&g->device));

    // -- validation ------------------------------------------------------
    LG_TRY(tmp.scratch(8, s));
    LG_TRY(status.scratch(4, s));
    LG_TRY(stats.scratch(8, s));
    LG_TRY(fill_u32(status.as<uint32_t>(), 0, 1, s));
    LG_TRY(fill_u32(stats.as<uint32_t>(), 0, 2, s));
    LG_LAUNCH(validate_offsets_kernel, grid_for(n, 256, 1u << 16), 256, 0, s, n, m, row_offsets,
              status.as<uint32_t>());
    LG_CHECK_LAUNCH();
    uint32_t bad = 0;
    LG_CHECK_HIP(hipMemcpyAsync(&bad, status.p, 4, hipMemcpyDeviceToHost, s));
    LG_CHECK_HIP(hipStreamSynchronize(s));
    WalkTable walk;
    DevBuf low;  // entries below the diagonal per row (the symmetry check's split)
    if (!bad) {  // the offsets are sound: walk the lists
        LG_TRY(walk_table(n, row_offsets, walk, tmp, s));
        LG_TRY(low.scratch((uint64_t)n * 4, s));
        LG_TRY(fill_u32(low.as<uint32_t>(), 0, n, s));
        LG_LAUNCH(validate_edges_kernel, walk.grid, 256, 0, s, n, row_offsets, col, walk.items,
                  walk.map.as<uint32_t>(), walk.coff.as<uint64_t>(), status.as<uint32_t>(), low.as<uint32_t>());
        LG_CHECK_LAUNCH();
        LG_CHECK_HIP(hipMemcpyAsync(&bad, status.p, 4, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
    }
    if (!bad && m) {
        // the offsets of the entries below the diagonal (counted by the validation walk)
        DevBuf lowoff;
        LG_TRY(lowoff.scratch(((uint64_t)n + 1) * 8, s));
        LG_TRY(exclusive_scan_u32(low.as<uint32_t>(), lowoff.as<uint64_t>(), n, tmp, s));
        uint64_t half = 0;
        LG_CHECK_HIP(hipMemcpyAsync(&half, lowoff.as<uint64_t>() + n, 8, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
        if (2 * half != m) {
            bad = kAsymmetric;  // the two halves differ in size
        } else {
            DevBuf key, val, key2, val2;
            LG_TRY(key.scratch(half * 4, s));
            LG_TRY(val.scratch(half * 4, s));
            LG_TRY(key2.scratch(half * 4, s));
            LG_TRY(val2.scratch(half * 4, s));
            LG_LAUNCH(sym_emit_kernel, walk.grid, 256, 0, s, n, row_offsets, col, walk.items,
                      walk.map.as<uint32_t>(), walk.coff.as<uint64_t>(), (const uint64_t *)lowoff.p,
                      key.as<uint32_t>(), val.as<uint32_t>());
            LG_CHECK_LAUNCH();
            int alt = 0;
            LG_TRY(radix_sort_pairs(key.as<uint32_t>(), val.as<uint32_t>(), key2.as<uint32_t>(),
                                    val2.as<uint32_t>(), half, bitlen_u64(n - 1), tmp, s, &alt));
            LG_LAUNCH(sym_check_kernel, walk.grid, 256, 0, s, n, row_offsets, col, walk.items,
                      walk.map.as<uint32_t>(), walk.coff.as<uint64_t>(), (const uint64_t *)lowoff.p, half,
                      (alt ? key2 : key).as<uint32_t>(), (alt ? val2 : val).as<uint32_t>(), status.as<uint32_t>());
            LG_CHECK_LAUNCH();
            LG_CHECK_HIP(hipMemcpyAsync(&bad, status.p, 4, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
        }
    }
    if (bad) {
        set_error("invalid input graph:%s%s%s%s%s", (bad & kBadOffsets) ? " bad-offsets" : "",
                  (bad & kBadId) ? " id>=n" : "", (bad & kSelfLoop) ? " self-loop" : "",
                  (bad & kUnsorted) ? " unsorted-or-duplicate" : "", (bad & kAsymmetric) ? " not-symmetric" : "");
        return LG_ERR_INVALID;
    }
    LG_TRY(deg.scratch((uint64_t)n * 4, s));
    LG_LAUNCH(degree_kernel, grid_for(n, 256, 4096), 256, 0, s, n, row_offsets, deg.as<uint32_t>(), stats.as<uint32_t>());
    LG_CHECK_LAUNCH();
    uint32_t st[2];
    LG_CHECK_HIP(hipMemcpyAsync(st, stats.p, 8, hipMemcpyDeviceToHost, s));
    LG_CHECK_HIP(hipStreamSynchronize(s));
    g->max_degree = st[0];
    g->isolated = st[1];
    if (weights) {
        g->weighted = true;
        uint32_t wmax = 0;
        if (m) {
            LG_TRY(fill_u32(stats.as<uint32_t>(), 0, 1, s));
            LG_LAUNCH(max_u32_kernel, grid_for(m, 256, 4096), 256, 0, s, m, weights, stats.as<uint32_t>());
            LG_CHECK_LAUNCH();
            LG_CHECK_HIP(hipMemcpyAsync(&wmax, stats.p, 4, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
        }
        g->omega = wmax ? bitlen_u64(wmax) : 1u;
    }

    // -- relabeling --------------------------------------------------------
    const uint64_t *cur_off = row_offsets;
    const uint32_t *cur_col = col;
    DevBuf off_new, col_new;
    const uint32_t idbits = bitlen_u64(n - 1);
    if (o.relabel != LG_RELABEL_NONE) {
        DevBuf deg_new;
        LG_TRY(g->perm.scratch((uint64_t)n * 4, s));
        LG_TRY(g->inv.scratch((uint64_t)n * 4, s));
        LG_TRY(deg_new.scratch((uint64_t)n * 4, s));
        if (o.relabel == LG_RELABEL_DEGREE) {
            DevBuf k1, k2, v2;
            LG_TRY(k1.scratch((uint64_t)n * 4, s));
            LG_TRY(k2.scratch((uint64_t)n * 4, s));
            LG_TRY(v2.scratch((uint64_t)n * 4, s));
            LG_LAUNCH(dm_keys_kernel, grid1(n), 256, 0, s, n, deg.as<uint32_t>(), k1.as<uint32_t>(),
                      g->perm.as<uint32_t>());
            LG_CHECK_LAUNCH();
            LG_TRY(radix_sort_pairs(k1.as<uint32_t>(), g->perm.as<uint32_t>(), k2.as<uint32_t>(),
                                    v2.as<uint32_t>(), n, idbits, tmp, s));
        } else {
            LG_TRY(greedy_permutation(n, row_offsets, col, deg, g->max_degree, walk, g->perm.as<uint32_t>(), tmp,
                                      s));
        }
        LG_LAUNCH(dm_inverse_kernel, grid1(n), 256, 0, s, n, g->perm.as<uint32_t>(), deg.as<uint32_t>(),
                  g->inv.as<uint32_t>(), deg_new.as<uint32_t>());
        LG_CHECK_LAUNCH();
        LG_TRY(off_new.scratch(((uint64_t)n + 1) * 8, s));
        LG_TRY(exclusive_scan_u32(deg_new.as<uint32_t>(), off_new.as<uint64_t>(), n, tmp, s));
        if (m) {
            DevBuf key, key2, val2;
            LG_TRY(key.scratch(m * 4, s));
            LG_TRY(col_new.scratch(m * 4, s));
            LG_TRY(key2.scratch(m * 4, s));
            LG_TRY(val2.scratch(m * 4, s));
            WalkTable wnew;
            LG_TRY(walk_table(n, off_new.as<uint64_t>(), wnew, tmp, s));
            // key: original target; col_new (as values): new source row
            LG_LAUNCH(dm_emit_kernel, wnew.grid, 256, 0, s, n, g->perm.as<uint32_t>(), row_offsets, col,
                      off_new.as<uint64_t>(), wnew.items, wnew.map.as<uint32_t>(), wnew.coff.as<uint64_t>(),
                      key.as<uint32_t>(), col_new.as<uint32_t>());
            LG_CHECK_LAUNCH();
            int alt = 0;
            LG_TRY(radix_sort_pairs(key.as<uint32_t>(), col_new.as<uint32_t>(), key2.as<uint32_t>(),
                                    val2.as<uint32_t>(), m, idbits, tmp, s, &alt));
            // the grouped values now sit in col_new (or val2); place them by new row into the other buffer
            DevBuf &grouped = alt ? val2 : col_new;
            DevBuf &placed = alt ? col_new : key2;
            LG_LAUNCH(dm_place_kernel, wnew.grid, 256, 0, s, n, g->perm.as<uint32_t>(), row_offsets,
                      grouped.as<uint32_t>(), off_new.as<uint64_t>(), wnew.items, wnew.map.as<uint32_t>(),
                      wnew.coff.as<uint64_t>(), placed.as<uint32_t>());
            LG_CHECK_LAUNCH();
            if (!alt) std::swap(col_new, key2);  // col_new holds the relabeled lists
            LG_CHECK_HIP(hipStreamSynchronize(s));
        }
        LG_CHECK_HIP(hipStreamSynchronize(s));
        cur_off = off_new.as<uint64_t>();
        cur_col = col_new.as<uint32_t>();
        if (weights && m) {  // the weights follow their edges
            LG_TRY(wt_new.scratch(m * 4, s));
            DevBuf miss;
            LG_TRY(miss.scratch(8, s));
            LG_TRY(fill_u32(miss.as<uint32_t>(), 0, 1, s));
            LG_LAUNCH(relabel_weights_kernel, grid1(m), 256, 0, s, n, m, cur_off, cur_col, g->perm.as<uint32_t>(),
                      row_offsets, col, weights, wt_new.as<uint32_t>(), miss.as<uint32_t>());
            LG_CHECK_LAUNCH();
            uint32_t missed = 0;
            LG_CHECK_HIP(hipMemcpyAsync(&missed, miss.p, 4, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
            if (missed) {
                set_error("lg_encode_weighted: a relabeled entry has no edge in its original list");
                return LG_ERR_DEVICE;
            }
            weights = wt_new.as<uint32_t>();
        }
    }

    // -- heavy vertex list (shared by the traversal kernels) -------------
    {
        DevBuf flag, pos;
        LG_TRY(flag.scratch((uint64_t)n * 4, s));
        LG_TRY(pos.scratch(((uint64_t)n + 1) * 8, s));
        LG_LAUNCH(heavy_flag_kernel, grid1(n), 256, 0, s, n, cur_off, g->heavy_threshold, flag.as<uint32_t>());
        LG_CHECK_LAUNCH();
        LG_TRY(exclusive_scan_u32(flag.as<uint32_t>(), pos.as<uint64_t>(), n, tmp, s));
        uint64_t nh = 0;
        LG_CHECK_HIP(hipMemcpyAsync(&nh, pos.as<uint64_t>() + n, 8, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
        g->n_heavy = (uint32_t)nh;
        LG_TRY(g->heavy.scratch((nh ? nh : 1) * 4, s));
        LG_LAUNCH(heavy_scatter_kernel, grid1(n), 256, 0, s, n, flag.as<uint32_t>(), pos.as<uint64_t>(),
                  g->heavy.as<uint32_t>());
        LG_CHECK_LAUNCH();
        const uint64_t words = ((uint64_t)n + 63) / 64;
        LG_TRY(g->iso.scratch(words * 8, s));
        LG_LAUNCH(isolated_bitmap_kernel, grid_for(words * kWave, 256, 1u << 16), 256, 0, s, n, cur_off,
                  g->iso.as<uint64_t>());
        LG_CHECK_LAUNCH();
        LG_CHECK_HIP(hipStreamSynchronize(s));
    }

    // -- plain CSR baseline ----------------------------------------------
    if (o.layout == LG_LAYOUT_PLAIN) {
        g->poff64 = m >= (1ull << 32);
        if (g->poff64) {
            LG_TRY(g->poff.scratch(((uint64_t)n + 1) * 8, s));
            LG_CHECK_HIP(hipMemcpyAsync(g->poff.p, cur_off, ((uint64_t)n + 1) * 8, hipMemcpyDeviceToDevice, s));
        } else {
            LG_TRY(g->poff.scratch(((uint64_t)n + 1) * 4, s));
            LG_LAUNCH(offsets_to_u32_kernel, grid1(n + 1ull), 256, 0, s, (uint64_t)n + 1, cur_off,
                      g->poff.as<uint32_t>());
            LG_CHECK_LAUNCH();
        }
        if (col_new.p) {
            g->pcol = std::move(col_new);
        } else {
            LG_TRY(g->pcol.scratch((m ? m : 1) * 4, s));
            if (m) LG_CHECK_HIP(hipMemcpyAsync(g->pcol.p, cur_col, m * 4, hipMemcpyDeviceToDevice, s));
        }
        if (weights) {
            LG_TRY(g->pwt.scratch((m ? m : 1) * 4, s));
            if (m) LG_CHECK_HIP(hipMemcpyAsync(g->pwt.p, weights, m * 4, hipMemcpyDeviceToDevice, s));
        }
        LG_CHECK_HIP(hipStreamSynchronize(s));
        return LG_OK;
    }

    // -- packed representation ---------------------------------------------
    g->s = idbits ? idbits : 1;
    if (o.id_mode == LG_IDS_VARINT_FULL || o.id_mode == LG_IDS_VARINT_DIFF) {
        const bool diff = o.id_mode == LG_IDS_VARINT_DIFF;
        DevBuf P;
        LG_TRY(P.scratch(((uint64_t)n + 1) * 8, s));
        uint64_t total = 0;
        if (m) {
            DevBuf head, len, pos;
            LG_TRY(head.scratch((m + 3) & ~3ull, s));
            LG_TRY(len.scratch(m * 4, s));
            LG_TRY(pos.scratch((m + 1) * 8, s));
            LG_TRY(fill_u32(head.as<uint32_t>(), 0, (m + 3) / 4, s));
            LG_LAUNCH(varint_head_kernel, grid1(n), 256, 0, s, n, cur_off, head.as<uint8_t>());
            LG_CHECK_LAUNCH();
            if (diff)
                LG_LAUNCH(varint_len_kernel<true>, grid1(m), 256, 0, s, m, cur_col, head.as<uint8_t>(),
                          len.as<uint32_t>());
            else
                LG_LAUNCH(varint_len_kernel<false>, grid1(m), 256, 0, s, m, cur_col, head.as<uint8_t>(),
                          len.as<uint32_t>());
            LG_CHECK_LAUNCH();
            LG_TRY(exclusive_scan_u32(len.as<uint32_t>(), pos.as<uint64_t>(), m, tmp, s));
            LG_CHECK_HIP(hipMemcpyAsync(&total, pos.as<uint64_t>() + m, 8, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
            g->A_words = (total + 7) / 8 + 1;
            LG_TRY(g->A.scratch(g->A_words * 8, s));
            LG_TRY(fill_u64(g->A.as<uint64_t>(), 0, g->A_words, s));
            if (diff)
                LG_LAUNCH(varint_write_kernel<true>, grid1(m), 256, 0, s, m, cur_col, head.as<uint8_t>(),
                          pos.as<uint64_t>(), g->A.as<uint8_t>());
            else
                LG_LAUNCH(varint_write_kernel<false>, grid1(m), 256, 0, s, m, cur_col, head.as<uint8_t>(),
                          pos.as<uint64_t>(), g->A.as<uint8_t>());
            LG_CHECK_LAUNCH();
            LG_LAUNCH(varint_starts_kernel, grid1(n + 1ull), 256, 0, s, n, cur_off, pos.as<uint64_t>(),
                      P.as<uint64_t>());
            LG_CHECK_LAUNCH();
            LG_CHECK_HIP(hipStreamSynchronize(s));
        } else {
            g->A_words = 1;
            LG_TRY(g->A.scratch(8, s));
            LG_TRY(fill_u64(g->A.as<uint64_t>(), 0, 1, s));
            LG_TRY(fill_u64(P.as<uint64_t>(), 0, (uint64_t)n + 1, s));
        }
        g->U = total * 8;
        LG_TRY(build_offsets(g, P.as<uint64_t>(), total, tmp, s));
    } else if (o.id_mode == LG_IDS_GLOBAL && weights) {
        g->U = m * (uint64_t)(g->s + g->omega);
        g->A_words = (g->U + 63) / 64 + 1;
        LG_TRY(g->A.scratch(g->A_words * 8, s));
        LG_TRY(fill_u64(g->A.as<uint64_t>(), 0, g->A_words, s));
        if (m) {
            LG_LAUNCH(pack_weighted_kernel<false>, grid1(m), 256, 0, s, n, m, cur_off, cur_col, weights,
                      (const uint8_t *)nullptr, (const uint64_t *)nullptr, g->s, g->omega,
                      g->A.as<unsigned long long>());
            LG_CHECK_LAUNCH();
        }
        LG_TRY(build_offsets(g, cur_off, m, tmp, s));
    } else if (o.id_mode == LG_IDS_LOCAL && weights) {
        g->F = bitlen_u64(g->s);
        DevBuf w8, len, P;
        LG_TRY(w8.scratch((uint64_t)n, s));
        LG_TRY(len.scratch((uint64_t)n * 8, s));
        LG_TRY(P.scratch(((uint64_t)n + 1) * 8, s));
        LG_LAUNCH(local_width_kernel, grid1(n), 256, 0, s, n, cur_off, cur_col, w8.as<uint8_t>(),
                  len.as<uint64_t>());
        LG_CHECK_LAUNCH();
        LG_LAUNCH(weighted_len_kernel, grid1(n), 256, 0, s, n, cur_off, w8.as<uint8_t>(), g->omega,
                  len.as<uint64_t>());
        LG_CHECK_LAUNCH();
        LG_TRY(exclusive_scan_u64(len.as<uint64_t>(), P.as<uint64_t>(), n, tmp, s));
        LG_CHECK_HIP(hipMemcpyAsync(&g->U, P.as<uint64_t>() + n, 8, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
        LG_TRY(pack_fixed(SrcU8{w8.as<uint8_t>()}, n, g->F, g->W, g->W_words, s));
        g->A_words = (g->U + 63) / 64 + 1;
        LG_TRY(g->A.scratch(g->A_words * 8, s));
        LG_TRY(fill_u64(g->A.as<uint64_t>(), 0, g->A_words, s));
        if (m) {
            LG_LAUNCH(pack_weighted_kernel<true>, grid1(m), 256, 0, s, n, m, cur_off, cur_col, weights,
                      w8.as<uint8_t>(), P.as<uint64_t>(), g->s, g->omega, g->A.as<unsigned long long>());
            LG_CHECK_LAUNCH();
        }
        LG_TRY(build_offsets(g, P.as<uint64_t>(), g->U, tmp, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
    } else if (o.id_mode == LG_IDS_GLOBAL) {
        g->U = m * g->s;
        LG_TRY(pack_fixed(SrcU32{cur_col}, m, g->s, g->A, g->A_words, s));
        LG_TRY(build_offsets(g, cur_off, m, tmp, s));
    } else {
        g->F = bitlen_u64(g->s);
        DevBuf w8, len, P;
        LG_TRY(w8.scratch((uint64_t)n, s));
        LG_TRY(len.scratch((uint64_t)n * 8, s));
        LG_TRY(P.scratch(((uint64_t)n + 1) * 8, s));
        LG_LAUNCH(local_width_kernel, grid1(n), 256, 0, s, n, cur_off, cur_col, w8.as<uint8_t>(),
                  len.as<uint64_t>());
        LG_CHECK_LAUNCH();
        WalkTable wp;
        LG_TRY(walk_table(n, cur_off, wp, tmp, s));
        const bool gap = o.id_mode == LG_IDS_LOCAL_GAP;
        DevBuf g8, gmax;
        if (gap) {  // gap widths, and bit lengths w_v + (d_v - 1) g_v
            LG_TRY(g8.scratch((uint64_t)n, s));
            LG_TRY(gmax.scratch((uint64_t)n * 4, s));
            LG_TRY(fill_u32(gmax.as<uint32_t>(), 0, n, s));
            if (m) {
                LG_LAUNCH(gap_max_kernel, wp.grid, 256, 0, s, n, cur_off, cur_col, wp.items, wp.map.as<uint32_t>(),
                          wp.coff.as<uint64_t>(), gmax.as<uint32_t>());
                LG_CHECK_LAUNCH();
            }
            LG_LAUNCH(gap_len_kernel, grid1(n), 256, 0, s, n, cur_off, w8.as<uint8_t>(), gmax.as<uint32_t>(),
                      g8.as<uint8_t>(), len.as<uint64_t>());
            LG_CHECK_LAUNCH();
        }
        LG_TRY(exclusive_scan_u64(len.as<uint64_t>(), P.as<uint64_t>(), n, tmp, s));
        LG_CHECK_HIP(hipMemcpyAsync(&g->U, P.as<uint64_t>() + n, 8, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
        LG_TRY(pack_fixed(SrcU8{w8.as<uint8_t>()}, n, g->F, g->W, g->W_words, s));
        if (gap) LG_TRY(pack_fixed(SrcU8{g8.as<uint8_t>()}, n, g->F, g->G, g->G_words, s));
        g->A_words = (g->U + 63) / 64 + 1;
        LG_TRY(g->A.scratch(g->A_words * 8, s));
        LG_TRY(fill_u64(g->A.as<uint64_t>(), 0, g->A_words, s));
        if (gap)
            LG_LAUNCH((pack_walk_kernel<true>), wp.grid, 256, 0, s, n, cur_off, cur_col, w8.as<uint8_t>(),
                      g8.as<uint8_t>(), P.as<uint64_t>(), wp.items, wp.map.as<uint32_t>(), wp.coff.as<uint64_t>(),
                      g->A.as<unsigned long long>());
        else
            LG_LAUNCH((pack_walk_kernel<false>), wp.grid, 256, 0, s, n, cur_off, cur_col, w8.as<uint8_t>(),
                      (const uint8_t *)nullptr, P.as<uint64_t>(), wp.items, wp.map.as<uint32_t>(),
                      wp.coff.as<uint64_t>(), g->A.as<unsigned long long>());
        LG_CHECK_LAUNCH();
        LG_TRY(build_offsets(g, P.as<uint64_t>(), g->U, tmp, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
    }
    LG_CHECK_HIP(hipStreamSynchronize(s));
    return LG_OK;
}

static lg_status encode_entry(uint32_t n, uint64_t m, const uint64_t *row_offsets, const uint32_t *col,
                              const uint32_t *weights, const lg_encode_opts *opts, hipStream_t stream,
                              lg_graph **out);

}  // namespace lg

extern "C" lg_status lg_encode(uint32_t n, uint64_t m, const uint64_t *row_offsets, const uint32_t *col,
                               const lg_encode_opts *opts, hipStream_t stream, lg_graph **out) {
    return lg::encode_entry(n, m, row_offsets, col, nullptr, opts, stream, out);
}

extern "C" lg_status lg_encode_weighted(uint32_t n, uint64_t m, const uint64_t *row_offsets, const uint32_t *col,
                                        const uint32_t *weights, const lg_encode_opts *opts, hipStream_t stream,
                                        lg_graph **out) {
    using namespace lg;
    if (!weights && m) {
        if (out) *out = nullptr;
        set_error("lg_encode_weighted: weights is NULL");
        return LG_ERR_INVALID;
    }
    lg_encode_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.layout == LG_LAYOUT_PACKED && o.id_mode != LG_IDS_GLOBAL && o.id_mode != LG_IDS_LOCAL) {
        if (out) *out = nullptr;
        set_error("lg_encode_weighted: weighted graphs take global or local IDs (or the plain layout)");
        return LG_ERR_UNSUPPORTED;
    }
    // a non-NULL marker when there are no entries, so the graph is weighted
    static const uint32_t kNone = 0;
    return encode_entry(n, m, row_offsets, col, weights ? weights : &kNone, opts, stream, out);
}

namespace lg {

static lg_status encode_entry(uint32_t n, uint64_t m, const uint64_t *row_offsets, const uint32_t *col,
                              const uint32_t *weights, const lg_encode_opts *opts, hipStream_t stream,
                              lg_graph **out) {
    if (!out) { set_error("lg_encode: out is NULL"); return LG_ERR_INVALID; }
    *out = nullptr;
    lg_encode_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (n == 0 || n >= (1u << 31)) { set_error("lg_encode: n must be in [1, 2^31)"); return LG_ERR_INVALID; }
    if (m >= (1ull << 36)) { set_error("lg_encode: m must be below 2^36"); return LG_ERR_UNSUPPORTED; }
    if (!row_offsets || (m && !col)) { set_error("lg_encode: NULL input array"); return LG_ERR_INVALID; }
    if (o.layout > LG_LAYOUT_PLAIN || o.id_mode > LG_IDS_VARINT_DIFF || o.offset_mode > LG_OFFS_INTERLEAVED_BV ||
        o.relabel > LG_RELABEL_GREEDY || o.flags || o.reserved[0] || o.reserved[1] || o.reserved[2]) {
        set_error("lg_encode: unknown option value");
        return LG_ERR_INVALID;
    }
    if (o.layout == LG_LAYOUT_PACKED && o.offset_mode == LG_OFFS_INTERLEAVED_BV &&
        (weights || (o.id_mode != LG_IDS_GLOBAL && o.id_mode != LG_IDS_LOCAL))) {
        set_error("lg_encode: interleaved bit-vector offsets take global or local IDs without weights");
        return LG_ERR_UNSUPPORTED;
    }
    lg_graph *g = new (std::nothrow) lg_graph();
    if (!g) { set_error("lg_encode: host allocation failed"); return LG_ERR_OOM; }
    g->n = n;
    g->m = m;
    g->layout = o.layout;
    g->id_mode = o.layout == LG_LAYOUT_PACKED ? o.id_mode : 0;
    g->offset_mode = o.layout == LG_LAYOUT_PACKED ? o.offset_mode : 0;
    g->relabel = o.relabel;
    lg_status st = encode_impl(n, m, row_offsets, col, weights, o, stream, g);
    // gap and Varint lists: the segment tables of the long lists serve the
    // traversals too (several BFS lanes may run at once), so build them here
    if (st == LG_OK && g->layout == LG_LAYOUT_PACKED && g->id_mode == LG_IDS_LOCAL_GAP)
        st = ensure_heavy_segments(g, stream);
    if (st == LG_OK && g->layout == LG_LAYOUT_PACKED &&
        (g->id_mode == LG_IDS_VARINT_FULL || g->id_mode == LG_IDS_VARINT_DIFF))
        st = build_varint_segments(g, stream);
    if (st == LG_OK && hipEventCreateWithFlags(&g->last_use, hipEventDisableTiming) != hipSuccess) {
        g->last_use = nullptr;
        set_error("lg_encode: hipEventCreateWithFlags failed");
        st = LG_ERR_DEVICE;
    }
    if (st == LG_OK) st = mark_use(g, stream);
    if (st != LG_OK) {
        (void)hipStreamSynchronize(stream);
        lg_free(g);
        return st;
    }
    *out = g;
    return LG_OK;
}

}  // namespace lg
