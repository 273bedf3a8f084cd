// lg_bfs: direction-optimizing breadth-first search over the packed (or
// plain) adjacency array, decoding neighbor lists inside the frontier
// kernels (BFS of section "Considered Algorithms"; the edge extraction of
// subsection "Accessing An Edge").
//
// Top-down level d:
//   prepare  per frontier vertex: (first bit, degree, width) from the offset
//            structure; exclusive scan of the degrees
//   expand   every block takes a fixed tile of frontier edges, stages the
//            frontier entries the tile touches in LDS, and each lane decodes
//            one edge (u), skips u if visited before this level, claims
//            depth[u] with a CAS, records the smallest-label parent with
//            atomicMin, and winners are appended to the next queue with one
//            atomic per wave (ballot + mbcnt)
// Bottom-up level d:
//   each wave owns 64 consecutive vertices (one visited word); an unvisited
//   vertex decodes its list in ascending order and stops at the first
//   neighbor in the frontier bitmap, which is its smallest-label parent
// The switch between the two follows the edge-count heuristic of
// direction-optimizing BFS; it changes the running time only.
// Gap and Varint lists, whose entries can only be read in order, take the
// same level loop with in-order kernels (bfs_one_inorder): a wave per
// frontier list or per segment of a long list top-down, a lane per list
// with a wave pass for long lists bottom-up.
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lg_device.hpp"
#include "lg_varint.hpp"

namespace lg {

uint64_t BfsWork::bytes() const {
    return qa.bytes + qb.bytes + fstart.bytes + fdeg.bytes + fw.bytes + fscan.bytes + visited.bytes + curr.bytes +
           next.bytes + counters.bytes + sample.bytes + depth_i.bytes + parent_i.bytes + scan_tmp.bytes + pv.bytes + pstart.bytes +
           pdeg.bytes + pw.bytes + pseg_cnt.bytes + pseg_off.bytes;
}

BfsWork::~BfsWork() {
    if (host) (void)hipHostFree(host);
}

BfsPool::~BfsPool() {
    for (BfsLane *l : lanes) {
        if (l->stream) {
            (void)hipStreamSynchronize(l->stream);
            (void)hipStreamDestroy(l->stream);
        }
        if (l->done) (void)hipEventDestroy(l->done);
        delete l;
    }
    if (start) (void)hipEventDestroy(start);
}

uint64_t BfsPool::bytes() const {
    uint64_t b = ms.bytes();
    for (const BfsLane *l : lanes) b += l->work.bytes();
    return b;
}

uint64_t bfs_bytes(const lg_graph *g) { return g->bfs ? g->bfs->bytes() : 0; }

lg_status bfs_free(lg_graph *g) {
    delete g->bfs;
    g->bfs = nullptr;
    return LG_OK;
}

lg_status bfs_workspace_ensure(BfsWork &w, uint64_t n, uint64_t n_heavy, bool relabel, bool need_parent) {
    if (!w.host) {
        if (hipHostMalloc((void **)&w.host, 8 * sizeof(uint64_t)) != hipSuccess) {
            w.host = nullptr;
            set_error("lg_bfs: pinned host allocation failed");
            return LG_ERR_OOM;
        }
    }
    const uint64_t words = (n + 63) / 64;
    LG_TRY(w.qa.ensure(n * 4));
    LG_TRY(w.qb.ensure(n * 4));
    LG_TRY(w.fstart.ensure(n * 8));
    LG_TRY(w.fdeg.ensure(n * 4));
    LG_TRY(w.fw.ensure(n * 4));
    LG_TRY(w.fscan.ensure((n + 1) * 8));
    LG_TRY(w.visited.ensure(words * 8));
    LG_TRY(w.curr.ensure(words * 8));
    LG_TRY(w.next.ensure(words * 8));
    LG_TRY(w.counters.ensure(8 * 8));
    LG_TRY(w.sample.ensure(8 * 8));
    const uint64_t nh = n_heavy ? n_heavy : 1;
    LG_TRY(w.pv.ensure(nh * 4));
    LG_TRY(w.pstart.ensure(nh * 8));
    LG_TRY(w.pdeg.ensure(nh * 4));
    LG_TRY(w.pw.ensure(nh * 4));
    LG_TRY(w.pseg_cnt.ensure(nh * 4));
    LG_TRY(w.pseg_off.ensure((nh + 1) * 8));
    if (relabel) {
        LG_TRY(w.depth_i.ensure(n * 4));
        if (need_parent) LG_TRY(w.parent_i.ensure(n * 4));
    }
    return LG_OK;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// visited starts as the root plus every vertex without edges (never reached,
// never a neighbor), so bottom-up sweeps skip words of such vertices
// The root arrives as its original ID and is mapped to its label here (inv,
// when relabeled), so that no host round trip is needed.
__global__ void bfs_init_kernel(uint32_t n, int32_t *__restrict__ depth, uint32_t *__restrict__ parent,
                                const uint64_t *__restrict__ iso, uint64_t *__restrict__ visited, uint32_t root_id,
                                const uint32_t *__restrict__ inv, uint32_t *__restrict__ queue,
                                uint64_t *__restrict__ counters) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint32_t root = inv ? inv[root_id] : root_id;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        depth[i] = i == root ? 0 : -1;
        if (parent) parent[i] = i == root ? root : 0xFFFFFFFFu;
        if (i < words) visited[i] = iso[i] | ((i == (root >> 6)) ? (1ull << (root & 63)) : 0ull);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        queue[0] = root;
        for (int i = 0; i < 5; ++i) counters[i] = 0;  // queue count and both bottom-up pairs
    }
}

// Degrees of a fixed sample of a large frontier: kDirSample vertices at
// evenly spaced queue positions, a partial sum per block.  Decoding every
// frontier vertex's offsets only to learn that the search turns bottom-up
// is the costliest step of that level with Elias-Fano offsets.
constexpr uint32_t kDirSampleBlocks = 8;
constexpr uint32_t kDirSampleThreads = 512;
constexpr uint32_t kDirSample = kDirSampleBlocks * kDirSampleThreads;
static_assert(kDirSampleBlocks <= 8, "the partial sums are read back into the 8-word host staging area");

template <class Acc>
__global__ __launch_bounds__(kDirSampleThreads) void td_sample_kernel(Acc acc, const uint32_t *__restrict__ queue,
                                                                      uint64_t qsize, uint64_t *__restrict__ part) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long d = acc.info(queue[i * qsize / kDirSample]).deg;
    const unsigned long long t = block_sum_u64(d);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Bottom-up cost of the next level on a sample: kDirSample vertices at evenly
// spaced labels; one not yet visited reads its list in order until its first
// neighbour in the frontier bitmap (at most kBuSampleWalk entries), as the
// bottom-up sweep would; its cost is one (its offsets) plus the entries read.
// Partial sums per block.
constexpr uint32_t kBuSampleWalk = 1024;

template <class Acc>
__global__ __launch_bounds__(kDirSampleThreads) void bu_cost_sample_kernel(Acc acc, uint32_t n,
                                                                           const uint64_t *__restrict__ visited,
                                                                           const uint64_t *__restrict__ curr,
                                                                           uint64_t *__restrict__ part) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t v = (uint32_t)(((2 * i + 1) * (uint64_t)n) / (2ull * kDirSample));
    unsigned long long cost = 0;
    if (v < n && !((visited[v >> 6] >> (v & 63)) & 1ull)) {
        const VInfo vi = acc.info(v);
        const uint32_t st = Acc::step(vi.w), mk = Acc::mask(vi.w);
        const uint32_t lim = vi.deg < kBuSampleWalk ? vi.deg : kBuSampleWalk;
        cost = 1;
        for (uint32_t j = 0; j < lim; ++j) {
            const uint32_t u = acc.get(vi.start + (uint64_t)j * st, mk);
            ++cost;
            if (u < n && ((curr[u >> 6] >> (u & 63)) & 1ull)) break;
        }
    }
    const unsigned long long t = block_sum_u64(cost);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <class Acc>
__global__ void td_prepare_kernel(Acc acc, const uint32_t *__restrict__ queue, uint32_t qsize,
                                  uint64_t *__restrict__ fstart, uint32_t *__restrict__ fdeg,
                                  uint32_t *__restrict__ fw) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < qsize; i += stride) {
        const VInfo vi = acc.info(queue[i]);
        fstart[i] = vi.start;
        fdeg[i] = vi.deg;
        fw[i] = vi.w;
    }
}

constexpr uint32_t kStrideBlocks = 4096;  // grid of the grid-stride sweep kernels
constexpr int kTdThreads = 256;
constexpr int kTdEdgesPerThread = 4;
constexpr uint32_t kTdTile = kTdThreads * kTdEdgesPerThread;

// largest i in [lo, hi] with a[i] <= x (a non-decreasing, a[lo] <= x)
template <class T>
__device__ __forceinline__ uint32_t last_le(const T *a, uint32_t lo, uint32_t hi, uint64_t x) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo + 1) >> 1);
        if ((uint64_t)a[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// kMin: a level large enough that a pass over every vertex is cheap beside
// it.  Each edge to an unvisited vertex does one atomicMin of the parent
// (whose result nobody waits for; without parents, a plain store of the
// depth, the same value from every writer) instead of a CAS on the depth,
// the atomicMin and a queue append: td_finish_kernel then finds the new
// vertices.  The smallest label among the level's claimants is the parent
// either way.
template <class Acc, bool kParent, bool kMin = false>
__global__ __launch_bounds__(kTdThreads) void td_expand_kernel(
    Acc acc, const uint32_t *__restrict__ queue, uint32_t qsize, const uint64_t *__restrict__ fstart,
    const uint32_t *__restrict__ fw, const uint64_t *__restrict__ fscan, uint64_t edges,
    const uint64_t *__restrict__ visited, int32_t *__restrict__ depth, uint32_t *__restrict__ parent,
    int32_t next_depth, uint32_t *__restrict__ queue_out, unsigned long long *__restrict__ tail) {
    __shared__ uint64_t s_scan[kTdTile + 1];
    __shared__ uint64_t s_start[kTdTile];
    __shared__ uint32_t s_w[kTdTile];
    __shared__ uint32_t s_v[kTdTile];
    __shared__ uint32_t s_range[2];
    __shared__ uint32_t s_wsum[kTdThreads / kWave];
    __shared__ unsigned long long s_base;
    const uint32_t lane = lane_id();
    for (uint64_t t = blockIdx.x; t * kTdTile < edges; t += gridDim.x) {
        const uint64_t e0 = t * kTdTile;
        const uint64_t e1 = e0 + kTdTile < edges ? e0 + kTdTile : edges;
        if (threadIdx.x == 0) s_range[0] = last_le(fscan, 0, qsize - 1, e0);
        if (threadIdx.x == 1) s_range[1] = last_le(fscan, 0, qsize - 1, e1 - 1);
        __syncthreads();
        const uint32_t i0 = s_range[0];
        const uint32_t span = s_range[1] - i0 + 1;
        const bool staged = span <= kTdTile;
        if (staged) {
            for (uint32_t j = threadIdx.x; j < span; j += kTdThreads) {
                s_scan[j] = fscan[i0 + j];
                s_start[j] = fstart[i0 + j];
                s_w[j] = fw[i0 + j];
                s_v[j] = queue[i0 + j];
            }
        }
        __syncthreads();
        // every thread decodes its (up to) kTdEdgesPerThread edges, keeps the
        // vertices it claimed, and the block reserves queue space once
        // in phases, so that a thread's list loads and then its bitmap loads
        // are in flight together: a load under a per-edge branch waits for its
        // data before the branch ends.  An idle slot reads stream position 0
        // with mask 0 (the level has edges, so the stream holds one) and then
        // bitmap word 0.
        uint64_t epos[kTdEdgesPerThread];
        uint32_t msk[kTdEdgesPerThread], src[kTdEdgesPerThread];
        uint32_t live = 0;
#pragma unroll
        for (int r = 0; r < kTdEdgesPerThread; ++r) {
            const uint64_t e = e0 + (uint64_t)r * kTdThreads + threadIdx.x;
            epos[r] = 0;
            msk[r] = src[r] = 0;
            if (e < e1) {
                uint64_t base_e, start;
                uint32_t w, v;
                if (staged) {
                    const uint32_t j = last_le(s_scan, 0, span - 1, e);
                    base_e = s_scan[j]; start = s_start[j]; w = s_w[j]; v = s_v[j];
                } else {
                    const uint32_t j = last_le(fscan, i0, s_range[1], e);
                    base_e = fscan[j]; start = fstart[j]; w = fw[j]; v = queue[j];
                }
                epos[r] = start + (e - base_e) * Acc::step(w);
                msk[r] = Acc::mask(w);
                src[r] = v;
                live |= 1u << r;
            }
        }
        uint32_t u[kTdEdgesPerThread];
        uint64_t vw[kTdEdgesPerThread];
#pragma unroll
        for (int r = 0; r < kTdEdgesPerThread; ++r) u[r] = acc.get(epos[r], msk[r]);
#pragma unroll
        for (int r = 0; r < kTdEdgesPerThread; ++r) vw[r] = visited[u[r] >> 6];
        if constexpr (kMin) {
#pragma unroll
            for (int r = 0; r < kTdEdgesPerThread; ++r) {
                if (((live >> r) & 1u) && !((vw[r] >> (u[r] & 63)) & 1ull)) {
                    if constexpr (kParent) atomicMin(&parent[u[r]], src[r]);
                    else depth[u[r]] = next_depth;
                }
            }
            __syncthreads();  // the next tile rewrites the staged ranges
            continue;
        }
        uint32_t won[kTdEdgesPerThread];
        uint32_t nwon = 0;
#pragma unroll
        for (int r = 0; r < kTdEdgesPerThread; ++r) {
            if (((live >> r) & 1u) && !((vw[r] >> (u[r] & 63)) & 1ull)) {
                const int32_t old = atomicCAS(&depth[u[r]], -1, next_depth);
                if (kParent && (old == -1 || old == next_depth)) atomicMin(&parent[u[r]], src[r]);
                if (old == -1) won[nwon++] = u[r];
            }
        }
        // block exclusive scan of the claim counts, one atomic per tile
        const uint32_t incl = wave_incl_scan(nwon);
        if (lane == kWave - 1) s_wsum[threadIdx.x / kWave] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < kTdThreads / kWave; ++w) { const uint32_t c = s_wsum[w]; s_wsum[w] = tot; tot += c; }
            s_base = tot ? atomicAdd(tail, (unsigned long long)tot) : 0ull;
        }
        __syncthreads();
        unsigned long long pos = s_base + s_wsum[threadIdx.x / kWave] + (incl - nwon);
        for (uint32_t i = 0; i < nwon; ++i) queue_out[pos + i] = won[i];
        __syncthreads();
    }
}

// After a claim-only level (td_expand_kernel<..., kMin = true>): a wave per
// 64-vertex word finds the vertices not visited before whose parent (or,
// without parents, depth) the level set, writes their depth, and writes the
// word of the next frontier's bitmap and the visited one.  Past n the
// visited bits are set (the isolated-vertex bitmap pads them).
template <bool kParent>
__global__ void td_finish_kernel(uint32_t n, uint64_t *__restrict__ visited, const uint32_t *__restrict__ parent,
                                 int32_t *__restrict__ depth, int32_t next_depth, uint64_t *__restrict__ frontier) {
    const uint32_t lane = lane_id();
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wstride = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t w = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; w < words; w += wstride) {
        const uint64_t v = w * 64 + lane;
        const uint64_t vc = v < n ? v : n - 1;
        // both loads at once (a load under a branch waits before the branch ends)
        const uint64_t vis = visited[w];
        uint32_t pv = 0;
        int32_t dv = 0;
        if constexpr (kParent) pv = parent[vc];
        else dv = depth[vc];
        const bool fresh = !((vis >> lane) & 1ull) && (kParent ? pv != 0xFFFFFFFFu : dv == next_depth);
        if (kParent && fresh) depth[v] = next_depth;
        const uint64_t m = __ballot(fresh);
        if (lane == 0) {
            frontier[w] = m;
            if (m) visited[w] = vis | m;
        }
    }
}

// A small top-down level in one launch: a wave per frontier vertex decodes
// its list and claims neighbors by the same rule as td_expand_kernel (skip
// vertices visited before this level, CAS the depth, smallest parent label
// among the claimants of the level).  Used for the small frontiers at the end
// of a search, where the prepare / scan / expand launches and their host
// round trips would cost more than the work.
template <class Acc, bool kParent>
__global__ void td_small_kernel(Acc acc, const uint32_t *__restrict__ queue, uint32_t qsize,
                                const uint64_t *__restrict__ visited, int32_t *__restrict__ depth,
                                uint32_t *__restrict__ parent, int32_t next_depth, uint32_t *__restrict__ queue_out,
                                unsigned long long *__restrict__ tail) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t i = wave; i < qsize; i += nwaves) {
        const uint32_t v = queue[i];
        const VInfo vi = acc.info(v);
        const uint32_t st = Acc::step(vi.w), mk = Acc::mask(vi.w);
        for (uint64_t e0 = 0; e0 < vi.deg; e0 += kWave) {
            const uint64_t e = e0 + lane;
            bool won = false;
            uint32_t u = 0;
            if (e < vi.deg) {
                u = acc.get(vi.start + e * st, mk);
                if (!((visited[u >> 6] >> (u & 63)) & 1ull)) {
                    const int32_t old = atomicCAS(&depth[u], -1, next_depth);
                    if (kParent && (old == -1 || old == next_depth)) atomicMin(&parent[u], v);
                    won = old == -1;
                }
            }
            const uint64_t m = __ballot(won);
            if (m) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(tail, (unsigned long long)__popcll(m));
                base = __shfl(base, 0, kWave) + popc_below(m);
                if (won) queue_out[base] = u;
            }
        }
    }
}

constexpr uint32_t kSmallFrontier = 16384;  // frontier size up to which late levels take td_small_kernel

// Marks the q queued vertices in a bitmap.  The queue counter was read by
// the host already: the kernel clears it for the next level's appends.
__global__ void mark_queue_kernel(const uint32_t *__restrict__ queue, uint64_t q, unsigned long long *__restrict__ bits,
                                  unsigned long long *__restrict__ counter) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < q; i += stride) {
        const uint32_t u = queue[i];
        atomicOr(&bits[u >> 6], 1ull << (u & 63));
    }
}

// The bitmaps of a level whose queue holds a large share of the vertices,
// streamed from the depth array (a wave per 64-vertex word, one coalesced
// read): `frontier` = the vertices at depth d, `visited` = every reached
// vertex and every vertex without edges.  One atomic per queued vertex costs
// far more once the queue holds millions of vertices (30 M at one level of a
// uniform random graph of 67 M vertices: 2.5 ms against 0.1 ms).  Either
// bitmap may be NULL.  Clears the queue counter as mark_queue_kernel does.
__global__ void level_bitmaps_kernel(uint32_t n, const int32_t *__restrict__ depth, int32_t d,
                                     const uint64_t *__restrict__ iso, uint64_t *__restrict__ frontier,
                                     uint64_t *__restrict__ visited, unsigned long long *__restrict__ counter) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
    const uint32_t lane = lane_id();
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wstride = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t w = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; w < words; w += wstride) {
        const uint64_t v = w * 64 + lane;
        const int32_t dv = v < n ? depth[v] : -1;
        const uint64_t at = __ballot(dv == d);
        const uint64_t reached = __ballot(dv >= 0);
        if (lane == 0) {
            if (frontier) frontier[w] = at;
            if (visited) visited[w] = reached | iso[w];
        }
    }
}

// Sweep over all vertices, a lane per vertex: an unvisited vertex decodes
// the first min(d_v, threshold) entries of its list (its smallest labels),
// four at a time, and stops at the first frontier neighbor -- its parent.
// A vertex with more entries and no hit among them is appended to the
// pending list for the segment pass.
template <class Acc, bool kParent>
__global__ void bu_step_kernel(Acc acc, uint32_t n, uint32_t threshold, const uint64_t *__restrict__ curr,
                               uint64_t *__restrict__ visited, uint64_t *__restrict__ next,
                               int32_t *__restrict__ depth, uint32_t *__restrict__ parent, int32_t next_depth,
                               unsigned long long *__restrict__ counters, unsigned long long *__restrict__ next_counters,
                               uint32_t *__restrict__ pv, uint64_t *__restrict__ pstart, uint32_t *__restrict__ pdeg,
                               uint32_t *__restrict__ pw) {
    const uint32_t lane = lane_id();
    // the next bottom-up level counts into the other pair: clear it here
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        next_counters[1] = 0;
        next_counters[2] = 0;
    }
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    unsigned long long woke = 0;
    for (uint64_t q = wave; q < words; q += nwaves) {
        const uint64_t vis = visited[q];
        // the offset decode's select samples do not depend on the visited
        // word: issue their loads together with it
        EFSamples smp{0, 0};
        if constexpr (Acc::kPacked && Acc::kEF) smp = ef_samples(acc.pv.ef, q * 64, n + 1);
        if (vis == ~0ull) {  // every word of next is written: no clearing launch
            if (lane == 0) next[q] = 0;
            continue;
        }
        const VInfo vi = wave_info(acc, q * 64, n, &smp);
        const uint64_t v = q * 64 + lane;
        bool found = false, pending = false;
        uint32_t par = 0;
        if (v < n && !((vis >> lane) & 1ull) && vi.deg) {
            const uint32_t st = Acc::step(vi.w), mk = Acc::mask(vi.w);
            const uint32_t lim = vi.deg < threshold ? vi.deg : threshold;
            for (uint32_t i = 0; i < lim && !found; i += 4) {
                // four list loads, then four frontier-bitmap loads, with no
                // branch between them (entries past the limit re-read the
                // first one, which exists: d_v >= 1)
                uint32_t u[4];
                uint64_t cw[4];
                bool f[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) u[b] = acc.get(vi.start + (uint64_t)(i + b < lim ? i + b : 0u) * st, mk);
#pragma unroll
                for (int b = 0; b < 4; ++b) cw[b] = curr[u[b] >> 6];
#pragma unroll
                for (int b = 0; b < 4; ++b) f[b] = i + b < lim && ((cw[b] >> (u[b] & 63)) & 1ull);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    if (f[b] && !found) { found = true; par = u[b]; }
                }
            }
            pending = !found && vi.deg > threshold;
        }
        const uint64_t fm = __ballot(found);
        if (found) {
            depth[v] = next_depth;
            if (kParent) parent[v] = par;
        }
        if (lane == 0) next[q] = fm;
        if (lane == 0 && fm) {
            visited[q] |= fm;
            woke += (unsigned long long)__popcll(fm);
        }
        const uint64_t pm = __ballot(pending);
        if (pm) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&counters[2], (unsigned long long)__popcll(pm));
            base = __shfl(base, 0, kWave) + popc_below(pm);
            if (pending) {
                pv[base] = (uint32_t)v;
                pstart[base] = vi.start;
                pdeg[base] = vi.deg;
                pw[base] = vi.w;
            }
        }
    }
    woke = block_sum_u64(woke);
    if (threadIdx.x == 0 && woke) atomicAdd(&counters[1], woke);
}

constexpr uint32_t kPendingSeg = 1024;  // entries per segment of the pending pass

__global__ void bu_pending_count_kernel(const unsigned long long *__restrict__ counters, uint32_t threshold,
                                        const uint32_t *__restrict__ pdeg, uint32_t *__restrict__ cnt) {
    const uint64_t np = counters[2];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride)
        cnt[i] = (pdeg[i] - threshold + kPendingSeg - 1) / kPendingSeg;
}

// Segment pass over the pending heavy vertices' entries [threshold, d):
// one wave per segment of kPendingSeg entries, 64 per probe.  Lists ascend,
// so a segment's first frontier neighbor is its smallest and the smallest
// over the segments is the parent (atomicMin); a segment whose first label
// already exceeds the best parent found skips its scan.
template <class Acc, bool kParent>
__global__ void bu_pending_kernel(Acc acc, uint32_t threshold, uint64_t np, const uint64_t *__restrict__ pseg_off,
                                  const uint32_t *__restrict__ pv, const uint64_t *__restrict__ pstart,
                                  const uint32_t *__restrict__ pdeg, const uint32_t *__restrict__ pw,
                                  const uint64_t *__restrict__ curr, unsigned long long *__restrict__ visited,
                                  unsigned long long *__restrict__ next, int32_t *__restrict__ depth,
                                  uint32_t *__restrict__ parent, int32_t next_depth,
                                  unsigned long long *__restrict__ counters) {
    const uint32_t lane = lane_id();
    const uint64_t nseg = pseg_off[np];
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    unsigned long long woke = 0;
    for (uint64_t k = wave; k < nseg; k += nwaves) {
        uint32_t lo = 0, hi = (uint32_t)np - 1;  // pending vertex owning segment k
        while (lo < hi) {
            const uint32_t mid = lo + ((hi - lo + 1) >> 1);
            if (pseg_off[mid] <= k) lo = mid; else hi = mid - 1;
        }
        const uint32_t v = pv[lo];
        const uint32_t w = pw[lo];
        const uint32_t st = Acc::step(w), mk = Acc::mask(w);
        const uint64_t start = pstart[lo];
        const uint64_t d = pdeg[lo];
        const uint64_t e0 = threshold + (k - pseg_off[lo]) * kPendingSeg;
        const uint64_t e1 = e0 + kPendingSeg < d ? e0 + kPendingSeg : d;
        if (kParent) {
            if (parent[v] < acc.get(start + e0 * st, mk)) continue;
        } else if (depth[v] == next_depth) {
            continue;
        }
        for (uint64_t base = e0; base < e1; base += kWave) {
            const uint64_t i = base + lane;
            uint32_t u = 0;
            bool hit = false;
            if (i < e1) {
                u = acc.get(start + i * st, mk);
                hit = (curr[u >> 6] >> (u & 63)) & 1ull;
            }
            const uint64_t m = __ballot(hit);
            if (m) {
                const uint32_t first = (uint32_t)__ffsll((long long)m) - 1;
                const uint32_t par = __shfl(u, first, kWave);
                if (lane == 0) {
                    if (kParent) atomicMin(&parent[v], par);
                    if (atomicCAS(&depth[v], -1, next_depth) == -1) {
                        atomicOr(&next[v >> 6], 1ull << (v & 63));
                        atomicOr(&visited[v >> 6], 1ull << (v & 63));
                        ++woke;
                    }
                }
                break;
            }
        }
    }
    woke = block_sum_u64(woke);
    if (threadIdx.x == 0 && woke) atomicAdd(&counters[1], woke);
}

// frontier bitmap -> queue.  A wave takes 64 consecutive words (one per
// lane), reserves their entries with one atomic and writes them in order,
// 64 consecutive queue slots per step: slot j's word is the one whose
// prefix count range holds j (a binary search of the wave's inclusive
// counts), its bit the (j - count before)-th one of that word.  One lane
// writing its word's ones one after another scattered every store.
__global__ void bitmap_to_queue_kernel(uint64_t words, const uint64_t *__restrict__ bits,
                                       uint32_t *__restrict__ queue, unsigned long long *__restrict__ tail) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t w0 = wave * kWave; w0 < words; w0 += nwaves * kWave) {
        const uint64_t q = w0 + lane;
        const uint64_t b = q < words ? bits[q] : 0ull;
        const uint32_t c = (uint32_t)__popcll(b);
        const uint32_t incl = wave_incl_scan(c);
        const uint32_t total = __shfl(incl, kWave - 1, kWave);
        if (total == 0) continue;  // wave-uniform
        unsigned long long off = 0;
        if (lane == 0) off = atomicAdd(tail, (unsigned long long)total);
        off = __shfl(off, 0, kWave);
        for (uint32_t j0 = 0; j0 < total; j0 += kWave) {
            const uint32_t j = j0 + lane;
            // the number of words whose inclusive count is <= j (at most 63:
            // the last word's count is total > j); power-of-two steps keep
            // every shuffle index in the wave
            uint32_t k = 0;
#pragma unroll
            for (uint32_t step = kWave / 2; step > 0; step >>= 1)
                if (__shfl(incl, k + step - 1, kWave) <= j) k += step;
            const uint64_t x = __shfl(b, k, kWave);
            const uint32_t before = __shfl(incl, k, kWave) - __shfl(c, k, kWave);
            if (j < total) queue[off + j] = (uint32_t)((w0 + k) * 64 + select_in_word(x, j - before));
        }
    }
}

// ---------------------------------------------------------------------------
// gap-encoded lists (subsection "Adding Fixed-Size Gap Encoding"): an entry
// is the difference to the one before, so every list is read from its
// start.  Top-down, a wave per frontier vertex takes 64 entries per step
// and a wave prefix sum; bottom-up, a lane per unvisited vertex adds up to
// `threshold` differences, four loads at a time, and a wave per longer
// list without a hit goes on from there.  Depths and parents follow the
// rules of the other encodings (the smallest label one level up).
// ---------------------------------------------------------------------------

template <class Acc>
__global__ __launch_bounds__(kDirSampleThreads) void inorder_sample_kernel(Acc acc, const uint32_t *__restrict__ queue,
                                                                           uint64_t qsize, uint64_t *__restrict__ part) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t v = queue[i * qsize / kDirSample];
    unsigned long long d;
    if constexpr (IsGapAcc<Acc>::value) {
        d = acc.info(v).deg;
    } else {
        uint64_t b0, b1;
        acc.offsets(v, b0, b1);
        d = b1 - b0;
    }
    const unsigned long long t = block_sum_u64(d);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <class Acc>
__global__ void gap_frontier_edges_kernel(Acc acc, const uint32_t *__restrict__ queue, uint64_t qsize,
                                          unsigned long long *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long e = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < qsize; i += stride)
        e += acc.info(queue[i]).deg;
    e = block_sum_u64(e);
    if (threadIdx.x == 0 && e) atomicAdd(out, e);
}

template <class Acc, bool kParent>
__global__ void td_gap_kernel(Acc acc, uint32_t n, uint32_t split, const uint32_t *__restrict__ queue, uint64_t qsize,
                              const uint64_t *__restrict__ visited, int32_t *__restrict__ depth,
                              uint32_t *__restrict__ parent, int32_t next_depth, uint32_t *__restrict__ queue_out,
                              unsigned long long *__restrict__ tail) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t i = wave; i < qsize; i += nwaves) {
        const uint32_t v = queue[i];
        const GapInfo gi = acc.info(v);
        if (gi.deg > split) continue;  // a segmented list: td_gap_seg_kernel
        uint32_t carry = 0;
        for (uint64_t j0 = 0; j0 < gi.deg; j0 += kWave) {
            const uint64_t j = j0 + lane;
            const bool valid = j < gi.deg;
            const uint32_t x = valid ? acc.get(Acc::entry_bit(gi, j), j ? gi.g : gi.w) : 0u;
            const uint32_t val = wave_incl_scan(x) + carry;
            carry = __shfl(val, kWave - 1, kWave);
            // a stored label is < n; the clamp keeps every access in bounds
            // whatever the stream holds
            const uint32_t u = val < n ? val : n - 1;
            bool won = false;
            if (valid && !((visited[u >> 6] >> (u & 63)) & 1ull)) {
                const int32_t old = atomicCAS(&depth[u], -1, next_depth);
                if (kParent && (old == -1 || old == next_depth)) atomicMin(&parent[u], v);
                won = old == -1;
            }
            const uint64_t m = __ballot(won);
            if (m) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(tail, (unsigned long long)__popcll(m));
                base = __shfl(base, 0, kWave) + popc_below(m);
                if (won) queue_out[base] = u;
            }
        }
    }
}

// The lists longer than `split` of the frontier, one wave per segment of
// seg_size entries (the graph's tables: segment k of heavy vertex
// seg_map[k], whose prefix starts from seg_base[k]); a segment whose vertex
// is not in the frontier bitmap is skipped.
template <class Acc, bool kParent>
__global__ void td_gap_seg_kernel(Acc acc, uint32_t n, uint64_t n_seg, uint32_t seg_size,
                                  const uint32_t *__restrict__ seg_map, const uint64_t *__restrict__ seg_off,
                                  const uint32_t *__restrict__ heavy, const uint64_t *__restrict__ hstart,
                                  const uint32_t *__restrict__ hdeg, const uint32_t *__restrict__ hw,
                                  const uint32_t *__restrict__ hg, const uint32_t *__restrict__ seg_base,
                                  const uint64_t *__restrict__ frontier, const uint64_t *__restrict__ visited,
                                  int32_t *__restrict__ depth, uint32_t *__restrict__ parent, int32_t next_depth,
                                  uint32_t *__restrict__ queue_out, unsigned long long *__restrict__ tail) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t k = wave; k < n_seg; k += nwaves) {
        const uint32_t h = seg_map[k];
        const uint32_t v = heavy[h];
        if (!((frontier[v >> 6] >> (v & 63)) & 1ull)) continue;  // same for every lane
        const uint64_t d = hdeg[h];
        const uint64_t e0 = (k - seg_off[h]) * seg_size;
        const uint64_t e1 = e0 + seg_size < d ? e0 + seg_size : d;
        const GapInfo gi{hstart[h], (uint32_t)d, hw[h], hg[h]};
        uint32_t carry = seg_base[k];
        for (uint64_t j0 = e0; j0 < e1; j0 += kWave) {
            const uint64_t j = j0 + lane;
            const bool valid = j < e1;
            const uint32_t x = valid ? acc.get(Acc::entry_bit(gi, j), j ? gi.g : gi.w) : 0u;
            const uint32_t val = wave_incl_scan(x) + carry;
            carry = __shfl(val, kWave - 1, kWave);
            const uint32_t u = val < n ? val : n - 1;
            bool won = false;
            if (valid && !((visited[u >> 6] >> (u & 63)) & 1ull)) {
                const int32_t old = atomicCAS(&depth[u], -1, next_depth);
                if (kParent && (old == -1 || old == next_depth)) atomicMin(&parent[u], v);
                won = old == -1;
            }
            const uint64_t m = __ballot(won);
            if (m) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(tail, (unsigned long long)__popcll(m));
                base = __shfl(base, 0, kWave) + popc_below(m);
                if (won) queue_out[base] = u;
            }
        }
    }
}

template <class Acc, bool kParent>
__global__ void bu_gap_kernel(Acc acc, uint32_t n, uint32_t threshold, const uint64_t *__restrict__ curr,
                              uint64_t *__restrict__ visited, uint64_t *__restrict__ next,
                              int32_t *__restrict__ depth, uint32_t *__restrict__ parent, int32_t next_depth,
                              unsigned long long *__restrict__ counters, unsigned long long *__restrict__ next_counters,
                              uint32_t *__restrict__ pv, uint64_t *__restrict__ pstart, uint32_t *__restrict__ pdeg,
                              uint32_t *__restrict__ pwg, uint32_t *__restrict__ pcarry) {
    const uint32_t lane = lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        next_counters[1] = 0;
        next_counters[2] = 0;
    }
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    unsigned long long woke = 0;
    for (uint64_t q = wave; q < words; q += nwaves) {
        const uint64_t vis = visited[q];
        if (vis == ~0ull) {
            if (lane == 0) next[q] = 0;
            continue;
        }
        const uint64_t v = q * 64 + lane;
        const bool open = v < n && !((vis >> lane) & 1ull);
        uint64_t o0, o1;
        wave_offsets(acc.base, q * 64, n, o0, o1);
        GapInfo gi{0, 0, 0, 0};
        if (open && o1 > o0) {
            gi.start = o0;
            gi.w = acc.base.width((uint32_t)v);
            gi.g = acc.gap_width((uint32_t)v);
            gi.deg = gi.g == 0 ? 1u : 1u + exact_div_width(o1 - o0 - gi.w, gi.g);
        }
        bool found = false, pending = false;
        uint32_t par = 0, val = 0;
        if (open && gi.deg) {
            const uint32_t lim = gi.deg < threshold ? gi.deg : threshold;
            for (uint32_t i = 0; i < lim && !found; i += 4) {
                uint32_t x[4], u[4];
                uint64_t cw[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t e = i + b < lim ? i + b : 0u;  // past the limit: entry 0 again, dropped
                    x[b] = acc.get(Acc::entry_bit(gi, e), e ? gi.g : gi.w);
                }
                uint32_t run = val;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    run += i + b < lim ? x[b] : 0u;
                    u[b] = run < n ? run : n - 1;
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) cw[b] = curr[u[b] >> 6];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    if (!found && i + b < lim) {
                        val += x[b];
                        if ((cw[b] >> (u[b] & 63)) & 1ull) { found = true; par = u[b]; }
                    }
                }
            }
            pending = !found && gi.deg > threshold;
        }
        const uint64_t fm = __ballot(found);
        if (found) {
            depth[v] = next_depth;
            if (kParent) parent[v] = par;
        }
        if (lane == 0) next[q] = fm;
        if (lane == 0 && fm) {
            visited[q] |= fm;
            woke += (unsigned long long)__popcll(fm);
        }
        const uint64_t pm = __ballot(pending);
        if (pm) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&counters[2], (unsigned long long)__popcll(pm));
            base = __shfl(base, 0, kWave) + popc_below(pm);
            if (pending) {
                pv[base] = (uint32_t)v;
                pstart[base] = gi.start;
                pdeg[base] = gi.deg;
                pwg[base] = gi.w | (gi.g << 8);
                pcarry[base] = val;  // the label of entry threshold - 1
            }
        }
    }
    woke = block_sum_u64(woke);
    if (threadIdx.x == 0 && woke) atomicAdd(&counters[1], woke);
}

// the pending lists from entry `threshold` on, a wave each, 64 entries per
// step; the first frontier neighbor is the smallest, the parent
template <class Acc, bool kParent>
__global__ void bu_gap_pending_kernel(Acc acc, uint32_t n, uint32_t threshold, uint64_t np,
                                      const uint32_t *__restrict__ pv, const uint64_t *__restrict__ pstart,
                                      const uint32_t *__restrict__ pdeg, const uint32_t *__restrict__ pwg,
                                      const uint32_t *__restrict__ pcarry, const uint64_t *__restrict__ curr,
                                      unsigned long long *__restrict__ visited, unsigned long long *__restrict__ next,
                                      int32_t *__restrict__ depth, uint32_t *__restrict__ parent, int32_t next_depth,
                                      unsigned long long *__restrict__ counters) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    unsigned long long woke = 0;
    for (uint64_t p = wave; p < np; p += nwaves) {
        const uint32_t v = pv[p];
        const uint32_t wg = pwg[p];
        const GapInfo gi{pstart[p], pdeg[p], wg & 255u, wg >> 8};
        uint32_t carry = pcarry[p];
        for (uint64_t e0 = threshold; e0 < gi.deg; e0 += kWave) {
            const uint64_t i = e0 + lane;
            const bool valid = i < gi.deg;
            const uint32_t x = valid ? acc.get(Acc::entry_bit(gi, i), gi.g) : 0u;
            const uint32_t val = wave_incl_scan(x) + carry;
            carry = __shfl(val, kWave - 1, kWave);
            const uint32_t u = val < n ? val : n - 1;
            const bool hit = valid && ((curr[u >> 6] >> (u & 63)) & 1ull);
            const uint64_t m = __ballot(hit);
            if (m) {
                const uint32_t first = (uint32_t)__ffsll((long long)m) - 1;
                const uint32_t par = __shfl(u, first, kWave);
                if (lane == 0) {
                    depth[v] = next_depth;
                    if (kParent) parent[v] = par;
                    atomicOr(&next[v >> 6], 1ull << (v & 63));
                    atomicOr(&visited[v >> 6], 1ull << (v & 63));
                    ++woke;
                }
                break;
            }
        }
    }
    woke = block_sum_u64(woke);
    if (threadIdx.x == 0 && woke) atomicAdd(&counters[1], woke);
}

// ---------------------------------------------------------------------------
// Varint lists (subsection "Incorporating Degree-Minimizing (DM)"): byte
// streams of base-128 values, read in order like gap lists.  The direction
// rule counts list bytes instead of entries (it changes the time, never the
// result).  Top-down, a wave per frontier vertex takes 64 bytes per step: a
// lane holding a value's last byte assembles the value from the (at most
// four) continuation bytes before it, DMd adds a wave prefix sum; bottom-up,
// a lane per unvisited vertex decodes up to `threshold` values from 8-byte
// windows and stops at the first frontier neighbor, and a wave per longer
// list without a hit goes on from the byte and label it reached.
// ---------------------------------------------------------------------------

template <class Acc>
__global__ void varint_frontier_bytes_kernel(Acc acc, const uint32_t *__restrict__ queue, uint64_t qsize,
                                             unsigned long long *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long e = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < qsize; i += stride) {
        uint64_t b0, b1;
        acc.offsets(queue[i], b0, b1);
        e += b1 - b0;
    }
    e = block_sum_u64(e);
    if (threadIdx.x == 0 && e) atomicAdd(out, e);
}

template <class Acc, bool kParent>
__global__ void td_varint_kernel(Acc acc, uint32_t n, uint64_t split, const uint32_t *__restrict__ queue, uint64_t qsize,
                                 const uint64_t *__restrict__ visited, int32_t *__restrict__ depth,
                                 uint32_t *__restrict__ parent, int32_t next_depth, uint32_t *__restrict__ queue_out,
                                 unsigned long long *__restrict__ tail) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t i = wave; i < qsize; i += nwaves) {
        const uint32_t v = queue[i];
        uint64_t b0, b1;
        acc.offsets(v, b0, b1);
        if (b1 - b0 > split) continue;  // a chunked list: td_varint_seg_kernel
        uint32_t prevb = 0, carry = 0;
        for (uint64_t p0 = b0; p0 < b1; p0 += kWave) {
            uint32_t x;
            const bool end = varint_step(acc, p0, b1, prevb, x);
            uint32_t label = x;
            if constexpr (Acc::kDifferences) {
                const uint32_t sc = wave_incl_scan(end ? x : 0u);
                label = carry + sc;
                carry += __shfl(sc, kWave - 1, kWave);
            }
            // a stored label is < n; the clamp keeps every access in bounds
            const uint32_t u = label < n ? label : n - 1;
            bool won = false;
            if (end && !((visited[u >> 6] >> (u & 63)) & 1ull)) {
                const int32_t old = atomicCAS(&depth[u], -1, next_depth);
                if (kParent && (old == -1 || old == next_depth)) atomicMin(&parent[u], v);
                won = old == -1;
            }
            const uint64_t m = __ballot(won);
            if (m) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(tail, (unsigned long long)__popcll(m));
                base = __shfl(base, 0, kWave) + popc_below(m);
                if (won) queue_out[base] = u;
            }
        }
    }
}

template <class Acc>
__global__ void varint_seg_info_kernel(Acc acc, const uint32_t *__restrict__ heavy, uint32_t n_heavy, uint64_t split,
                                       uint32_t chunk, uint64_t *__restrict__ hb0, uint64_t *__restrict__ hb1,
                                       uint32_t *__restrict__ segcnt) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n_heavy; h += stride) {
        uint64_t b0, b1;
        acc.offsets(heavy[h], b0, b1);
        hb0[h] = b0;
        hb1[h] = b1;
        segcnt[h] = b1 - b0 > split ? (uint32_t)((b1 - b0 + chunk - 1) / chunk) : 0u;
    }
}

__global__ void varint_seg_map_kernel(uint32_t n_heavy, const uint64_t *__restrict__ seg_off,
                                      uint32_t *__restrict__ seg_map) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n_heavy; h += stride)
        for (uint64_t k = seg_off[h]; k < seg_off[h + 1]; ++k) seg_map[k] = (uint32_t)h;
}

// sum of the differences ending in each chunk (DMd), a wave per chunk
template <class Acc>
__global__ void varint_seg_sum_kernel(Acc acc, uint64_t n_seg, uint32_t chunk, const uint32_t *__restrict__ seg_map,
                                      const uint64_t *__restrict__ seg_off, const uint64_t *__restrict__ hb0,
                                      const uint64_t *__restrict__ hb1, uint32_t *__restrict__ seg_sum) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t k = wave; k < n_seg; k += nwaves) {
        const uint32_t h = seg_map[k];
        const uint64_t b0 = hb0[h], b1 = hb1[h];
        const uint64_t c0 = b0 + (k - seg_off[h]) * chunk;
        const uint64_t c1 = c0 + chunk < b1 ? c0 + chunk : b1;
        uint32_t prevb = varint_chunk_prevb(acc, b0, c0), sum = 0;
        for (uint64_t p0 = c0; p0 < c1; p0 += kWave) {
            uint32_t x;
            const bool end = varint_step(acc, p0, c1, prevb, x);
            sum += end ? x : 0u;
        }
        sum = wave_sum(sum);
        if (lane == 0) seg_sum[k] = sum;
    }
}

__global__ void varint_seg_base_kernel(uint64_t n_seg, const uint32_t *__restrict__ seg_map,
                                       const uint64_t *__restrict__ seg_off, const uint64_t *__restrict__ scan,
                                       uint32_t *__restrict__ seg_base) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_seg; k += stride)
        seg_base[k] = (uint32_t)(scan[k] - scan[seg_off[seg_map[k]]]);
}

template <class Acc, bool kParent>
__global__ void td_varint_seg_kernel(Acc acc, uint32_t n, uint64_t n_seg, uint32_t chunk,
                                     const uint32_t *__restrict__ seg_map, const uint64_t *__restrict__ seg_off,
                                     const uint32_t *__restrict__ heavy, const uint64_t *__restrict__ hb0,
                                     const uint64_t *__restrict__ hb1, const uint32_t *__restrict__ seg_base,
                                     const uint64_t *__restrict__ frontier, const uint64_t *__restrict__ visited,
                                     int32_t *__restrict__ depth, uint32_t *__restrict__ parent, int32_t next_depth,
                                     uint32_t *__restrict__ queue_out, unsigned long long *__restrict__ tail) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t k = wave; k < n_seg; k += nwaves) {
        const uint32_t h = seg_map[k];
        const uint32_t v = heavy[h];
        if (!((frontier[v >> 6] >> (v & 63)) & 1ull)) continue;  // same for every lane
        const uint64_t b0 = hb0[h], b1 = hb1[h];
        const uint64_t c0 = b0 + (k - seg_off[h]) * chunk;
        const uint64_t c1 = c0 + chunk < b1 ? c0 + chunk : b1;
        uint32_t prevb = varint_chunk_prevb(acc, b0, c0), carry = seg_base[k];
        for (uint64_t p0 = c0; p0 < c1; p0 += kWave) {
            uint32_t x;
            const bool end = varint_step(acc, p0, c1, prevb, x);
            uint32_t label = x;
            if constexpr (Acc::kDifferences) {
                const uint32_t sc = wave_incl_scan(end ? x : 0u);
                label = carry + sc;
                carry += __shfl(sc, kWave - 1, kWave);
            }
            const uint32_t u = label < n ? label : n - 1;
            bool won = false;
            if (end && !((visited[u >> 6] >> (u & 63)) & 1ull)) {
                const int32_t old = atomicCAS(&depth[u], -1, next_depth);
                if (kParent && (old == -1 || old == next_depth)) atomicMin(&parent[u], v);
                won = old == -1;
            }
            const uint64_t m = __ballot(won);
            if (m) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(tail, (unsigned long long)__popcll(m));
                base = __shfl(base, 0, kWave) + popc_below(m);
                if (won) queue_out[base] = u;
            }
        }
    }
}

template <class Acc, bool kParent>
__global__ void bu_varint_kernel(Acc acc, uint32_t n, uint32_t threshold, const uint64_t *__restrict__ curr,
                                 uint64_t *__restrict__ visited, uint64_t *__restrict__ next,
                                 int32_t *__restrict__ depth, uint32_t *__restrict__ parent, int32_t next_depth,
                                 unsigned long long *__restrict__ counters,
                                 unsigned long long *__restrict__ next_counters, uint32_t *__restrict__ pv,
                                 uint64_t *__restrict__ ppos, uint64_t *__restrict__ pend,
                                 uint32_t *__restrict__ plabel) {
    const uint32_t lane = lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        next_counters[1] = 0;
        next_counters[2] = 0;
    }
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    unsigned long long woke = 0;
    for (uint64_t q = wave; q < words; q += nwaves) {
        const uint64_t vis = visited[q];
        if (vis == ~0ull) {
            if (lane == 0) next[q] = 0;
            continue;
        }
        const uint64_t v = q * 64 + lane;
        const bool open = v < n && !((vis >> lane) & 1ull);
        uint64_t b0, b1;
        wave_offsets(acc.base, q * 64, n, b0, b1);
        if (!open) b1 = b0;
        bool found = false, pending = false;
        uint32_t par = 0, label = 0, count = 0;
        uint64_t pos = b0;
        uint32_t acc_v = 0, shift = 0;
        while (pos < b1 && count < threshold && !found) {
            // the 8 stream bytes from pos (two aligned words and a funnel
            // shift; the pad word keeps the second one in bounds)
            const uint64_t k = pos >> 3;
            const uint32_t sh = (uint32_t)(pos & 7) * 8;
            const uint64_t w0 = acc.word(k * 8), w1 = acc.word(k * 8 + 8);
            const uint64_t win = sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0;
            const uint32_t avail = b1 - pos < 8 ? (uint32_t)(b1 - pos) : 8u;
            for (uint32_t j = 0; j < avail && count < threshold && !found; ++j) {
                const uint32_t b = (uint32_t)(win >> (8 * j)) & 255u;
                acc_v |= (b & 127u) << shift;
                shift += 7;
                ++pos;
                if (!(b & 128u)) {
                    label = Acc::kDifferences && count ? label + acc_v : acc_v;
                    ++count;
                    acc_v = 0;
                    shift = 0;
                    const uint32_t u = label < n ? label : n - 1;
                    if ((curr[u >> 6] >> (u & 63)) & 1ull) { found = true; par = u; }
                }
            }
        }
        // a list cut at `threshold` values ends on a value boundary
        pending = open && !found && pos < b1;
        const uint64_t fm = __ballot(found);
        if (found) {
            depth[v] = next_depth;
            if (kParent) parent[v] = par;
        }
        if (lane == 0) next[q] = fm;
        if (lane == 0 && fm) {
            visited[q] |= fm;
            woke += (unsigned long long)__popcll(fm);
        }
        const uint64_t pm = __ballot(pending);
        if (pm) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&counters[2], (unsigned long long)__popcll(pm));
            base = __shfl(base, 0, kWave) + popc_below(pm);
            if (pending) {
                pv[base] = (uint32_t)v;
                ppos[base] = pos;
                pend[base] = b1;
                plabel[base] = label;  // the last label read (DMd continues from it)
            }
        }
    }
    woke = block_sum_u64(woke);
    if (threadIdx.x == 0 && woke) atomicAdd(&counters[1], woke);
}

template <class Acc, bool kParent>
__global__ void bu_varint_pending_kernel(Acc acc, uint32_t n, uint64_t np, const uint32_t *__restrict__ pv,
                                         const uint64_t *__restrict__ ppos, const uint64_t *__restrict__ pend,
                                         const uint32_t *__restrict__ plabel, const uint64_t *__restrict__ curr,
                                         unsigned long long *__restrict__ visited,
                                         unsigned long long *__restrict__ next, int32_t *__restrict__ depth,
                                         uint32_t *__restrict__ parent, int32_t next_depth,
                                         unsigned long long *__restrict__ counters) {
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    unsigned long long woke = 0;
    for (uint64_t p = wave; p < np; p += nwaves) {
        const uint32_t v = pv[p];
        const uint64_t b1 = pend[p];
        uint32_t prevb = 0, carry = plabel[p];
        for (uint64_t p0 = ppos[p]; p0 < b1; p0 += kWave) {
            uint32_t x;
            const bool end = varint_step(acc, p0, b1, prevb, x);
            uint32_t label = x;
            if constexpr (Acc::kDifferences) {
                const uint32_t sc = wave_incl_scan(end ? x : 0u);
                label = carry + sc;
                carry += __shfl(sc, kWave - 1, kWave);
            }
            const uint32_t u = label < n ? label : n - 1;
            const bool hit = end && ((curr[u >> 6] >> (u & 63)) & 1ull);
            const uint64_t m = __ballot(hit);
            if (m) {
                const uint32_t first = (uint32_t)__ffsll((long long)m) - 1;
                const uint32_t par = __shfl(u, first, kWave);
                if (lane == 0) {
                    depth[v] = next_depth;
                    if (kParent) parent[v] = par;
                    atomicOr(&next[v >> 6], 1ull << (v & 63));
                    atomicOr(&visited[v >> 6], 1ull << (v & 63));
                    ++woke;
                }
                break;
            }
        }
    }
    woke = block_sum_u64(woke);
    if (threadIdx.x == 0 && woke) atomicAdd(&counters[1], woke);
}

// results in original IDs: depth_out[o] = depth[inv[o]], parent through perm
// (unreached vertices, among them every edgeless one, need no parent lookup)
__global__ void bfs_unpermute_kernel(uint32_t n, const uint32_t *__restrict__ inv, const uint32_t *__restrict__ perm,
                                     const int32_t *__restrict__ depth_i, const uint32_t *__restrict__ parent_i,
                                     int32_t *__restrict__ depth, int32_t *__restrict__ parent) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += stride) {
        const uint32_t x = inv[o];
        const int32_t d = depth_i[x];
        depth[o] = d;
        if (parent) parent[o] = d < 0 ? -1 : (int32_t)perm[parent_i[x]];
    }
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------

// bottom-up -> top-down when the frontier shrinks below n / kBfsBeta
constexpr double kBfsBeta = 18.0;

template <class Acc>
static lg_status bfs_one(lg_graph *g, BfsWork &w, Acc acc, uint32_t root_id, const uint32_t *inv, int32_t *depth,
                         uint32_t *parent, int32_t max_depth, uint32_t flags, double alpha, hipStream_t s) {
    const uint32_t n = g->n;
    const uint64_t words = ((uint64_t)n + 63) / 64;
    uint32_t *qin = w.qa.as<uint32_t>(), *qout = w.qb.as<uint32_t>();
    uint64_t *visited = w.visited.as<uint64_t>(), *curr = w.curr.as<uint64_t>(), *next = w.next.as<uint64_t>();
    unsigned long long *ctr = w.counters.as<unsigned long long>();
    const uint32_t gsz = grid_for(n, 256, 1u << 16);

    LG_LAUNCH(bfs_init_kernel, gsz, 256, 0, s, n, depth, parent, g->iso.as<uint64_t>(), visited, root_id, inv, qin,
              (uint64_t *)ctr);
    LG_CHECK_LAUNCH();

    uint64_t qsize = 1;
    uint64_t edges_to_check = g->m;
    uint64_t awake = 0;
    int32_t level = 0;
    bool topdown = true;
    bool bu_done = false;  // a bottom-up phase is over: the frontier only shrinks from here
    uint32_t bu_pair = 0;  // counter pair of the next bottom-up level
    // queues above this size mark their bitmaps by a streaming pass over the
    // depths instead of one atomic per vertex
    const uint64_t stream_marks = std::max<uint64_t>(4096, n / 64);
    const uint32_t wgrid = grid_for(words * kWave, 256, kStrideBlocks);
    int32_t curr_level = -1;  // the level whose frontier curr holds (-1: none)
    // the frontier bitmap of the queue qin (what a bottom-up level reads)
    auto mark_frontier = [&]() -> lg_status {
        if (curr_level == level) return LG_OK;
        if (qsize > stream_marks) {
            LG_LAUNCH(level_bitmaps_kernel, wgrid, 256, 0, s, n, (const int32_t *)depth, level,
                      g->iso.as<uint64_t>(), curr, (uint64_t *)nullptr, ctr);
        } else {
            LG_TRY(fill_u64(curr, 0, words, s));
            LG_LAUNCH(mark_queue_kernel, grid_for(qsize, 256, 1u << 16), 256, 0, s, qin, qsize,
                      (unsigned long long *)curr, ctr);
        }
        LG_CHECK_LAUNCH();
        curr_level = level;
        return LG_OK;
    };
    // Between the switch points, is a bottom-up level cheaper than expanding
    // `td_cost` frontier edges?  Builds the frontier bitmap as a side effect.
    auto bottom_up_cheaper = [&](double td_cost, bool &cheaper) -> lg_status {
        LG_TRY(mark_frontier());
        LG_LAUNCH(bu_cost_sample_kernel<Acc>, kDirSampleBlocks, kDirSampleThreads, 0, s, acc, n, visited, curr,
                  w.sample.as<uint64_t>());
        LG_CHECK_LAUNCH();
        LG_CHECK_HIP(hipMemcpyAsync(w.host, w.sample.p, kDirSampleBlocks * 8, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
        uint64_t sampled = 0;
        for (uint32_t b = 0; b < kDirSampleBlocks; ++b) sampled += w.host[b];
        const double bu_cost = (double)sampled * ((double)n / (double)kDirSample);
        cheaper = td_cost > kBfsProbeCost * bu_cost;
        return LG_OK;
    };
    // with a late switch point beyond the early one, the band between them is sampled
    const bool banded = flags == LG_BFS_DIRECTION_OPT && alpha > kBfsAlphaLate;
    int32_t sampled_level = -1;  // the level whose sample chose top-down
    for (;;) {
        if (max_depth >= 0 && level >= max_depth) break;
        // ctr[0], the queue counter, is zero at every level's start: bfs_init
        // clears it, and every level that appends clears it again when it
        // marks its queue (the queue built after a bottom-up phase counts
        // into ctr[5] instead)
        if (topdown && qsize && bu_done && qsize <= kSmallFrontier) {
            const uint32_t grid = grid_for(qsize * kWave, 256, kStrideBlocks);
            if (parent)
                LG_LAUNCH((td_small_kernel<Acc, true>), grid, 256, 0, s, acc, qin, (uint32_t)qsize, visited, depth,
                          parent, level + 1, qout, ctr);
            else
                LG_LAUNCH((td_small_kernel<Acc, false>), grid, 256, 0, s, acc, qin, (uint32_t)qsize, visited, depth,
                          parent, level + 1, qout, ctr);
            LG_CHECK_LAUNCH();
            LG_CHECK_HIP(hipMemcpyAsync(w.host, ctr, 8, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
            qsize = w.host[0];
            if (qsize) {
                LG_LAUNCH(mark_queue_kernel, grid_for(qsize, 256, 1u << 16), 256, 0, s, qout, qsize,
                          (unsigned long long *)visited, ctr);
                LG_CHECK_LAUNCH();
            }
            std::swap(qin, qout);
            ++level;
            continue;
        }
        if (topdown) {
            if (qsize == 0) break;
            if (flags == LG_BFS_DIRECTION_OPT && qsize > 2 * (uint64_t)kDirSample) {
                // a large frontier: when a sample's degrees put its edges at
                // twice the switch point or more, turn bottom-up without
                // decoding the whole frontier (the direction changes the
                // time, never the result)
                LG_LAUNCH(td_sample_kernel<Acc>, kDirSampleBlocks, kDirSampleThreads, 0, s, acc, qin, qsize,
                          w.fscan.as<uint64_t>());
                LG_CHECK_LAUNCH();
                LG_CHECK_HIP(hipMemcpyAsync(w.host, w.fscan.p, kDirSampleBlocks * 8, hipMemcpyDeviceToHost, s));
                LG_CHECK_HIP(hipStreamSynchronize(s));
                uint64_t sampled = 0;
                for (uint32_t b = 0; b < kDirSampleBlocks; ++b) sampled += w.host[b];
                const double est = (double)sampled * ((double)qsize / (double)kDirSample);
                if (est > 2.0 * (double)edges_to_check / alpha) {
                    bool cheaper = true;
                    if (banded && est <= 2.0 * (double)edges_to_check / kBfsAlphaLate) {
                        LG_TRY(bottom_up_cheaper(est, cheaper));
                        sampled_level = level;
                    } else {
                        LG_TRY(mark_frontier());
                    }
                    if (cheaper) {
                        awake = qsize;
                        topdown = false;
                        continue;
                    }
                }
            }
            LG_LAUNCH(td_prepare_kernel<Acc>, grid_for(qsize, 256, 1u << 16), 256, 0, s, acc, qin, (uint32_t)qsize,
                      w.fstart.as<uint64_t>(), w.fdeg.as<uint32_t>(), w.fw.as<uint32_t>());
            LG_CHECK_LAUNCH();
            LG_TRY(exclusive_scan_u32(w.fdeg.as<uint32_t>(), w.fscan.as<uint64_t>(), qsize, w.scan_tmp, s));
            LG_CHECK_HIP(hipMemcpyAsync(w.host, w.fscan.as<uint64_t>() + qsize, 8, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
            const uint64_t fedges = w.host[0];
            bool go_bu = (flags == LG_BFS_BOTTOM_UP && level >= 1) ||
                         (flags == LG_BFS_DIRECTION_OPT && (double)fedges > (double)edges_to_check / alpha);
            bool marked = false;
            if (go_bu && banded && (double)fedges <= (double)edges_to_check / kBfsAlphaLate) {
                // in the band: measured unless this level's sample already
                // chose top-down
                if (sampled_level == level) {
                    go_bu = false;
                } else {
                    LG_TRY(bottom_up_cheaper((double)fedges, go_bu));
                    marked = true;
                }
            }
            if (go_bu) {
                if (!marked) LG_TRY(mark_frontier());
                awake = qsize;
                topdown = false;
                continue;
            }
            edges_to_check = edges_to_check > fedges ? edges_to_check - fedges : 0;
            // a level of more than n/16 edges claims without CAS or queue
            // appends; a pass over the vertices then finds the new ones
            const bool claim_min = fedges > (uint64_t)n / 16;
            if (fedges) {
                const uint32_t tiles = grid_for(fedges, kTdTile, 1u << 20);
                if (claim_min) {
                    if (parent)
                        LG_LAUNCH((td_expand_kernel<Acc, true, true>), tiles, kTdThreads, 0, s, acc, qin,
                                  (uint32_t)qsize, w.fstart.as<uint64_t>(), w.fw.as<uint32_t>(),
                                  w.fscan.as<uint64_t>(), fedges, visited, depth, parent, level + 1, qout, ctr);
                    else
                        LG_LAUNCH((td_expand_kernel<Acc, false, true>), tiles, kTdThreads, 0, s, acc, qin,
                                  (uint32_t)qsize, w.fstart.as<uint64_t>(), w.fw.as<uint32_t>(),
                                  w.fscan.as<uint64_t>(), fedges, visited, depth, parent, level + 1, qout, ctr);
                } else if (parent) {
                    LG_LAUNCH((td_expand_kernel<Acc, true>), tiles, kTdThreads, 0, s, acc, qin, (uint32_t)qsize,
                              w.fstart.as<uint64_t>(), w.fw.as<uint32_t>(), w.fscan.as<uint64_t>(), fedges, visited,
                              depth, parent, level + 1, qout, ctr);
                } else {
                    LG_LAUNCH((td_expand_kernel<Acc, false>), tiles, kTdThreads, 0, s, acc, qin, (uint32_t)qsize,
                              w.fstart.as<uint64_t>(), w.fw.as<uint32_t>(), w.fscan.as<uint64_t>(), fedges, visited,
                              depth, parent, level + 1, qout, ctr);
                }
                LG_CHECK_LAUNCH();
            }
            if (claim_min) {
                // the next frontier's bitmap and the visited one from the pass,
                // its queue from the bitmap (the queue counter is zero here)
                if (parent)
                    LG_LAUNCH(td_finish_kernel<true>, wgrid, 256, 0, s, n, visited, (const uint32_t *)parent, depth,
                              level + 1, curr);
                else
                    LG_LAUNCH(td_finish_kernel<false>, wgrid, 256, 0, s, n, visited, (const uint32_t *)parent, depth,
                              level + 1, curr);
                LG_CHECK_LAUNCH();
                LG_LAUNCH(bitmap_to_queue_kernel, grid_for(words, 256, 1u << 16), 256, 0, s, words, curr, qout, ctr);
                LG_CHECK_LAUNCH();
                LG_CHECK_HIP(hipMemcpyAsync(w.host, ctr, 8, hipMemcpyDeviceToHost, s));
                LG_CHECK_HIP(hipStreamSynchronize(s));
                qsize = w.host[0];
                LG_TRY(fill_u64((uint64_t *)ctr, 0, 1, s));  // the next level's queue counter
                curr_level = level + 1;
                std::swap(qin, qout);
                ++level;
                continue;
            }
            LG_CHECK_HIP(hipMemcpyAsync(w.host, ctr, 8, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
            qsize = w.host[0];
            if (qsize > stream_marks) {
                // the next frontier's bitmap comes with the visited one
                LG_LAUNCH(level_bitmaps_kernel, wgrid, 256, 0, s, n, (const int32_t *)depth, level + 1,
                          g->iso.as<uint64_t>(), curr, visited, ctr);
                LG_CHECK_LAUNCH();
                curr_level = level + 1;
            } else if (qsize) {
                LG_LAUNCH(mark_queue_kernel, grid_for(qsize, 256, 1u << 16), 256, 0, s, qout, qsize,
                          (unsigned long long *)visited, ctr);
                LG_CHECK_LAUNCH();
            }
            std::swap(qin, qout);
            ++level;
        } else {
            // bottom-up levels alternate between two counter pairs (woken,
            // pending) at ctr[1..2] and ctr[3..4]; each level's sweep clears
            // the pair of the next one (bfs_init clears both)
            unsigned long long *bc = ctr + 2 * bu_pair;
            unsigned long long *bc_next = ctr + 2 * (bu_pair ^ 1u);
            bu_pair ^= 1u;
            const uint32_t grid = grid_for(words * kWave, 256, kStrideBlocks);
            if (parent)
                LG_LAUNCH((bu_step_kernel<Acc, true>), grid, 256, 0, s, acc, n, g->heavy_threshold, curr, visited,
                          next, depth, parent, level + 1, bc, bc_next, w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(),
                          w.pdeg.as<uint32_t>(), w.pw.as<uint32_t>());
            else
                LG_LAUNCH((bu_step_kernel<Acc, false>), grid, 256, 0, s, acc, n, g->heavy_threshold, curr, visited,
                          next, depth, parent, level + 1, bc, bc_next, w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(),
                          w.pdeg.as<uint32_t>(), w.pw.as<uint32_t>());
            LG_CHECK_LAUNCH();
            LG_CHECK_HIP(hipMemcpyAsync(w.host, bc + 1, 16, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
            const uint64_t np = w.host[1];
            if (np) {
                LG_LAUNCH(bu_pending_count_kernel, grid_for(np, 256, 1u << 16), 256, 0, s, bc, g->heavy_threshold,
                          w.pdeg.as<uint32_t>(), w.pseg_cnt.as<uint32_t>());
                LG_CHECK_LAUNCH();
                LG_TRY(exclusive_scan_u32(w.pseg_cnt.as<uint32_t>(), w.pseg_off.as<uint64_t>(), np, w.scan_tmp, s));
                if (parent)
                    LG_LAUNCH((bu_pending_kernel<Acc, true>), kStrideBlocks, 256, 0, s, acc, g->heavy_threshold, np,
                              w.pseg_off.as<uint64_t>(), w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(),
                              w.pdeg.as<uint32_t>(), w.pw.as<uint32_t>(), curr, (unsigned long long *)visited,
                              (unsigned long long *)next, depth, parent, level + 1, bc);
                else
                    LG_LAUNCH((bu_pending_kernel<Acc, false>), kStrideBlocks, 256, 0, s, acc, g->heavy_threshold, np,
                              w.pseg_off.as<uint64_t>(), w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(),
                              w.pdeg.as<uint32_t>(), w.pw.as<uint32_t>(), curr, (unsigned long long *)visited,
                              (unsigned long long *)next, depth, parent, level + 1, bc);
                LG_CHECK_LAUNCH();
                LG_CHECK_HIP(hipMemcpyAsync(w.host, bc + 1, 8, hipMemcpyDeviceToHost, s));
                LG_CHECK_HIP(hipStreamSynchronize(s));
            }
            const uint64_t now = w.host[0];
            std::swap(curr, next);
            ++level;
            curr_level = level;  // the sweep wrote this level's frontier
            if (now == 0) break;
            const bool back = flags == LG_BFS_DIRECTION_OPT && now < awake && (double)now <= (double)n / kBfsBeta;
            awake = now;
            if (back) {
                bu_done = true;
                LG_TRY(fill_u64((uint64_t *)ctr + 5, 0, 1, s));
                LG_LAUNCH(bitmap_to_queue_kernel, grid_for(words, 256, 1u << 16), 256, 0, s, words, curr, qin,
                          ctr + 5);
                LG_CHECK_LAUNCH();
                qsize = now;
                topdown = true;
            }
        }
    }
    return LG_OK;
}

// The traversal over gap or Varint lists: the same level structure and
// direction rule as bfs_one, with the in-order kernels above (the frontier's
// edge count, from every frontier vertex's degree, or its list bytes for
// Varint lists, decides the direction).
template <class Acc>
static lg_status bfs_one_inorder(lg_graph *g, BfsWork &w, Acc acc, uint32_t root_id, const uint32_t *inv,
                                 int32_t *depth, uint32_t *parent, int32_t max_depth, uint32_t flags, double alpha,
                                 hipStream_t s) {
    constexpr bool kGap = IsGapAcc<Acc>::value;
    const uint32_t n = g->n;
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint32_t thr = g->heavy_threshold;
    uint32_t *qin = w.qa.as<uint32_t>(), *qout = w.qb.as<uint32_t>();
    uint64_t *visited = w.visited.as<uint64_t>(), *curr = w.curr.as<uint64_t>(), *next = w.next.as<uint64_t>();
    unsigned long long *ctr = w.counters.as<unsigned long long>();
    LG_LAUNCH(bfs_init_kernel, grid_for(n, 256, 1u << 16), 256, 0, s, n, depth, parent, g->iso.as<uint64_t>(),
              visited, root_id, inv, qin, (uint64_t *)ctr);
    LG_CHECK_LAUNCH();
    uint64_t qsize = 1, edges_to_check = kGap ? g->m : g->U / 8, awake = 0;
    int32_t level = 0;
    bool topdown = true;
    uint32_t bu_pair = 0;
    for (;;) {
        if (max_depth >= 0 && level >= max_depth) break;
        if (topdown) {
            if (qsize == 0) break;
            bool go_bu = flags == LG_BFS_BOTTOM_UP && level >= 1;
            if (flags == LG_BFS_DIRECTION_OPT && qsize > 2 * (uint64_t)kDirSample) {
                // a large frontier: a sample at twice the switch point or
                // more turns the search bottom-up without the exact count
                LG_LAUNCH(inorder_sample_kernel<Acc>, kDirSampleBlocks, kDirSampleThreads, 0, s, acc, qin, qsize,
                          w.fscan.as<uint64_t>());
                LG_CHECK_LAUNCH();
                LG_CHECK_HIP(hipMemcpyAsync(w.host, w.fscan.p, kDirSampleBlocks * 8, hipMemcpyDeviceToHost, s));
                LG_CHECK_HIP(hipStreamSynchronize(s));
                uint64_t sampled = 0;
                for (uint32_t b = 0; b < kDirSampleBlocks; ++b) sampled += w.host[b];
                const double est = (double)sampled * ((double)qsize / (double)kDirSample);
                go_bu = est > 2.0 * (double)edges_to_check / alpha;
            }
            if (flags == LG_BFS_DIRECTION_OPT && !go_bu) {
                LG_TRY(fill_u64(w.fscan.as<uint64_t>(), 0, 1, s));
                if constexpr (kGap)
                    LG_LAUNCH(gap_frontier_edges_kernel<Acc>, grid_for(qsize, 256, 1024), 256, 0, s, acc, qin, qsize,
                              w.fscan.as<unsigned long long>());
                else
                    LG_LAUNCH(varint_frontier_bytes_kernel<Acc>, grid_for(qsize, 256, 1024), 256, 0, s, acc, qin,
                              qsize, w.fscan.as<unsigned long long>());
                LG_CHECK_LAUNCH();
                LG_CHECK_HIP(hipMemcpyAsync(w.host, w.fscan.p, 8, hipMemcpyDeviceToHost, s));
                LG_CHECK_HIP(hipStreamSynchronize(s));
                const uint64_t fedges = w.host[0];
                go_bu = (double)fedges > (double)edges_to_check / alpha;
                if (!go_bu) edges_to_check = edges_to_check > fedges ? edges_to_check - fedges : 0;
            }
            if (go_bu) {
                LG_TRY(fill_u64(curr, 0, words, s));
                LG_LAUNCH(mark_queue_kernel, grid_for(qsize, 256, 1u << 16), 256, 0, s, qin, qsize,
                          (unsigned long long *)curr, ctr);
                LG_CHECK_LAUNCH();
                awake = qsize;
                topdown = false;
                continue;
            }
            const uint32_t grid = grid_for(qsize * kWave, 256, kStrideBlocks);
            if constexpr (kGap) {
                // lists above pr_split go by segments (tables built with the
                // encoding), the rest a wave per list
                const uint32_t split = g->n_seg ? g->pr_split : 0xFFFFFFFFu;
                if (g->n_seg) {
                    LG_TRY(fill_u64(curr, 0, words, s));
                    LG_LAUNCH(mark_queue_kernel, grid_for(qsize, 256, 1u << 16), 256, 0, s, qin, qsize,
                              (unsigned long long *)curr, ctr);
                    LG_CHECK_LAUNCH();
                    const uint32_t sgrid = grid_for(g->n_seg * kWave, 256, kStrideBlocks);
                    if (parent)
                        LG_LAUNCH((td_gap_seg_kernel<Acc, true>), sgrid, 256, 0, s, acc, n, g->n_seg, g->seg_size,
                                  g->seg_map.as<uint32_t>(), g->seg_off.as<uint64_t>(), g->heavy.as<uint32_t>(),
                                  g->hstart.as<uint64_t>(), g->hdeg.as<uint32_t>(), g->hw.as<uint32_t>(),
                                  g->hg.as<uint32_t>(), g->seg_base.as<uint32_t>(), curr, visited, depth, parent,
                                  level + 1, qout, ctr);
                    else
                        LG_LAUNCH((td_gap_seg_kernel<Acc, false>), sgrid, 256, 0, s, acc, n, g->n_seg, g->seg_size,
                                  g->seg_map.as<uint32_t>(), g->seg_off.as<uint64_t>(), g->heavy.as<uint32_t>(),
                                  g->hstart.as<uint64_t>(), g->hdeg.as<uint32_t>(), g->hw.as<uint32_t>(),
                                  g->hg.as<uint32_t>(), g->seg_base.as<uint32_t>(), curr, visited, depth, parent,
                                  level + 1, qout, ctr);
                    LG_CHECK_LAUNCH();
                }
                if (parent)
                    LG_LAUNCH((td_gap_kernel<Acc, true>), grid, 256, 0, s, acc, n, split, qin, qsize, visited, depth,
                              parent, level + 1, qout, ctr);
                else
                    LG_LAUNCH((td_gap_kernel<Acc, false>), grid, 256, 0, s, acc, n, split, qin, qsize, visited, depth,
                              parent, level + 1, qout, ctr);
            } else {
                // lists above vseg_split bytes go by chunks, the rest a wave
                // per list
                const uint64_t split = g->n_vseg ? g->vseg_split : ~0ull;
                if (g->n_vseg) {
                    LG_TRY(fill_u64(curr, 0, words, s));
                    LG_LAUNCH(mark_queue_kernel, grid_for(qsize, 256, 1u << 16), 256, 0, s, qin, qsize,
                              (unsigned long long *)curr, ctr);
                    LG_CHECK_LAUNCH();
                    const uint32_t sgrid = grid_for(g->n_vseg * kWave, 256, kStrideBlocks);
                    if (parent)
                        LG_LAUNCH((td_varint_seg_kernel<Acc, true>), sgrid, 256, 0, s, acc, n, g->n_vseg,
                                  g->vseg_bytes, g->vseg_map.as<uint32_t>(), g->vseg_off.as<uint64_t>(),
                                  g->heavy.as<uint32_t>(), g->vhb0.as<uint64_t>(), g->vhb1.as<uint64_t>(),
                                  g->vseg_base.as<uint32_t>(), curr, visited, depth, parent, level + 1, qout, ctr);
                    else
                        LG_LAUNCH((td_varint_seg_kernel<Acc, false>), sgrid, 256, 0, s, acc, n, g->n_vseg,
                                  g->vseg_bytes, g->vseg_map.as<uint32_t>(), g->vseg_off.as<uint64_t>(),
                                  g->heavy.as<uint32_t>(), g->vhb0.as<uint64_t>(), g->vhb1.as<uint64_t>(),
                                  g->vseg_base.as<uint32_t>(), curr, visited, depth, parent, level + 1, qout, ctr);
                    LG_CHECK_LAUNCH();
                }
                if (parent)
                    LG_LAUNCH((td_varint_kernel<Acc, true>), grid, 256, 0, s, acc, n, split, qin, qsize, visited,
                              depth, parent, level + 1, qout, ctr);
                else
                    LG_LAUNCH((td_varint_kernel<Acc, false>), grid, 256, 0, s, acc, n, split, qin, qsize, visited,
                              depth, parent, level + 1, qout, ctr);
            }
            LG_CHECK_LAUNCH();
            LG_CHECK_HIP(hipMemcpyAsync(w.host, ctr, 8, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
            qsize = w.host[0];
            if (qsize) {
                LG_LAUNCH(mark_queue_kernel, grid_for(qsize, 256, 1u << 16), 256, 0, s, qout, qsize,
                          (unsigned long long *)visited, ctr);
                LG_CHECK_LAUNCH();
            }
            std::swap(qin, qout);
            ++level;
        } else {
            unsigned long long *bc = ctr + 2 * bu_pair;
            unsigned long long *bc_next = ctr + 2 * (bu_pair ^ 1u);
            bu_pair ^= 1u;
            const uint32_t grid = grid_for(words * kWave, 256, kStrideBlocks);
            // pending lists: gap -- vertex, list start, degree, widths, label
            // of entry threshold - 1; Varint -- vertex, next byte, end byte,
            // last label
            if constexpr (kGap) {
                if (parent)
                    LG_LAUNCH((bu_gap_kernel<Acc, true>), grid, 256, 0, s, acc, n, thr, curr, visited, next, depth,
                              parent, level + 1, bc, bc_next, w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(),
                              w.pdeg.as<uint32_t>(), w.pw.as<uint32_t>(), w.pseg_cnt.as<uint32_t>());
                else
                    LG_LAUNCH((bu_gap_kernel<Acc, false>), grid, 256, 0, s, acc, n, thr, curr, visited, next, depth,
                              parent, level + 1, bc, bc_next, w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(),
                              w.pdeg.as<uint32_t>(), w.pw.as<uint32_t>(), w.pseg_cnt.as<uint32_t>());
            } else {
                if (parent)
                    LG_LAUNCH((bu_varint_kernel<Acc, true>), grid, 256, 0, s, acc, n, thr, curr, visited, next, depth,
                              parent, level + 1, bc, bc_next, w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(),
                              w.pseg_off.as<uint64_t>(), w.pseg_cnt.as<uint32_t>());
                else
                    LG_LAUNCH((bu_varint_kernel<Acc, false>), grid, 256, 0, s, acc, n, thr, curr, visited, next,
                              depth, parent, level + 1, bc, bc_next, w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(),
                              w.pseg_off.as<uint64_t>(), w.pseg_cnt.as<uint32_t>());
            }
            LG_CHECK_LAUNCH();
            LG_CHECK_HIP(hipMemcpyAsync(w.host, bc + 1, 16, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
            const uint64_t np = w.host[1];
            if (np) {
                const uint32_t pgrid = grid_for(np * kWave, 256, kStrideBlocks);
                if constexpr (kGap) {
                    if (parent)
                        LG_LAUNCH((bu_gap_pending_kernel<Acc, true>), pgrid, 256, 0, s, acc, n, thr, np,
                                  w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(), w.pdeg.as<uint32_t>(),
                                  w.pw.as<uint32_t>(), w.pseg_cnt.as<uint32_t>(), curr, (unsigned long long *)visited,
                                  (unsigned long long *)next, depth, parent, level + 1, bc);
                    else
                        LG_LAUNCH((bu_gap_pending_kernel<Acc, false>), pgrid, 256, 0, s, acc, n, thr, np,
                                  w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(), w.pdeg.as<uint32_t>(),
                                  w.pw.as<uint32_t>(), w.pseg_cnt.as<uint32_t>(), curr, (unsigned long long *)visited,
                                  (unsigned long long *)next, depth, parent, level + 1, bc);
                } else {
                    if (parent)
                        LG_LAUNCH((bu_varint_pending_kernel<Acc, true>), pgrid, 256, 0, s, acc, n, np,
                                  w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(), w.pseg_off.as<uint64_t>(),
                                  w.pseg_cnt.as<uint32_t>(), curr, (unsigned long long *)visited,
                                  (unsigned long long *)next, depth, parent, level + 1, bc);
                    else
                        LG_LAUNCH((bu_varint_pending_kernel<Acc, false>), pgrid, 256, 0, s, acc, n, np,
                                  w.pv.as<uint32_t>(), w.pstart.as<uint64_t>(), w.pseg_off.as<uint64_t>(),
                                  w.pseg_cnt.as<uint32_t>(), curr, (unsigned long long *)visited,
                                  (unsigned long long *)next, depth, parent, level + 1, bc);
                }
                LG_CHECK_LAUNCH();
                LG_CHECK_HIP(hipMemcpyAsync(w.host, bc + 1, 8, hipMemcpyDeviceToHost, s));
                LG_CHECK_HIP(hipStreamSynchronize(s));
            }
            const uint64_t now = w.host[0];
            std::swap(curr, next);
            ++level;
            if (now == 0) break;
            const bool back = flags == LG_BFS_DIRECTION_OPT && now < awake && (double)now <= (double)n / kBfsBeta;
            awake = now;
            if (back) {
                LG_TRY(fill_u64((uint64_t *)ctr + 5, 0, 1, s));
                LG_LAUNCH(bitmap_to_queue_kernel, grid_for(words, 256, 1u << 16), 256, 0, s, words, curr, qin,
                          ctr + 5);
                LG_CHECK_LAUNCH();
                qsize = now;
                topdown = true;
            }
        }
    }
    return LG_OK;
}

// Chunk tables of the long Varint lists (see lg_graph), built once with the
// encoding: per heavy vertex its byte range and chunk count, a scan, the
// chunk map, and for differences the label before every chunk (a wave sum
// per chunk, a scan, a per-list subtraction).
lg_status build_varint_segments(lg_graph *g, hipStream_t s) {
    const uint32_t nh = g->n_heavy;
    g->n_vseg = 0;
    LG_TRY(g->vhb0.scratch((uint64_t)(nh ? nh : 1) * 8, s));
    LG_TRY(g->vhb1.scratch((uint64_t)(nh ? nh : 1) * 8, s));
    LG_TRY(g->vseg_off.scratch(((uint64_t)nh + 1) * 8, s));
    DevBuf tmp;
    if (!nh) return fill_u64(g->vseg_off.as<uint64_t>(), 0, 1, s);
    return dispatch_acc_dec(g, [&](auto acc) -> lg_status {
        using Acc = decltype(acc);
        if constexpr (IsVarintAcc<Acc>::value) {
            DevBuf segcnt;
            LG_TRY(segcnt.scratch((uint64_t)nh * 4, s));
            LG_LAUNCH(varint_seg_info_kernel<Acc>, grid_for(nh, 256, 1u << 16), 256, 0, s, acc,
                      g->heavy.as<uint32_t>(), nh, (uint64_t)g->vseg_split, g->vseg_bytes, g->vhb0.as<uint64_t>(),
                      g->vhb1.as<uint64_t>(), segcnt.as<uint32_t>());
            LG_CHECK_LAUNCH();
            LG_TRY(exclusive_scan_u32(segcnt.as<uint32_t>(), g->vseg_off.as<uint64_t>(), nh, tmp, s));
            LG_CHECK_HIP(hipMemcpyAsync(&g->n_vseg, g->vseg_off.as<uint64_t>() + nh, 8, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
            LG_TRY(g->vseg_map.scratch((g->n_vseg ? g->n_vseg : 1) * 4, s));
            LG_TRY(g->vseg_base.scratch((g->n_vseg ? g->n_vseg : 1) * 4, s));
            if (!g->n_vseg) return LG_OK;
            LG_LAUNCH(varint_seg_map_kernel, grid_for(nh, 256, 1u << 16), 256, 0, s, nh,
                      g->vseg_off.as<uint64_t>(), g->vseg_map.as<uint32_t>());
            LG_CHECK_LAUNCH();
            if constexpr (Acc::kDifferences) {
                DevBuf ssum, sscan;
                LG_TRY(ssum.scratch(g->n_vseg * 4, s));
                LG_TRY(sscan.scratch((g->n_vseg + 1) * 8, s));
                LG_LAUNCH(varint_seg_sum_kernel<Acc>, grid_for(g->n_vseg * kWave, 256, 1u << 16), 256, 0, s, acc,
                          g->n_vseg, g->vseg_bytes, g->vseg_map.as<uint32_t>(), g->vseg_off.as<uint64_t>(),
                          g->vhb0.as<uint64_t>(), g->vhb1.as<uint64_t>(), ssum.as<uint32_t>());
                LG_CHECK_LAUNCH();
                LG_TRY(exclusive_scan_u32(ssum.as<uint32_t>(), sscan.as<uint64_t>(), g->n_vseg, tmp, s));
                LG_LAUNCH(varint_seg_base_kernel, grid_for(g->n_vseg, 256, 1u << 16), 256, 0, s, g->n_vseg,
                          g->vseg_map.as<uint32_t>(), g->vseg_off.as<uint64_t>(), sscan.as<uint64_t>(),
                          g->vseg_base.as<uint32_t>());
                LG_CHECK_LAUNCH();
            } else {
                LG_TRY(fill_u32(g->vseg_base.as<uint32_t>(), 0, g->n_vseg, s));
            }
            LG_CHECK_HIP(hipStreamSynchronize(s));
            return LG_OK;
        }
        return LG_ERR_UNSUPPORTED;
    });
}

lg_status bfs_run(lg_graph *g, BfsWork &w, const uint32_t *roots, uint32_t r, int32_t *depth, int32_t *parent,
                  int32_t max_depth, uint32_t flags, hipStream_t stream, double alpha) {
    if (r == 0) return LG_OK;
    LG_TRY(bfs_workspace_ensure(w, g->n, g->n_heavy, g->relabel != LG_RELABEL_NONE, parent != nullptr));
    const bool rel = g->relabel != LG_RELABEL_NONE;
    const uint32_t *inv = rel ? g->inv.as<uint32_t>() : nullptr;
    return dispatch_acc_dec(g, [&](auto acc) -> lg_status {
        // one traversal: the in-order kernels for gap and Varint lists, else
        // the general ones
        auto one = [&](uint32_t root, int32_t *d, uint32_t *p) -> lg_status {
            using A = decltype(acc);
            if constexpr (IsGapAcc<A>::value || IsVarintAcc<A>::value)
                return bfs_one_inorder(g, w, acc, root, inv, d, p, max_depth, flags, alpha, stream);
            else
                return bfs_one(g, w, acc, root, inv, d, p, max_depth, flags, alpha, stream);
        };
        for (uint32_t i = 0; i < r; ++i) {
            int32_t *d_out = depth + (uint64_t)i * g->n;
            int32_t *p_out = parent ? parent + (uint64_t)i * g->n : nullptr;
            if (rel) {
                LG_TRY(one(roots[i], w.depth_i.as<int32_t>(), p_out ? w.parent_i.as<uint32_t>() : nullptr));
                LG_LAUNCH(bfs_unpermute_kernel, grid_for(g->n, 256, 1u << 16), 256, 0, stream, g->n,
                          g->inv.as<uint32_t>(), g->perm.as<uint32_t>(), w.depth_i.as<int32_t>(),
                          p_out ? w.parent_i.as<uint32_t>() : nullptr, d_out, p_out);
                LG_CHECK_LAUNCH();
            } else {
                LG_TRY(one(roots[i], d_out, reinterpret_cast<uint32_t *>(p_out)));
            }
        }
        return LG_OK;
    });
}

// ---------------------------------------------------------------------------
// Multi-source BFS: the roots of one call (up to 64 at a time) in one
// traversal.  Every vertex holds 64-bit masks, bit i for root i: vis (the
// searches that reached it), fr (those with it in this level's frontier),
// nx (the next level's).  A level either marks candidates top-down (every
// frontier edge (u, v) ORs fr[u] & ~vis[v] into nx[v] and offers u as the
// parent of each bit so set, the smallest offer winning), or finds the next
// frontier bottom-up over every vertex with open bits, reading its list in
// order and taking for each bit the first neighbor whose frontier mask
// holds it.  Either way the parent is the neighbor one level up with the
// smallest label, so every row equals the search from its root alone.  A
// bottom-up level reads each open vertex's list once for all roots.
// ---------------------------------------------------------------------------

constexpr uint32_t kMsRoots = 64;
constexpr uint32_t kMsLaneLimit = 256;  // entries a lane reads before a wave finishes its list
constexpr int kMsThreads = 256;

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long x) {
    const uint32_t lo = wave_or((uint32_t)x), hi = wave_or((uint32_t)(x >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// the roots (original IDs, mapped to labels through inv when relabeled):
// reached at depth 0, their own parents, in the first frontier
__global__ void ms_roots_kernel(uint32_t r, const uint32_t *__restrict__ roots, const uint32_t *__restrict__ inv,
                                uint64_t n, unsigned long long *__restrict__ vis, unsigned long long *__restrict__ fr,
                                int32_t *__restrict__ depth, int32_t *__restrict__ parent) {
    const uint32_t i = threadIdx.x;
    if (i >= r) return;
    const uint32_t x = inv ? inv[roots[i]] : roots[i];
    atomicOr(&vis[x], 1ull << i);
    atomicOr(&fr[x], 1ull << i);
    depth[(uint64_t)i * n + x] = 0;
    if (parent) parent[(uint64_t)i * n + x] = (int32_t)x;
}

// bitmap of the vertices with a non-empty mask
__global__ void ms_bits_kernel(uint32_t n, const unsigned long long *__restrict__ fr, uint64_t *__restrict__ bits) {
    const uint32_t lane = lane_id();
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wstride = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t q = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; q < words; q += wstride) {
        const uint64_t v = q * 64 + lane;
        const uint64_t m = __ballot(v < n && fr[v < n ? v : n - 1] != 0ull);
        if (lane == 0) bits[q] = m;
    }
}

// Top-down marking over the frontier's edges, tiled as td_expand_kernel
// tiles them: nx[v] |= fr[u] & ~vis[v] for every frontier edge (u, v), and
// for each bit b so set parent[b][v] = min(parent[b][v], u).  The rows hold
// -1 (the largest value unsigned) where no parent is set yet, so the row
// ends with the smallest frontier neighbour: the first in v's sorted list,
// the parent a search from root b alone takes.
template <class Acc, bool kParent>
__global__ __launch_bounds__(kTdThreads) void ms_mark_kernel(
    Acc acc, const uint32_t *__restrict__ queue, uint32_t qsize, const uint64_t *__restrict__ fstart,
    const uint32_t *__restrict__ fw, const uint64_t *__restrict__ fscan, uint64_t edges,
    const unsigned long long *__restrict__ fr, const unsigned long long *__restrict__ vis,
    unsigned long long *__restrict__ nx, uint64_t n, uint32_t *__restrict__ parent) {
    __shared__ uint64_t s_scan[kTdTile + 1];
    __shared__ uint64_t s_start[kTdTile];
    __shared__ uint32_t s_w[kTdTile];
    __shared__ unsigned long long s_fr[kTdTile];
    __shared__ uint32_t s_q[kParent ? kTdTile : 1];
    __shared__ uint32_t s_range[2];
    for (uint64_t t = blockIdx.x; t * kTdTile < edges; t += gridDim.x) {
        const uint64_t e0 = t * kTdTile;
        const uint64_t e1 = e0 + kTdTile < edges ? e0 + kTdTile : edges;
        if (threadIdx.x == 0) s_range[0] = last_le(fscan, 0, qsize - 1, e0);
        if (threadIdx.x == 1) s_range[1] = last_le(fscan, 0, qsize - 1, e1 - 1);
        __syncthreads();
        const uint32_t i0 = s_range[0];
        const uint32_t span = s_range[1] - i0 + 1;
        const bool staged = span <= kTdTile;
        if (staged) {
            for (uint32_t j = threadIdx.x; j < span; j += kTdThreads) {
                s_scan[j] = fscan[i0 + j];
                s_start[j] = fstart[i0 + j];
                s_w[j] = fw[i0 + j];
                const uint32_t q = queue[i0 + j];
                s_fr[j] = fr[q];
                if constexpr (kParent) s_q[j] = q;
            }
        }
        __syncthreads();
        // in phases, so that the list loads and then the mask loads of a
        // thread's edges are in flight together (idle slots: position 0 with
        // mask 0, an empty frontier mask)
        uint64_t epos[kTdEdgesPerThread];
        uint32_t msk[kTdEdgesPerThread], src[kTdEdgesPerThread];
        unsigned long long fm[kTdEdgesPerThread];
#pragma unroll
        for (int r = 0; r < kTdEdgesPerThread; ++r) {
            const uint64_t e = e0 + (uint64_t)r * kTdThreads + threadIdx.x;
            epos[r] = 0;
            msk[r] = 0;
            fm[r] = 0ull;
            src[r] = 0;
            if (e < e1) {
                uint64_t base_e, start;
                uint32_t w, q = 0;
                unsigned long long f;
                if (staged) {
                    const uint32_t j = last_le(s_scan, 0, span - 1, e);
                    base_e = s_scan[j]; start = s_start[j]; w = s_w[j]; f = s_fr[j];
                    if constexpr (kParent) q = s_q[j];
                } else {
                    const uint32_t j = last_le(fscan, i0, s_range[1], e);
                    q = queue[j];
                    base_e = fscan[j]; start = fstart[j]; w = fw[j]; f = fr[q];
                }
                epos[r] = start + (e - base_e) * Acc::step(w);
                msk[r] = Acc::mask(w);
                fm[r] = f;
                src[r] = q;
            }
        }
        uint32_t u[kTdEdgesPerThread];
        unsigned long long vw[kTdEdgesPerThread];
#pragma unroll
        for (int r = 0; r < kTdEdgesPerThread; ++r) u[r] = acc.get(epos[r], msk[r]);
#pragma unroll
        for (int r = 0; r < kTdEdgesPerThread; ++r) vw[r] = vis[u[r]];
#pragma unroll
        for (int r = 0; r < kTdEdgesPerThread; ++r) {
            const unsigned long long add = fm[r] & ~vw[r];
            if (add) {
                atomicOr(&nx[u[r]], add);
                if constexpr (kParent) {
                    for (unsigned long long h = add; h; h &= h - 1)
                        atomicMin(&parent[(uint64_t)(__ffsll((long long)h) - 1) * n + u[r]], src[r]);
                }
            }
        }
        __syncthreads();  // the next tile rewrites the staged ranges
    }
}

// One level's depths (and, bottom-up, parents), a lane per vertex over
// 64-vertex words.  Top-down, the candidates nx[v] are the level's new bits
// (their parents came with the marking).  Bottom-up, the open bits P are
// every unreached bit of a search still running: the lane reads its list in
// order, four entries per step, until every open bit is found or
// kMsLaneLimit entries; a longer list goes to ms_pending_kernel with the
// bits still open.  A lane keeps, per root, the
// list position of the parent (one byte: positions stay under kMsLaneLimit)
// in LDS until its vertex is done; rows are then written four roots at a
// time, so that the lanes of a wave write one row's consecutive entries
// together and the parents' list reads are in flight together.  The byte
// stage and the register bound let eight waves share a SIMD, which skewed
// graphs need to hide lanes waiting on long lists (the host caps the grid
// on even-degree graphs, where more waves only evict the lanes' list lines).
constexpr uint32_t kMsParStride = kMsRoots + 4;  // bytes per lane: 17 words, so lanes fall on distinct banks
static_assert(kMsLaneLimit <= 256, "a parent's list position is kept in one byte");

// (the Elias-Fano offset lookup of wave_info needs more registers: five waves)
template <class A> struct MsWavesPerEU { static constexpr int value = 8; };
template <int I, int O> struct MsWavesPerEU<PackedAcc<I, O>> { static constexpr int value = O == kOffsEF ? 5 : 8; };

template <class Acc, bool kParent, bool kTD>
__global__ __launch_bounds__(kMsThreads, MsWavesPerEU<Acc>::value) void ms_resolve_kernel(
    Acc acc, uint32_t n, int32_t next_depth, unsigned long long active, const unsigned long long *__restrict__ fr,
    unsigned long long *__restrict__ vis, unsigned long long *__restrict__ nx, int32_t *__restrict__ depth,
    int32_t *__restrict__ parent, uint64_t *__restrict__ bits, uint32_t *__restrict__ pend_v,
    unsigned long long *__restrict__ pend_m, unsigned long long *__restrict__ ctr) {
    __shared__ uint8_t s_par[kParent ? kMsThreads * kMsParStride : 4];
    __shared__ unsigned long long s_act[kMsThreads / kWave];
    uint8_t *par = &s_par[kParent ? threadIdx.x * kMsParStride : 0];
    const uint32_t lane = lane_id();
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wstride = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    unsigned long long act = 0ull;  // searches with a vertex in the next frontier
    for (uint64_t q = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; q < words; q += wstride) {
        const uint64_t v = q * 64 + lane;
        const bool valid = v < n;
        const uint64_t vc = valid ? v : n - 1;
        unsigned long long P;
        if constexpr (kTD) P = valid ? nx[vc] : 0ull;
        else P = valid ? (~vis[vc] & active) : 0ull;
        if (__ballot(P != 0ull) == 0) {  // wave-uniform: nothing open in this word
            if constexpr (!kTD) {
                if (valid) nx[v] = 0ull;
            }
            if (lane == 0) bits[q] = 0ull;
            continue;
        }
        unsigned long long found = kTD ? P : 0ull;
        bool pending = false;
        const VInfo vi = kTD ? VInfo{0, 0, 0} : wave_info(acc, q * 64, n);
        const uint32_t st = Acc::step(vi.w), mk = Acc::mask(vi.w);
        if (!kTD && P && vi.deg) {
            const uint32_t lim = vi.deg < kMsLaneLimit ? vi.deg : kMsLaneLimit;
            for (uint32_t i = 0; i < lim && found != P; i += 4) {
                // four list loads, then four mask loads (entries past the
                // limit re-read the first one, which exists)
                uint32_t u[4];
                unsigned long long m[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) u[b] = acc.get(vi.start + (uint64_t)(i + b < lim ? i + b : 0u) * st, mk);
#pragma unroll
                for (int b = 0; b < 4; ++b) m[b] = fr[u[b]];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    unsigned long long h = (i + b < lim) ? (m[b] & P & ~found) : 0ull;
                    found |= h;
                    if constexpr (kParent) {
                        while (h) {
                            par[__ffsll((long long)h) - 1] = (uint8_t)(i + b);
                            h &= h - 1;
                        }
                    }
                }
            }
            pending = found != P && vi.deg > lim;
        }
        // the rows of the roots found here, four roots at a time (a found
        // bit implies a non-empty list, so its position names an entry; the
        // other lanes read the array's first entry, which exists whenever
        // any bit is found, and drop it)
        for (unsigned long long bb = wave_or64(found); bb;) {
            uint32_t rr[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                rr[k] = bb ? (uint32_t)__ffsll((long long)bb) - 1 : kMsRoots;
                bb &= bb - 1;
            }
            bool has[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) has[k] = rr[k] < kMsRoots && ((found >> rr[k]) & 1ull);
            uint32_t pu[4];
            if constexpr (kParent && !kTD) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint64_t pos = has[k] ? vi.start + (uint64_t)par[rr[k]] * st : 0ull;
                    pu[k] = acc.get(pos, mk);
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (has[k]) {
                    depth[(uint64_t)rr[k] * n + v] = next_depth;
                    if constexpr (kParent && !kTD) parent[(uint64_t)rr[k] * n + v] = (int32_t)pu[k];
                }
            }
        }
        if (valid) {
            if constexpr (kTD) {
                vis[v] |= P;  // every candidate is reached at this level
            } else {
                vis[v] |= found;
                nx[v] = found;
            }
        }
        act |= kTD ? P : found;
        const uint64_t pm = __ballot(pending);
        if (pm) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&ctr[3], (unsigned long long)__popcll(pm));
            base = __shfl(base, 0, kWave) + popc_below(pm);
            if (pending) {
                pend_v[base] = (uint32_t)v;
                pend_m[base] = P & ~found;
            }
        }
        // the next frontier's words: a pending bottom-up vertex may still
        // find bits (counting it costs nothing if it does not)
        const uint64_t fw_bits = __ballot(valid && (kTD ? P != 0ull : (found != 0ull || pending)));
        if (lane == 0) bits[q] = fw_bits;
    }
    act = wave_or64(act);
    if (lane == 0) s_act[threadIdx.x / kWave] = act;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0ull;
        for (int i = 0; i < kMsThreads / kWave; ++i) a |= s_act[i];
        if (a) atomicOr(&ctr[2], a);
    }
}

// The long lists left by ms_resolve_kernel: a wave per vertex reads the rest
// of the list 64 entries per step; for each open bit the first lane holding
// it gives the parent.
template <class Acc, bool kParent>
__global__ void ms_pending_kernel(Acc acc, uint32_t n, int32_t next_depth, const unsigned long long *__restrict__ fr,
                                  unsigned long long *__restrict__ vis, unsigned long long *__restrict__ nx,
                                  int32_t *__restrict__ depth, int32_t *__restrict__ parent,
                                  const uint32_t *__restrict__ pend_v, const unsigned long long *__restrict__ pend_m,
                                  unsigned long long *__restrict__ ctr) {
    const uint32_t lane = lane_id();
    const uint64_t np = ctr[3];
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    unsigned long long act = 0ull;
    for (uint64_t k = wave; k < np; k += nwaves) {
        const uint32_t v = pend_v[k];
        unsigned long long P = pend_m[k];
        const VInfo vi = acc.info(v);
        const uint32_t st = Acc::step(vi.w), mk = Acc::mask(vi.w);
        unsigned long long got = 0ull;
        for (uint64_t e0 = kMsLaneLimit; e0 < vi.deg && P; e0 += kWave) {
            const uint64_t idx = e0 + lane;
            const bool in = idx < vi.deg;
            const uint32_t u = acc.get(vi.start + (in ? idx : 0ull) * st, mk);
            const unsigned long long m = in ? (fr[u] & P) : 0ull;
            const unsigned long long uni = wave_or64(m);
            for (unsigned long long bb = uni; bb; bb &= bb - 1) {
                const uint32_t r = (uint32_t)__ffsll((long long)bb) - 1;
                const uint64_t holders = __ballot((m >> r) & 1ull);
                const uint32_t first = (uint32_t)__ffsll((long long)holders) - 1;
                const uint32_t pu = __shfl(u, first, kWave);
                if (lane == 0) {
                    depth[(uint64_t)r * n + v] = next_depth;
                    if constexpr (kParent) parent[(uint64_t)r * n + v] = (int32_t)pu;
                }
            }
            P &= ~uni;
            got |= uni;
        }
        if (lane == 0 && got) {
            atomicOr(&nx[v], got);
            atomicOr(&vis[v], got);
        }
        act |= got;
    }
    if (lane == 0 && act) atomicOr(&ctr[2], act);
}

// After the last level: -1 in the rows of the searches that never reached v.
__global__ void ms_finish_kernel(uint32_t n, uint32_t r, const unsigned long long *__restrict__ vis,
                                 int32_t *__restrict__ depth, int32_t *__restrict__ parent) {
    const uint32_t lane = lane_id();
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wstride = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    const unsigned long long all = r >= 64 ? ~0ull : ((1ull << r) - 1ull);
    for (uint64_t q = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; q < words; q += wstride) {
        const uint64_t v = q * 64 + lane;
        const unsigned long long open = v < n ? (~vis[v] & all) : 0ull;
        for (unsigned long long bb = wave_or64(open); bb; bb &= bb - 1) {
            const uint32_t i = (uint32_t)__ffsll((long long)bb) - 1;
            if ((open >> i) & 1ull) {
                depth[(uint64_t)i * n + v] = -1;
                if (parent) parent[(uint64_t)i * n + v] = -1;
            }
        }
    }
}

// One batch of at most 64 roots.  The rows are computed in label space.  On
// a relabeled graph they are then unpermuted into original IDs
// (bfs_unpermute_kernel, as for a single root): from the workspace rows
// `ws` (depth rows, then parent rows) when the caller has them, else each
// row is first copied to a one-row workspace.  The host reads two counters
// per level: the next frontier's size and the searches still running.
template <class Acc>
static lg_status bfs_ms_batch(lg_graph *g, BfsWork &w, MsWork &ms, Acc acc, const uint32_t *roots, uint32_t r,
                              int32_t *depth_out, int32_t *parent_out, int32_t max_depth, int32_t *ws,
                              hipStream_t s) {
    const uint32_t n = g->n;
    const bool rel = g->relabel != LG_RELABEL_NONE;
    int32_t *depth = rel && ws ? ws : depth_out;
    int32_t *parent = parent_out ? (rel && ws ? ws + (uint64_t)r * n : parent_out) : nullptr;
    const uint64_t words = ((uint64_t)n + 63) / 64;
    unsigned long long *vis = ms.vis.as<unsigned long long>();
    unsigned long long *fr = ms.fr.as<unsigned long long>();
    unsigned long long *nx = ms.nx.as<unsigned long long>();
    uint64_t *bits = ms.bits.as<uint64_t>();
    unsigned long long *ctr = w.counters.as<unsigned long long>();
    uint32_t *queue = w.qa.as<uint32_t>();
    const uint32_t wgrid = grid_for(words * kWave, 256, kStrideBlocks);
    LG_TRY(fill_u64((uint64_t *)vis, 0, n, s));
    LG_TRY(fill_u64((uint64_t *)fr, 0, n, s));
    LG_TRY(fill_u64((uint64_t *)ctr, 0, 8, s));
    // top-down levels take parents by atomic minimum over rows that start at -1
    if (parent) LG_TRY(fill_u32(reinterpret_cast<uint32_t *>(parent), 0xFFFFFFFFu, (uint64_t)r * n, s));
    LG_CHECK_HIP(hipMemcpyAsync(ms.roots.p, roots, (uint64_t)r * 4, hipMemcpyHostToDevice, s));
    LG_LAUNCH(ms_roots_kernel, 1, kMsRoots, 0, s, r, ms.roots.as<uint32_t>(), rel ? g->inv.as<uint32_t>() : nullptr,
              (uint64_t)n, vis, fr, depth, parent);
    LG_CHECK_LAUNCH();
    LG_LAUNCH(ms_bits_kernel, wgrid, 256, 0, s, n, (const unsigned long long *)fr, bits);
    LG_CHECK_LAUNCH();
    LG_LAUNCH(bitmap_to_queue_kernel, grid_for(words, 256, 1u << 16), 256, 0, s, words, bits, queue, ctr);
    LG_CHECK_LAUNCH();
    LG_CHECK_HIP(hipMemcpyAsync(w.host, ctr, 8, hipMemcpyDeviceToHost, s));
    LG_CHECK_HIP(hipStreamSynchronize(s));
    uint64_t fsize = w.host[0];
    unsigned long long active = r >= 64 ? ~0ull : ((1ull << r) - 1ull);
    // the resolve grid: on graphs with even degrees two workgroups per CU
    // (more waves only evict the lanes' list lines under the random mask
    // reads: measured slower); on skewed ones, where lanes of a wave wait
    // on each other's long lists, the full grid hides the latency
    int cus = 0;
    LG_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
    const bool skewed = (uint64_t)g->n_heavy * 256 > n;
    const uint32_t rgrid = grid_for(words * kWave, kMsThreads, skewed ? kStrideBlocks : (uint32_t)std::max(1, 2 * cus));
    for (int32_t level = 0; fsize && active && (max_depth < 0 || level < max_depth); ++level) {
        // top-down while the frontier's edges are under a third of the
        // graph's: a top-down edge costs a mask read and one or two atomics,
        // a bottom-up level reads every open vertex's list until its open
        // bits are found, in the early levels the whole list (measured at
        // Erdos-Renyi scale 26, 64 roots: the level with 3% of the edges on
        // the frontier took 45 ms bottom-up, 10 ms top-down)
        bool td = fsize <= (uint64_t)n / 4;
        uint64_t fedges = 0;
        if (td) {
            LG_LAUNCH(td_prepare_kernel<Acc>, grid_for(fsize, 256, 1u << 16), 256, 0, s, acc, queue, (uint32_t)fsize,
                      w.fstart.as<uint64_t>(), w.fdeg.as<uint32_t>(), w.fw.as<uint32_t>());
            LG_CHECK_LAUNCH();
            LG_TRY(exclusive_scan_u32(w.fdeg.as<uint32_t>(), w.fscan.as<uint64_t>(), fsize, w.scan_tmp, s));
            LG_CHECK_HIP(hipMemcpyAsync(w.host, w.fscan.as<uint64_t>() + fsize, 8, hipMemcpyDeviceToHost, s));
            LG_CHECK_HIP(hipStreamSynchronize(s));
            fedges = w.host[0];
            td = fedges * 3 < g->m;
        }
        LG_TRY(fill_u64((uint64_t *)ctr, 0, 8, s));  // [0] queue, [2] running searches, [3] pending
        if (td) {
            LG_TRY(fill_u64((uint64_t *)nx, 0, n, s));
            if (fedges) {
                auto mark = [&](auto kpar) -> lg_status {
                    LG_LAUNCH((ms_mark_kernel<Acc, decltype(kpar)::value>), grid_for(fedges, kTdTile, 1u << 20),
                              kTdThreads, 0, s, acc, queue, (uint32_t)fsize, w.fstart.as<uint64_t>(),
                              w.fw.as<uint32_t>(), w.fscan.as<uint64_t>(), fedges, (const unsigned long long *)fr,
                              (const unsigned long long *)vis, nx, (uint64_t)n, reinterpret_cast<uint32_t *>(parent));
                    LG_CHECK_LAUNCH();
                    return LG_OK;
                };
                if (parent) LG_TRY(mark(std::true_type{}));
                else LG_TRY(mark(std::false_type{}));
            }
        }
        auto resolve = [&](auto kpar, auto ktd) -> lg_status {
            constexpr bool P = decltype(kpar)::value, T = decltype(ktd)::value;
            LG_LAUNCH((ms_resolve_kernel<Acc, P, T>), rgrid, kMsThreads, 0, s, acc, n, level + 1, active,
                      (const unsigned long long *)fr, vis, nx, depth, parent, bits, ms.pend_v.as<uint32_t>(),
                      ms.pend_m.as<unsigned long long>(), ctr);
            LG_CHECK_LAUNCH();
            if constexpr (!T) {  // only bottom-up levels leave long lists
                LG_LAUNCH((ms_pending_kernel<Acc, P>), kStrideBlocks, 256, 0, s, acc, n, level + 1,
                          (const unsigned long long *)fr, vis, nx, depth, parent, (const uint32_t *)ms.pend_v.p,
                          (const unsigned long long *)ms.pend_m.p, ctr);
                LG_CHECK_LAUNCH();
            }
            return LG_OK;
        };
        if (parent) {
            if (td) LG_TRY(resolve(std::true_type{}, std::true_type{}));
            else LG_TRY(resolve(std::true_type{}, std::false_type{}));
        } else {
            if (td) LG_TRY(resolve(std::false_type{}, std::true_type{}));
            else LG_TRY(resolve(std::false_type{}, std::false_type{}));
        }
        LG_LAUNCH(bitmap_to_queue_kernel, grid_for(words, 256, 1u << 16), 256, 0, s, words, bits, queue, ctr);
        LG_CHECK_LAUNCH();
        LG_CHECK_HIP(hipMemcpyAsync(w.host, ctr, 24, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));
        fsize = w.host[0];
        active = w.host[2];
        std::swap(fr, nx);
    }
    LG_LAUNCH(ms_finish_kernel, wgrid, 256, 0, s, n, r, (const unsigned long long *)vis, depth, parent);
    LG_CHECK_LAUNCH();
    if (rel) {
        for (uint32_t i = 0; i < r; ++i) {
            int32_t *d_row = depth_out + (uint64_t)i * n;
            int32_t *p_row = parent_out ? parent_out + (uint64_t)i * n : nullptr;
            const int32_t *d_in = depth + (uint64_t)i * n;
            const uint32_t *p_in = parent ? reinterpret_cast<const uint32_t *>(parent + (uint64_t)i * n) : nullptr;
            if (!ws) {  // the row is its own output: copy it aside first
                int32_t *tmp_d = w.depth_i.as<int32_t>();
                uint32_t *tmp_p = parent ? w.parent_i.as<uint32_t>() : nullptr;
                LG_CHECK_HIP(hipMemcpyAsync(tmp_d, d_row, (uint64_t)n * 4, hipMemcpyDeviceToDevice, s));
                if (p_row) LG_CHECK_HIP(hipMemcpyAsync(tmp_p, p_row, (uint64_t)n * 4, hipMemcpyDeviceToDevice, s));
                d_in = tmp_d;
                p_in = tmp_p;
            }
            LG_LAUNCH(bfs_unpermute_kernel, grid_for(n, 256, 1u << 16), 256, 0, s, n, g->inv.as<uint32_t>(),
                      g->perm.as<uint32_t>(), d_in, p_in, d_row, p_row);
            LG_CHECK_LAUNCH();
        }
    }
    return LG_OK;
}

constexpr uint32_t kBfsLanes = 8;

// One set of lanes per device, shared by all graphs (workspaces grow to the
// largest graph and stay until lg_trim); a multi-root call holds it for its
// duration, so such calls on one device run one after the other.
namespace {
struct DevicePools {
    std::mutex mu;
    std::map<int, BfsPool *> pools;
    std::map<int, std::mutex *> locks;
};
DevicePools &device_pools() {
    static DevicePools *d = new DevicePools();  // never destroyed (streams may outlive static teardown)
    return *d;
}
}  // namespace

void bfs_pools_trim() {
    DevicePools &d = device_pools();
    std::lock_guard<std::mutex> g(d.mu);
    for (auto &kv : d.pools) {
        std::lock_guard<std::mutex> l(*d.locks[kv.first]);
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(kv.first);
        delete kv.second;
        (void)hipSetDevice(prev);
    }
    d.pools.clear();
}

static lg_status pool_ensure(BfsPool *&pp, uint32_t lanes) {
    if (!pp) {
        pp = new (std::nothrow) BfsPool();
        if (!pp) { set_error("lg_bfs: host allocation failed"); return LG_ERR_OOM; }
        LG_CHECK_HIP(hipEventCreateWithFlags(&pp->start, hipEventDisableTiming));
    }
    BfsPool &p = *pp;
    while (p.lanes.size() < lanes) {
        BfsLane *l = new (std::nothrow) BfsLane();
        if (!l) { set_error("lg_bfs: host allocation failed"); return LG_ERR_OOM; }
        p.lanes.push_back(l);
        LG_CHECK_HIP(hipStreamCreateWithFlags(&l->stream, hipStreamNonBlocking));
        LG_CHECK_HIP(hipEventCreateWithFlags(&l->done, hipEventDisableTiming));
    }
    return LG_OK;
}

// Several roots: lanes take the next root from a shared counter until none
// is left.  Work on `stream` before the call is complete before any lane
// starts, and `stream` waits for every lane before work queued after the
// call runs.  Every root's result is that of a run alone.
static lg_status bfs_run_lanes(lg_graph *g, const uint32_t *roots, uint32_t r, int32_t *depth, int32_t *parent,
                               int32_t max_depth, uint32_t flags, hipStream_t stream) {
    const uint32_t L = std::min<uint32_t>(r, kBfsLanes);
    DevicePools &dp = device_pools();
    std::mutex *dev_lock;
    BfsPool **slot;
    {
        std::lock_guard<std::mutex> gl(dp.mu);
        if (!dp.locks.count(g->device)) dp.locks[g->device] = new std::mutex();
        dev_lock = dp.locks[g->device];
        slot = &dp.pools[g->device];
    }
    std::lock_guard<std::mutex> hold(*dev_lock);
    LG_TRY(pool_ensure(*slot, L));
    BfsPool &p = **slot;
    LG_CHECK_HIP(hipEventRecord(p.start, stream));
    for (uint32_t i = 0; i < L; ++i) LG_CHECK_HIP(hipStreamWaitEvent(p.lanes[i]->stream, p.start, 0));
    std::atomic<uint32_t> next{0};
    std::vector<lg_status> st(L, LG_OK);
    std::vector<std::string> err(L);
    std::vector<std::thread> th;
    const uint64_t n = g->n;
    for (uint32_t i = 0; i < L; ++i) {
        th.emplace_back([&, i] {
            (void)hipSetDevice(g->device);
            BfsLane &ln = *p.lanes[i];
            for (uint32_t k = next++; k < r && st[i] == LG_OK; k = next++) {
                st[i] = bfs_run(g, ln.work, roots + k, 1, depth + (uint64_t)k * n,
                                parent ? parent + (uint64_t)k * n : nullptr, max_depth, flags, ln.stream);
                if (st[i] != LG_OK) err[i] = lg_last_error();
            }
            (void)hipEventRecord(ln.done, ln.stream);
        });
    }
    for (auto &t : th) t.join();
    for (uint32_t i = 0; i < L; ++i) LG_CHECK_HIP(hipStreamWaitEvent(stream, p.lanes[i]->done, 0));
    for (uint32_t i = 0; i < L; ++i)
        if (st[i] != LG_OK) {
            set_error("%s", err[i].c_str());
            return st[i];
        }
    return LG_OK;
}

// Several roots of a direction-optimizing search on a graph whose lists are
// not read in order only: the multi-source traversal, in batches of up to
// 64 roots while at least kMsMinRoots are left (fewer go to the lanes: a
// bottom-up multi-source level reads whole lists for every search still
// open, which the one-root searches beat below about 16 roots on the graphs
// measured).
// It runs on `stream` and holds the device's BFS pool (its lane 0
// workspace, the multi-source masks) for its duration.
constexpr uint32_t kMsMinRoots = 16;
constexpr uint64_t kMsRowsCap = 16ull << 30;  // bytes of label-space rows a relabeled batch may keep aside

static bool bfs_ms_graph(const lg_graph *g, uint32_t flags) {
    if (flags != LG_BFS_DIRECTION_OPT) return false;
    if (g->layout == LG_LAYOUT_PLAIN) return true;
    return !g->weighted && (g->id_mode == LG_IDS_GLOBAL || g->id_mode == LG_IDS_LOCAL) &&
           g->offset_mode != LG_OFFS_INTERLEAVED_BV;
}

// how many of r roots the multi-source batches take (the first ones)
static uint32_t bfs_ms_roots(uint32_t r) {
    uint32_t k = 0;
    while (r - k >= kMsMinRoots) k += std::min<uint32_t>(kMsRoots, r - k);
    return k;
}

static lg_status bfs_run_ms(lg_graph *g, const uint32_t *roots, uint32_t r, int32_t *depth, int32_t *parent,
                            int32_t max_depth, hipStream_t stream) {
    DevicePools &dp = device_pools();
    std::mutex *dev_lock;
    BfsPool **slot;
    {
        std::lock_guard<std::mutex> gl(dp.mu);
        if (!dp.locks.count(g->device)) dp.locks[g->device] = new std::mutex();
        dev_lock = dp.locks[g->device];
        slot = &dp.pools[g->device];
    }
    std::lock_guard<std::mutex> hold(*dev_lock);
    LG_TRY(pool_ensure(*slot, 1));
    BfsPool &p = **slot;
    BfsWork &w = p.lanes[0]->work;
    MsWork &ms = p.ms;
    // lane 0's workspace may still be in use by an earlier lanes call's
    // kernels on lane 0's stream (its event marks their end)
    LG_CHECK_HIP(hipStreamWaitEvent(stream, p.lanes[0]->done, 0));
    const uint64_t n = g->n, words = (n + 63) / 64;
    LG_TRY(bfs_workspace_ensure(w, n, g->n_heavy, g->relabel != LG_RELABEL_NONE, parent != nullptr));
    LG_TRY(ms.vis.ensure(n * 8));
    LG_TRY(ms.fr.ensure(n * 8));
    LG_TRY(ms.nx.ensure(n * 8));
    LG_TRY(ms.bits.ensure(words * 8));
    LG_TRY(ms.pend_v.ensure(n * 4));
    LG_TRY(ms.pend_m.ensure(n * 8));
    LG_TRY(ms.roots.ensure(kMsRoots * 4));
    // relabeled graphs: a batch's label-space rows in a workspace, so that
    // they unpermute straight into the caller's rows, when it stays within
    // kMsRowsCap (else every row is copied aside before its unpermute)
    int32_t *ws = nullptr;
    if (g->relabel != LG_RELABEL_NONE) {
        const uint64_t need = (uint64_t)std::min<uint32_t>(r, kMsRoots) * n * (parent ? 8 : 4);
        if (need <= kMsRowsCap) {
            LG_TRY(ms.rows.ensure(need));
            ws = ms.rows.as<int32_t>();
        }
    }
    // lane 0's stream is not used: everything runs on the caller's stream
    LG_TRY(dispatch_acc(g, [&](auto acc) -> lg_status {
        for (uint32_t b0 = 0; b0 < r; b0 += kMsRoots) {
            const uint32_t rb = std::min<uint32_t>(kMsRoots, r - b0);
            LG_TRY(bfs_ms_batch(g, w, ms, acc, roots + b0, rb, depth + (uint64_t)b0 * n,
                                parent ? parent + (uint64_t)b0 * n : nullptr, max_depth, ws, stream));
        }
        return LG_OK;  // batches follow each other on the caller's stream (shared masks and roots buffer)
    }));
    // the last batch's finishing kernels still read the masks: another call
    // may take them (on another stream) once the device lock is released
    LG_CHECK_HIP(hipStreamSynchronize(stream));
    return LG_OK;
}

}  // namespace lg

extern "C" lg_status lg_bfs(const lg_graph *gc, const uint32_t *roots, uint32_t r, int32_t *depth, int32_t *parent,
                            int32_t max_depth, uint32_t flags, hipStream_t stream) {
    using namespace lg;
    lg_graph *g = const_cast<lg_graph *>(gc);
    if (!g || (r && (!roots || !depth))) { set_error("lg_bfs: NULL argument"); return LG_ERR_INVALID; }
    if (flags > LG_BFS_BOTTOM_UP) { set_error("lg_bfs: unknown flags"); return LG_ERR_INVALID; }
    for (uint32_t i = 0; i < r; ++i)
        if (roots[i] >= g->n) { set_error("lg_bfs: root %u out of range", roots[i]); return LG_ERR_INVALID; }
    if (r == 0) return LG_OK;
    const uint32_t r_ms = bfs_ms_graph(g, flags) ? bfs_ms_roots(r) : 0;
    if (r_ms) {
        LG_TRY(bfs_run_ms(g, roots, r_ms, depth, parent, max_depth, stream));
        if (r_ms < r) {
            const uint64_t off = (uint64_t)r_ms * g->n;
            LG_TRY(bfs_run_lanes(g, roots + r_ms, r - r_ms, depth + off, parent ? parent + off : nullptr, max_depth,
                                 flags, stream));
        }
        return mark_use(g, stream);
    }
    if (r > 1) {
        // the lanes' work is joined back into `stream` before this returns
        LG_TRY(bfs_run_lanes(g, roots, r, depth, parent, max_depth, flags, stream));
        return mark_use(g, stream);
    }
    if (!g->bfs) {
        g->bfs = new (std::nothrow) BfsWork();
        if (!g->bfs) { set_error("lg_bfs: host allocation failed"); return LG_ERR_OOM; }
    }
    LG_TRY(bfs_run(g, *g->bfs, roots, r, depth, parent, max_depth, flags, stream));
    return mark_use(g, stream);
}
