// Internal declarations of liblg: the graph handle, device views of it,
// error plumbing, kernel-launch timing and shared utility launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "lg.h"

namespace lg {

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------

void set_error(const char *fmt, ...);

#define LG_CHECK_HIP(expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::lg::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),      \
                            __FILE__, __LINE__);                                        \
            return e_ == hipErrorOutOfMemory ? LG_ERR_OOM : LG_ERR_DEVICE;              \
        }                                                                               \
    } while (0)

#define LG_TRY(expr)                                                                    \
    do {                                                                                \
        lg_status s_ = (expr);                                                          \
        if (s_ != LG_OK) return s_;                                                     \
    } while (0)

// ---------------------------------------------------------------------------
// device memory owned by the library
// ---------------------------------------------------------------------------

// A device buffer with RAII release; on failure the status says OOM.
struct DevBuf {
    void *p = nullptr;
    uint64_t bytes = 0;
    hipStream_t pool_stream = nullptr;  // scratch from the pool: returns there on release
    bool pooled = false;
    bool borrowed = false;  // a view of memory the buffer does not own: never freed or grown
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept
        : p(o.p), bytes(o.bytes), pool_stream(o.pool_stream), pooled(o.pooled), borrowed(o.borrowed) {
        o.p = nullptr;
        o.bytes = 0;
        o.pooled = false;
        o.borrowed = false;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; bytes = o.bytes; pool_stream = o.pool_stream; pooled = o.pooled; borrowed = o.borrowed;
            o.p = nullptr; o.bytes = 0; o.pooled = false; o.borrowed = false;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release();
    // view [ptr, ptr + nbytes) of memory owned elsewhere: ensure() then only
    // checks the size (it fails with LG_ERR_UNSUPPORTED instead of
    // allocating) and release() forgets the view
    void borrow(void *ptr, uint64_t nbytes) {
        release();
        p = ptr;
        bytes = nbytes;
        borrowed = true;
    }
    lg_status alloc(uint64_t nbytes);          // release + allocate
    lg_status ensure(uint64_t nbytes);         // grow only
    // release + take a buffer of at least nbytes that is only ever used on
    // stream s, from the scratch pool when one fits (no allocation, no
    // device-wide synchronization when it is released again)
    lg_status scratch(uint64_t nbytes, hipStream_t s);
    template <class T> T *as() const { return static_cast<T *>(p); }
};

}  // namespace lg

#include "lg_views.hpp"

namespace lg {

// ---------------------------------------------------------------------------
// the graph handle
// ---------------------------------------------------------------------------

struct PrWork;
struct PbWork;
struct SsspWork;

// Device workspace of one BFS at a time (grow-only buffers).
struct BfsWork {
    DevBuf qa, qb;               // frontier queues (stored labels)
    DevBuf fstart, fdeg, fw;     // per frontier entry: first bit/element, degree, width
    DevBuf fscan;                // exclusive scan of fdeg
    DevBuf visited, curr, next;  // bitmaps, one bit per vertex
    DevBuf counters;             // [0] queue tail, [1] awakened count, [2] pending count
    DevBuf sample;               // partial sums of the sampled bottom-up cost (8 words)
    DevBuf pv, pstart, pdeg, pw; // bottom-up: heavy vertices left for the segment pass
    DevBuf pseg_cnt, pseg_off;
    DevBuf depth_i, parent_i;    // label-space results when relabeled
    DevBuf scan_tmp;
    uint64_t *host = nullptr;    // pinned readback slots
    BfsWork() = default;
    BfsWork(const BfsWork &) = delete;
    BfsWork &operator=(const BfsWork &) = delete;
    ~BfsWork();
    uint64_t bytes() const;
};

// Roots of one lg_bfs call run on a few lanes at once: each lane has its own
// stream (default priority), workspace and host thread, so that one root's
// host round trips between levels are covered by another root's kernels.
// One set of lanes per device (lg_bfs.hip), freed by lg_trim.
struct BfsLane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    BfsWork work;
};
// Multi-source BFS of up to 64 roots at once (lg_bfs.hip): per vertex a
// 64-bit mask per state (bit i: root i), a frontier bitmap, and the vertices
// whose long lists a whole wave finishes.
struct MsWork {
    DevBuf vis, fr, nx;          // u64[n]: reached, in this level's frontier, in the next one
    DevBuf bits;                 // u64[words]: vertices of the next frontier
    DevBuf pend_v, pend_m;       // u32[n], u64[n]: vertices left for the wave pass, their open bits
    DevBuf roots;                // u32[64]: the batch's roots
    DevBuf rows;                 // relabeled graphs: the batch's depth and parent rows in label space
    uint64_t bytes() const {
        return vis.bytes + fr.bytes + nx.bytes + bits.bytes + pend_v.bytes + pend_m.bytes + roots.bytes + rows.bytes;
    }
};
struct BfsPool {
    std::vector<BfsLane *> lanes;
    hipEvent_t start = nullptr;
    MsWork ms;
    ~BfsPool();
    uint64_t bytes() const;
};

// Device workspace of one neighbor decode at a time (grow-only buffers).
struct DecodeWork {
    DevBuf head;                 // labels, degrees, flag
    DevBuf scan_tmp, keys, keys2, vals, vals2, sort_tmp;
    uint64_t *host = nullptr;    // readback slots (pinned, allocated on first use, unless set by the caller)
    bool host_owned = true;      // host came from hipHostMalloc and is freed with the workspace
    DecodeWork() = default;
    DecodeWork(const DecodeWork &) = delete;
    DecodeWork &operator=(const DecodeWork &) = delete;
    ~DecodeWork();
    uint64_t bytes() const;
};

}  // namespace lg

struct lg_graph {
    uint32_t n = 0;
    uint64_t m = 0;
    uint32_t layout = 0, id_mode = 0, offset_mode = 0, relabel = 0;
    int device = 0;
    uint32_t max_degree = 0, isolated = 0;

    // packed layout
    uint32_t s = 0, F = 0, wO = 0, ef_l = 0;
    uint64_t U = 0, universe = 0, hbits = 0;
    lg::DevBuf A, O, W, G, L, H, rank_sb, sel;  // G: gap-width table (gap mode)
    uint64_t A_words = 0, O_words = 0, W_words = 0, G_words = 0, L_words = 0, H_words = 0, n_rank = 0, n_sel = 0;
    // interleaved bit-vector offsets (bvIL): 9 words per 512-bit block + 1
    lg::DevBuf IL;
    uint64_t IL_words = 0, il_blocks = 0;

    // plain layout
    lg::DevBuf poff, pcol;
    bool poff64 = false;

    // weighted graphs: omega = weight width (each packed entry is the ID,
    // then the weight); the plain layout keeps one uint32 weight per entry
    // in pwt
    bool weighted = false;
    uint32_t omega = 0;
    lg::DevBuf pwt;

    // relabeling: perm[new] = old, inv[old] = new
    lg::DevBuf perm, inv;

    // vertices whose degree exceeds heavy_threshold, ascending: the traversal
    // kernels give each of them a wave (bottom-up BFS) or several waves
    // (PageRank) instead of one lane
    lg::DevBuf heavy;
    uint32_t n_heavy = 0;
    // one bit per vertex (label space), set for vertices without edges and
    // for the padding past n: BFS starts with them marked visited, so sweeps
    // skip words that hold only such vertices
    lg::DevBuf iso;
    uint32_t heavy_threshold = 64;
    // PageRank work tables, built at the first lg_pagerank.  Per heavy
    // vertex: first bit/element, degree, width.  Vertices of degree above
    // pr_split have their lists cut into segments of seg_size edges
    // (seg_off[h] .. seg_off[h+1], seg_map[k] = h; seg_part[k] holds the
    // segment's sum in the current iteration).  The other vertices are taken
    // in units of consecutive vertices inside one 64-aligned block, at most
    // about pr_unit_edges edges each: unit k = [units[k], units[k+1]).
    // With gap-encoded lists also the gap width of each heavy vertex (hg) and
    // the value of the entry before each segment (seg_base; 0 for a list's
    // first segment).
    lg::DevBuf hstart, hdeg, hw, hg, seg_off, seg_map, seg_part, seg_base, units;
    uint64_t n_seg = 0, n_units = 0;
    uint32_t seg_size = 4096;       // a power of two keeping every vertex below 2^16 segments
    uint32_t pr_split = 4096;       // degree above which PageRank segments a list
    uint32_t pr_unit_edges = 8192;  // edge budget of a unit (plus at most one list of <= pr_split)
    uint64_t heavy_edges = 0, heavy_bits = 0;  // entries and bits (packed) of the heavy lists
    bool segs_built = false;
    // Varint lists longer than vseg_split bytes, in byte chunks of vseg_bytes
    // (built with the encoding): heavy vertex h's byte range [vhb0, vhb1),
    // its chunks vseg_off[h] .. vseg_off[h+1] (vseg_map[k] = h); a value
    // belongs to the chunk holding its last byte, and vseg_base[k] is the
    // label before chunk k (differences) or 0 (full labels)
    lg::DevBuf vhb0, vhb1, vseg_off, vseg_map, vseg_base;
    uint64_t n_vseg = 0;
    // PageRank over Varint lists (built at its first call): d_v per vertex,
    // the contribution ping-pong and one partial sum per chunk
    lg::DevBuf vdeg, vca, vcb, vpart;
    uint32_t vseg_bytes = 4096, vseg_split = 8192;

    // lazily allocated workspaces of the plain calls (lg_bfs, lg_pagerank,
    // lg_decode_neighbors); the server brings its own per worker
    lg::BfsWork *bfs = nullptr;
    lg::PrWork *pr = nullptr;
    lg::PbWork *pb = nullptr;  // PageRank by propagation blocking (lg_pagerank_pb.hip)
    lg::DecodeWork *dec = nullptr;
    lg::SsspWork *sssp = nullptr;
    std::mutex sssp_mu;  // lg_sssp calls on this graph share `sssp`: one at a time
    // recorded on the caller's stream at the end of every call that reads
    // the graph; lg_free waits for it (and nothing else) before the arrays
    // are released
    hipEvent_t last_use = nullptr;

    lg::PackedView packed_view() const;
    lg::PlainView plain_view() const;
    uint64_t device_bytes() const;
};

namespace lg {

// ---------------------------------------------------------------------------
// kernel timing (lg_prof_*)
// ---------------------------------------------------------------------------

bool prof_on();
struct ProfMark {
    hipEvent_t a = nullptr, b = nullptr;
    const char *name = nullptr;
    hipStream_t stream = nullptr;
};
ProfMark prof_begin(const char *name, hipStream_t stream);
void prof_end(ProfMark &m);

// Launch a kernel with timing when profiling is on.
#define LG_LAUNCH(kernel, grid, block, shmem, stream, ...)                              \
    do {                                                                                \
        ::lg::ProfMark pm_;                                                             \
        if (::lg::prof_on()) pm_ = ::lg::prof_begin(#kernel, stream);                   \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__); \
        if (pm_.a) ::lg::prof_end(pm_);                                                 \
    } while (0)

#define LG_CHECK_LAUNCH() LG_CHECK_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// utility launchers (lg_util.hip)
// ---------------------------------------------------------------------------

lg_status fill_u32(uint32_t *p, uint32_t value, uint64_t count, hipStream_t s);
lg_status fill_u64(uint64_t *p, uint64_t value, uint64_t count, hipStream_t s);

// Exclusive prefix sum: out[0..count] with out[count] = total.  `tmp` is
// grown as needed.
lg_status exclusive_scan_u32(const uint32_t *in, uint64_t *out, uint64_t count, DevBuf &tmp,
                             hipStream_t s);
lg_status exclusive_scan_u64(const uint64_t *in, uint64_t *out, uint64_t count, DevBuf &tmp,
                             hipStream_t s);

// Scratch bytes the scans and sorts below grow `tmp` to for `count` items
// (non-decreasing in count).
uint64_t scan_tmp_bytes(uint64_t count);
uint64_t radix_sort_tmp_bytes(uint64_t count);

// Stable LSD radix sort of (key, value) pairs on key bits [0, bits).  The
// buffers are ping-ponged with the alt ones; results end in keys/vals, or,
// when in_alt is not NULL, wherever the last pass wrote them (*in_alt = 1:
// in keys_alt/vals_alt), which saves a copy after an odd number of passes.
lg_status radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                           uint64_t count, uint32_t bits, DevBuf &tmp, hipStream_t s, int *in_alt = nullptr);

// Stable radix sort of (key, value) pairs whose keys are 64-bit: bits [0, bits).
lg_status radix_sort_pairs64(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                             uint64_t count, uint32_t bits, DevBuf &tmp, hipStream_t s, int *in_alt = nullptr);

// Grid size helper: blocks needed for `count` items at `per_block`, capped.
inline uint32_t grid_for(uint64_t count, uint64_t per_block, uint64_t cap = 1u << 30) {
    uint64_t g = (count + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

inline uint32_t bitlen_u64(uint64_t x) { return x ? 64u - (uint32_t)__builtin_clzll(x) : 0u; }

// Build the PageRank work tables of g (once); defined in lg_heavy.hip.
lg_status ensure_heavy_segments(lg_graph *g, hipStream_t s);
lg_status build_varint_segments(lg_graph *g, hipStream_t s);
lg_status pagerank_varint(lg_graph *g, float damping, uint32_t iters, float *scores, hipStream_t s);

// Record g->last_use on `stream` (the end of a call that read g).
lg_status mark_use(lg_graph *g, hipStream_t stream);

lg_status bfs_free(lg_graph *g);
void bfs_pools_trim();
lg_status bfs_workspace_ensure(BfsWork &w, uint64_t n, uint64_t n_heavy, bool relabel, bool need_parent);
// Direction switch of the direction-optimizing BFS: top-down -> bottom-up
// when the frontier's edges exceed the unexplored edges / alpha.
//   kBfsAlphaLatency  searches that have the device to themselves (lg_bfs).
//                     Timing 64-root searches on Kronecker scale 24 over
//                     alpha 5 .. 1000: 60 is 16 % faster than the customary
//                     15, anything in 60 .. 250 about equal.
//   kBfsAlphaShared   searches that share the device with unrelated queries
//                     (the query server).  Switching early shortens one
//                     search by sweeping every vertex a level sooner; the
//                     extra sweeps are device time the other queries wait
//                     for, and on the mixed serving input 15 serves 30 % more
//                     queries per second than 60 at a third of the p99.
constexpr double kBfsAlphaLatency = 60.0;
constexpr double kBfsAlphaShared = 15.0;
// Between the two switch points (frontier edges in (m_u/60, m_u/15]) the
// right direction depends on how soon an unvisited vertex meets the
// frontier: on a Kronecker graph whose lists start with the hubs, within a
// probe or two (bottom-up wins at 60), on a uniform random graph with a
// frontier of 1.5 % of the vertices, only after most of its list (top-down
// wins: bottom-up at that level cost 4x the search on Erdos-Renyi scale 26).
// There lg_bfs measures it: the bottom-up cost of a sample of vertices
// (entries read until the first frontier neighbour), scaled to the graph,
// against the top-down cost (the frontier's edges).  kBfsProbeCost is the
// cost of a bottom-up entry relative to a top-down edge (a sequential read
// and a bitmap probe against a random claim): about 1/6 on both graphs.
constexpr double kBfsAlphaLate = 15.0;
constexpr double kBfsProbeCost = 1.0 / 6.0;

// BFS from host roots on an explicit workspace (lg_bfs without argument checks)
lg_status bfs_run(lg_graph *g, BfsWork &w, const uint32_t *roots, uint32_t r, int32_t *depth, int32_t *parent,
                  int32_t max_depth, uint32_t flags, hipStream_t stream, double alpha = kBfsAlphaLatency);
// lg_decode_neighbors on an explicit workspace
lg_status decode_run(lg_graph *g, DecodeWork &w, const uint32_t *vertices, uint32_t k, uint64_t *out_off,
                     uint32_t *out_ids, uint64_t cap, uint32_t flags, hipStream_t stream, uint64_t *total);
lg_status pr_free(lg_graph *g);
// PageRank by propagation blocking: the graphs it serves, its driver, its
// workspace (lg_pagerank_pb.hip)
bool pb_applies(const lg_graph *g);
lg_status pagerank_pb(lg_graph *g, float damping, uint32_t iters, float *scores, hipStream_t s);
uint64_t pb_bytes(const lg_graph *g);
void pb_free(lg_graph *g);
void pb_trim();  // frees the bin buffers parked for the next graph
lg_status sssp_free(lg_graph *g);
uint64_t sssp_bytes(const lg_graph *g);

}  // namespace lg
