// PageRank by propagation blocking (the PR of section "Considered
// Algorithms", same iteration as lg_pagerank.hip), for graphs whose labels
// give the contribution gathers of the pull no locality: unrelabeled graphs
// of at least 2^22 vertices.
//
// The pull reads contrib[u] for every stored entry at a random place of a
// 4n-byte array; once that array outgrows the caches, every gather costs a
// line transfer and the iteration runs at the random-access rate of the
// memory side cache, not at the stream rate (Erdos-Renyi scale 26: 2.1e9
// gathers, 40 ms per iteration).  Propagation blocking turns the gathers
// into streams.  A symmetric graph's list of u is also the set of vertices
// whose lists hold u, so reading the lists in order and sending contrib[u]
// to every neighbour v computes the same sums:
//
//   level 1  the lists are read in storage order, a workgroup per equal range
//            of entries; every entry (v, contrib[u]) goes to coarse bin
//            v >> 20.  A workgroup takes 4,096 entries per round (their rows'
//            offsets all loaded at once, the list loads issued together),
//            counting-sorts them by bin in LDS and writes each bin's run
//            whole, so the writes are long runs, not scattered words.
//   level 2  each coarse bin is split into 64 fine bins of 2^14 vertices
//            the same way.
//   level 3  a workgroup per fine bin adds its entries in LDS and finalizes
//            its vertices.
//
// Every (workgroup, bin) writes into its own region, whose place is fixed
// once per graph by a counting pass (the graph does not change): no global
// atomics.  The sums are taken in 64-bit fixed point (units of 2^-60) with
// LDS integer atomics: exact whatever the order of the entries, so the
// scores repeat bit for bit and carry no summation error beyond the FP32
// rounding of each contribution.
#include <algorithm>

#include "lg_device.hpp"

namespace lg {

constexpr uint32_t kPbThreads = 1024;
constexpr uint32_t kPbWaves = kPbThreads / kWave;     // 16
// level 1: 64-entry steps per wave per round, 4,096 entries per round, so
// that its LDS (about 60 KB) lets two workgroups share a compute unit
constexpr uint32_t kPb1Steps = 4;
constexpr uint32_t kPb1Round = kPbThreads * kPb1Steps;
constexpr uint32_t kPb1PerCU = 2;
// level 1's grid: 16 workgroups per CU, two resident at a time.  Smaller
// entry ranges even out the workgroups' ends (windows cost more where rows
// are short); level 2 then takes kPb2Merge neighbouring level-1 regions per
// workgroup, so that its regions stay about two rounds long.  Measured at
// Erdos-Renyi scale 26 against one range per resident workgroup and one
// region per level-2 workgroup: 16.5 -> 15.4 ms per iteration (mean of
// three alternating runs, both layouts; the results are bit-identical)
constexpr uint32_t kPb1Grid = 16;
constexpr uint32_t kPb2Merge = 4;
constexpr uint32_t kFineShift = 14;                    // fine bin: 16,384 vertices
constexpr uint32_t kFine = 1u << kFineShift;
constexpr uint32_t kSubBins = 64;                      // fine bins per coarse bin
constexpr uint32_t kCoarseShift = kFineShift + 6;      // coarse bin: 2^20 vertices
constexpr uint32_t kPbMaxCoarse = 255;                 // coarse bins fit a byte below the 0xFF sentinel
constexpr double kFixScale = 1152921504606846976.0;    // 2^60
constexpr double kFixUnit = 1.0 / 1152921504606846976.0;

// Workgroup barrier that orders LDS only.  Threads of these kernels share
// data through LDS alone (the bins they write to global memory are read by
// the next kernel), so a barrier need not wait for their global stores, as
// __syncthreads() does: the stores of one round stay in flight while the
// next round runs.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves (the
// cross-lane scan of the GCN ISA: shifts by 1, 2, 4 and 8 lanes inside each
// row of 16, then the last lane of a row broadcast into the rows after it).
// Unlike a shuffle scan it needs no lane-address registers, which the
// compiler keeps live across the whole kernel: in the binning kernels,
// which run at the 64-VGPR limit, those registers forced a spill whose
// reload waited for every load in flight.
__device__ __forceinline__ uint32_t wave_scan_dpp(uint32_t x) {
    // dpp_ctrl: row_shr:n = 0x110 + n, row_bcast:15 = 0x142, row_bcast:31 = 0x143
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // rows 1, 3 += end of rows 0, 2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // rows 2, 3 += end of row 1
    return x;
}

// below this many vertices the pull's gathers stay in cache
constexpr uint32_t kPbMinVertices = 1u << 22;

struct PbWork {
    uint32_t nwg = 0;      // level-1 workgroups
    uint32_t nc = 0;       // coarse bins
    uint32_t nf = 0;       // fine bins
    DevBuf row_lo, k_lo;   // u32[nwg]: row holding each level-1 workgroup's first entry, entries before it
    DevBuf base1;          // u64[nwg * nc]: level-1 region start of (workgroup, coarse bin)
    DevBuf len1;           // u32[nwg * nc]: entries of that region
    DevBuf base2;          // u64[nwg * nc * 64]: level-2 region start of ((w, c), fine bin)
    DevBuf fstart;         // u64[nf + 1]: fine bin starts in the level-2 arrays
    DevBuf buf1;           // uint2[m]: (vertex within the coarse bin, contribution bits)
    DevBuf buf2;           // u16[m] vertex within the fine bin, then (at val_off) f32[m] contribution
    uint64_t val_off = 0;  // byte offset of the contributions in buf2
    DevBuf ca, cb;         // contribution ping-pong
    bool built = false;
};

uint64_t pb_bytes(const lg_graph *g) {
    if (!g->pb) return 0;
    const PbWork &w = *g->pb;
    return w.row_lo.bytes + w.k_lo.bytes + w.base1.bytes + w.len1.bytes + w.base2.bytes + w.fstart.bytes + w.buf1.bytes +
           w.buf2.bytes + w.ca.bytes + w.cb.bytes;
}

// The two bin buffers (8 B per stored entry each) outlive their graph in one
// slot per device: the next graph of about the same size takes them without
// an allocation, which at this size can stall for hundreds of milliseconds.
// lg_free parks them only after the graph's last use, so whoever takes them
// finds them idle; lg_trim frees them.
namespace {
constexpr int kPbSlots = 64;  // devices
struct PbSlot {
    DevBuf buf1, buf2;
};
std::mutex g_pb_slot_mu;
PbSlot *pb_slots() {
    static PbSlot *p = new PbSlot[kPbSlots];  // never destroyed: no frees during static teardown
    return p;
}
}  // namespace

void pb_free(lg_graph *g) {
    if (g->pb && g->pb->built && g->device >= 0 && g->device < kPbSlots) {
        std::lock_guard<std::mutex> lk(g_pb_slot_mu);
        PbSlot &sl = pb_slots()[g->device];
        if (!sl.buf1.p || sl.buf1.bytes < g->pb->buf1.bytes) {  // keep the larger pair
            sl.buf1 = std::move(g->pb->buf1);
            sl.buf2 = std::move(g->pb->buf2);
        }
    }
    delete g->pb;
    g->pb = nullptr;
}

void pb_trim() {
    std::lock_guard<std::mutex> lk(g_pb_slot_mu);
    for (int d = 0; d < kPbSlots; ++d) {
        pb_slots()[d].buf1.release();
        pb_slots()[d].buf2.release();
    }
}

// bin buffers of `bytes1` and `bytes2`: the parked pair when it fits (at
// most a quarter larger), else new ones (a parked pair that does not fit is
// freed first, so that its memory is available)
static lg_status pb_take_bins(lg_graph *g, uint64_t bytes1, uint64_t bytes2) {
    PbWork &W = *g->pb;
    auto fits = [](const DevBuf &b, uint64_t need) { return b.p && b.bytes >= need && b.bytes <= need + need / 4; };
    if (g->device >= 0 && g->device < kPbSlots) {
        std::lock_guard<std::mutex> lk(g_pb_slot_mu);
        PbSlot &sl = pb_slots()[g->device];
        if (fits(sl.buf1, bytes1) && fits(sl.buf2, bytes2)) {
            W.buf1 = std::move(sl.buf1);
            W.buf2 = std::move(sl.buf2);
            return LG_OK;
        }
        sl.buf1.release();
        sl.buf2.release();
    }
    LG_TRY(W.buf1.alloc(bytes1));
    LG_TRY(W.buf2.alloc(bytes2));
    return LG_OK;
}

// Is propagation blocking the PageRank of this graph?  A rule of the graph
// alone (never of timing), so that results do not depend on the run.
bool pb_applies(const lg_graph *g) {
    if (g->relabel != LG_RELABEL_NONE || g->weighted || g->n < kPbMinVertices) return false;
    if (((uint64_t)g->n + (1u << kCoarseShift) - 1) >> kCoarseShift > kPbMaxCoarse) return false;
    if (g->layout == LG_LAYOUT_PLAIN) return true;
    return (g->id_mode == LG_IDS_GLOBAL || g->id_mode == LG_IDS_LOCAL) && g->offset_mode != LG_OFFS_INTERLEAVED_BV;
}

// ---------------------------------------------------------------------------
// level 1: workgroup w streams entries [w m / nwg, (w + 1) m / nwg) of the
// lists in storage order
// ---------------------------------------------------------------------------

// d_v of every vertex (a wave per 64 vertices)
template <class Acc>
__global__ void pb_degree_kernel(Acc acc, uint32_t n, uint32_t *__restrict__ deg) {
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t q = wave; q < words; q += nwaves) {
        const VInfo vi = wave_info(acc, q * 64, n);
        const uint64_t v = q * 64 + lane_id();
        if (v < n) deg[v] = vi.deg;
    }
}

// the row holding entry w m / nwg (the last row whose first entry is at or
// before it) and the entries of that row before it
__global__ void pb_row_lo_kernel(uint32_t n, uint64_t m, uint32_t nwg, const uint64_t *__restrict__ eoff,
                                 uint32_t *__restrict__ row_lo, uint32_t *__restrict__ k_lo) {
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwg) return;
    const uint64_t e = m * w / nwg;
    uint32_t lo = 0, hi = n - 1;  // eoff[0] = 0 <= e
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (eoff[mid] <= e) lo = mid; else hi = mid - 1;
    }
    row_lo[w] = lo;
    k_lo[w] = (uint32_t)(e - eoff[lo]);
}

// A window is 1,024 rows from the 64-aligned block of the first row with
// entries left: their offsets and contributions come in once, a workgroup
// scan gives each row's first entry within the window, and the rows with
// entries mark those first entries in a bitmap of the window's first
// kWinCap entries, with the marks before each 32-bit word alongside.  The
// window then serves rounds of up to 4,096 entries until its bitmap is used
// up: each thread takes kPb1Steps entries of the round, finds their rows by
// the rank of the bitmap (one popcount; a binary search per entry made the
// kernel bound by its instruction count) and issues their list loads
// together.  Write mode: entries (v & (2^20 - 1), contrib[u]) counting-sorted
// by coarse bin v >> 20 and written as runs at the workgroup's region
// cursors; the counts alternate between two arrays so that folding one
// round's counts into the cursors needs no barrier of its own.  Count mode:
// entries per fine bin.
constexpr uint32_t kWin = kPbThreads;           // rows per window
constexpr uint32_t kWinCap = 32 * kPbThreads;   // window entries with a bitmap bit (one word per thread)
constexpr uint32_t kPb1WavesPerEU = kPb1PerCU * kPbWaves / 4;  // waves per SIMD for kPb1PerCU workgroups per CU

template <class Acc, bool kCount>
__global__ __launch_bounds__(kPbThreads, kPb1WavesPerEU) void pb_bin1_kernel(
    Acc acc, uint32_t n, uint64_t m, uint32_t nwg, const float *__restrict__ cin,
    const uint32_t *__restrict__ row_lo, const uint32_t *__restrict__ k_lo, uint32_t nc,
    const uint64_t *__restrict__ base1, uint2 *__restrict__ buf1, uint32_t nf, uint32_t *__restrict__ hist_out) {
    extern __shared__ uint32_t s_fhist[];  // count mode: entries per fine bin
    __shared__ uint2 s_buf[kCount ? 1 : kPb1Round];   // (vertex, contribution bits) sorted by coarse bin
    __shared__ uint32_t s_hist[2][kCount ? 1 : kPbMaxCoarse + 1];
    __shared__ uint32_t s_start[kCount ? 1 : kPbMaxCoarse + 1];
    __shared__ uint64_t s_cur[kCount ? 1 : kPbMaxCoarse + 1];
    // window row t: stream position of its next entry (low word; high bits
    // with the element width in the top byte), first entry within the
    // window, contribution bits
    __shared__ uint4 s_row[kWin];
    __shared__ uint2 s_mk[kWinCap / 32];   // bitmap word, marks in the words before
    __shared__ uint16_t s_rowk[kWin];      // window row of the k-th row with entries
    __shared__ uint32_t s_wsum[kPbWaves], s_wnz[kPbWaves], s_wmk[kPbWaves];  // per-wave totals
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t w = blockIdx.x;
    const uint64_t e_end = m * (w + 1) / nwg;
    if constexpr (kCount) {
        for (uint32_t b = threadIdx.x; b < nf; b += kPbThreads) s_fhist[b] = 0;
    } else {
        for (uint32_t c = threadIdx.x; c < nc; c += kPbThreads) {
            s_hist[0][c] = s_hist[1][c] = 0;
            s_cur[c] = base1[(uint64_t)w * nc + c];
        }
    }
    // the next entry: row r0, entry k0 of its list, position e in the stream
    // (the same in every thread)
    uint32_t r0 = row_lo[w], k0 = k_lo[w];
    uint64_t e = m * w / nwg;
    uint32_t par = 0;
    // the number of bitmap marks at or before window entry j: the window row
    // of entry j is the one with that many marks
    auto row_of = [&](uint32_t j) -> uint32_t {
        const uint2 mk = s_mk[j >> 5];
        return s_rowk[mk.y + __popc(mk.x & (0xFFFFFFFFu >> (31u - (j & 31u)))) - 1];
    };
    while (e < e_end) {
        // -- the window
        if constexpr (kCount) lds_barrier();  // the last round's lookups are done
        const uint64_t a0 = r0 & ~(uint64_t)(kWave - 1);
        const uint64_t v = a0 + threadIdx.x;
        const VInfo vi = wave_info(acc, a0 + (uint64_t)wv * kWave, n);
        uint32_t d = (v >= r0 && v < n) ? vi.deg : 0u;
        uint64_t st = vi.start;
        if (v == r0) {
            d -= k0;
            st += (uint64_t)k0 * Acc::step(vi.w);
        }
        const float cl = cin[v < n ? v : n - 1];  // unconditional (see the entry loads below)
        const float cv = d ? cl : 0.f;
        // a row past the bitmap counts as kWinCap: the sum of 1,024 rows stays
        // in 32 bits, and every row the bitmap reaches keeps its exact start
        const uint32_t dc = d < kWinCap ? d : kWinCap;
        const uint32_t incl = wave_scan_dpp(dc);
        const uint32_t nzi = wave_scan_dpp(d ? 1u : 0u);
        if (lane == kWave - 1) {
            s_wsum[wv] = incl;
            s_wnz[wv] = nzi;
        }
        s_mk[threadIdx.x].x = 0;
        lds_barrier();
        // every wave scans the 16 wave totals itself (no barrier for a scan by one wave)
        uint32_t total, E, k_nz;
        {
            const uint32_t x = lane < kPbWaves ? s_wsum[lane] : 0u;
            const uint32_t y = lane < kPbWaves ? s_wnz[lane] : 0u;
            const uint32_t xi = wave_scan_dpp(x), yi = wave_scan_dpp(y);
            total = __builtin_amdgcn_readfirstlane(__shfl(xi, kPbWaves - 1, kWave));  // uniform: a scalar register
            E = __shfl(xi - x, wv, kWave) + incl - dc;
            k_nz = __shfl(yi - y, wv, kWave) + nzi - 1;
        }
        const uint32_t jn = total < kWinCap ? total : kWinCap;
        if (d) {
            if (E < kWinCap) atomicOr(&s_mk[E >> 5].x, 1u << (E & 31));
            s_rowk[k_nz] = (uint16_t)threadIdx.x;
        }
        s_row[threadIdx.x] = make_uint4((uint32_t)st, (uint32_t)(st >> 32) | (vi.w << 24), E, __float_as_uint(cv));
        lds_barrier();
        const uint32_t pc = __popc(s_mk[threadIdx.x].x);
        const uint32_t pci = wave_scan_dpp(pc);
        if (lane == kWave - 1) s_wmk[wv] = pci;
        lds_barrier();
        {
            const uint32_t x = lane < kPbWaves ? s_wmk[lane] : 0u;
            const uint32_t xi = wave_scan_dpp(x);
            s_mk[threadIdx.x].y = __shfl(xi - x, wv, kWave) + pci - pc;
        }
        lds_barrier();
        // where the next window starts
        uint32_t nr0, nk0;
        if (total < kWinCap) {  // the window's rows have no entries past its bitmap (a capped row makes total >= kWinCap)
            nr0 = (uint32_t)(a0 + kWin < n ? a0 + kWin : n);
            nk0 = 0;
        } else {  // the bitmap ends inside row t
            const uint32_t t = __builtin_amdgcn_readfirstlane(row_of(kWinCap - 1));
            nk0 = (a0 + t == r0 ? k0 : 0u) + (kWinCap - __builtin_amdgcn_readfirstlane(s_row[t].z));
            nr0 = (uint32_t)(a0 + t);
        }
        // -- rounds over the window's entries [j0, jn).  The next round's
        // list loads go out while this round sorts and writes; every thread
        // issues the same loads and stores in every round (idle slots read
        // stream position 0 with mask 0 and store to the sink entry m), so
        // that the wait for the next round's entries, on the counter that
        // loads and stores share in order, need not wait for this round's
        // stores
        auto round_len = [&](uint32_t jb, uint64_t eb) -> uint32_t {
            uint32_t R = jn - jb;
            if (R > kPb1Round) R = kPb1Round;
            const uint64_t left = e_end - eb;
            if (R > left) R = (uint32_t)left;
            return R;
        };
        // slot q of a round: the list words holding its entry, and its window
        // row | bit offset << 10 | width << 16 | valid << 31
        uint32_t nlo[kPb1Steps], nhi[kPb1Steps], nmeta[kPb1Steps];
        auto issue = [&](uint32_t jb, uint32_t Rb) {
            uint64_t pos[kPb1Steps];
#pragma unroll
            for (uint32_t q = 0; q < kPb1Steps; ++q) {
                const uint32_t i = threadIdx.x + q * kPbThreads;
                pos[q] = 0;
                nmeta[q] = 0;
                if (i < Rb) {
                    const uint32_t j = jb + i;
                    const uint32_t t = row_of(j);
                    const uint4 ri = s_row[t];
                    const uint32_t ww = ri.y >> 24;
                    const uint64_t rs = ((uint64_t)(ri.y & 0xFFFFFFu) << 32) | ri.x;
                    pos[q] = rs + (uint64_t)(j - ri.z) * Acc::step(ww);
                    nmeta[q] = t | (((uint32_t)pos[q] & 31u) << 10) | (ww << 16) | (1u << 31);
                }
            }
#pragma unroll
            for (uint32_t q = 0; q < kPb1Steps; ++q) {
                if constexpr (Acc::kPacked) {
                    const uint64_t k = pos[q] >> 5;  // the pad word keeps k + 1 in bounds
                    nlo[q] = acc.pv.A32[k];
                    nhi[q] = acc.pv.A32[k + 1];
                } else {
                    nlo[q] = acc.pv.col[pos[q]];
                    nhi[q] = 0;
                }
            }
        };
        // the round's entries from the loaded words (the loop is rotated:
        // each round's entries are taken at the end of the round before, where
        // only that round's stores follow their loads)
        uint32_t e_v[kPb1Steps], e_meta[kPb1Steps], e_rank[kPb1Steps];
        auto take = [&]() {
#pragma unroll
            for (uint32_t q = 0; q < kPb1Steps; ++q) {
                e_meta[q] = nmeta[q];
                if constexpr (Acc::kPacked) {
                    const uint32_t ww = (e_meta[q] >> 16) & 63u;
                    e_v[q] = __builtin_amdgcn_alignbit(nhi[q], nlo[q], (e_meta[q] >> 10) & 31u) & width_mask(ww);
                } else {
                    e_v[q] = nlo[q];
                }
            }
        };
        uint32_t j0 = 0;
        issue(0, e < e_end ? round_len(0, e) : 0u);
        take();
        while (j0 < jn && e < e_end) {
            const uint32_t R = round_len(j0, e);
#pragma unroll
            for (uint32_t q = 0; q < kPb1Steps; ++q) {
                e_rank[q] = 0;
                if (!(e_meta[q] >> 31)) continue;
                e_v[q] = e_v[q] < n ? e_v[q] : n - 1;  // a stored ID is < n; keeps a corrupt stream in bounds
                if constexpr (kCount) atomicAdd(&s_fhist[e_v[q] >> kFineShift], 1u);
                else e_rank[q] = atomicAdd(&s_hist[par][e_v[q] >> kCoarseShift], 1u);
            }
            {  // the next round of this window (none: every slot idle)
                const uint32_t jb = j0 + R;
                const uint64_t eb = e + R;
                issue(jb, (jb < jn && eb < e_end) ? round_len(jb, eb) : 0u);
            }
            if constexpr (!kCount) {
                lds_barrier();  // ranks taken; the last round's copy-out is done
                if (wv == 0) {
                    // the last round's counts move the cursors; this round's give the run starts
                    uint32_t carry = 0;
                    for (uint32_t c0 = 0; c0 < nc; c0 += kWave) {
                        const uint32_t c = c0 + lane;
                        uint32_t h = 0;
                        if (c < nc) {
                            s_cur[c] += s_hist[par ^ 1][c];
                            s_hist[par ^ 1][c] = 0;
                            h = s_hist[par][c];
                        }
                        const uint32_t hi = wave_scan_dpp(h);
                        if (c < nc) s_start[c] = carry + hi - h;
                        carry += __shfl(hi, kWave - 1, kWave);
                    }
                }
                lds_barrier();
#pragma unroll
                for (uint32_t q = 0; q < kPb1Steps; ++q)
                    if (e_meta[q] >> 31)
                        s_buf[s_start[e_v[q] >> kCoarseShift] + e_rank[q]] =
                            make_uint2(e_v[q], s_row[e_meta[q] & 0x3FFu].w);
                lds_barrier();
#pragma unroll
                for (uint32_t q = 0; q < kPb1Steps; ++q) {
                    const uint32_t i = threadIdx.x + q * kPbThreads;
                    const uint2 x = s_buf[i < R ? i : 0u];
                    const uint32_t c = x.x >> kCoarseShift;
                    const uint64_t dst = i < R ? s_cur[c] + (i - s_start[c]) : m;
                    buf1[dst] = make_uint2(x.x & ((1u << kCoarseShift) - 1u), x.y);
                }
                par ^= 1u;
            }
            j0 += R;
            e += R;
            take();
        }
        r0 = nr0;
        k0 = nk0;
    }
    if constexpr (kCount) {
        lds_barrier();
        for (uint32_t b = threadIdx.x; b < nf; b += kPbThreads) hist_out[(uint64_t)w * nf + b] = s_fhist[b];
    }
}

// ---------------------------------------------------------------------------
// level 2: one workgroup per kPb2Merge neighbouring level-1 regions
// (w .. w + kPb2Merge - 1, c), 64 fine bins.  Those regions are one range of
// the level-1 buffer (regions are placed coarse-major) and their chunks of
// every fine bin one range of the level-2 arrays (placed fine-major), so
// the workgroup streams them as one region.
// ---------------------------------------------------------------------------

static_assert(kSubBins == kWave, "level 2 scans its fine bins with one wave");
// level 2: one 1,024-thread workgroup per CU, 16 entries per thread, rounds
// of 16,384 entries (runs of 256 entries per fine bin)
constexpr uint32_t kPb2Threads = 1024;
constexpr uint32_t kPb2Steps = 16;
constexpr uint32_t kPb2Round = kPb2Threads * kPb2Steps;
constexpr uint32_t kPb2WavesPerEU = (kPb2Threads / kWave) / 4;

__global__ __launch_bounds__(kPb2Threads, kPb2WavesPerEU) void pb_bin2_kernel(const uint2 *__restrict__ buf1,
                                                                             const uint64_t *__restrict__ base1,
                                                                             const uint32_t *__restrict__ len1,
                                                                             const uint64_t *__restrict__ base2,
                                                                             uint16_t *__restrict__ loc2,
                                                                             float *__restrict__ val2,
                                                                             uint64_t sink, uint32_t nwg,
                                                                             uint32_t nc) {
    __shared__ uint2 s_buf[kPb2Round];  // entries sorted by fine bin (bits 14..19 of the local vertex)
    __shared__ uint32_t s_hist[2][kSubBins];
    __shared__ uint32_t s_start[kSubBins];
    __shared__ uint64_t s_cur[kSubBins];
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t w0 = blockIdx.x / nc * kPb2Merge, c = blockIdx.x % nc;
    const uint64_t r = (uint64_t)w0 * nc + c;  // the first of the merged regions
    const uint64_t b0 = base1[r];
    uint32_t len = 0;
    for (uint32_t k = 0; k < kPb2Merge && w0 + k < nwg; ++k) len += len1[r + (uint64_t)k * nc];
    if (threadIdx.x < kSubBins) {
        s_hist[0][threadIdx.x] = s_hist[1][threadIdx.x] = 0;
        s_cur[threadIdx.x] = base2[r * kSubBins + threadIdx.x];
    }
    // round k + 1's entries are loaded while round k is sorted and written.
    // Loads and stores share one in-order counter: so that the wait for the
    // next round's entries need not wait for this round's stores, every
    // thread issues the same loads and stores in every round (a slot past
    // the region reads its first entry, and stores to the sink entry m of
    // the level-2 arrays).
    uint2 nx[kPb2Steps];
    auto load = [&](uint32_t at) {
#pragma unroll
        for (uint32_t st = 0; st < kPb2Steps; ++st) {
            const uint32_t i = at + st * kPb2Threads + threadIdx.x;
            nx[st] = buf1[b0 + (i < len ? i : 0u)];
            if (i >= len) nx[st].x = 0xFFFFFFFFu;
        }
    };
    load(0);
    lds_barrier();
    uint32_t par = 0;
    for (uint32_t at = 0; at < len; at += kPb2Round) {
        uint2 e[kPb2Steps];
        uint32_t rank[kPb2Steps];
#pragma unroll
        for (uint32_t st = 0; st < kPb2Steps; ++st) {
            e[st] = nx[st];
            rank[st] = e[st].x != 0xFFFFFFFFu ? atomicAdd(&s_hist[par][e[st].x >> kFineShift], 1u) : 0u;
        }
        load(at + kPb2Round);  // past the region: slots marked empty
        lds_barrier();  // ranks taken; the last round's copy-out is done
        if (wv == 0) {  // the last round's counts move the cursors; this round's give the run starts
            s_cur[lane] += s_hist[par ^ 1][lane];
            s_hist[par ^ 1][lane] = 0;
            const uint32_t h = s_hist[par][lane];
            s_start[lane] = wave_scan_dpp(h) - h;
        }
        lds_barrier();
#pragma unroll
        for (uint32_t st = 0; st < kPb2Steps; ++st)
            if (e[st].x != 0xFFFFFFFFu) s_buf[s_start[e[st].x >> kFineShift] + rank[st]] = e[st];
        lds_barrier();
        const uint32_t total = len - at < kPb2Round ? len - at : kPb2Round;
#pragma unroll
        for (uint32_t st = 0; st < kPb2Steps; ++st) {
            const uint32_t i = st * kPb2Threads + threadIdx.x;
            const uint2 x = s_buf[i < total ? i : 0u];
            const uint32_t f = x.x >> kFineShift;
            const uint64_t at2 = i < total ? s_cur[f] + (i - s_start[f]) : sink;
            loc2[at2] = (uint16_t)(x.x & (kFine - 1u));
            val2[at2] = __uint_as_float(x.y);
        }
        par ^= 1u;
    }
}

// ---------------------------------------------------------------------------
// level 3: one workgroup per fine bin, exact sums, finalize
// ---------------------------------------------------------------------------

template <class Acc>
__global__ __launch_bounds__(kPbThreads) void pb_accum_kernel(Acc acc, uint32_t n, const uint64_t *__restrict__ fstart,
                                                              const uint16_t *__restrict__ loc2,
                                                              const float *__restrict__ val2, float base, float alpha,
                                                              const uint64_t *__restrict__ iso, float *__restrict__ cout,
                                                              float *__restrict__ scores,
                                                              const uint32_t *__restrict__ perm) {
    __shared__ unsigned long long s_acc[kFine];
    const uint32_t b = blockIdx.x;
    for (uint32_t i = threadIdx.x; i < kFine; i += kPbThreads) s_acc[i] = 0ull;
    lds_barrier();
    const uint64_t a = fstart[b], z = fstart[b + 1];
    constexpr uint32_t kIn = 8;  // independent loads in flight per thread (one workgroup per CU)
    for (uint64_t i = a + threadIdx.x; i < z; i += (uint64_t)kPbThreads * kIn) {
        // unconditional loads at clamped indexes: a load under a branch waits
        // for its data before the branch ends, one load per wave in flight
        uint32_t lv[kIn];
        float xv[kIn];
#pragma unroll
        for (uint32_t q = 0; q < kIn; ++q) {
            const uint64_t k = i + (uint64_t)q * kPbThreads;
            const uint64_t kk = k < z ? k : z - 1;
            lv[q] = loc2[kk];
            xv[q] = val2[kk];
        }
#pragma unroll
        for (uint32_t q = 0; q < kIn; ++q) {
            // a contribution is in [0, 1]: its fixed-point value fits
            const double x = (double)xv[q] * kFixScale;
            if (xv[q] != 0.0f && i + (uint64_t)q * kPbThreads < z)
                atomicAdd(&s_acc[lv[q] & (kFine - 1u)], (unsigned long long)__double2ll_rn(x));
        }
    }
    lds_barrier();
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t v_lo = (uint64_t)b * kFine;
    for (uint32_t q = wv; q < kFine / kWave; q += kPbWaves) {
        const uint64_t w0 = v_lo + (uint64_t)q * kWave;
        if (w0 >= n) break;
        const bool all_iso = iso[w0 / kWave] == ~0ull;
        if (all_iso && !scores) continue;
        const uint64_t v = w0 + lane;
        const VInfo vi = all_iso ? VInfo{0, 0, 0} : wave_info(acc, w0, n);
        if (v < n) {
            const double sum = (double)(long long)s_acc[q * kWave + lane] * kFixUnit;
            const float pr = (float)((double)base + (double)alpha * sum);
            if (!all_iso) cout[v] = vi.deg ? pr / (float)vi.deg : 0.0f;
            if (scores) scores[perm ? perm[v] : v] = pr;
        }
    }
}

// contrib_0 = PR_0 / d (0 for vertices without edges)
template <class Acc>
__global__ void pb_init_kernel(Acc acc, uint32_t n, double inv_n, float *__restrict__ ca, float *__restrict__ cb) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v0 = (uint64_t)blockIdx.x * blockDim.x; v0 < n; v0 += stride) {
        const uint64_t w0 = v0 + (threadIdx.x & ~(uint64_t)(kWave - 1));
        const uint64_t v = w0 + lane_id();
        const uint32_t deg = wave_info(acc, w0, n).deg;
        if (v < n) {
            const float c = deg ? (float)(inv_n / (double)deg) : 0.0f;
            ca[v] = c;
            cb[v] = c;
        }
    }
}

// ---------------------------------------------------------------------------
// region tables from the counting pass (hist[w][b]: workgroup w's entries in
// fine bin b = 64 c + f)
// ---------------------------------------------------------------------------

// level-1 region lengths len1[w][c], and the same counts in coarse-major
// order (c, w) for the scan that places the level-1 regions; the counts in
// fine-major order (b, w) for the scan that places the level-2 regions
__global__ void pb_tables_count_kernel(const uint32_t *__restrict__ hist, uint32_t nwg, uint32_t nc, uint32_t nf,
                                       uint32_t *__restrict__ len1, uint32_t *__restrict__ len1_cw,
                                       uint32_t *__restrict__ hist_bw) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t cells = (uint64_t)nwg * nf;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += stride) {
        const uint32_t w = (uint32_t)(i / nf), b = (uint32_t)(i % nf);
        hist_bw[(uint64_t)b * nwg + w] = hist[i];
    }
    const uint64_t regions = (uint64_t)nwg * nc;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < regions; i += stride) {
        const uint32_t w = (uint32_t)(i / nc), c = (uint32_t)(i % nc);
        uint32_t sum = 0;
        for (uint32_t b = c * kSubBins; b < (c + 1) * kSubBins && b < nf; ++b) sum += hist[(uint64_t)w * nf + b];
        len1[i] = sum;
        len1_cw[(uint64_t)c * nwg + w] = sum;
    }
}

// region starts from the two exclusive scans: base1[w][c] (level 1,
// coarse-major), base2[w][c][f] and fstart[b] (level 2, fine-major)
__global__ void pb_tables_place_kernel(const uint64_t *__restrict__ scan_cw, const uint64_t *__restrict__ scan_bw,
                                       uint32_t nwg, uint32_t nc, uint32_t nf, uint64_t *__restrict__ base1,
                                       uint64_t *__restrict__ base2, uint64_t *__restrict__ fstart) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t cells = (uint64_t)nwg * nc * kSubBins;  // base2 slots, fine bins past nf included
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += stride) {
        const uint32_t w = (uint32_t)(i / ((uint64_t)nc * kSubBins)), b = (uint32_t)(i % ((uint64_t)nc * kSubBins));
        base2[i] = b < nf ? scan_bw[(uint64_t)b * nwg + w] : scan_bw[(uint64_t)nf * nwg];
        if (w == 0 && b < nf) fstart[b] = scan_bw[(uint64_t)b * nwg];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) fstart[nf] = scan_bw[(uint64_t)nf * nwg];
    const uint64_t regions = (uint64_t)nwg * nc;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < regions; i += stride) {
        const uint32_t w = (uint32_t)(i / nc), c = (uint32_t)(i % nc);
        base1[i] = scan_cw[(uint64_t)c * nwg + w];
    }
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------

template <class Acc>
static lg_status pb_build(lg_graph *g, Acc acc, hipStream_t s) {
    PbWork &W = *g->pb;
    const uint32_t n = g->n;
    int cus = 0;
    LG_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
    W.nwg = (uint32_t)std::max(1, cus) * kPb1Grid;
    W.nf = (uint32_t)(((uint64_t)n + kFine - 1) >> kFineShift);
    W.nc = (W.nf + kSubBins - 1) / kSubBins;
    // first row of every level-1 workgroup's entry range, from the element
    // offsets (degrees, then a scan)
    {
        DevBuf deg, eoff, tmp;
        LG_TRY(deg.scratch((uint64_t)n * 4, s));
        LG_TRY(eoff.scratch(((uint64_t)n + 1) * 8, s));
        LG_LAUNCH(pb_degree_kernel<Acc>, grid_for(((uint64_t)n + 63) / 64 * kWave, 256, 1u << 16), 256, 0, s, acc,
                  n, deg.as<uint32_t>());
        LG_CHECK_LAUNCH();
        LG_TRY(exclusive_scan_u32(deg.as<uint32_t>(), eoff.as<uint64_t>(), n, tmp, s));
        LG_TRY(W.row_lo.scratch((uint64_t)W.nwg * 4, s));
        LG_TRY(W.k_lo.scratch((uint64_t)W.nwg * 4, s));
        LG_LAUNCH(pb_row_lo_kernel, grid_for(W.nwg, 256, 1u << 16), 256, 0, s, n, g->m, W.nwg,
                  (const uint64_t *)eoff.as<uint64_t>(), W.row_lo.as<uint32_t>(), W.k_lo.as<uint32_t>());
        LG_CHECK_LAUNCH();
        LG_CHECK_HIP(hipStreamSynchronize(s));  // the temporaries are freed here
    }
    // counting pass: entries of each workgroup per fine bin
    DevBuf hist;
    LG_TRY(hist.scratch((uint64_t)W.nwg * W.nf * 4, s));
    LG_LAUNCH((pb_bin1_kernel<Acc, true>), W.nwg, kPbThreads, W.nf * 4, s, acc, n, g->m, W.nwg,
              (const float *)W.ca.p, W.row_lo.as<uint32_t>(), W.k_lo.as<uint32_t>(), W.nc,
              (const uint64_t *)nullptr, (uint2 *)nullptr, W.nf, hist.as<uint32_t>());
    LG_CHECK_LAUNCH();
    // regions: coarse bin c's level-1 data is the concatenation over w of
    // region (w, c); fine bin b's level-2 data the concatenation over the
    // regions (w, c) of their part for b (both laid out by exclusive scans on
    // the device; the host reads back the two totals only)
    const uint32_t nwg = W.nwg, nc = W.nc, nf = W.nf;
    {
        DevBuf len1_cw, hist_bw, scan_cw, scan_bw, tmp;
        LG_TRY(W.len1.scratch((uint64_t)nwg * nc * 4, s));
        LG_TRY(W.base1.scratch((uint64_t)nwg * nc * 8, s));
        LG_TRY(W.base2.scratch((uint64_t)nwg * nc * kSubBins * 8, s));
        LG_TRY(W.fstart.scratch(((uint64_t)nf + 1) * 8, s));
        LG_TRY(len1_cw.scratch((uint64_t)nwg * nc * 4, s));
        LG_TRY(hist_bw.scratch((uint64_t)nwg * nf * 4, s));
        LG_TRY(scan_cw.scratch(((uint64_t)nwg * nc + 1) * 8, s));
        LG_TRY(scan_bw.scratch(((uint64_t)nwg * nf + 1) * 8, s));
        const uint32_t grid = grid_for((uint64_t)nwg * nc * kSubBins, 256, 1u << 14);
        LG_LAUNCH(pb_tables_count_kernel, grid, 256, 0, s, (const uint32_t *)hist.as<uint32_t>(), nwg, nc, nf,
                  W.len1.as<uint32_t>(), len1_cw.as<uint32_t>(), hist_bw.as<uint32_t>());
        LG_CHECK_LAUNCH();
        LG_TRY(exclusive_scan_u32(len1_cw.as<uint32_t>(), scan_cw.as<uint64_t>(), (uint64_t)nwg * nc, tmp, s));
        LG_TRY(exclusive_scan_u32(hist_bw.as<uint32_t>(), scan_bw.as<uint64_t>(), (uint64_t)nwg * nf, tmp, s));
        LG_LAUNCH(pb_tables_place_kernel, grid, 256, 0, s, (const uint64_t *)scan_cw.as<uint64_t>(),
                  (const uint64_t *)scan_bw.as<uint64_t>(), nwg, nc, nf, W.base1.as<uint64_t>(),
                  W.base2.as<uint64_t>(), W.fstart.as<uint64_t>());
        LG_CHECK_LAUNCH();
        uint64_t tot[2] = {0, 0};
        LG_CHECK_HIP(hipMemcpyAsync(&tot[0], scan_cw.as<uint64_t>() + (uint64_t)nwg * nc, 8, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipMemcpyAsync(&tot[1], scan_bw.as<uint64_t>() + (uint64_t)nwg * nf, 8, hipMemcpyDeviceToHost, s));
        LG_CHECK_HIP(hipStreamSynchronize(s));  // the temporaries are released here
        if (tot[0] != g->m || tot[1] != g->m) {
            set_error("lg_pagerank: propagation-blocking counts %llu, %llu differ from %llu entries",
                      (unsigned long long)tot[0], (unsigned long long)tot[1], (unsigned long long)g->m);
            return LG_ERR_DEVICE;
        }
    }
    // level 2 keeps a fine-bin vertex in 16 bits and its contribution in a
    // second array: 6 B per entry instead of 8 for level 2's writes and the
    // accumulation's reads
    // (one more entry in each: the sink that idle slots of a round store to)
    const uint64_t me = g->m + 1;
    W.val_off = (me * 2 + 255) & ~255ull;
    LG_TRY(pb_take_bins(g, me * 8, W.val_off + me * 4));
    W.built = true;
    return LG_OK;
}

lg_status pagerank_pb(lg_graph *g, float damping, uint32_t iters, float *scores, hipStream_t s) {
    if (!g->pb) {
        g->pb = new (std::nothrow) PbWork();
        if (!g->pb) { set_error("lg_pagerank: host allocation failed"); return LG_ERR_OOM; }
    }
    PbWork &W = *g->pb;
    const uint32_t n = g->n;
    if (W.ca.bytes < (uint64_t)n * 4) LG_TRY(W.ca.alloc((uint64_t)n * 4));
    if (W.cb.bytes < (uint64_t)n * 4) LG_TRY(W.cb.alloc((uint64_t)n * 4));
    const uint32_t *perm = g->relabel != LG_RELABEL_NONE ? g->perm.as<uint32_t>() : nullptr;
    const double nd = (double)n, a = damping, z = g->isolated;
    return dispatch_acc(g, [&](auto acc) -> lg_status {
        using Acc = decltype(acc);
        if (!W.built) LG_TRY(pb_build<Acc>(g, acc, s));
        float *cin = W.ca.as<float>(), *cout = W.cb.as<float>();
        LG_LAUNCH(pb_init_kernel<Acc>, grid_for(n, 256, 1u << 16), 256, 0, s, acc, n, 1.0 / nd, cin, cout);
        LG_CHECK_LAUNCH();
        double D = z / nd;
        for (uint32_t t = 0; t < iters; ++t) {
            const double b = (1.0 - a) / nd + a * D / nd;
            const bool last = t + 1 == iters;
            if (g->m) {
                LG_LAUNCH((pb_bin1_kernel<Acc, false>), W.nwg, kPbThreads, 0, s, acc, n, g->m, W.nwg,
                          (const float *)cin, W.row_lo.as<uint32_t>(), W.k_lo.as<uint32_t>(), W.nc,
                          W.base1.as<uint64_t>(), W.buf1.as<uint2>(), W.nf, (uint32_t *)nullptr);
                LG_CHECK_LAUNCH();
                LG_LAUNCH(pb_bin2_kernel, (W.nwg + kPb2Merge - 1) / kPb2Merge * W.nc, kPb2Threads, 0, s,
                          (const uint2 *)W.buf1.p, W.base1.as<uint64_t>(), W.len1.as<uint32_t>(),
                          W.base2.as<uint64_t>(), W.buf2.as<uint16_t>(), (float *)((char *)W.buf2.p + W.val_off),
                          g->m, W.nwg, W.nc);
                LG_CHECK_LAUNCH();
            }
            LG_LAUNCH(pb_accum_kernel<Acc>, W.nf, kPbThreads, 0, s, acc, n, W.fstart.as<uint64_t>(),
                      (const uint16_t *)W.buf2.p, (const float *)((char *)W.buf2.p + W.val_off), (float)b, (float)a,
                      g->iso.as<uint64_t>(), cout,
                      last ? scores : (float *)nullptr, last ? perm : (const uint32_t *)nullptr);
            LG_CHECK_LAUNCH();
            D = z * b;
            std::swap(cin, cout);
        }
        return LG_OK;
    });
}

}  // namespace lg
