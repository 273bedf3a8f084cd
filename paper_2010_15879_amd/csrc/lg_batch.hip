// lg_bfs_batch_*: many BFS queries over many (small) graphs in one
// persistent launch.
//
// Every workgroup is a worker: it takes the next job (graph, root) from a
// device counter, runs that BFS to the end itself (level-synchronous, with
// workgroup barriers between levels), and takes the next job until none is
// left -- so the exit condition is reached by every workgroup.  A level is
// taken `chunk` frontier vertices at a time: a vertex of degree below
// `wave_threshold` is expanded by one thread, a larger one by a whole wave
// (lanes over its list, coalesced).  Both knobs are picked per plan by
// timing candidate settings on the actual batch.  Visiting is the BFS rule
// of the single-query path (CAS on depth, smallest-label parent by
// atomicMin), so every result equals the per-query result bit for bit.
//
// A plan captures "reset the job counter + the persistent launch" in a HIP
// graph, replayed by lg_bfs_batch_run.
#include <algorithm>
#include <cstring>
#include <vector>

#include "lg_device.hpp"
#include "lg_varint.hpp"

struct lg_batch_plan;

namespace lg {

constexpr uint32_t kMaxChunk = 1024;

template <class Acc>
struct BatchGraph {
    Acc acc;
    uint32_t n;
};

struct BatchJob {
    uint32_t graph;
    uint32_t root;
    uint64_t out_offset;
};

template <class Acc>
__device__ __forceinline__ void batch_visit(uint32_t u, uint32_t v, int32_t nd, int32_t *__restrict__ D,
                                            uint32_t *__restrict__ P, uint32_t *__restrict__ qnext,
                                            uint32_t *s_tail) {
    // a plain read first: most edges of later levels reach vertices settled
    // at earlier levels, which the CAS would only confirm
    const int32_t seen = __builtin_nontemporal_load(&D[u]);
    if (seen != -1 && seen != nd) return;
    const int32_t old = atomicCAS(&D[u], -1, nd);
    if (P && (old == -1 || old == nd)) atomicMin(&P[u], v);
    if (old == -1) qnext[atomicAdd(s_tail, 1u)] = u;
}

template <class Acc, int kThreads>
__global__ __launch_bounds__(kThreads) void bfs_batch_kernel(
    const BatchGraph<Acc> *__restrict__ graphs, const BatchJob *__restrict__ jobs, uint32_t num_jobs,
    uint32_t *__restrict__ job_counter, int32_t *__restrict__ depth, int32_t *__restrict__ parent,
    int32_t max_depth, uint32_t *__restrict__ queues, uint64_t qcap, uint32_t chunk, uint32_t wave_threshold) {
    __shared__ uint32_t s_job, s_fsize, s_tail, s_nheavy;
    __shared__ uint32_t s_heavy[kMaxChunk];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wv = tid / kWave;
    constexpr uint32_t kWaves = kThreads / kWave;
    uint32_t *qa = queues + (uint64_t)blockIdx.x * 2 * qcap;
    uint32_t *qb = qa + qcap;
    for (;;) {
        if (tid == 0) s_job = atomicAdd(job_counter, 1u);
        __syncthreads();
        const uint32_t job = s_job;
        if (job >= num_jobs) break;
        const BatchJob jb = jobs[job];
        const BatchGraph<Acc> G = graphs[jb.graph];
        const uint32_t n = G.n;
        int32_t *D = depth + jb.out_offset;
        uint32_t *P = parent ? reinterpret_cast<uint32_t *>(parent + jb.out_offset) : nullptr;
        for (uint32_t v = tid; v < n; v += kThreads) {
            D[v] = v == jb.root ? 0 : -1;
            if (P) P[v] = v == jb.root ? jb.root : 0xFFFFFFFFu;
        }
        if (tid == 0) {
            qa[0] = jb.root;
            s_fsize = 1;
        }
        __syncthreads();
        int32_t level = 0;
        uint32_t *qin = qa, *qout = qb;
        for (;;) {
            const uint32_t F = s_fsize;
            if (F == 0 || (max_depth >= 0 && level >= max_depth)) break;
            __syncthreads();  // everyone has read s_fsize
            if (tid == 0) s_tail = 0;
            const int32_t nd = level + 1;
            for (uint32_t c0 = 0; c0 < F; c0 += chunk) {
                const uint32_t c1 = c0 + chunk < F ? c0 + chunk : F;
                if (tid == 0) s_nheavy = 0;
                __syncthreads();
                for (uint32_t i = c0 + tid; i < c1; i += kThreads) {
                    const uint32_t v = qin[i];
                    if constexpr (IsGapAcc<Acc>::value) {
                        // gap lists: a running sum of the differences
                        const GapInfo gi = G.acc.info(v);
                        if (gi.deg >= wave_threshold) {
                            s_heavy[atomicAdd(&s_nheavy, 1u)] = v;
                        } else {
                            uint32_t val = 0;
                            for (uint32_t e = 0; e < gi.deg; ++e) {
                                val += G.acc.get(Acc::entry_bit(gi, e), e ? gi.g : gi.w);
                                batch_visit<Acc>(val < n ? val : n - 1, v, nd, D, P, qout, &s_tail);
                            }
                        }
                    } else if constexpr (IsVarintAcc<Acc>::value) {
                        // Varint lists: bytes from 8-byte windows (the list's
                        // byte count stands in for its degree)
                        uint64_t b0, b1;
                        G.acc.offsets(v, b0, b1);
                        if (b1 - b0 >= wave_threshold) {
                            s_heavy[atomicAdd(&s_nheavy, 1u)] = v;
                        } else {
                            uint32_t label = 0, accv = 0, shift = 0, count = 0;
                            for (uint64_t pos = b0; pos < b1;) {
                                const uint64_t k = pos >> 3;
                                const uint32_t sh = (uint32_t)(pos & 7) * 8;
                                const uint64_t w0 = G.acc.word(k * 8), w1 = G.acc.word(k * 8 + 8);
                                const uint64_t win = sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0;
                                const uint32_t avail = b1 - pos < 8 ? (uint32_t)(b1 - pos) : 8u;
                                for (uint32_t j = 0; j < avail; ++j) {
                                    const uint32_t b = (uint32_t)(win >> (8 * j)) & 255u;
                                    accv |= (b & 127u) << shift;
                                    shift += 7;
                                    if (!(b & 128u)) {
                                        label = Acc::kDifferences && count ? label + accv : accv;
                                        ++count;
                                        accv = 0;
                                        shift = 0;
                                        batch_visit<Acc>(label < n ? label : n - 1, v, nd, D, P, qout, &s_tail);
                                    }
                                }
                                pos += avail;
                            }
                        }
                    } else {
                        const VInfo vi = G.acc.info(v);
                        if (vi.deg >= wave_threshold) {
                            s_heavy[atomicAdd(&s_nheavy, 1u)] = v;
                        } else {
                            const uint32_t st = Acc::step(vi.w), mk = Acc::mask(vi.w);
                            uint64_t pos = vi.start;
                            for (uint32_t e = 0; e < vi.deg; ++e, pos += st)
                                batch_visit<Acc>(G.acc.get(pos, mk), v, nd, D, P, qout, &s_tail);
                        }
                    }
                }
                __syncthreads();
                const uint32_t nh = s_nheavy;
                for (uint32_t h = wv; h < nh; h += kWaves) {
                    const uint32_t v = s_heavy[h];
                    if constexpr (IsGapAcc<Acc>::value) {
                        // 64 entries per step, a wave prefix sum
                        const GapInfo gi = G.acc.info(v);
                        uint32_t carry = 0;
                        for (uint64_t e0 = 0; e0 < gi.deg; e0 += kWave) {
                            const uint64_t e = e0 + lane;
                            const bool valid = e < gi.deg;
                            const uint32_t x = valid ? G.acc.get(Acc::entry_bit(gi, e), e ? gi.g : gi.w) : 0u;
                            const uint32_t val = wave_incl_scan(x) + carry;
                            carry = __shfl(val, kWave - 1, kWave);
                            if (valid) batch_visit<Acc>(val < n ? val : n - 1, v, nd, D, P, qout, &s_tail);
                        }
                    } else if constexpr (IsVarintAcc<Acc>::value) {
                        // 64 bytes per step (value assembly of varint_step)
                        uint64_t b0, b1;
                        G.acc.offsets(v, b0, b1);
                        uint32_t prevb = 0, carry = 0;
                        for (uint64_t p0 = b0; p0 < b1; p0 += kWave) {
                            uint32_t x;
                            const bool end = varint_step(G.acc, p0, b1, prevb, x);
                            uint32_t label = x;
                            if constexpr (Acc::kDifferences) {
                                const uint32_t sc = wave_incl_scan(end ? x : 0u);
                                label = carry + sc;
                                carry += __shfl(sc, kWave - 1, kWave);
                            }
                            if (end) batch_visit<Acc>(label < n ? label : n - 1, v, nd, D, P, qout, &s_tail);
                        }
                    } else {
                        const VInfo vi = G.acc.info(v);
                        const uint32_t st = Acc::step(vi.w), mk = Acc::mask(vi.w);
                        for (uint32_t e = lane; e < vi.deg; e += kWave)
                            batch_visit<Acc>(G.acc.get(vi.start + (uint64_t)e * st, mk), v, nd, D, P, qout,
                                             &s_tail);
                    }
                }
                __syncthreads();
            }
            if (tid == 0) s_fsize = s_tail;
            uint32_t *t = qin; qin = qout; qout = t;
            ++level;
            __syncthreads();
        }
        __syncthreads();  // s_job is rewritten next
    }
}

__global__ void batch_reset_kernel(uint32_t *__restrict__ counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

}  // namespace lg

// ---------------------------------------------------------------------------
// the plan
// ---------------------------------------------------------------------------

struct lg_batch_plan {
    int device = 0;
    uint32_t layout = 0, id_mode = 0, offset_mode = 0;
    uint32_t num_graphs = 0, num_jobs = 0;
    uint64_t qcap = 0;
    int32_t *depth = nullptr, *parent = nullptr;
    int32_t max_depth = -1;
    uint32_t threads = 256, chunk = 256, wave_threshold = 32, workgroups = 0;
    double tuned_ms = 0.0;
    uint32_t candidates = 0;
    lg::DevBuf graphs, jobs, counter, queues;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<lg_graph *> handles;  // the plan's graphs (each run is one use of each)
    hipEvent_t last_run = nullptr;    // recorded after every replay
};

namespace lg {

template <class Acc>
static lg_status batch_launch(lg_batch_plan *p, hipStream_t s) {
    LG_LAUNCH(batch_reset_kernel, 1, 64, 0, s, p->counter.as<uint32_t>());
    LG_CHECK_LAUNCH();
    const auto *G = p->graphs.as<const BatchGraph<Acc>>();
    const auto *J = p->jobs.as<const BatchJob>();
    if (p->threads == 256)
        LG_LAUNCH((bfs_batch_kernel<Acc, 256>), p->workgroups, 256, 0, s, G, J, p->num_jobs, p->counter.as<uint32_t>(),
                  p->depth, p->parent, p->max_depth, p->queues.as<uint32_t>(), p->qcap, p->chunk, p->wave_threshold);
    else
        LG_LAUNCH((bfs_batch_kernel<Acc, 512>), p->workgroups, 512, 0, s, G, J, p->num_jobs, p->counter.as<uint32_t>(),
                  p->depth, p->parent, p->max_depth, p->queues.as<uint32_t>(), p->qcap, p->chunk, p->wave_threshold);
    LG_CHECK_LAUNCH();
    return LG_OK;
}

template <class Acc>
static lg_status batch_workgroups(lg_batch_plan *p, uint32_t &wg) {
    int cus = 0, per = 0;
    LG_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device));
    if (p->threads == 256)
        LG_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, bfs_batch_kernel<Acc, 256>, 256, 0));
    else
        LG_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, bfs_batch_kernel<Acc, 512>, 512, 0));
    if (per < 1) per = 1;
    wg = (uint32_t)std::min<uint64_t>((uint64_t)cus * per, p->num_jobs ? p->num_jobs : 1);
    return LG_OK;
}

// (Re)allocate the per-workgroup queues for p->workgroups workers.
static lg_status batch_queues(lg_batch_plan *p) {
    return p->queues.ensure((uint64_t)p->workgroups * 2 * p->qcap * 4);
}

template <class Acc>
static lg_status batch_build(lg_batch_plan *p, const lg_graph *const *gs, bool autotune, hipStream_t s) {
    std::vector<BatchGraph<Acc>> hg(p->num_graphs);
    for (uint32_t i = 0; i < p->num_graphs; ++i) {
        const lg_graph *g = gs[i];
        if constexpr (IsGapAcc<Acc>::value || IsVarintAcc<Acc>::value) hg[i].acc = Acc{{g->packed_view()}};
        else if constexpr (Acc::kPacked) hg[i].acc = Acc{g->packed_view()};
        else hg[i].acc = Acc{g->plain_view()};
        hg[i].n = g->n;
    }
    LG_TRY(p->graphs.alloc(sizeof(BatchGraph<Acc>) * hg.size()));
    LG_CHECK_HIP(hipMemcpy(p->graphs.p, hg.data(), sizeof(BatchGraph<Acc>) * hg.size(), hipMemcpyHostToDevice));

    struct Cfg { uint32_t threads, chunk, wt; };
    std::vector<Cfg> cands;
    if (autotune) {
        for (uint32_t th : {256u, 512u})
            for (uint32_t ch : {256u, 1024u})
                for (uint32_t wt : {8u, 32u, 128u}) cands.push_back({th, ch, wt});
    } else {
        cands.push_back({p->threads, p->chunk, p->wave_threshold});
    }
    p->candidates = (uint32_t)cands.size();
    hipEvent_t e0, e1;
    LG_CHECK_HIP(hipEventCreate(&e0));
    LG_CHECK_HIP(hipEventCreate(&e1));
    float best = -1.f;
    Cfg bestc = cands[0];
    lg_status st = LG_OK;
    for (const Cfg &c : cands) {
        p->threads = c.threads;
        p->chunk = c.chunk;
        p->wave_threshold = c.wt;
        if ((st = batch_workgroups<Acc>(p, p->workgroups)) != LG_OK) break;
        if ((st = batch_queues(p)) != LG_OK) break;
        if (cands.size() > 1) {
            if ((st = batch_launch<Acc>(p, s)) != LG_OK) break;  // warm-up
        }
        (void)hipEventRecord(e0, s);
        if ((st = batch_launch<Acc>(p, s)) != LG_OK) break;
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) { st = LG_ERR_DEVICE; set_error("batch: sync failed"); break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (best < 0.f || ms < best) { best = ms; bestc = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    LG_TRY(st);
    p->threads = bestc.threads;
    p->chunk = bestc.chunk;
    p->wave_threshold = bestc.wt;
    p->tuned_ms = best;
    LG_TRY(batch_workgroups<Acc>(p, p->workgroups));
    LG_TRY(batch_queues(p));
    // capture reset + launch into a graph, on a private stream (the legacy
    // default stream cannot be captured; capturing executes nothing, and the
    // graph is launched later on the caller's stream)
    LG_CHECK_HIP(hipStreamSynchronize(s));
    hipStream_t cs = nullptr;
    LG_CHECK_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    hipGraph_t gr = nullptr;
    if (ce == hipSuccess) {
        st = batch_launch<Acc>(p, cs);
        ce = hipStreamEndCapture(cs, &gr);
    }
    (void)hipStreamDestroy(cs);
    LG_TRY(st);
    if (ce != hipSuccess) { set_error("batch: graph capture failed: %s", hipGetErrorString(ce)); return LG_ERR_DEVICE; }
    p->graph = gr;
    LG_CHECK_HIP(hipGraphInstantiate(&p->exec, gr, nullptr, nullptr, 0));
    return LG_OK;
}

}  // namespace lg

extern "C" lg_status lg_bfs_batch_plan(const lg_graph *const *graphs, uint32_t num_graphs, const lg_bfs_job *jobs,
                                       uint32_t num_jobs, int32_t *depth, int32_t *parent, int32_t max_depth,
                                       uint32_t flags, hipStream_t stream, lg_batch_plan **out) {
    using namespace lg;
    if (!out) { set_error("lg_bfs_batch_plan: out is NULL"); return LG_ERR_INVALID; }
    *out = nullptr;
    if (!graphs || !num_graphs || (num_jobs && (!jobs || !depth))) {
        set_error("lg_bfs_batch_plan: NULL argument");
        return LG_ERR_INVALID;
    }
    if (flags & ~(uint32_t)LG_BATCH_AUTOTUNE) { set_error("lg_bfs_batch_plan: unknown flags"); return LG_ERR_INVALID; }
    const lg_graph *g0 = graphs[0];
    uint64_t qcap = 1;
    for (uint32_t i = 0; i < num_graphs; ++i) {
        const lg_graph *g = graphs[i];
        if (!g) { set_error("lg_bfs_batch_plan: NULL graph"); return LG_ERR_INVALID; }
        if (g->layout != g0->layout || g->id_mode != g0->id_mode || g->offset_mode != g0->offset_mode ||
            (g->layout == LG_LAYOUT_PLAIN && g->poff64 != g0->poff64)) {
            set_error("lg_bfs_batch_plan: all graphs must share one layout and encoding");
            return LG_ERR_UNSUPPORTED;
        }
        if (g->relabel != LG_RELABEL_NONE) {
            set_error("lg_bfs_batch_plan: relabeled graphs are not supported in batches");
            return LG_ERR_UNSUPPORTED;
        }
        if (g->layout == LG_LAYOUT_PACKED && g->weighted) {
            set_error("lg_bfs_batch_plan: packed weighted graphs are read by lg_sssp only");
            return LG_ERR_UNSUPPORTED;
        }
        qcap = std::max<uint64_t>(qcap, g->n);
    }
    std::vector<BatchJob> hj(num_jobs);
    for (uint32_t j = 0; j < num_jobs; ++j) {
        if (jobs[j].graph >= num_graphs || jobs[j].root >= graphs[jobs[j].graph]->n) {
            set_error("lg_bfs_batch_plan: job %u has a bad graph index or root", j);
            return LG_ERR_INVALID;
        }
        hj[j] = BatchJob{jobs[j].graph, jobs[j].root, jobs[j].out_offset};
    }
    // largest graphs first: long jobs start early, short ones fill the tail
    std::stable_sort(hj.begin(), hj.end(), [&](const BatchJob &a, const BatchJob &b) {
        return graphs[a.graph]->m > graphs[b.graph]->m;
    });
    lg_batch_plan *p = new (std::nothrow) lg_batch_plan();
    if (!p) { set_error("lg_bfs_batch_plan: host allocation failed"); return LG_ERR_OOM; }
    lg_status st = LG_OK;
    do {
        if (hipGetDevice(&p->device) != hipSuccess) { st = LG_ERR_DEVICE; set_error("hipGetDevice failed"); break; }
        p->layout = g0->layout;
        p->id_mode = g0->id_mode;
        p->offset_mode = g0->offset_mode;
        p->num_graphs = num_graphs;
        p->num_jobs = num_jobs;
        p->qcap = qcap;
        p->depth = depth;
        p->parent = parent;
        p->max_depth = max_depth;
        for (uint32_t i = 0; i < num_graphs; ++i) p->handles.push_back(const_cast<lg_graph *>(graphs[i]));
        if (hipEventCreateWithFlags(&p->last_run, hipEventDisableTiming) != hipSuccess) {
            p->last_run = nullptr;
            st = LG_ERR_DEVICE;
            set_error("lg_bfs_batch_plan: hipEventCreateWithFlags failed");
            break;
        }
        if ((st = p->jobs.alloc(sizeof(BatchJob) * (num_jobs ? num_jobs : 1))) != LG_OK) break;
        if (num_jobs && hipMemcpy(p->jobs.p, hj.data(), sizeof(BatchJob) * num_jobs, hipMemcpyHostToDevice) != hipSuccess) {
            st = LG_ERR_DEVICE;
            set_error("lg_bfs_batch_plan: job upload failed");
            break;
        }
        if ((st = p->counter.alloc(8)) != LG_OK) break;
        st = dispatch_acc_dec(g0, [&](auto acc) -> lg_status {
            return batch_build<decltype(acc)>(p, graphs, (flags & LG_BATCH_AUTOTUNE) != 0, stream);
        });
    } while (0);
    if (st != LG_OK) {
        (void)hipStreamSynchronize(stream);
        lg_bfs_batch_free(p);
        return st;
    }
    *out = p;
    return LG_OK;
}

extern "C" lg_status lg_bfs_batch_run(lg_batch_plan *p, hipStream_t stream) {
    if (!p || !p->exec) { lg::set_error("lg_bfs_batch_run: bad plan"); return LG_ERR_INVALID; }
    LG_CHECK_HIP(hipGraphLaunch(p->exec, stream));
    // the plan's scratch and graphs are in use until this point of `stream`
    if (p->last_run) LG_CHECK_HIP(hipEventRecord(p->last_run, stream));
    for (lg_graph *g : p->handles) LG_TRY(lg::mark_use(g, stream));
    return LG_OK;
}

extern "C" lg_status lg_bfs_batch_info(const lg_batch_plan *p, lg_batch_info *out) {
    if (!p || !out) { lg::set_error("lg_bfs_batch_info: NULL argument"); return LG_ERR_INVALID; }
    std::memset(out, 0, sizeof(*out));
    out->num_jobs = p->num_jobs;
    out->workgroups = p->workgroups;
    out->threads = p->threads;
    out->chunk = p->chunk;
    out->wave_threshold = p->wave_threshold;
    out->candidates = p->candidates;
    out->tuned_ms = p->tuned_ms;
    out->scratch_bytes = p->queues.bytes;
    return LG_OK;
}

extern "C" void lg_bfs_batch_free(lg_batch_plan *p) {
    if (!p) return;
    // wait for the plan's own last replay, not for the whole device
    if (p->last_run) {
        (void)hipEventSynchronize(p->last_run);
        (void)hipEventDestroy(p->last_run);
    }
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
}
