// lg_server_*: a query server over graphs resident in HBM.
//
// Queries (neighbor-list fetch, k-hop expansion, full BFS) are submitted from
// any host thread and served by worker threads.  Each worker owns one HIP
// stream (default priority) and grow-only device workspaces, so queries run
// by different workers overlap on the device.  Before a worker runs a query it
// grows each of its buffers to the size that query can use at most, so the
// bytes it holds are known exactly before the launch.  Admission is FIFO: the
// query at the head starts on a free worker when the resident graphs plus
// every worker's buffers, after that growth, fit under the budget; a worker
// drops its own buffers, or asks idle workers to drop theirs, when that is
// what it takes; a query that could not fit even on an otherwise empty device
// is rejected (LG_ERR_CAPACITY).  A worker that takes a neighbor fetch also takes the
// other queued neighbor fetches on the same graph (up to max_batch) and
// serves them with one decode launch: requests that arrive while others run
// join the next batch.  Every result equals the result of the same query run
// alone (the kernels are deterministic).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lg_device.hpp"

namespace lg {

uint64_t bfs_bytes(const lg_graph *g);
uint64_t pr_bytes(const lg_graph *g);

// ---------------------------------------------------------------------------
// admission (host logic only; shared with lg_admission_simulate)
// ---------------------------------------------------------------------------

enum AdmitDecision { kAdmit, kShrink, kWait, kReclaim, kReject };

// Idle worker w looks at the head query.  need: bytes of the buffers the query
// uses, when the worker starts from nothing; grow: bytes the worker's total
// grows by if it keeps what it holds.  held[i]: bytes worker i holds;
// busy[i]: worker i is running a query.  Invariant: resident + sum(held) <=
// budget.
//   admit    the growth fits now
//   shrink   it fits once w drops its own buffers
//   reject   it cannot fit even if no worker held anything
//   reclaim  idle workers hold enough to make it fit: ask them to drop theirs
//   wait     only running workers could make room: wait for a completion
static AdmitDecision admit_decision(uint64_t budget, uint64_t resident, const std::vector<uint64_t> &held,
                                    const std::vector<bool> &busy, uint32_t w, uint64_t need, uint64_t grow) {
    uint64_t in_use = resident;
    for (uint64_t h : held) in_use += h;
    const uint64_t others = in_use - held[w];
    if (in_use + grow <= budget) return kAdmit;
    if (others + need <= budget) return kShrink;
    if (resident + need > budget) return kReject;
    uint64_t idle_other = 0;
    bool any_busy = false;
    for (size_t i = 0; i < held.size(); ++i) {
        if (i == w) continue;
        if (busy[i]) any_busy = true;
        else idle_other += held[i];
    }
    if (idle_other > 0 && (others - idle_other + need <= budget || !any_busy)) return kReclaim;
    return any_busy ? kWait : kReject;  // not reachable without busy workers: would have fit
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// vertices v with 1 <= depth[v] <= k, ascending: wave q handles v in [64q, 64q+64)
__global__ void khop_count_kernel(uint32_t n, const int32_t *__restrict__ depth, int32_t k,
                                  uint32_t *__restrict__ cnt) {
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    const uint32_t lane = lane_id();
    for (uint64_t q = wave; q < words; q += nwaves) {
        const uint64_t v = q * 64 + lane;
        const int32_t d = v < n ? depth[v] : -1;
        const uint64_t m = __ballot(d >= 1 && d <= k);
        if (lane == 0) cnt[q] = (uint32_t)__popcll(m);
    }
}

__global__ void khop_write_kernel(uint32_t n, const int32_t *__restrict__ depth, int32_t k,
                                  const uint64_t *__restrict__ woff, uint32_t *__restrict__ out) {
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    const uint32_t lane = lane_id();
    for (uint64_t q = wave; q < words; q += nwaves) {
        const uint64_t v = q * 64 + lane;
        const int32_t d = v < n ? depth[v] : -1;
        const bool in = d >= 1 && d <= k;
        const uint64_t m = __ballot(in);
        if (in) out[woff[q] + popc_below(m)] = (uint32_t)v;
    }
}

__device__ __forceinline__ uint64_t mix_u64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// order-independent digest of a BFS result: sum over v of mix(v, depth, parent),
// plus the reached count and the largest depth
__global__ void bfs_digest_kernel(uint32_t n, const int32_t *__restrict__ depth, const int32_t *__restrict__ parent,
                                  unsigned long long *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long dig = 0, reached = 0;
    int32_t mx = -1;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t d = depth[v];
        const int32_t p = parent ? parent[v] : 0;
        dig += mix_u64((v << 32) ^ ((uint64_t)(uint32_t)d * 0x9E3779B97F4A7C15ull) ^ (uint64_t)(uint32_t)p);
        reached += d >= 0;
        mx = d > mx ? d : mx;
    }
    dig = block_sum_u64(dig);
    reached = block_sum_u64(reached);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const int32_t t = __shfl_xor(mx, o, kWave);
        mx = t > mx ? t : mx;
    }
    __shared__ int32_t s_mx[16];
    if (lane_id() == 0) s_mx[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t w = 1; w < blockDim.x / kWave; ++w) mx = s_mx[w] > mx ? s_mx[w] : mx;
        atomicAdd(&out[0], dig);
        atomicAdd(&out[1], reached);
        atomicMax(reinterpret_cast<int *>(&out[2]), mx);
    }
}

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace lg

// ---------------------------------------------------------------------------
// the server
// ---------------------------------------------------------------------------

struct lg_server {
    struct Query {
        uint64_t ticket;
        lg_query q;
        double t_submit;
    };
    struct Result {
        lg_query_result r{};
        std::vector<uint32_t> ids;
        std::vector<int32_t> depth, parent;
    };
    struct Worker {
        std::thread th;
        hipStream_t stream = nullptr;
        lg::BfsWork bfs;
        lg::DecodeWork dec;
        lg::DevBuf depth, parent, vin, off, ids, kcnt, koff, dig, scan_tmp;
        uint64_t *pinned = nullptr;  // host staging for small readbacks
        uint64_t bytes() const {
            return bfs.bytes() + dec.bytes() + depth.bytes + parent.bytes + vin.bytes + off.bytes + ids.bytes +
                   kcnt.bytes + koff.bytes + dig.bytes + scan_tmp.bytes;
        }
        void drop() {
            bfs.~BfsWork();
            new (&bfs) lg::BfsWork();
            dec.~DecodeWork();
            new (&dec) lg::DecodeWork();
            depth.release(); parent.release(); vin.release(); off.release(); ids.release();
            kcnt.release(); koff.release(); dig.release(); scan_tmp.release();
        }
    };
    // one buffer of a worker and the size a query can grow it to at most
    struct Reserve {
        lg::DevBuf *buf;
        uint64_t bytes;
    };

    int device = 0;
    std::vector<lg_graph *> graphs;
    uint64_t budget = 0, resident = 0, peak = 0;
    uint32_t max_batch = 64;
    uint32_t overruns = 0;  // a worker held more than admission accounted for (never expected)
    std::mutex mu;
    std::condition_variable cv;  // every state change: queue, completion, release
    std::deque<Query> pending;
    std::unordered_map<uint64_t, Result> done;
    std::deque<uint64_t> completed_order;
    std::vector<Worker *> workers;
    std::vector<uint64_t> held;
    std::vector<bool> busy;
    std::vector<bool> release_req;
    uint64_t next_ticket = 1, submitted = 0, completed = 0, rejected = 0, batches = 0;
    bool stop = false;

    void plan(Worker &W, const lg_query &q, uint32_t batch, std::vector<Reserve> &out) const;
    void run_worker(uint32_t w);
    lg_status serve_neighbors(Worker &W, lg_graph *g, const std::vector<Query> &qs, std::vector<Result> &res);
    lg_status serve_bfs(Worker &W, lg_graph *g, const Query &q, Result &res);
};

// The buffers a query uses and the most each can be grown to while it runs
// (the same sizes bfs_workspace_ensure, decode_run and the scans and sorts
// ask for, at their largest for this graph and batch).
void lg_server::plan(Worker &W, const lg_query &q, uint32_t batch, std::vector<Reserve> &out) const {
    using namespace lg;
    const lg_graph *g = graphs[q.graph];
    const uint64_t n = g->n;
    const bool rel = g->relabel != LG_RELABEL_NONE;
    out.clear();
    if (q.kind == LG_QUERY_NEIGHBORS) {
        const uint64_t k = batch;
        const uint64_t cap = k * std::max<uint32_t>(g->max_degree, 1);
        out.push_back({&W.vin, k * 4});
        out.push_back({&W.off, (k + 1) * 8});
        out.push_back({&W.ids, cap * 4});
        out.push_back({&W.dec.head, (k * 8 + 8 + 7) & ~7ull});
        out.push_back({&W.dec.scan_tmp, scan_tmp_bytes(k)});
        if (rel) {  // sorted output of a relabeled graph: keyed radix sort
            out.push_back({&W.dec.keys, cap * 8});
            out.push_back({&W.dec.keys2, cap * 8});
            out.push_back({&W.dec.vals, cap * 4});
            out.push_back({&W.dec.vals2, cap * 4});
            out.push_back({&W.dec.sort_tmp, radix_sort_tmp_bytes(cap)});
        }
        return;
    }
    const bool khop = q.kind == LG_QUERY_KHOP;
    const uint64_t words = (n + 63) / 64;
    const uint64_t nh = g->n_heavy ? g->n_heavy : 1;
    BfsWork &b = W.bfs;
    out.push_back({&b.qa, n * 4});
    out.push_back({&b.qb, n * 4});
    out.push_back({&b.fstart, n * 8});
    out.push_back({&b.fdeg, n * 4});
    out.push_back({&b.fw, n * 4});
    out.push_back({&b.fscan, (n + 1) * 8});
    out.push_back({&b.visited, words * 8});
    out.push_back({&b.curr, words * 8});
    out.push_back({&b.next, words * 8});
    out.push_back({&b.counters, 8 * 8});
    out.push_back({&b.sample, 8 * 8});
    out.push_back({&b.pv, nh * 4});
    out.push_back({&b.pstart, nh * 8});
    out.push_back({&b.pdeg, nh * 4});
    out.push_back({&b.pw, nh * 4});
    out.push_back({&b.pseg_cnt, nh * 4});
    out.push_back({&b.pseg_off, (nh + 1) * 8});
    out.push_back({&b.scan_tmp, scan_tmp_bytes(std::max<uint64_t>(n, nh))});
    if (rel) {
        out.push_back({&b.depth_i, n * 4});
        if (!khop) out.push_back({&b.parent_i, n * 4});
    }
    out.push_back({&W.depth, n * 4});
    if (khop) {
        out.push_back({&W.kcnt, words * 4});
        out.push_back({&W.koff, (words + 1) * 8});
        out.push_back({&W.scan_tmp, scan_tmp_bytes(words)});
        out.push_back({&W.ids, std::max<uint64_t>(n, 1) * 4});
    } else {
        out.push_back({&W.parent, n * 4});
        out.push_back({&W.dig, 3 * 8});
    }
}

lg_status lg_server::serve_neighbors(Worker &W, lg_graph *g, const std::vector<Query> &qs,
                                     std::vector<Result> &res) {
    using namespace lg;
    const uint32_t k = (uint32_t)qs.size();
    const uint64_t cap = (uint64_t)k * std::max<uint32_t>(g->max_degree, 1);
    LG_TRY(W.vin.ensure((uint64_t)k * 4));
    LG_TRY(W.off.ensure(((uint64_t)k + 1) * 8));
    LG_TRY(W.ids.ensure(cap * 4));
    std::vector<uint32_t> vs(k);
    for (uint32_t i = 0; i < k; ++i) vs[i] = qs[i].q.vertex;
    LG_CHECK_HIP(hipMemcpyAsync(W.vin.p, vs.data(), (uint64_t)k * 4, hipMemcpyHostToDevice, W.stream));
    uint64_t total = 0;
    LG_TRY(decode_run(g, W.dec, W.vin.as<uint32_t>(), k, W.off.as<uint64_t>(), W.ids.as<uint32_t>(), cap,
                      LG_DECODE_SORTED, W.stream, &total));
    std::vector<uint64_t> off(k + 1);
    LG_CHECK_HIP(hipMemcpyAsync(off.data(), W.off.p, ((uint64_t)k + 1) * 8, hipMemcpyDeviceToHost, W.stream));
    std::vector<uint32_t> ids(total);
    if (total) LG_CHECK_HIP(hipMemcpyAsync(ids.data(), W.ids.p, total * 4, hipMemcpyDeviceToHost, W.stream));
    LG_CHECK_HIP(hipStreamSynchronize(W.stream));
    for (uint32_t i = 0; i < k; ++i) {
        res[i].ids.assign(ids.begin() + off[i], ids.begin() + off[i + 1]);
        res[i].r.count = off[i + 1] - off[i];
    }
    return LG_OK;
}

lg_status lg_server::serve_bfs(Worker &W, lg_graph *g, const Query &q, Result &res) {
    using namespace lg;
    const uint64_t n = g->n;
    const bool khop = q.q.kind == LG_QUERY_KHOP;
    LG_TRY(W.depth.ensure(n * 4));
    if (!khop) LG_TRY(W.parent.ensure(n * 4));
    const uint32_t root = q.q.vertex;
    LG_TRY(bfs_run(g, W.bfs, &root, 1, W.depth.as<int32_t>(), khop ? nullptr : W.parent.as<int32_t>(),
                   khop ? q.q.k : -1, LG_BFS_DIRECTION_OPT, W.stream, kBfsAlphaShared));
    res.r.n = n;
    if (khop) {
        const uint64_t words = (n + 63) / 64;
        LG_TRY(W.kcnt.ensure(words * 4));
        LG_TRY(W.koff.ensure((words + 1) * 8));
        LG_LAUNCH(khop_count_kernel, grid_for(words * kWave, 256, 4096), 256, 0, W.stream, (uint32_t)n,
                  W.depth.as<int32_t>(), q.q.k, W.kcnt.as<uint32_t>());
        LG_CHECK_LAUNCH();
        LG_TRY(exclusive_scan_u32(W.kcnt.as<uint32_t>(), W.koff.as<uint64_t>(), words, W.scan_tmp, W.stream));
        LG_CHECK_HIP(hipMemcpyAsync(W.pinned, W.koff.as<uint64_t>() + words, 8, hipMemcpyDeviceToHost, W.stream));
        LG_CHECK_HIP(hipStreamSynchronize(W.stream));
        const uint64_t cnt = W.pinned[0];
        LG_TRY(W.ids.ensure(std::max<uint64_t>(cnt, 1) * 4));
        LG_LAUNCH(khop_write_kernel, grid_for(words * kWave, 256, 4096), 256, 0, W.stream, (uint32_t)n,
                  W.depth.as<int32_t>(), q.q.k, W.koff.as<uint64_t>(), W.ids.as<uint32_t>());
        LG_CHECK_LAUNCH();
        res.ids.resize(cnt);
        if (cnt) LG_CHECK_HIP(hipMemcpyAsync(res.ids.data(), W.ids.p, cnt * 4, hipMemcpyDeviceToHost, W.stream));
        LG_CHECK_HIP(hipStreamSynchronize(W.stream));
        res.r.count = cnt;
        return LG_OK;
    }
    LG_TRY(W.dig.ensure(3 * 8));
    LG_TRY(fill_u64(W.dig.as<uint64_t>(), 0, 2, W.stream));
    LG_TRY(fill_u64(W.dig.as<uint64_t>() + 2, 0xFFFFFFFFull, 1, W.stream));  // max depth starts at -1
    LG_LAUNCH(bfs_digest_kernel, grid_for(n, 256, 4096), 256, 0, W.stream, (uint32_t)n, W.depth.as<int32_t>(),
              W.parent.as<int32_t>(), W.dig.as<unsigned long long>());
    LG_CHECK_LAUNCH();
    LG_CHECK_HIP(hipMemcpyAsync(W.pinned, W.dig.p, 24, hipMemcpyDeviceToHost, W.stream));
    if (q.q.flags & LG_QUERY_KEEP_ARRAYS) {
        res.depth.resize(n);
        res.parent.resize(n);
        LG_CHECK_HIP(hipMemcpyAsync(res.depth.data(), W.depth.p, n * 4, hipMemcpyDeviceToHost, W.stream));
        LG_CHECK_HIP(hipMemcpyAsync(res.parent.data(), W.parent.p, n * 4, hipMemcpyDeviceToHost, W.stream));
    }
    LG_CHECK_HIP(hipStreamSynchronize(W.stream));
    res.r.digest = W.pinned[0];
    res.r.count = W.pinned[1];
    res.r.max_depth = (int32_t)(uint32_t)W.pinned[2];
    return LG_OK;
}

void lg_server::run_worker(uint32_t w) {
    using namespace lg;
    (void)hipSetDevice(device);
    Worker &W = *workers[w];
    std::vector<Reserve> rsv;
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        if (release_req[w]) {  // drop buffers (asked by a worker that needs the room)
            release_req[w] = false;
            lk.unlock();
            (void)hipStreamSynchronize(W.stream);
            W.drop();
            lk.lock();
            held[w] = 0;
            cv.notify_all();
            continue;
        }
        if (stop) break;
        if (pending.empty()) {
            cv.wait(lk);
            continue;
        }
        // head of the queue, plus the queued neighbor fetches on the same graph
        const Query head = pending.front();
        uint32_t batch = 1;
        if (head.q.kind == LG_QUERY_NEIGHBORS) {
            for (size_t i = 1; i < pending.size() && batch < max_batch; ++i)
                if (pending[i].q.kind == LG_QUERY_NEIGHBORS && pending[i].q.graph == head.q.graph) ++batch;
        }
        AdmitDecision d;
        uint64_t grow = 0;
        while (true) {  // a batch that could never fit is halved before anything is rejected
            plan(W, head.q, batch, rsv);
            uint64_t need = 0;
            grow = 0;
            for (const Reserve &r : rsv) {
                need += r.bytes;
                grow += r.bytes > r.buf->bytes ? r.bytes - r.buf->bytes : 0;
            }
            d = admit_decision(budget, resident, held, busy, w, need, grow);
            if (d != kReject || batch == 1) break;
            batch = (batch + 1) / 2;
        }
        if (d == kReject) {
            pending.pop_front();
            Result res;
            res.r.status = LG_ERR_CAPACITY;
            res.r.kind = head.q.kind;
            res.r.queue_ms = res.r.latency_ms = now_ms() - head.t_submit;
            done[head.ticket] = std::move(res);
            completed_order.push_back(head.ticket);
            ++rejected;
            ++completed;
            cv.notify_all();
            continue;
        }
        if (d == kShrink) {  // drop own buffers, then look at the queue again
            lk.unlock();
            (void)hipStreamSynchronize(W.stream);
            W.drop();
            lk.lock();
            held[w] = 0;
            cv.notify_all();
            continue;
        }
        if (d == kReclaim) {
            for (size_t i = 0; i < workers.size(); ++i)
                if (i != w && !busy[i] && held[i] > 0) release_req[i] = true;
            cv.notify_all();
            cv.wait(lk);
            continue;
        }
        if (d == kWait) {
            cv.wait(lk);
            continue;
        }
        // admitted: take the queries, account the bytes, grow the buffers, run unlocked
        std::vector<Query> qs;
        qs.push_back(head);
        pending.pop_front();
        if (head.q.kind == LG_QUERY_NEIGHBORS) {
            for (auto it = pending.begin(); it != pending.end() && qs.size() < batch;) {
                if (it->q.kind == LG_QUERY_NEIGHBORS && it->q.graph == head.q.graph) {
                    qs.push_back(*it);
                    it = pending.erase(it);
                } else {
                    ++it;
                }
            }
        }
        held[w] += grow;
        uint64_t in_use = resident;
        for (uint64_t h : held) in_use += h;
        peak = std::max(peak, in_use);
        busy[w] = true;
        ++batches;
        lk.unlock();

        const double t_start = now_ms();
        lg_graph *g = graphs[head.q.graph];
        std::vector<Result> res(qs.size());
        lg_status st = LG_OK;
        for (const Reserve &r : rsv)
            if (st == LG_OK) st = r.buf->ensure(r.bytes);
        if (st == LG_OK) {
            if (head.q.kind == LG_QUERY_NEIGHBORS) st = serve_neighbors(W, g, qs, res);
            else st = serve_bfs(W, g, qs[0], res[0]);
        }
        const double t_end = now_ms();
        const uint64_t actual = W.bytes();

        lk.lock();
        if (actual > held[w]) ++overruns;
        held[w] = std::max(held[w], actual);
        busy[w] = false;
        for (size_t i = 0; i < qs.size(); ++i) {
            Result &r = res[i];
            r.r.status = st;
            r.r.kind = qs[i].q.kind;
            r.r.batch = (uint32_t)qs.size();
            r.r.queue_ms = t_start - qs[i].t_submit;
            r.r.service_ms = t_end - t_start;
            r.r.latency_ms = t_end - qs[i].t_submit;
            done[qs[i].ticket] = std::move(r);
            completed_order.push_back(qs[i].ticket);
            ++completed;
        }
        cv.notify_all();
    }
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" lg_status lg_server_create(const lg_graph *const *graphs, uint32_t num_graphs, const lg_server_opts *opts,
                                      lg_server **out) {
    using namespace lg;
    if (!out || !graphs || !num_graphs) { set_error("lg_server_create: NULL argument"); return LG_ERR_INVALID; }
    *out = nullptr;
    lg_server_opts o{};
    if (opts) o = *opts;
    if (o.workers == 0) o.workers = 8;
    if (o.max_batch == 0) o.max_batch = 64;
    lg_server *S = new (std::nothrow) lg_server();
    if (!S) { set_error("lg_server_create: host allocation failed"); return LG_ERR_OOM; }
    (void)hipGetDevice(&S->device);
    for (uint32_t i = 0; i < num_graphs; ++i) {
        if (!graphs[i]) { delete S; set_error("lg_server_create: NULL graph"); return LG_ERR_INVALID; }
        S->graphs.push_back(const_cast<lg_graph *>(graphs[i]));
    }
    for (lg_graph *g : S->graphs) S->resident += g->device_bytes() + bfs_bytes(g) + pr_bytes(g);
    S->budget = o.budget_bytes ? o.budget_bytes : ~0ull;
    S->max_batch = o.max_batch;
    if (S->resident > S->budget) {
        delete S;
        set_error("lg_server_create: the resident graphs alone exceed the budget");
        return LG_ERR_CAPACITY;
    }
    S->held.assign(o.workers, 0);
    S->busy.assign(o.workers, false);
    S->release_req.assign(o.workers, false);
    lg_status st = LG_OK;
    for (uint32_t w = 0; w < o.workers && st == LG_OK; ++w) {
        auto *W = new (std::nothrow) lg_server::Worker();
        if (!W) { st = LG_ERR_OOM; set_error("lg_server_create: host allocation failed"); break; }
        S->workers.push_back(W);
        if (hipStreamCreateWithFlags(&W->stream, hipStreamNonBlocking) != hipSuccess ||
            hipHostMalloc((void **)&W->pinned, 8 * sizeof(uint64_t)) != hipSuccess) {
            st = LG_ERR_DEVICE;
            set_error("lg_server_create: stream or pinned allocation failed");
        }
    }
    if (st != LG_OK) {
        for (auto *W : S->workers) {
            if (W->stream) (void)hipStreamDestroy(W->stream);
            if (W->pinned) (void)hipHostFree(W->pinned);
            delete W;
        }
        delete S;
        return st;
    }
    for (uint32_t w = 0; w < o.workers; ++w) S->workers[w]->th = std::thread([S, w] { S->run_worker(w); });
    *out = S;
    return LG_OK;
}

extern "C" lg_status lg_server_submit(lg_server *S, const lg_query *q, uint64_t *ticket) {
    using namespace lg;
    if (!S || !q || !ticket) { set_error("lg_server_submit: NULL argument"); return LG_ERR_INVALID; }
    if (q->kind > LG_QUERY_BFS || q->graph >= S->graphs.size() || q->vertex >= S->graphs[q->graph]->n ||
        (q->kind == LG_QUERY_KHOP && q->k < 0)) {
        set_error("lg_server_submit: bad query");
        return LG_ERR_INVALID;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    *ticket = S->next_ticket++;
    S->pending.push_back(lg_server::Query{*ticket, *q, now_ms()});
    ++S->submitted;
    S->cv.notify_all();
    return LG_OK;
}

static void fill_result(lg_server::Result &r, lg_query_result *out) {
    *out = r.r;
    out->ids = r.ids.empty() ? nullptr : r.ids.data();
    out->depth = r.depth.empty() ? nullptr : r.depth.data();
    out->parent = r.parent.empty() ? nullptr : r.parent.data();
}

extern "C" lg_status lg_server_wait(lg_server *S, uint64_t ticket, lg_query_result *out) {
    if (!S || !out) { lg::set_error("lg_server_wait: NULL argument"); return LG_ERR_INVALID; }
    std::unique_lock<std::mutex> lk(S->mu);
    if (ticket == 0 || ticket >= S->next_ticket) { lg::set_error("lg_server_wait: unknown ticket"); return LG_ERR_INVALID; }
    while (S->done.find(ticket) == S->done.end()) S->cv.wait(lk);
    fill_result(S->done[ticket], out);
    return LG_OK;
}

extern "C" lg_status lg_server_result(lg_server *S, uint64_t ticket, lg_query_result *out) {
    if (!S || !out) { lg::set_error("lg_server_result: NULL argument"); return LG_ERR_INVALID; }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->done.find(ticket);
    if (it == S->done.end()) { lg::set_error("lg_server_result: not completed"); return LG_ERR_INVALID; }
    fill_result(it->second, out);
    return LG_OK;
}

extern "C" lg_status lg_server_poll(lg_server *S, uint64_t *tickets, uint32_t cap, uint32_t *count) {
    if (!S || !count || (cap && !tickets)) { lg::set_error("lg_server_poll: NULL argument"); return LG_ERR_INVALID; }
    std::lock_guard<std::mutex> lk(S->mu);
    uint32_t c = 0;
    while (c < cap && !S->completed_order.empty()) {
        tickets[c++] = S->completed_order.front();
        S->completed_order.pop_front();
    }
    *count = c;
    return LG_OK;
}

extern "C" lg_status lg_server_release(lg_server *S, uint64_t ticket) {
    if (!S) { lg::set_error("lg_server_release: NULL argument"); return LG_ERR_INVALID; }
    std::lock_guard<std::mutex> lk(S->mu);
    S->done.erase(ticket);
    return LG_OK;
}

extern "C" lg_status lg_server_get_stats(lg_server *S, lg_server_stats *out) {
    if (!S || !out) { lg::set_error("lg_server_get_stats: NULL argument"); return LG_ERR_INVALID; }
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->rejected = S->rejected;
    out->queued = S->pending.size();
    uint64_t running = 0, in_use = S->resident;
    for (size_t i = 0; i < S->busy.size(); ++i) {
        running += S->busy[i];
        in_use += S->held[i];
    }
    out->running = running;
    out->budget_bytes = S->budget;
    out->resident_bytes = S->resident;
    out->in_use_bytes = in_use;
    out->peak_bytes = S->peak;
    out->workers = (uint32_t)S->workers.size();
    out->overruns = S->overruns;
    out->batches = S->batches;
    return LG_OK;
}

extern "C" void lg_server_free(lg_server *S) {
    if (!S) return;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        // drain: every submitted query completes first
        while (S->completed < S->submitted) S->cv.wait(lk);
        S->stop = true;
        S->cv.notify_all();
    }
    for (auto *W : S->workers) {
        if (W->th.joinable()) W->th.join();
        (void)hipStreamSynchronize(W->stream);
        (void)hipStreamDestroy(W->stream);
        (void)hipHostFree(W->pinned);
        delete W;
    }
    delete S;
}

// Host-only admission simulator: FIFO queries with arrival times, buffer
// sizes and fixed service times on `workers` workers, using the server's
// admission rule (without batching; each worker holds one grow-only buffer).  Outputs start/finish times, the
// per-query status (LG_OK or LG_ERR_CAPACITY) and the peak accounted bytes.
extern "C" lg_status lg_admission_simulate(const double *arrival, const uint64_t *need, const double *service,
                                           uint32_t count, uint64_t budget, uint64_t resident, uint32_t workers,
                                           double *start, double *finish, int32_t *status, uint64_t *peak) {
    using namespace lg;
    if (!workers || (count && (!arrival || !need || !service || !start || !finish || !status)) || !peak) {
        set_error("lg_admission_simulate: bad arguments");
        return LG_ERR_INVALID;
    }
    std::vector<uint64_t> held(workers, 0);
    std::vector<bool> busy(workers, false);
    std::vector<double> free_at(workers, 0.0);
    std::vector<int64_t> running(workers, -1);
    *peak = resident;
    double t = 0.0;
    uint32_t next = 0;  // next query in FIFO order (arrivals assumed sorted)
    uint32_t safety = 0;
    while (next < count) {
        if (++safety > 100u * count + 1000u) { set_error("lg_admission_simulate: no progress"); return LG_ERR_DEVICE; }
        // retire everything finished by t
        for (uint32_t w = 0; w < workers; ++w)
            if (busy[w] && free_at[w] <= t) busy[w] = false;
        if (arrival[next] > t) {
            // idle until the next arrival or completion
            double nt = arrival[next];
            for (uint32_t w = 0; w < workers; ++w)
                if (busy[w]) nt = std::min(nt, free_at[w]);
            t = std::max(t, nt);
            continue;
        }
        int32_t w_idle = -1;
        for (uint32_t w = 0; w < workers; ++w)
            if (!busy[w]) { w_idle = (int32_t)w; break; }
        if (w_idle < 0) {  // wait for the first completion
            double nt = 1e300;
            for (uint32_t w = 0; w < workers; ++w) nt = std::min(nt, free_at[w]);
            t = std::max(t, nt);
            continue;
        }
        const uint64_t grow = need[next] > held[w_idle] ? need[next] - held[w_idle] : 0;
        const AdmitDecision d = admit_decision(budget, resident, held, busy, (uint32_t)w_idle, need[next], grow);
        if (d == kReject) {
            status[next] = LG_ERR_CAPACITY;
            start[next] = finish[next] = t;
            ++next;
            continue;
        }
        if (d == kShrink) {
            held[w_idle] = 0;
            continue;
        }
        if (d == kReclaim) {
            for (uint32_t w = 0; w < workers; ++w)
                if ((int32_t)w != w_idle && !busy[w]) held[w] = 0;
            continue;
        }
        if (d == kWait) {
            double nt = 1e300;
            for (uint32_t w = 0; w < workers; ++w)
                if (busy[w]) nt = std::min(nt, free_at[w]);
            t = std::max(t, nt);
            continue;
        }
        held[w_idle] += grow;
        uint64_t in_use = resident;
        for (uint64_t h : held) in_use += h;
        *peak = std::max(*peak, in_use);
        busy[w_idle] = true;
        start[next] = t;
        finish[next] = t + service[next];
        free_at[w_idle] = finish[next];
        status[next] = LG_OK;
        ++next;
    }
    return LG_OK;
}
