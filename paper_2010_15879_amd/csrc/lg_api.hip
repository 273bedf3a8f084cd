// liblg support code: error strings, device buffers, graph views, lg_info,
// lg_export, lg_free and the kernel-timing facility.
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lg_internal.hpp"

namespace lg {

static thread_local char t_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_err, sizeof(t_err), fmt, ap);
    va_end(ap);
}

// ---------------------------------------------------------------------------
// scratch pool: released scratch buffers stay allocated for the next request
// on the same device and stream (work on one stream runs in order, so a
// buffer taken again there is only touched after the earlier work)
// ---------------------------------------------------------------------------

namespace {
struct Cached {
    int device;
    hipStream_t stream;
    uint64_t bytes;
    void *p;
};
struct Pool {
    std::mutex mu;
    std::vector<Cached> list;
    uint64_t total = 0;
};
Pool &pool() {
    static Pool *p = new Pool();  // never destroyed: buffers may outlive static teardown
    return *p;
}
constexpr uint64_t kPoolCap = 64ull << 30;  // bytes the pool keeps at most
}  // namespace

void DevBuf::release() {
    if (borrowed) {
        p = nullptr;
        bytes = 0;
        borrowed = false;
        return;
    }
    if (p) {
        if (pooled) {
            int dev = 0;
            (void)hipGetDevice(&dev);
            Pool &pl = pool();
            std::lock_guard<std::mutex> g(pl.mu);
            while (pl.total + bytes > kPoolCap && !pl.list.empty()) {
                (void)hipFree(pl.list.front().p);
                pl.total -= pl.list.front().bytes;
                pl.list.erase(pl.list.begin());
            }
            if (bytes <= kPoolCap) {
                pl.list.push_back(Cached{dev, pool_stream, bytes, p});
                pl.total += bytes;
            } else {
                (void)hipFree(p);
            }
        } else {
            (void)hipFree(p);
        }
    }
    p = nullptr;
    bytes = 0;
    pooled = false;
}

lg_status DevBuf::scratch(uint64_t nbytes, hipStream_t s) {
    release();
    if (nbytes == 0) nbytes = 8;
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        Pool &pl = pool();
        std::lock_guard<std::mutex> g(pl.mu);
        size_t best = pl.list.size();
        for (size_t i = 0; i < pl.list.size(); ++i) {
            const Cached &c = pl.list[i];
            if (c.device == dev && c.stream == s && c.bytes >= nbytes && c.bytes <= nbytes + nbytes / 4 + (2u << 20) &&
                (best == pl.list.size() || c.bytes < pl.list[best].bytes))
                best = i;
        }
        if (best < pl.list.size()) {
            p = pl.list[best].p;
            bytes = pl.list[best].bytes;
            pl.total -= bytes;
            pl.list.erase(pl.list.begin() + (long)best);
            pool_stream = s;
            pooled = true;
            return LG_OK;
        }
    }
    LG_TRY(alloc(nbytes));
    pool_stream = s;
    pooled = true;
    return LG_OK;
}

// Free every cached scratch buffer of the current device (out of memory).
static void pool_drop_device() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    Pool &pl = pool();
    std::lock_guard<std::mutex> g(pl.mu);
    for (size_t i = 0; i < pl.list.size();) {
        if (pl.list[i].device == dev) {
            (void)hipFree(pl.list[i].p);
            pl.total -= pl.list[i].bytes;
            pl.list.erase(pl.list.begin() + (long)i);
        } else {
            ++i;
        }
    }
}

lg_status DevBuf::alloc(uint64_t nbytes) {
    release();
    if (nbytes == 0) nbytes = 8;
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {  // the scratch cache may hold the memory: give it back, try once more
        (void)hipGetLastError();
        pool_drop_device();
        e = hipMalloc(&p, nbytes);
    }
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        set_error("hipMalloc(%llu bytes) failed: %s", (unsigned long long)nbytes, hipGetErrorString(e));
        return LG_ERR_OOM;
    }
    bytes = nbytes;
    return LG_OK;
}

lg_status DevBuf::ensure(uint64_t nbytes) {
    if (p && bytes >= nbytes) return LG_OK;
    if (borrowed) {
        set_error("a fixed scratch region of %llu bytes cannot hold %llu", (unsigned long long)bytes,
                  (unsigned long long)nbytes);
        return LG_ERR_UNSUPPORTED;
    }
    if (pooled) return scratch(nbytes, pool_stream);
    return alloc(nbytes);
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------

namespace {
struct ProfState {
    std::mutex mu;
    bool on = false;
    char filter[128] = "";  // time only launches whose kernel name contains this (empty: all)
    std::vector<ProfMark> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<uint64_t, double>> done;
};
ProfState &prof() {
    static ProfState *st = new ProfState();  // never destroyed: events may outlive static teardown
    return *st;
}
hipEvent_t pool_get(ProfState &st) {
    if (!st.pool.empty()) {
        hipEvent_t e = st.pool.back();
        st.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
// fold completed marks into the totals; with wait, wait for all of them
void drain(ProfState &st, bool wait) {
    std::vector<ProfMark> keep;
    for (auto &m : st.pending) {
        if (!wait && hipEventQuery(m.b) != hipSuccess) { keep.push_back(m); continue; }
        if (wait) (void)hipEventSynchronize(m.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
            auto &d = st.done[m.name];
            d.first += 1;
            d.second += ms;
        }
        st.pool.push_back(m.a);
        st.pool.push_back(m.b);
    }
    st.pending.swap(keep);
}
}  // namespace

bool prof_on() { return prof().on; }

// does the kernel name contain one of the '|'-separated filter parts?
static bool prof_match(const char *filter, const char *name) {
    char part[sizeof(ProfState::filter)];
    const char *p = filter;
    while (*p) {
        size_t k = 0;
        while (p[k] && p[k] != '|') ++k;
        std::memcpy(part, p, k);
        part[k] = 0;
        if (k && std::strstr(name, part)) return true;
        p += k;
        if (*p == '|') ++p;
    }
    return false;
}

ProfMark prof_begin(const char *name, hipStream_t stream) {
    ProfState &st = prof();
    if (st.filter[0] && !prof_match(st.filter, name)) return ProfMark{};
    std::lock_guard<std::mutex> g(st.mu);
    ProfMark m;
    if (st.pending.size() > 4096) drain(st, false);
    m.a = pool_get(st);
    m.b = pool_get(st);
    if (!m.a || !m.b) return ProfMark{};
    m.name = name;
    m.stream = stream;
    (void)hipEventRecord(m.a, stream);
    return m;
}

void prof_end(ProfMark &m) {
    ProfState &st = prof();
    std::lock_guard<std::mutex> g(st.mu);
    (void)hipEventRecord(m.b, m.stream);
    st.pending.push_back(m);
}

}  // namespace lg

// ---------------------------------------------------------------------------
// graph views and accounting
// ---------------------------------------------------------------------------

lg::PackedView lg_graph::packed_view() const {
    lg::PackedView v;
    v.A32 = A.as<uint32_t>();
    v.W = W.as<uint64_t>();
    v.G = G.as<uint64_t>();
    v.s = s;
    v.F = F;
    v.po.O = O.as<uint64_t>();
    v.po.w = wO;
    v.ef.L = L.as<uint64_t>();
    v.ef.H = H.as<uint64_t>();
    v.ef.rank_sb = rank_sb.as<uint32_t>();
    v.ef.sel = sel.as<uint32_t>();
    v.ef.l = ef_l;
    v.ef.n_sel = (uint32_t)n_sel;
    v.ef.n_sb = n_rank ? (uint32_t)(n_rank - 1) : 0;
    v.ef.n_hw = (uint32_t)H_words;
    v.il.W = IL.as<uint64_t>();
    v.il.blocks = il_blocks;
    return v;
}

lg::PlainView lg_graph::plain_view() const {
    lg::PlainView v;
    v.off = poff.p;
    v.col = pcol.as<uint32_t>();
    return v;
}

uint64_t lg_graph::device_bytes() const {
    uint64_t b = A.bytes + O.bytes + W.bytes + G.bytes + L.bytes + H.bytes + rank_sb.bytes + sel.bytes + IL.bytes +
                 poff.bytes +
                 pcol.bytes + pwt.bytes + perm.bytes + inv.bytes + heavy.bytes + iso.bytes + hstart.bytes + hdeg.bytes + hw.bytes +
                 hg.bytes + seg_off.bytes + seg_map.bytes + seg_part.bytes + seg_base.bytes + units.bytes +
                 vhb0.bytes + vhb1.bytes + vseg_off.bytes + vseg_map.bytes + vseg_base.bytes + vdeg.bytes +
                 vca.bytes + vcb.bytes + vpart.bytes + (dec ? dec->bytes() : 0);
    return b;
}

namespace lg {
uint64_t bfs_bytes(const lg_graph *g);
uint64_t pr_bytes(const lg_graph *g);
}  // namespace lg

namespace lg {
lg_status mark_use(lg_graph *g, hipStream_t stream) {
    if (g->last_use) LG_CHECK_HIP(hipEventRecord(g->last_use, stream));
    return LG_OK;
}
}  // namespace lg

extern "C" void lg_free(lg_graph *g) {
    if (!g) return;
    // Wait for the graph's own last use only (calls on one graph do not
    // overlap, so the last one recorded finishes after every earlier one);
    // work on other streams and graphs goes on.  The arrays then go back to
    // the scratch pool, or are freed.
    if (g->last_use) {
        (void)hipEventSynchronize(g->last_use);
        (void)hipEventDestroy(g->last_use);
        g->last_use = nullptr;
    }
    lg::bfs_free(g);
    lg::pr_free(g);
    lg::pb_free(g);
    lg::sssp_free(g);
    delete g->dec;
    delete g;
}

extern "C" lg_status lg_info(const lg_graph *g, lg_graph_info *out) {
    if (!g || !out) { lg::set_error("lg_info: NULL argument"); return LG_ERR_INVALID; }
    std::memset(out, 0, sizeof(*out));
    out->n = g->n;
    out->m = g->m;
    out->layout = g->layout;
    out->id_mode = g->id_mode;
    out->offset_mode = g->offset_mode;
    out->relabel = g->relabel;
    out->s = g->s;
    out->F = g->F;
    out->max_degree = g->max_degree;
    out->isolated = g->isolated;
    out->heavy_threshold = g->heavy_threshold;
    out->n_heavy = g->n_heavy;
    out->n_segments = g->n_seg;
    out->heavy_edges = g->heavy_edges;
    out->heavy_bits = g->heavy_bits;
    if (g->layout == LG_LAYOUT_PLAIN) {
        out->bytes_adj = g->m * 4;
        out->bytes_offsets = ((uint64_t)g->n + 1) * (g->poff64 ? 8 : 4);
    } else {
        out->w_offset = g->offset_mode == LG_OFFS_PACKED ? g->wO : 0;
        out->ef_l = g->ef_l;
        out->universe = g->universe;
        out->adj_bits = g->U;
        out->ef_high_bits = g->hbits;
        out->bytes_adj = g->A_words * 8;
        out->bytes_offsets = g->offset_mode == LG_OFFS_PACKED           ? g->O_words * 8
                             : g->offset_mode == LG_OFFS_INTERLEAVED_BV ? g->IL_words * 8
                                 : g->L_words * 8 + g->H_words * 8 + g->n_rank * 4 + g->n_sel * 4;
        out->bytes_widths = (g->W_words + g->G_words) * 8;
    }
    out->bytes_perm = g->perm.bytes + g->inv.bytes;
    out->device_bytes = g->device_bytes() + lg::bfs_bytes(g) + lg::pr_bytes(g) + lg::pb_bytes(g) + lg::sssp_bytes(g);
    out->weight_bits = g->omega;
    out->bytes_weights = g->pwt.bytes;
    return LG_OK;
}

static bool export_src(const lg_graph *g, uint32_t which, const void **p, uint64_t *bytes) {
    *p = nullptr;
    *bytes = 0;
    const bool packed = g->layout == LG_LAYOUT_PACKED;
    switch (which) {
        case LG_EXPORT_ADJ:
            if (packed) { *p = g->A.p; *bytes = g->A_words * 8; }
            else { *p = g->pcol.p; *bytes = g->m * 4; }
            return true;
        case LG_EXPORT_OFFSETS:
            if (packed) {
                if (g->offset_mode != LG_OFFS_PACKED) return false;
                *p = g->O.p; *bytes = g->O_words * 8;
            } else {
                *p = g->poff.p; *bytes = ((uint64_t)g->n + 1) * (g->poff64 ? 8 : 4);
            }
            return true;
        case LG_EXPORT_WIDTHS:
            if (!packed || (g->id_mode != LG_IDS_LOCAL && g->id_mode != LG_IDS_LOCAL_GAP)) return false;
            *p = g->W.p; *bytes = g->W_words * 8;
            return true;
        case LG_EXPORT_WEIGHTS:
            if (packed || !g->weighted) return false;
            *p = g->pwt.p; *bytes = g->m * 4;
            return true;
        case LG_EXPORT_GAP_WIDTHS:
            if (!packed || g->id_mode != LG_IDS_LOCAL_GAP) return false;
            *p = g->G.p; *bytes = g->G_words * 8;
            return true;
        case LG_EXPORT_EF_LOW:
        case LG_EXPORT_EF_HIGH:
        case LG_EXPORT_EF_RANK:
        case LG_EXPORT_EF_SELECT:
            if (!packed || (g->offset_mode != LG_OFFS_SUCCINCT && g->offset_mode != LG_OFFS_PLAIN_BV)) return false;
            if (which == LG_EXPORT_EF_LOW && g->offset_mode != LG_OFFS_SUCCINCT) return false;
            if (which == LG_EXPORT_EF_LOW) { *p = g->L.p; *bytes = g->L_words * 8; }
            if (which == LG_EXPORT_EF_HIGH) { *p = g->H.p; *bytes = g->H_words * 8; }
            if (which == LG_EXPORT_EF_RANK) { *p = g->rank_sb.p; *bytes = g->n_rank * 4; }
            if (which == LG_EXPORT_EF_SELECT) { *p = g->sel.p; *bytes = g->n_sel * 4; }
            return true;
        case LG_EXPORT_BV_INTERLEAVED:
            if (!packed || g->offset_mode != LG_OFFS_INTERLEAVED_BV) return false;
            *p = g->IL.p; *bytes = g->IL_words * 8;
            return true;
        case LG_EXPORT_PERM:
        case LG_EXPORT_INV:
            if (g->relabel == LG_RELABEL_NONE) return false;
            *p = which == LG_EXPORT_PERM ? g->perm.p : g->inv.p;
            *bytes = (uint64_t)g->n * 4;
            return true;
        default:
            return false;
    }
}

extern "C" uint64_t lg_export_bytes(const lg_graph *g, uint32_t which) {
    if (!g) return 0;
    const void *p;
    uint64_t bytes;
    return export_src(g, which, &p, &bytes) ? bytes : 0;
}

extern "C" lg_status lg_export(const lg_graph *g, uint32_t which, void *host_dst, uint64_t bytes) {
    if (!g || !host_dst) { lg::set_error("lg_export: NULL argument"); return LG_ERR_INVALID; }
    const void *p;
    uint64_t want;
    if (!export_src(g, which, &p, &want)) { lg::set_error("lg_export: array %u not held", which); return LG_ERR_INVALID; }
    if (bytes != want) {
        lg::set_error("lg_export: %llu bytes requested, array has %llu", (unsigned long long)bytes,
                      (unsigned long long)want);
        return LG_ERR_INVALID;
    }
    if (!bytes) return LG_OK;
    LG_CHECK_HIP(hipDeviceSynchronize());
    LG_CHECK_HIP(hipMemcpy(host_dst, p, bytes, hipMemcpyDeviceToHost));
    return LG_OK;
}

extern "C" const char *lg_last_error(void) { return lg::t_err; }

extern "C" void lg_trim(void) {
    lg::bfs_pools_trim();
    lg::pb_trim();
    lg::Pool &pl = lg::pool();
    std::lock_guard<std::mutex> g(pl.mu);
    for (const lg::Cached &c : pl.list) (void)hipFree(c.p);
    pl.list.clear();
    pl.total = 0;
}

extern "C" lg_status lg_prof_enable(int on) {
    auto &st = lg::prof();
    std::lock_guard<std::mutex> g(st.mu);
    st.on = on != 0;
    return LG_OK;
}

extern "C" lg_status lg_prof_filter(const char *substr) {
    auto &st = lg::prof();
    std::lock_guard<std::mutex> g(st.mu);
    if (!substr) substr = "";
    if (std::strlen(substr) >= sizeof(st.filter)) { lg::set_error("lg_prof_filter: name too long"); return LG_ERR_INVALID; }
    std::strcpy(st.filter, substr);
    return LG_OK;
}

extern "C" lg_status lg_prof_reset(void) {
    auto &st = lg::prof();
    std::lock_guard<std::mutex> g(st.mu);
    lg::drain(st, true);
    st.done.clear();
    return LG_OK;
}

extern "C" lg_status lg_prof_query(const char *kernel, uint64_t *launches, double *total_ms) {
    if (!kernel || !launches || !total_ms) { lg::set_error("lg_prof_query: NULL argument"); return LG_ERR_INVALID; }
    auto &st = lg::prof();
    std::lock_guard<std::mutex> g(st.mu);
    lg::drain(st, true);
    *launches = 0;
    *total_ms = 0.0;
    for (auto &kv : st.done) {
        // names are recorded as written at the launch site, possibly with
        // template arguments; match on the leading identifier
        std::string nm = kv.first;
        if (!nm.empty() && nm[0] == '(') nm.erase(0, 1);
        const size_t len = std::strlen(kernel);
        if (nm.compare(0, len, kernel) == 0 && (nm.size() == len || nm[len] == '<' || nm[len] == ')')) {
            *launches += kv.second.first;
            *total_ms += kv.second.second;
        }
    }
    return LG_OK;
}

extern "C" lg_status lg_prof_names(char *buf, uint64_t bytes) {
    if (!buf || !bytes) { lg::set_error("lg_prof_names: NULL argument"); return LG_ERR_INVALID; }
    auto &st = lg::prof();
    std::lock_guard<std::mutex> g(st.mu);
    lg::drain(st, true);
    std::string all;
    for (auto &kv : st.done) { all += kv.first; all += '\n'; }
    std::strncpy(buf, all.c_str(), bytes - 1);
    buf[bytes - 1] = 0;
    return all.size() < bytes ? LG_OK : LG_ERR_CAPACITY;
}
