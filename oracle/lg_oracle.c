/*
 * Log(Graph) CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately obvious implementation of what the packed
 * graph path computes, used to check the GPU library.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never calls into it.  It shares no code, header or table
 * with the GPU library.
 *
 * Conventions (the paper leaves these open; each reading is stated where it
 * is used):
 *   - vertex IDs are 0-based unsigned 32-bit integers;
 *   - bl(x) is the bit length of x, bl(0) = 0;
 *   - a packed bit stream stores its bit b as bit (b mod 64) of little-endian
 *     64-bit word floor(b / 64); a value's bit k goes to stream bit start + k
 *     (this is the byte/bit addressing of the edge-access listing in the
 *     "Accessing An Edge" subsection, read with an x86 bit-field extract);
 *     unused bits are zero and every stream carries one extra zero word.
 *
 * Every read and write of a packed stream below goes one bit at a time, on
 * purpose unlike any word-level implementation.
 *
 * Parity status: every function here is pinned by the CPU test suite
 * (closed forms, brute force, textbook library routines, hand-computed
 * fixtures); none is "parity unpinned".
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* bit helpers                                                          */
/* ------------------------------------------------------------------ */

static unsigned bitlen(uint64_t x) {
    unsigned b = 0;
    while (x) { b++; x >>= 1; }
    return b;
}

ORC_API unsigned orc_bitlen(uint64_t x) { return bitlen(x); }

static void put_bit(uint64_t *words, uint64_t pos) {
    words[pos / 64] |= (uint64_t)1 << (pos % 64);
}

static int get_bit(const uint64_t *words, uint64_t pos) {
    return (int)((words[pos / 64] >> (pos % 64)) & 1u);
}

/* write `width` low bits of value at stream bit `start`, one bit at a time */
static void put_bits(uint64_t *words, uint64_t start, uint64_t value, unsigned width) {
    for (unsigned k = 0; k < width; k++)
        if ((value >> k) & 1u) put_bit(words, start + k);
}

static uint64_t get_bits(const uint64_t *words, uint64_t start, unsigned width) {
    uint64_t v = 0;
    for (unsigned k = 0; k < width; k++)
        if (get_bit(words, start + k)) v |= (uint64_t)1 << k;
    return v;
}

/* number of 64-bit words of a stream of `bits` bits, plus the zero pad word */
ORC_API uint64_t orc_stream_words(uint64_t bits) { return (bits + 63) / 64 + 1; }

ORC_API uint64_t orc_get_bits(const uint64_t *words, uint64_t start, unsigned width) {
    return get_bits(words, start, width);
}

/* ------------------------------------------------------------------ */
/* vertex ID widths -- section "Logarithmization of Vertex IDs"          */
/* ------------------------------------------------------------------ */

/* Global approach: ceil(log2 n) bits per ID.  Reading: for n = 1 the
 * formula gives 0, so the width is max(1, bl(n - 1)), which equals
 * ceil(log2 n) for every n >= 2. */
ORC_API unsigned orc_global_width(uint64_t n) {
    unsigned s = n ? bitlen(n - 1) : 0;
    return s ? s : 1;
}

/* Local approach: the list of v is stored with enough bits for its largest
 * ID.  Reading: ceil(log2 maxN_v) undercounts when maxN_v is a power of two
 * and gives 0 for maxN_v in {0, 1}; the width is max(1, bl(maxN_v)) for a
 * non-empty list and 0 for an empty one.  The maximum is found by scanning,
 * not by assuming the list is sorted. */
ORC_API void orc_local_widths(uint64_t n, const uint64_t *off, const uint32_t *col, uint8_t *w) {
    for (uint64_t v = 0; v < n; v++) {
        if (off[v + 1] == off[v]) { w[v] = 0; continue; }
        uint32_t mx = 0;
        for (uint64_t i = off[v]; i < off[v + 1]; i++)
            if (col[i] > mx) mx = col[i];
        unsigned b = bitlen(mx);
        w[v] = (uint8_t)(b ? b : 1);
    }
}

/* Local widths of the relabeled graph, read off the original lists: row x
 * is the list of perm[x] renamed through inv, so its largest entry is the
 * largest inv[u] over that list.  deg2[x] receives the row length. */
ORC_API void orc_relabeled_local_widths(uint64_t n, const uint64_t *off, const uint32_t *col,
                                        const uint32_t *perm, const uint32_t *inv, uint8_t *w,
                                        uint64_t *deg2) {
    for (uint64_t x = 0; x < n; x++) {
        uint32_t v = perm[x];
        deg2[x] = off[v + 1] - off[v];
        if (deg2[x] == 0) { w[x] = 0; continue; }
        uint32_t mx = 0;
        for (uint64_t i = off[v]; i < off[v + 1]; i++)
            if (inv[col[i]] > mx) mx = inv[col[i]];
        unsigned b = bitlen(mx);
        w[x] = (uint8_t)(b ? b : 1);
    }
}

/* bits of the per-vertex width field: enough to write the global width */
ORC_API unsigned orc_width_field_bits(uint64_t n) { return bitlen(orc_global_width(n)); }

/* ------------------------------------------------------------------ */
/* packed adjacency -- "Vertex IDs: The Global/Local Approach" and the   */
/* edge-access listing of "Accessing An Edge"                            */
/* ------------------------------------------------------------------ */

/* Bit length of every neighbor list laid end to end: |A| = 2m*s (global)
 * or sum_v d_v * w_v (local).  w == NULL selects the global width s. */
ORC_API uint64_t orc_adjacency_bits(uint64_t n, const uint64_t *off, const uint8_t *w, unsigned s) {
    uint64_t U = 0;
    for (uint64_t v = 0; v < n; v++)
        U += (off[v + 1] - off[v]) * (uint64_t)(w ? w[v] : s);
    return U;
}

/* Bit start P_v of every list (v = 0..n): the running total of the list
 * bit lengths before v. */
ORC_API void orc_bit_starts(uint64_t n, const uint64_t *off, const uint8_t *w, unsigned s, uint64_t *P) {
    uint64_t acc = 0;
    for (uint64_t v = 0; v < n; v++) {
        P[v] = acc;
        acc += (off[v + 1] - off[v]) * (uint64_t)(w ? w[v] : s);
    }
    P[n] = acc;
}

/* Element i of the list of v occupies stream bits [P_v + i*w_v, + w_v).
 * `words` must hold orc_stream_words(U) zeroed words. */
ORC_API void orc_pack_adjacency(uint64_t n, const uint64_t *off, const uint32_t *col,
                                const uint8_t *w, unsigned s, uint64_t *words) {
    uint64_t pos = 0;
    for (uint64_t v = 0; v < n; v++) {
        unsigned wv = w ? w[v] : s;
        for (uint64_t i = off[v]; i < off[v + 1]; i++) {
            put_bits(words, pos, col[i], wv);
            pos += wv;
        }
    }
}

/* Words [k0, k1) of the same stream, computed without building the rest:
 * every element is visited in order and only its bits that fall inside
 * [64*k0, 64*k1) are written.  `out` holds k1 - k0 zeroed words. */
ORC_API void orc_pack_adjacency_words(uint64_t n, const uint64_t *off, const uint32_t *col,
                                      const uint8_t *w, unsigned s, uint64_t k0, uint64_t k1,
                                      uint64_t *out) {
    uint64_t lo = 64 * k0, hi = 64 * k1, pos = 0;
    for (uint64_t v = 0; v < n && pos < hi; v++) {
        unsigned wv = w ? w[v] : s;
        uint64_t d = off[v + 1] - off[v];
        if (pos + d * wv <= lo) { pos += d * wv; continue; }
        for (uint64_t i = off[v]; i < off[v + 1]; i++) {
            for (unsigned k = 0; k < wv; k++) {
                uint64_t b = pos + k;
                if (b >= lo && b < hi && ((col[i] >> k) & 1u)) put_bit(out, b - lo);
            }
            pos += wv;
        }
    }
}

/* Fixed-size gap encoding, local approach (subsection "Adding Fixed-Size Gap
 * Encoding"): the differences between consecutive neighbors of A_v, all at
 * the width of the largest difference in A_v.  Readings: the first element
 * is stored as is, at the local width w_v of "The Local Approach"
 * (max(1, bl(max N_v))); the gap width is g_v = bl(largest difference)
 * (>= 1, the lists being strictly increasing) for d_v >= 2 and 0 for
 * shorter lists; the list of v then takes w_v + (d_v - 1) g_v bits (0 when
 * d_v = 0). */
ORC_API void orc_gap_widths(uint64_t n, const uint64_t *off, const uint32_t *col, uint8_t *g) {
    for (uint64_t v = 0; v < n; v++) {
        uint32_t mx = 0;
        for (uint64_t i = off[v] + 1; i < off[v + 1]; i++)
            if (col[i] - col[i - 1] > mx) mx = col[i] - col[i - 1];
        g[v] = (uint8_t)bitlen(mx);
    }
}

ORC_API void orc_gap_bit_starts(uint64_t n, const uint64_t *off, const uint8_t *w, const uint8_t *g, uint64_t *P) {
    uint64_t acc = 0;
    for (uint64_t v = 0; v < n; v++) {
        P[v] = acc;
        const uint64_t d = off[v + 1] - off[v];
        if (d) acc += w[v] + (d - 1) * (uint64_t)g[v];
    }
    P[n] = acc;
}

/* The gap stream: per list the first element at w_v bits, then each
 * difference at g_v bits, LSB-first.  `words` holds orc_stream_words(U)
 * zeroed words. */
ORC_API void orc_pack_gap(uint64_t n, const uint64_t *off, const uint32_t *col, const uint8_t *w,
                          const uint8_t *g, uint64_t *words) {
    uint64_t pos = 0;
    for (uint64_t v = 0; v < n; v++) {
        for (uint64_t i = off[v]; i < off[v + 1]; i++) {
            if (i == off[v]) {
                put_bits(words, pos, col[i], w[v]);
                pos += w[v];
            } else {
                put_bits(words, pos, col[i] - col[i - 1], g[v]);
                pos += g[v];
            }
        }
    }
}

/* A gap-encoded list of d elements starting at stream bit `start`: the
 * first element, then running sums of the differences. */
ORC_API void orc_decode_gap_list(const uint64_t *words, uint64_t start, uint64_t d, unsigned w, unsigned g,
                                 uint32_t *out) {
    if (d == 0) return;
    uint32_t x = (uint32_t)orc_get_bits(words, start, w);
    out[0] = x;
    for (uint64_t i = 1; i < d; i++) {
        x += (uint32_t)orc_get_bits(words, start + w + (i - 1) * g, g);
        out[i] = x;
    }
}

/* ------------------------------------------------------------------ */
/* Varint lists -- subsection "Incorporating Degree-Minimizing (DM)":   */
/* DMf stores every label of a list, DMd the first label and then the   */
/* differences of consecutive labels, each value as a Varint.  Reading  */
/* (the paper names the code but not its byte layout): the common       */
/* little-endian base-128 form, 7 value bits per byte, the lowest group */
/* first, the top bit of a byte set when another byte of the same value */
/* follows.  Lists follow each other in vertex order, byte-aligned; the */
/* offsets are byte starts.                                              */
/* ------------------------------------------------------------------ */

/* The value entry i of row v stores. */
static uint32_t varint_value(const uint64_t *off, const uint32_t *col, uint64_t v, uint64_t i, int diff) {
    if (!diff || i == off[v]) return col[i];
    return col[i] - col[i - 1];
}

ORC_API unsigned orc_varint_len(uint32_t x) {
    unsigned b = 1;
    while (x >= 128) {
        x >>= 7;
        b++;
    }
    return b;
}

/* Byte start of every list (count n + 1, the last one the stream length). */
ORC_API void orc_varint_byte_starts(uint64_t n, const uint64_t *off, const uint32_t *col, int diff, uint64_t *P) {
    uint64_t acc = 0;
    for (uint64_t v = 0; v < n; v++) {
        P[v] = acc;
        for (uint64_t i = off[v]; i < off[v + 1]; i++) acc += orc_varint_len(varint_value(off, col, v, i, diff));
    }
    P[n] = acc;
}

/* The byte stream; `bytes` holds at least P[n] bytes. */
ORC_API void orc_pack_varint(uint64_t n, const uint64_t *off, const uint32_t *col, int diff, uint8_t *bytes) {
    uint64_t pos = 0;
    for (uint64_t v = 0; v < n; v++) {
        for (uint64_t i = off[v]; i < off[v + 1]; i++) {
            uint32_t x = varint_value(off, col, v, i, diff);
            for (;;) {
                const uint8_t low = (uint8_t)(x & 127u);
                x >>= 7;
                if (x) {
                    bytes[pos++] = (uint8_t)(low | 128u);
                } else {
                    bytes[pos++] = low;
                    break;
                }
            }
        }
    }
}

/* The list held in bytes [b0, b1): returns its length, the labels in out
 * (out must hold b1 - b0 values, the most a list of that size can have). */
ORC_API uint64_t orc_decode_varint_list(const uint8_t *bytes, uint64_t b0, uint64_t b1, int diff, uint32_t *out) {
    uint64_t count = 0;
    uint64_t acc = 0;
    unsigned shift = 0;
    for (uint64_t p = b0; p < b1; p++) {
        acc |= (uint64_t)(bytes[p] & 127u) << shift;
        shift += 7;
        if (!(bytes[p] & 128u)) {
            uint32_t x = (uint32_t)acc;
            if (diff && count) x += out[count - 1];
            out[count++] = x;
            acc = 0;
            shift = 0;
        }
    }
    return count;
}

/* ------------------------------------------------------------------ */
/* Weighted lists -- subsections "Logarithmization of Edge Weights" and */
/* "Accessing an Edge Weight": each entry is the neighbor ID followed   */
/* directly by the edge's weight.  Reading: one weight width for the    */
/* graph, omega = max(1, bl(largest weight)); the ID keeps its global   */
/* (s) or local (w_v) width, so an entry takes s + omega or w_v + omega */
/* bits.                                                                 */
/* ------------------------------------------------------------------ */

ORC_API unsigned orc_weight_width(uint64_t m, const uint32_t *wt) {
    uint32_t mx = 0;
    for (uint64_t i = 0; i < m; i++)
        if (wt[i] > mx) mx = wt[i];
    const unsigned b = bitlen(mx);
    return b ? b : 1;
}

/* w == NULL selects the global width s; `words` holds zeroed words. */
ORC_API void orc_pack_weighted(uint64_t n, const uint64_t *off, const uint32_t *col, const uint32_t *wt,
                               const uint8_t *w, unsigned s, unsigned omega, uint64_t *words) {
    uint64_t pos = 0;
    for (uint64_t v = 0; v < n; v++) {
        const unsigned wv = w ? w[v] : s;
        for (uint64_t i = off[v]; i < off[v + 1]; i++) {
            put_bits(words, pos, col[i], wv);
            pos += wv;
            put_bits(words, pos, wt[i], omega);
            pos += omega;
        }
    }
}

ORC_API void orc_decode_weighted_list(const uint64_t *words, uint64_t start, uint64_t d, unsigned w,
                                      unsigned omega, uint32_t *ids, uint32_t *wts) {
    for (uint64_t i = 0; i < d; i++) {
        const uint64_t b = start + i * (uint64_t)(w + omega);
        ids[i] = (uint32_t)get_bits(words, b, w);
        wts[i] = (uint32_t)get_bits(words, b + w, omega);
    }
}

/* ------------------------------------------------------------------ */
/* SSSP (section "Considered Algorithms"): the distances themselves,    */
/* by Dijkstra's algorithm with a binary heap (lazy deletion).  Entry i */
/* of row u is the edge u -> col[i] of weight wt[i]; dist = -1 where    */
/* the root does not reach.                                              */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t d;
    uint32_t v;
} heap_item;

static void heap_push(heap_item *h, uint64_t *size, heap_item x) {
    uint64_t i = (*size)++;
    h[i] = x;
    while (i > 0) {
        const uint64_t p = (i - 1) / 2;
        if (h[p].d <= h[i].d) break;
        const heap_item t = h[p];
        h[p] = h[i];
        h[i] = t;
        i = p;
    }
}

static heap_item heap_pop(heap_item *h, uint64_t *size) {
    const heap_item top = h[0];
    h[0] = h[--(*size)];
    uint64_t i = 0;
    for (;;) {
        const uint64_t l = 2 * i + 1, r = l + 1;
        uint64_t m = i;
        if (l < *size && h[l].d < h[m].d) m = l;
        if (r < *size && h[r].d < h[m].d) m = r;
        if (m == i) break;
        const heap_item t = h[m];
        h[m] = h[i];
        h[i] = t;
        i = m;
    }
    return top;
}

ORC_API int orc_sssp(uint64_t n, const uint64_t *off, const uint32_t *col, const uint32_t *wt, uint32_t root,
                     int64_t *dist) {
    if (root >= n) return -1;
    heap_item *h = (heap_item *)malloc(sizeof(heap_item) * (off[n] + 1));
    if (!h) return -2;
    for (uint64_t v = 0; v < n; v++) dist[v] = -1;
    uint64_t size = 0;
    dist[root] = 0;
    heap_push(h, &size, (heap_item){0, root});
    while (size) {
        const heap_item it = heap_pop(h, &size);
        if (it.d != dist[it.v]) continue;  // a stale entry
        for (uint64_t i = off[it.v]; i < off[it.v + 1]; i++) {
            const int64_t nd = it.d + (int64_t)wt[i];
            const uint32_t x = col[i];
            if (dist[x] < 0 || nd < dist[x]) {
                dist[x] = nd;
                heap_push(h, &size, (heap_item){nd, x});
            }
        }
    }
    free(h);
    return 0;
}

/* Element i of a list whose first element starts at stream bit `start`. */
ORC_API void orc_decode_list(const uint64_t *words, uint64_t start, uint64_t d, unsigned w, uint32_t *out) {
    for (uint64_t i = 0; i < d; i++)
        out[i] = (uint32_t)get_bits(words, start + i * (uint64_t)w, w);
}

/* Fixed-width packing of a value sequence: value j at bits [j*width, +width).
 * Used for the packed offsets ("Logarithmization of Single Offsets"), the
 * Elias-Fano low bits and the per-vertex width table. */
ORC_API void orc_pack_fixed(const uint64_t *vals, uint64_t count, unsigned width, uint64_t *words) {
    for (uint64_t j = 0; j < count; j++)
        put_bits(words, j * (uint64_t)width, vals[j], width);
}

/* ------------------------------------------------------------------ */
/* bit vector queries -- subsection "Bit Vectors"                        */
/* ------------------------------------------------------------------ */

/* Reading of the conventions: rank1(i) counts the ones in positions [0, i)
 * (exclusive).  The paper's inclusive rank_S(x) equals rank1(x + 1).
 * select1(k) is the position of the k-th one, counting k from 0.  Both
 * are linear scans. */
ORC_API uint64_t orc_rank1(const uint64_t *words, uint64_t i) {
    uint64_t r = 0;
    for (uint64_t p = 0; p < i; p++) r += (uint64_t)get_bit(words, p);
    return r;
}

/* returns the position, or `nbits` when the vector has at most k ones */
ORC_API uint64_t orc_select1(const uint64_t *words, uint64_t nbits, uint64_t k) {
    uint64_t seen = 0;
    for (uint64_t p = 0; p < nbits; p++) {
        if (get_bit(words, p)) {
            if (seen == k) return p;
            seen++;
        }
    }
    return nbits;
}

/* ------------------------------------------------------------------ */
/* Elias-Fano offsets -- sections "Logarithmizing Offsets" and           */
/* "Succinct Bit Vectors in Log(Graph)" (sparse bit vector bvSD)        */
/* ------------------------------------------------------------------ */

/* The offsets x_0 <= x_1 <= ... <= x_n (universe u = x_n) are kept as an
 * Elias-Fano sequence.  Reading (the paper sets one bit per list start,
 * which cannot mark two starts at the same place; the non-decreasing
 * sequence formulation allows repeats): the low l bits of every x_v are
 * stored verbatim, and the high part sets bit (x_v >> l) + v of the upper
 * bit vector H, which therefore holds exactly n + 1 ones.
 * l = floor(log2(u / (n + 1))) when u >= n + 1, else 0. */
ORC_API unsigned orc_ef_low_bits(uint64_t count, uint64_t universe) {
    if (universe < count || count == 0) return 0;
    return bitlen(universe / count) - 1;
}

ORC_API uint64_t orc_ef_upper_bits(uint64_t count, uint64_t universe, unsigned l) {
    return (universe >> l) + count;
}

/* Directory over H, checkable bit-exactly because every entry is a plain
 * rank or select value:
 *   rank_sb[b] = rank1(512 * b) for b = 0 .. ceil(|H| / 512)  (one extra
 *                entry at the end, which equals the number of ones);
 *   sel[j]     = select1(64 * j) for j = 0 .. ceil((n + 1) / 64) - 1.     */
ORC_API uint64_t orc_ef_rank_entries(uint64_t hbits) { return (hbits + 511) / 512 + 1; }
ORC_API uint64_t orc_ef_select_entries(uint64_t count) { return (count + 63) / 64; }

ORC_API void orc_ef_build(const uint64_t *x, uint64_t count, uint64_t universe,
                          uint64_t *L, uint64_t *H, uint32_t *rank_sb, uint32_t *sel) {
    unsigned l = orc_ef_low_bits(count, universe);
    uint64_t hbits = orc_ef_upper_bits(count, universe, l);
    for (uint64_t v = 0; v < count; v++) {
        uint64_t low = l ? (x[v] & (((uint64_t)1 << l) - 1)) : 0;
        put_bits(L, v * (uint64_t)l, low, l);
        put_bit(H, (x[v] >> l) + v);
    }
    /* one running count over H gives both directory tables */
    uint64_t nr = orc_ef_rank_entries(hbits), ns = orc_ef_select_entries(count);
    uint64_t ones = 0;
    for (uint64_t p = 0; p <= hbits; p++) {
        if (p % 512 == 0 && p / 512 < nr) rank_sb[p / 512] = (uint32_t)ones;
        if (p == hbits) break;
        if (get_bit(H, p)) {
            if (ones % 64 == 0 && ones / 64 < ns) sel[ones / 64] = (uint32_t)p;
            ones++;
        }
    }
    rank_sb[nr - 1] = (uint32_t)ones; /* the extra last entry: all ones */
}

/* x_v recovered from L and H: ((select1(v) - v) << l) | L[v] */
ORC_API uint64_t orc_ef_get(const uint64_t *L, const uint64_t *H, uint64_t hbits, unsigned l, uint64_t v) {
    uint64_t pos = orc_select1(H, hbits, v);
    return ((pos - v) << l) | get_bits(L, v * (uint64_t)l, l);
}

/* ------------------------------------------------------------------ */
/* degree-minimizing relabeling -- "Incorporating Degree-Minimizing"   */
/* ------------------------------------------------------------------ */

/* Higher degree gets a lower label.  Reading of the unstated tie-break:
 * equal degrees keep their original order.  perm[new] = old and
 * inv[old] = new.  A plain insertion-free approach: qsort on (-d, id). */
static const uint64_t *g_sort_off;

static int cmp_dm(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    uint64_t dx = g_sort_off[x + 1] - g_sort_off[x];
    uint64_t dy = g_sort_off[y + 1] - g_sort_off[y];
    if (dx != dy) return dx > dy ? -1 : 1;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

ORC_API void orc_dm_permutation(uint64_t n, const uint64_t *off, uint32_t *perm, uint32_t *inv) {
    for (uint64_t v = 0; v < n; v++) perm[v] = (uint32_t)v;
    g_sort_off = off;
    qsort(perm, n, sizeof(uint32_t), cmp_dm);
    for (uint64_t x = 0; x < n; x++) inv[perm[x]] = (uint32_t)x;
}

/* The greedy relabeling heuristic of subsection "Adding Integer Linear
 * Programming" (its listing of a greedy heuristic for vertex relabeling):
 * visit the vertices in increasing order of degree; each visited vertex
 * hands the next unused label to every neighbor, in list order, that has no
 * label yet; vertices that never received one (no edges) take the remaining
 * labels in ID order.  Readings of the printed listing: the vertex IDs are
 * ordered by their degrees (ties by ID; the listing sorts the two arrays
 * independently), the loops start at vertex 0 and labels start at 0 (the
 * listing starts both at 1), and the leftover loop labels vertex i.
 * perm[x] = vertex with new label x, inv[v] = new label of v. */
ORC_API void orc_greedy_permutation(uint64_t n, const uint64_t *off, const uint32_t *col, uint32_t *perm,
                                    uint32_t *inv) {
    if (n == 0) return;
    uint64_t maxd = 0;
    for (uint64_t v = 0; v < n; v++) {
        const uint64_t d = off[v + 1] - off[v];
        if (d > maxd) maxd = d;
    }
    /* IDs ordered by degree ascending, stable (counting sort by degree) */
    uint64_t *start = (uint64_t *)calloc(maxd + 2, sizeof(uint64_t));
    uint32_t *order = (uint32_t *)malloc(n * sizeof(uint32_t));
    unsigned char *visit = (unsigned char *)calloc(n, 1);
    for (uint64_t v = 0; v < n; v++) start[off[v + 1] - off[v] + 1]++;
    for (uint64_t d = 1; d <= maxd + 1; d++) start[d] += start[d - 1];
    for (uint64_t v = 0; v < n; v++) order[start[off[v + 1] - off[v]]++] = (uint32_t)v;
    uint32_t nl = 0;
    for (uint64_t i = 0; i < n; i++) {
        const uint32_t v = order[i];
        for (uint64_t e = off[v]; e < off[v + 1]; e++) {
            const uint32_t id = col[e];
            if (!visit[id]) {
                inv[id] = nl;
                perm[nl] = id;
                nl++;
                visit[id] = 1;
            }
        }
    }
    for (uint64_t i = 0; i < n; i++)
        if (!visit[i]) {
            inv[i] = nl;
            perm[nl] = (uint32_t)i;
            nl++;
        }
    free(start);
    free(order);
    free(visit);
}

/* The relabeled adjacency array: row x is the list of perm[x] with every
 * neighbor renamed through inv and re-sorted ascending (lists are kept
 * sorted, subsection "Adjacency Array Data Structures"). */
ORC_API void orc_relabel(uint64_t n, const uint64_t *off, const uint32_t *col,
                         const uint32_t *perm, const uint32_t *inv,
                         uint64_t *off2, uint32_t *col2) {
    off2[0] = 0;
    for (uint64_t x = 0; x < n; x++) {
        uint32_t v = perm[x];
        uint64_t d = off[v + 1] - off[v];
        off2[x + 1] = off2[x] + d;
        for (uint64_t i = 0; i < d; i++) col2[off2[x] + i] = inv[col[off[v] + i]];
        qsort(col2 + off2[x], d, sizeof(uint32_t), cmp_u32);
    }
}

/* One row of the relabeled adjacency array (row x = list of perm[x]). */
ORC_API void orc_relabel_row(const uint64_t *off, const uint32_t *col, const uint32_t *perm,
                             const uint32_t *inv, uint32_t x, uint32_t *out) {
    uint32_t v = perm[x];
    uint64_t d = off[v + 1] - off[v];
    for (uint64_t i = 0; i < d; i++) out[i] = inv[col[off[v] + i]];
    qsort(out, d, sizeof(uint32_t), cmp_u32);
}

/* ------------------------------------------------------------------ */
/* BFS -- section "Considered Algorithms"                               */
/* ------------------------------------------------------------------ */

/* Textbook FIFO breadth-first search.  depth[v] = hop distance from the
 * root, -1 when unreachable.  Reading of the (non-unique) BFS tree: the
 * parent of a reached v != root is its neighbor of depth depth[v] - 1 whose
 * stored label is smallest; parent[root] = root; parent of an unreached
 * vertex is -1.  `label` gives the stored label of every vertex (NULL: the
 * vertex's own ID); depths do not depend on labels.  With max_depth >= 0
 * every vertex deeper than max_depth is reported as -1 / -1 (k-hop). */
ORC_API int orc_bfs_labels(uint64_t n, const uint64_t *off, const uint32_t *col, uint32_t root,
                           int32_t max_depth, const uint32_t *label, int32_t *depth, int32_t *parent) {
    if (root >= n) return -1;
    uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!queue) return -2;
    for (uint64_t v = 0; v < n; v++) depth[v] = -1;
    uint64_t head = 0, tail = 0;
    depth[root] = 0;
    queue[tail++] = root;
    while (head < tail) {
        uint32_t v = queue[head++];
        for (uint64_t i = off[v]; i < off[v + 1]; i++) {
            uint32_t u = col[i];
            if (depth[u] < 0) {
                depth[u] = depth[v] + 1;
                queue[tail++] = u;
            }
        }
    }
    free(queue);
    for (uint64_t v = 0; v < n; v++) {
        parent[v] = -1;
        if (depth[v] < 0) continue;
        if (v == root) { parent[v] = (int32_t)root; continue; }
        uint32_t best = UINT32_MAX, best_label = UINT32_MAX;
        for (uint64_t i = off[v]; i < off[v + 1]; i++) {
            uint32_t u = col[i];
            uint32_t lu = label ? label[u] : u;
            if (depth[u] == depth[v] - 1 && lu < best_label) { best_label = lu; best = u; }
        }
        parent[v] = (int32_t)best;
    }
    if (max_depth >= 0)
        for (uint64_t v = 0; v < n; v++)
            if (depth[v] > max_depth) { depth[v] = -1; parent[v] = -1; }
    return 0;
}

ORC_API int orc_bfs(uint64_t n, const uint64_t *off, const uint32_t *col, uint32_t root,
                    int32_t max_depth, int32_t *depth, int32_t *parent) {
    return orc_bfs_labels(n, off, col, root, max_depth, NULL, depth, parent);
}

/* BFS when the graph is stored under the degree-minimizing relabeling:
 * the smallest-label rule applies to the new labels; results stay in
 * original IDs. */
ORC_API int orc_bfs_relabeled(uint64_t n, const uint64_t *off, const uint32_t *col, uint32_t root,
                              int32_t max_depth, int32_t *depth, int32_t *parent) {
    if (root >= n) return -1;
    uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t *inv = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    int rc = -2;
    if (perm && inv) {
        orc_dm_permutation(n, off, perm, inv);
        rc = orc_bfs_labels(n, off, col, root, max_depth, inv, depth, parent);
    }
    free(perm); free(inv);
    return rc;
}

/* ------------------------------------------------------------------ */
/* PageRank -- section "Considered Algorithms" (pull variant)           */
/* ------------------------------------------------------------------ */

/* FP64 power iteration on the undirected graph.  Readings of what the
 * paper leaves unstated: PR_0 = 1/n; the rank of vertices without edges
 * (dangling mass D_t) is spread uniformly; exactly `iters` iterations:
 *   PR_{t+1}(v) = (1 - a)/n + a * ( sum_{u in N_v} PR_t(u)/d_u + D_t/n ). */
ORC_API int orc_pagerank(uint64_t n, const uint64_t *off, const uint32_t *col,
                         double alpha, uint32_t iters, double *pr) {
    if (n == 0) return 0;
    double *next = (double *)malloc(sizeof(double) * n);
    if (!next) return -2;
    for (uint64_t v = 0; v < n; v++) pr[v] = 1.0 / (double)n;
    for (uint32_t t = 0; t < iters; t++) {
        double dangling = 0.0;
        for (uint64_t u = 0; u < n; u++)
            if (off[u + 1] == off[u]) dangling += pr[u];
        for (uint64_t v = 0; v < n; v++) {
            double sum = 0.0;
            for (uint64_t i = off[v]; i < off[v + 1]; i++) {
                uint32_t u = col[i];
                sum += pr[u] / (double)(off[u + 1] - off[u]);
            }
            next[v] = (1.0 - alpha) / (double)n + alpha * (sum + dangling / (double)n);
        }
        memcpy(pr, next, sizeof(double) * n);
    }
    free(next);
    return 0;
}

/* ------------------------------------------------------------------ */
/* The same two results on every host core (OpenMP), for graphs where  */
/* the one-thread loops above take minutes.  They compute the same     */
/* definitions; the tests hold them to the one-thread versions and to  */
/* the same independent pins.                                           */
/* ------------------------------------------------------------------ */

/* PageRank as orc_pagerank, bit for bit: the dangling mass is summed in the
 * same vertex order on one thread, each PR_t(u)/d_u is the same division
 * (taken once per vertex instead of once per edge), and each vertex's sum
 * runs over its list in the same order; only different vertices go to
 * different threads.  threads <= 0 takes OpenMP's default. */
ORC_API int orc_pagerank_par(uint64_t n, const uint64_t *off, const uint32_t *col, double alpha, uint32_t iters,
                             double *pr, int threads) {
    if (n == 0) return 0;
    double *next = (double *)malloc(sizeof(double) * n);
    double *contrib = (double *)malloc(sizeof(double) * n);
    if (!next || !contrib) { free(next); free(contrib); return -2; }
    if (threads > 0) omp_set_num_threads(threads);
    const int64_t nn = (int64_t)n;
    for (uint64_t v = 0; v < n; v++) pr[v] = 1.0 / (double)n;
    for (uint32_t t = 0; t < iters; t++) {
        double dangling = 0.0;
        for (uint64_t u = 0; u < n; u++)
            if (off[u + 1] == off[u]) dangling += pr[u];
#pragma omp parallel for schedule(static)
        for (int64_t u = 0; u < nn; u++) {
            const uint64_t d = off[u + 1] - off[u];
            contrib[u] = d ? pr[u] / (double)d : 0.0;
        }
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t v = 0; v < nn; v++) {
            double sum = 0.0;
            for (uint64_t i = off[v]; i < off[v + 1]; i++) sum += contrib[col[i]];
            next[v] = (1.0 - alpha) / (double)n + alpha * (sum + dangling / (double)n);
        }
        memcpy(pr, next, sizeof(double) * n);
    }
    free(next);
    free(contrib);
    return 0;
}

/* Level-synchronous breadth-first search: level d + 1 is every unreached
 * neighbor of a level-d vertex (frontier vertices on several threads; a
 * vertex is claimed by one compare-and-swap of its depth).  Depths equal the
 * FIFO search's; parents follow the same rule as orc_bfs_labels (smallest
 * stored label one level up), taken after the depths are final.  `label`
 * NULL: the vertex's own ID.  With max_depth >= 0 the search stops after
 * that level. */
ORC_API int orc_bfs_levels(uint64_t n, const uint64_t *off, const uint32_t *col, uint32_t root, int32_t max_depth,
                           const uint32_t *label, int32_t *depth, int32_t *parent, int threads) {
    if (root >= n) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    const int64_t nn = (int64_t)n;
    uint32_t *front = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *nextf = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!front || !nextf) { free(front); free(nextf); return -2; }
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nn; v++) depth[v] = -1;
    depth[root] = 0;
    front[0] = root;
    uint64_t fsize = 1, nsize = 0;
    for (int32_t d = 0; fsize > 0 && (max_depth < 0 || d < max_depth); d++) {
        nsize = 0;
#pragma omp parallel
        {
            /* claimed vertices gather in a small local buffer, then move to
             * the next frontier in one reservation */
            uint32_t buf[1024];
            uint64_t nb = 0;
#pragma omp for schedule(dynamic, 64)
            for (int64_t k = 0; k < (int64_t)fsize; k++) {
                const uint32_t v = front[k];
                for (uint64_t i = off[v]; i < off[v + 1]; i++) {
                    const uint32_t u = col[i];
                    int32_t expect = -1;
                    if (__atomic_load_n(&depth[u], __ATOMIC_RELAXED) == -1 &&
                        __atomic_compare_exchange_n(&depth[u], &expect, d + 1, 0, __ATOMIC_RELAXED,
                                                    __ATOMIC_RELAXED)) {
                        buf[nb++] = u;
                        if (nb == 1024) {
                            const uint64_t at = __atomic_fetch_add(&nsize, nb, __ATOMIC_RELAXED);
                            memcpy(nextf + at, buf, nb * sizeof(uint32_t));
                            nb = 0;
                        }
                    }
                }
            }
            if (nb) {
                const uint64_t at = __atomic_fetch_add(&nsize, nb, __ATOMIC_RELAXED);
                memcpy(nextf + at, buf, nb * sizeof(uint32_t));
            }
        }
        uint32_t *t = front; front = nextf; nextf = t;
        fsize = nsize;
    }
    free(front);
    free(nextf);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < nn; v++) {
        parent[v] = -1;
        if (depth[v] < 0) continue;
        if ((uint64_t)v == root) { parent[v] = (int32_t)root; continue; }
        uint32_t best = UINT32_MAX, best_label = UINT32_MAX;
        for (uint64_t i = off[v]; i < off[v + 1]; i++) {
            const uint32_t u = col[i];
            const uint32_t lu = label ? label[u] : u;
            if (depth[u] == depth[v] - 1 && lu < best_label) { best_label = lu; best = u; }
        }
        parent[v] = (int32_t)best;
    }
    return 0;
}

/* Threads OpenMP would use by default (the host's cores unless limited). */
ORC_API int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Plain and interleaved bit vectors for O -- subsection "Arrays of    */
/* Offsets vs. Bit Vectors for O" and its table of offset structures   */
/* (bvPL, bvIL)                                                         */
/* ------------------------------------------------------------------ */

/* Both hold the offsets x_0 <= x_1 <= ... <= x_n (universe u = x_n) as one
 * plain bit vector in which the one of list v marks where that list starts.
 * Reading (the paper sets the bit of the block where a list starts, which
 * cannot mark two lists starting at the same place, i.e. empty lists): as
 * for the Elias-Fano upper bits, the one of list v goes to position
 * x_v + v, so the vector has u + n + 1 bits, exactly n + 1 ones, and
 * select1(v) - v = x_v.  The blocks are the units of the offsets themselves:
 * elements with global IDs, bits with local IDs. */
ORC_API uint64_t orc_bv_bits(uint64_t count, uint64_t universe) { return universe + count; }

/* bvPL: the plain bit vector plus a directory for select, kept in the same
 * form as the Elias-Fano one so that every entry is a plain rank or select
 * value: rank_sb[b] = rank1(512 b) for b = 0 .. ceil(bits / 512) (the extra
 * last entry holds all n + 1 ones) and sel[j] = select1(64 j) for
 * j < ceil((n + 1) / 64).  `bits` holds orc_stream_words(orc_bv_bits(..))
 * zeroed words; positions must stay below 2^32 (sel is 32-bit). */
ORC_API void orc_bv_plain_build(const uint64_t *x, uint64_t count, uint64_t universe, uint64_t *bits,
                                uint32_t *rank_sb, uint32_t *sel) {
    const uint64_t nbits = orc_bv_bits(count, universe);
    for (uint64_t v = 0; v < count; v++) put_bit(bits, x[v] + v);
    const uint64_t nr = orc_ef_rank_entries(nbits), ns = orc_ef_select_entries(count);
    uint64_t ones = 0;
    for (uint64_t p = 0; p <= nbits; p++) {
        if (p % 512 == 0 && p / 512 < nr) rank_sb[p / 512] = (uint32_t)ones;
        if (p == nbits) break;
        if (get_bit(bits, p)) {
            if (ones % 64 == 0 && ones / 64 < ns) sel[ones / 64] = (uint32_t)p;
            ones++;
        }
    }
    rank_sb[nr - 1] = (uint32_t)ones;
}

/* x_v from the plain bit vector: select1(v) - v (linear scan) */
ORC_API uint64_t orc_bv_plain_get(const uint64_t *bits, uint64_t nbits, uint64_t v) {
    return orc_select1(bits, nbits, v) - v;
}

/* bvIL: the same bit vector cut into blocks of 512 bits, each block preceded
 * by one 64-bit word holding the number of ones before it (the cumulative
 * sums the paper interleaves with the data every L bits; L = 512 here).
 * Block j takes words [9 j, 9 j + 9): word 9 j = rank1(512 j), words
 * 9 j + 1 .. 9 j + 8 = bits [512 j, 512 j + 512) of the vector.  One word
 * after the last block holds the total, n + 1.  `words` holds
 * orc_bvil_words(..) zeroed words. */
ORC_API uint64_t orc_bvil_words(uint64_t nbits) { return ((nbits + 511) / 512) * 9 + 1; }

ORC_API void orc_bvil_build(const uint64_t *x, uint64_t count, uint64_t universe, uint64_t *words) {
    const uint64_t nbits = orc_bv_bits(count, universe);
    const uint64_t blocks = (nbits + 511) / 512;
    for (uint64_t v = 0; v < count; v++) {
        const uint64_t p = x[v] + v;                      /* bit p of the vector */
        const uint64_t j = p / 512, in = p % 512;         /* block j, bit `in` of its data */
        put_bit(words, (9 * j + 1) * 64 + in);
    }
    uint64_t ones = 0;
    for (uint64_t j = 0; j < blocks; j++) {
        words[9 * j] = ones;
        for (uint64_t in = 0; in < 512; in++) ones += (uint64_t)get_bit(words, (9 * j + 1) * 64 + in);
    }
    words[9 * blocks] = ones;
}

/* x_v from the interleaved layout: the v-th one, found by walking the data
 * bits of the blocks in order (the count words are not used), minus v */
ORC_API uint64_t orc_bvil_get(const uint64_t *words, uint64_t nbits, uint64_t v) {
    uint64_t seen = 0;
    for (uint64_t p = 0; p < nbits; p++) {
        if (get_bit(words, (9 * (p / 512) + 1) * 64 + p % 512)) {
            if (seen == v) return p - v;
            seen++;
        }
    }
    return UINT64_MAX;
}
