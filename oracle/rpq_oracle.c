/*
 * CPU oracle for regular path queries -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code.  It shares nothing with the HIP library: its own graph
 * layout, its own automaton format (an epsilon-NFA with explicit
 * epsilon-closures, so Thompson automata run unchanged) and its own hash.
 *
 * What it computes (paper, Section 2.1, Definition 1, and the automata-based
 * evaluation of Section 2.2): for every source s, the set of vertices y such
 * that some walk s -> ... -> y has a label word accepted by the automaton.
 * The search is a plain breadth-first search over the product of the data
 * graph and the automaton, one visited set of (vertex, state) pairs per
 * source; a pair (s, y) is recorded whenever a final state is reached at y.
 * A zero-length walk counts: if the closure of the start state holds a final
 * state, (s, s) is in the result.  Walks, not simple paths; no hop bound
 * unless one is asked for.
 *
 * Length-bounded RPQs (the extension the paper's conclusion names: a length
 * constraint enforced by controlling the traversal depth): with max_len = k
 * only walks of at most k edges count.  The search is breadth-first, so a
 * product pair first reached at depth d has a walk of exactly d edges and none
 * shorter; pairs at depth k are recorded but not expanded.
 *
 * Result keys are (s << 32) | y, emitted per source in ascending y.  The
 * checksum of a key is one SplitMix64 output (Steele, Lea, Flood, OOPSLA
 * 2014) for state = key; sums are taken modulo 2^64.
 *
 * Product edges examined: for each dequeued (v, q) that is expanded, each
 * labelled transition (q, l, p) and each edge (v, l, w) counts one.  On an
 * epsilon-free automaton this is the sum over expanded (v, q) of
 * sum_l deg_l(v) * |delta(q, l)| (every reached pair is expanded unless a
 * length bound stops it).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t oracle_splitmix64_output(uint64_t state)
{
    /* SplitMix64: advance the state by the golden-ratio increment, then mix. */
    uint64_t z = state + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t oracle_mix64(uint64_t x) { return oracle_splitmix64_output(x); }

/* Checksum of a key sequence: the sum of mix64(key) modulo 2^64 (order-free). */
uint64_t oracle_hash_keys(const uint64_t* keys, uint64_t n)
{
    uint64_t h = 0;
    for (uint64_t i = 0; i < n; ++i) h += oracle_splitmix64_output(keys[i]);
    return h;
}

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

static int cmp_u32(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

/*
 * Adjacency for the oracle: per source vertex, its distinct (label, dst)
 * pairs sorted by label then dst.  off has n_vertices+1 entries; out_lab and
 * out_dst must hold n_edges entries.  Returns the number of distinct edges.
 */
uint64_t oracle_graph_build(uint32_t n_vertices, uint64_t n_edges, const uint32_t* src,
                            const uint8_t* lab, const uint32_t* dst,
                            uint64_t* off, uint32_t* out_lab, uint32_t* out_dst)
{
    uint64_t* cnt = (uint64_t*)calloc((size_t)n_vertices + 1, sizeof(uint64_t));
    uint64_t* key = (uint64_t*)malloc((size_t)(n_edges ? n_edges : 1) * sizeof(uint64_t));
    uint64_t* pos = (uint64_t*)malloc(((size_t)n_vertices + 1) * sizeof(uint64_t));
    for (uint64_t e = 0; e < n_edges; ++e) cnt[src[e] + 1]++;
    for (uint32_t v = 0; v < n_vertices; ++v) cnt[v + 1] += cnt[v];
    memcpy(pos, cnt, ((size_t)n_vertices + 1) * sizeof(uint64_t));
    for (uint64_t e = 0; e < n_edges; ++e)
        key[pos[src[e]]++] = ((uint64_t)lab[e] << 32) | dst[e];
    uint64_t out = 0;
    off[0] = 0;
    for (uint32_t v = 0; v < n_vertices; ++v) {
        uint64_t b = cnt[v], e = cnt[v + 1];
        qsort(key + b, (size_t)(e - b), sizeof(uint64_t), cmp_u64);
        for (uint64_t i = b; i < e; ++i) {
            if (i > b && key[i] == key[i - 1]) continue;
            out_lab[out] = (uint32_t)(key[i] >> 32);
            out_dst[out] = (uint32_t)(key[i] & 0xffffffffULL);
            ++out;
        }
        off[v + 1] = out;
    }
    free(cnt); free(key); free(pos);
    return out;
}

/* first index in [b, e) whose label is >= l */
static uint64_t label_lower(const uint32_t* g_lab, uint64_t b, uint64_t e, uint32_t l)
{
    while (b < e) {
        uint64_t m = b + (e - b) / 2;
        if (g_lab[m] < l) b = m + 1; else e = m;
    }
    return b;
}

typedef struct { uint64_t* a; uint64_t n, cap; } vec64;

static int vpush(vec64* v, uint64_t x)
{
    if (v->n == v->cap) {
        uint64_t nc = v->cap ? 2 * v->cap : 1024;
        uint64_t* na = (uint64_t*)realloc(v->a, (size_t)nc * sizeof(uint64_t));
        if (!na) return -1;
        v->a = na; v->cap = nc;
    }
    v->a[v->n++] = x;
    return 0;
}

/*
 * Evaluate the query from each source in sources[0..n_sources).
 *
 * Automaton: states 0..n_states-1, start state `start`, is_final[q] != 0 for
 * final states, labelled transitions grouped by origin state: transitions of
 * state q are t_label[t], t_to[t] for t in [t_off[q], t_off[q+1]).
 * eps_closure[i * n_states + j] != 0 iff j is in the epsilon-closure of i
 * (every state is in its own closure).
 *
 * Outputs (any pointer may be NULL):
 *   pairs[0..pairs_cap)      keys in (source order, ascending y); keys past the
 *                            capacity are counted but not written
 *   per_source[2*i+0/1]      count and checksum of source i
 *   totals[0..4)             count, checksum, product edges, max hops
 * max_len: the longest walk (in edges) that counts; UINT64_MAX for none.
 * Returns 0, or -1 when memory runs out.
 */
int oracle_rpq_eval(uint32_t n_vertices, const uint64_t* g_off, const uint32_t* g_lab,
                    const uint32_t* g_dst, uint32_t n_states, uint32_t start,
                    const uint8_t* is_final, const uint32_t* t_off, const uint32_t* t_label,
                    const uint32_t* t_to, const uint8_t* eps_closure, const uint32_t* sources,
                    uint64_t n_sources, uint64_t* pairs, uint64_t pairs_cap,
                    uint64_t* per_source, uint64_t* totals, uint64_t max_len)
{
    const uint64_t S = n_states;
    uint8_t* seen = (uint8_t*)calloc((size_t)n_vertices * S, 1);
    uint8_t* hit = (uint8_t*)calloc((size_t)n_vertices, 1);
    vec64 queue = {0, 0, 0};
    vec64 found = {0, 0, 0};
    if (!seen || !hit) { free(seen); free(hit); return -1; }
    uint64_t total_count = 0, total_hash = 0, prod_edges = 0, max_hops = 0, written = 0;

    for (uint64_t si = 0; si < n_sources; ++si) {
        const uint32_t s = sources[si];
        queue.n = 0; found.n = 0;
        /* level 0: the closure of the start state at the source */
        for (uint32_t q = 0; q < n_states; ++q) {
            if (!eps_closure[(uint64_t)start * S + q]) continue;
            seen[(uint64_t)s * S + q] = 1;
            if (vpush(&queue, (uint64_t)s * S + q)) goto oom;
            if (is_final[q] && !hit[s]) { hit[s] = 1; if (vpush(&found, s)) goto oom; }
        }
        uint64_t head = 0, level_end = queue.n, hops = 0;
        while (head < queue.n) {
            if (head == level_end) { ++hops; level_end = queue.n; }
            const uint64_t pv = queue.a[head++];
            const uint32_t v = (uint32_t)(pv / S), q = (uint32_t)(pv % S);
            if (hops >= max_len) continue;   /* its walks already have max_len edges */
            for (uint32_t t = t_off[q]; t < t_off[q + 1]; ++t) {
                const uint32_t l = t_label[t], p = t_to[t];
                uint64_t e = label_lower(g_lab, g_off[v], g_off[v + 1], l);
                for (; e < g_off[v + 1] && g_lab[e] == l; ++e) {
                    const uint32_t w = g_dst[e];
                    ++prod_edges;
                    for (uint32_t r = 0; r < n_states; ++r) {
                        if (!eps_closure[(uint64_t)p * S + r]) continue;
                        const uint64_t idx = (uint64_t)w * S + r;
                        if (seen[idx]) continue;
                        seen[idx] = 1;
                        if (vpush(&queue, idx)) goto oom;
                        if (is_final[r] && !hit[w]) { hit[w] = 1; if (vpush(&found, w)) goto oom; }
                    }
                }
            }
        }
        if (hops > max_hops) max_hops = hops;
        /* ordered distinct destinations of s */
        uint32_t* ys = (uint32_t*)malloc((size_t)(found.n ? found.n : 1) * sizeof(uint32_t));
        if (!ys) goto oom;
        for (uint64_t i = 0; i < found.n; ++i) ys[i] = (uint32_t)found.a[i];
        qsort(ys, (size_t)found.n, sizeof(uint32_t), cmp_u32);
        uint64_t c = 0, h = 0;
        for (uint64_t i = 0; i < found.n; ++i) {
            const uint64_t key = ((uint64_t)s << 32) | ys[i];
            ++c;
            h += oracle_splitmix64_output(key);
            if (pairs && written < pairs_cap) pairs[written] = key;
            ++written;
        }
        free(ys);
        if (per_source) { per_source[2 * si] = c; per_source[2 * si + 1] = h; }
        total_count += c; total_hash += h;
        /* reset the visited set and the hit marks touched by this source */
        for (uint64_t i = 0; i < queue.n; ++i) seen[queue.a[i]] = 0;
        for (uint64_t i = 0; i < found.n; ++i) hit[found.a[i]] = 0;
    }
    if (totals) { totals[0] = total_count; totals[1] = total_hash; totals[2] = prod_edges; totals[3] = max_hops; }
    free(seen); free(hit); free(queue.a); free(found.a);
    return 0;
oom:
    free(seen); free(hit); free(queue.a); free(found.a);
    return -1;
}
