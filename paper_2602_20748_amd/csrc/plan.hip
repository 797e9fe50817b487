// Split plans: a query head . tail evaluated through a materialized sub-result (WavePlan's
// loop-cache and start-in-the-middle plans, Section 2.3, as executed in Section 6: one sub-RPQ
// result is materialized in one direction, then joined with the rest of the expression).
//
// Walks split at the boundary between head and tail, so R(head . tail) is the composition of
// R(head) and R(tail): (x, y) is a result iff some middle vertex m has (x, m) in R(head) and
// (m, y) in R(tail).  The plan runs in three steps, each on the bit-parallel engine:
//   1. head from the sources, with pairs: their distinct targets are the middle vertices M;
//   2. tail from M (the start-in-the-middle exploration), with pairs: each (m, y) becomes an
//      edge m -lambda-> y of a new label lambda (the materialized relation, kept in out-edge
//      order, the slice direction the join walks);
//   3. head . lambda over the graph with lambda added: the join of the two relations, bit-parallel
//      over the sources, with the result keys in source order.
// The closure inside tail is explored once per middle vertex instead of once per unit of
// sources that reaches it.  This entry allocates device memory for its steps and the derived
// graph, frees it before returning, and synchronises the stream.
#include <hip/hip_runtime.h>

#include "internal.h"

#include <algorithm>
#include <cstring>
#include <vector>

namespace {

constexpr int kThreads = 256;

unsigned grid_for(uint64_t n, uint64_t cap = 16384) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + kThreads - 1) / kThreads, cap));
}

// every edge of a CSR as (src, label, dst); one thread per (vertex, label) row
__global__ void k_csr_edges(const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ dst, uint32_t V,
                            uint32_t L, uint32_t* __restrict__ es, uint8_t* __restrict__ el,
                            uint32_t* __restrict__ ed) {
    const uint64_t R = (uint64_t)V * L;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += stride) {
        const uint32_t v = (uint32_t)(r / L), l = (uint32_t)(r % L);
        for (uint32_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
            es[e] = v;
            el[e] = (uint8_t)l;
            ed[e] = dst[e];
        }
    }
}

// result keys (src << 32 | dst) as edges of one label, appended at offset `base`
__global__ void k_key_edges(const uint64_t* __restrict__ keys, uint64_t n, uint32_t label, uint64_t base,
                            uint32_t* __restrict__ es, uint8_t* __restrict__ el, uint32_t* __restrict__ ed) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        es[base + i] = (uint32_t)(keys[i] >> 32);
        el[base + i] = (uint8_t)label;
        ed[base + i] = (uint32_t)keys[i];
    }
}

// the set of targets of result keys: a bitmap of V bits
__global__ void k_target_bits(const uint64_t* __restrict__ keys, uint64_t n, uint64_t* __restrict__ bits) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t y = (uint32_t)keys[i];
        atomicOr(reinterpret_cast<unsigned long long*>(&bits[y >> 6]), 1ull << (y & 63));
    }
}

// bitmap -> ascending vertex list: per word its population count, then (after a scan) its vertices
__global__ void k_word_pop(const uint64_t* __restrict__ bits, uint64_t n_words, uint64_t* __restrict__ pop) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += stride)
        pop[i] = (uint64_t)__popcll(bits[i]);
}

__global__ void k_word_list(const uint64_t* __restrict__ bits, const uint64_t* __restrict__ pos, uint64_t n_words,
                            uint32_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += stride) {
        uint64_t w = bits[i], p = pos[i];
        while (w) {
            const int b = __ffsll((long long)w) - 1;
            w &= w - 1;
            out[p++] = (uint32_t)(i * 64 + b);
        }
    }
}

// device buffers of one plan, freed on every return path
struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    int get(T** out, uint64_t count) {
        void* p = nullptr;
        const hipError_t e = hipMalloc(&p, std::max<uint64_t>(8, count * sizeof(T)));
        if (e != hipSuccess) {
            rpq::set_error("hipMalloc(%llu) failed: %s", (unsigned long long)(count * sizeof(T)), hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? RPQ_ENOMEM : RPQ_EDEVICE;
        }
        ptrs.push_back(p);
        *out = static_cast<T*>(p);
        return RPQ_OK;
    }
};

struct GraphGuard {
    rpq_graph_t g = nullptr;
    ~GraphGuard() {
        if (g) (void)rpq_graph_destroy(g);
    }
};

// rpq_eval with its own workspace; keys (sorted, distinct) into a buffer sized by a count pass
int eval_keys(rpq_graph_t g, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources, uint32_t flags,
              const rpq_eval_opts* opts, Scratch& sc, uint64_t** keys, uint64_t* n_keys, hipStream_t s) {
    uint64_t ws_bytes = 0;
    RPQ_TRY(rpq_eval_workspace_size(g, nfa, n_sources, flags | RPQ_PAIRS, opts, &ws_bytes));
    uint8_t* ws = nullptr;
    RPQ_TRY(sc.get(&ws, ws_bytes));
    rpq_result r;
    std::memset(&r, 0, sizeof r);
    RPQ_TRY(rpq::eval_impl(g, nfa, sources, n_sources, flags & ~RPQ_PAIRS, opts, nullptr, ws, ws_bytes, &r, s));
    uint64_t* k = nullptr;
    RPQ_TRY(sc.get(&k, r.count));
    const uint64_t count = r.count;
    std::memset(&r, 0, sizeof r);
    r.pairs = k;
    r.capacity = count;
    RPQ_TRY(rpq::eval_impl(g, nfa, sources, n_sources, flags | RPQ_PAIRS, opts, nullptr, ws, ws_bytes, &r, s));
    *keys = k;
    *n_keys = count;
    return RPQ_OK;
}

int split_impl(rpq_graph_t g, const rpq_nfa* head, const rpq_nfa* tail, const uint32_t* sources, uint64_t n_sources,
               uint32_t flags, const rpq_eval_opts* opts, rpq_result* res, rpq_split_info* info, hipStream_t s) {
    if (!g || !head || !tail || !res) {
        rpq::set_error("graph, automata and result must be non-NULL");
        return RPQ_EINVAL;
    }
    if (flags & ~(RPQ_PAIRS | RPQ_PER_SOURCE | RPQ_ALL_SOURCES)) {
        rpq::set_error("split plans take RPQ_PAIRS, RPQ_PER_SOURCE and RPQ_ALL_SOURCES only");
        return RPQ_EUNSUPPORTED;
    }
    if (opts && (opts->visit > RPQ_VISIT_SEEN_OR)) {
        rpq::set_error("rpq_eval_opts.visit must be 0, RPQ_VISIT_TWO_READS or RPQ_VISIT_SEEN_OR");
        return RPQ_EINVAL;
    }
    if ((flags & RPQ_ALL_SOURCES) && n_sources == 0) n_sources = g->V;
    if (g->L >= RPQ_MAX_LABELS) {
        rpq::set_error("the graph has %u labels: no label id is left for the materialized relation", g->L);
        return RPQ_EUNSUPPORTED;
    }
    if (head->n_states >= RPQ_MAX_STATES) {
        rpq::set_error("head automaton has %u states; the plan adds one (at most %d)", head->n_states,
                       RPQ_MAX_STATES);
        return RPQ_EUNSUPPORTED;
    }
    // head . lambda: one more state, reached from every final state of head by the new label
    rpq_nfa joined;
    RPQ_TRY(rpq_nfa_append_label(head, g->L, &joined));
    const uint32_t lambda = g->L;
    const uint32_t pass = flags & RPQ_ALL_SOURCES;
    Scratch sc;
    // 1. head from the sources: the middle vertices
    uint64_t* hk = nullptr;
    uint64_t n_hk = 0;
    RPQ_TRY(eval_keys(g, head, sources, n_sources, pass, opts, sc, &hk, &n_hk, s));
    const uint64_t n_words = ((uint64_t)g->V + 63) / 64;
    uint64_t *bits = nullptr, *pos = nullptr, *tmp = nullptr;
    RPQ_TRY(sc.get(&bits, n_words));
    RPQ_TRY(sc.get(&pos, n_words + 1));
    RPQ_TRY(sc.get(&tmp, rpq::scan_temp_elems(n_words)));
    RPQ_TRY(rpq::fill_u64(bits, n_words, 0, s));
    if (n_hk) {
        hipLaunchKernelGGL(k_target_bits, dim3(grid_for(n_hk)), dim3(kThreads), 0, s, hk, n_hk, bits);
        RPQ_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_word_pop, dim3(grid_for(n_words)), dim3(kThreads), 0, s, bits, n_words, pos);
    RPQ_LAUNCH_CHECK();
    RPQ_TRY(rpq::exclusive_scan_u64(pos, pos, n_words, tmp, pos + n_words, s));
    uint64_t n_mid = 0;
    RPQ_HIP(hipMemcpyAsync(&n_mid, pos + n_words, 8, hipMemcpyDeviceToHost, s));
    RPQ_HIP(hipStreamSynchronize(s));
    uint32_t* mid = nullptr;
    RPQ_TRY(sc.get(&mid, n_mid));
    hipLaunchKernelGGL(k_word_list, dim3(grid_for(n_words)), dim3(kThreads), 0, s, bits, pos, n_words, mid);
    RPQ_LAUNCH_CHECK();
    // 2. tail from the middle vertices: the relation to materialize
    uint64_t* tk = nullptr;
    uint64_t n_tk = 0;
    if (n_mid) RPQ_TRY(eval_keys(g, tail, mid, n_mid, 0, opts, sc, &tk, &n_tk, s));
    // 3. the graph with lambda, then head . lambda from the sources
    const uint64_t E = g->E, n_edges = E + n_tk;
    uint32_t *es = nullptr, *ed = nullptr;
    uint8_t* el = nullptr;
    RPQ_TRY(sc.get(&es, n_edges));
    RPQ_TRY(sc.get(&ed, n_edges));
    RPQ_TRY(sc.get(&el, n_edges));
    hipLaunchKernelGGL(k_csr_edges, dim3(grid_for((uint64_t)g->V * g->L)), dim3(kThreads), 0, s, g->out.row_ptr,
                       g->out.dst, g->V, g->L, es, el, ed);
    RPQ_LAUNCH_CHECK();
    if (n_tk) {
        hipLaunchKernelGGL(k_key_edges, dim3(grid_for(n_tk)), dim3(kThreads), 0, s, tk, n_tk, lambda, E, es, el, ed);
        RPQ_LAUNCH_CHECK();
    }
    GraphGuard g2;
    RPQ_TRY(rpq_graph_create(es, el, ed, n_edges, g->V, g->L + 1, nullptr, 0, s, &g2.g));
    uint64_t ws_bytes = 0;
    RPQ_TRY(rpq_eval_workspace_size(g2.g, &joined, n_sources, flags, opts, &ws_bytes));
    uint8_t* ws = nullptr;
    RPQ_TRY(sc.get(&ws, ws_bytes));
    const int rc = rpq::eval_impl(g2.g, &joined, sources, n_sources, flags, opts, nullptr, ws, ws_bytes, res, s);
    if (rc != RPQ_OK && rc != RPQ_EOVERFLOW) return rc;
    if (info) {
        info->head_pairs = n_hk;
        info->middle_vertices = n_mid;
        info->tail_pairs = n_tk;
        info->derived_edges = g2.g->E;
    }
    // the scratch (and the derived graph) go when this returns: their last users must be done
    RPQ_HIP(hipStreamSynchronize(s));
    return rc;
}

}  // namespace

extern "C" {

int rpq_nfa_append_label(const rpq_nfa* in, uint32_t label, rpq_nfa* out) {
    rpq::clear_error();
    if (!in || !out) {
        rpq::set_error("automaton is NULL");
        return RPQ_EINVAL;
    }
    if (in->n_states == 0 || in->n_states >= RPQ_MAX_STATES || label >= RPQ_MAX_LABELS ||
        in->n_labels > RPQ_MAX_LABELS) {
        rpq::set_error("append: automaton of 1..%d states and a label id below %d", RPQ_MAX_STATES - 1,
                       RPQ_MAX_LABELS);
        return RPQ_EINVAL;
    }
    rpq_nfa o = *in;
    const uint32_t f = in->n_states;
    o.n_states = f + 1;
    o.n_labels = std::max(in->n_labels, label + 1);
    for (uint32_t q = 0; q < in->n_states; ++q)
        if ((in->final_mask >> q) & 1) o.delta[q * RPQ_MAX_LABELS + label] |= 1u << f;
    o.final_mask = 1u << f;
    *out = o;
    return RPQ_OK;
}

int rpq_eval_split(rpq_graph_t g, const rpq_nfa* head, const rpq_nfa* tail, const uint32_t* sources,
                   uint64_t n_sources, uint32_t flags, const rpq_eval_opts* opts, rpq_result* result,
                   rpq_split_info* info, hipStream_t stream) {
    rpq::clear_error();
    const int rc = split_impl(g, head, tail, sources, n_sources, flags, opts, result, info, stream);
    if (rc != RPQ_OK && rc != RPQ_EOVERFLOW) (void)hipStreamSynchronize(stream);
    return rc;
}

}  // extern "C"
