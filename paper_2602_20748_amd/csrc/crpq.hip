// Conjunctive regular path queries (Definition 2): the atoms are evaluated first and their
// results joined, as in the paper's CRPQ processing (Section 6.2).
//
// Data, all in the caller's workspace (a stack arena; nothing is allocated):
//   domains    one bitmap of V bits per variable: binding, vertex label and sample intersected;
//              shrunk by every atom result that involves the variable (semi-join reduction)
//   relations  per atom, its distinct pairs as sorted uint64 keys (f(x) << 32 | f(y)); a
//              transposed copy (f(y) << 32 | f(x)) only when the join reaches the atom from y
//              (the paper's slice transpose)
//   table      the join's partial assignments, column-major uint32, one column per bound
//              variable, rows in no particular order
//
// Atom evaluation, from the smaller of its two domains (backwards over the in-CSR with the
// reversed automaton when that is the destination's):
//   edge scan  the language holds only one-label words: a CSR scan of the source domain
//   dense      up to 65,536 sources: the bit-parallel traversal of rpq_eval, with result
//              vertices filtered by the destination domain at extraction
//   sparse     more sources: a per-source breadth-first search over (source, state, vertex)
//              triples with a device hash set as the visited set, for atoms whose sources
//              are many but reach little (a reply chain from millions of messages)
//
// Join: variables are bound one at a time (a vertex-at-a-time join).  For each partial row
// the candidates of the new variable z come from the shortest of the sorted lists that the
// atoms connecting z to bound variables give for that row, and each candidate must appear in
// the other lists, in z's domain, and differ from the variables z must differ from.  Work is
// spread over the grid by a prefix sum of per-row candidate counts, so one row with millions
// of candidates does not serialise on one wave.
#include "internal.h"

#include <algorithm>
#include <cstring>
#include <vector>

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr unsigned long long kEmpty = ~0ull;
constexpr uint64_t kDenseMaxSources = 65536;
constexpr int kMaxConn = CRPQ_MAX_ATOMS;
constexpr int kTile = 1024;            // keys per block in the order-preserving compaction
constexpr uint32_t kMaxProbe = 4096;   // hash-set probes before an insert gives up

inline uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

inline unsigned grid_for(uint64_t threads, unsigned cap = 65535) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((threads + kBlock - 1) / kBlock, cap));
}

// ------------------------------------------------------------------------------------------------
// device helpers
// ------------------------------------------------------------------------------------------------
// Wave-aggregated append: lanes with keep get consecutive positions from *counter (one atomic
// per wave).  Every lane of the wave must call it.
__device__ __forceinline__ uint64_t wave_append(bool keep, unsigned long long* counter) {
    const uint64_t m = __ballot(keep);
    unsigned long long base = 0;
    if (__lane_id() == 0 && m) base = atomicAdd(counter, (unsigned long long)__popcll(m));
    base = __shfl(base, 0, 64);
    return base + (uint64_t)__popcll(m & rpqd::lanemask_lt());
}

// Last lane c whose exclusive prefix is <= item (the lane owning item).
__device__ __forceinline__ int wave_owner(uint64_t excl, uint64_t item) {
    int c = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
        const int cand = c + step;
        const uint64_t e = __shfl(excl, cand, 64);
        if (e <= item) c = cand;
    }
    return c;
}

// First index in [lo, hi) with keys[i] >= key.
__device__ __forceinline__ uint64_t lower_bound(const uint64_t* keys, uint64_t lo, uint64_t hi, uint64_t key) {
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool contains(const uint64_t* keys, uint64_t lo, uint64_t hi, uint64_t key) {
    const uint64_t i = lower_bound(keys, lo, hi, key);
    return i < hi && keys[i] == key;
}

__device__ __forceinline__ bool bit_of(const uint64_t* bits, uint64_t v) { return (bits[v >> 6] >> (v & 63)) & 1; }

__device__ __forceinline__ uint64_t gthread() { return (uint64_t)blockIdx.x * kBlock + threadIdx.x; }
__device__ __forceinline__ uint64_t gstride() { return (uint64_t)gridDim.x * kBlock; }
// first item of this thread's wave in a wave-uniform grid-stride loop
__device__ __forceinline__ uint64_t gwave_base() { return (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~63u); }

// ------------------------------------------------------------------------------------------------
// domains
// ------------------------------------------------------------------------------------------------
__global__ void k_dom_build(uint64_t* __restrict__ bits, uint64_t V, const uint8_t* __restrict__ vlabel,
                            int32_t label, int64_t bound) {
    const uint64_t n_words = (V + 63) / 64;
    const int lane = __lane_id();
    for (uint64_t w = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); w < n_words;
         w += (uint64_t)gridDim.x * kWaves) {
        const uint64_t v = w * 64 + lane;
        bool ok = v < V;
        if (ok && label >= 0) ok = vlabel[v] == (uint8_t)label;
        if (ok && bound >= 0) ok = v == (uint64_t)bound;
        const uint64_t word = __ballot(ok);
        if (lane == 0) bits[w] = word;
    }
}

__global__ void k_bits_from_list(uint64_t* __restrict__ tmp, const uint32_t* __restrict__ list, uint64_t n,
                                 uint64_t V, unsigned long long* __restrict__ err) {
    for (uint64_t i = gthread(); i < n; i += gstride()) {
        const uint32_t x = list[i];
        if (x >= V) atomicOr(err, 1ull);
        else atomicOr(reinterpret_cast<unsigned long long*>(&tmp[x >> 6]), 1ull << (x & 63));
    }
}

__global__ void k_bits_from_keys(uint64_t* __restrict__ tmp, const uint64_t* __restrict__ keys, uint64_t n,
                                 int hi) {
    for (uint64_t i = gthread(); i < n; i += gstride()) {
        const uint64_t v = hi ? (keys[i] >> 32) : (keys[i] & 0xFFFFFFFFull);
        atomicOr(reinterpret_cast<unsigned long long*>(&tmp[v >> 6]), 1ull << (v & 63));
    }
}

__global__ void k_and(uint64_t* __restrict__ bits, const uint64_t* __restrict__ tmp, uint64_t n_words) {
    for (uint64_t i = gthread(); i < n_words; i += gstride()) bits[i] &= tmp[i];
}

__global__ void k_word_popc(const uint64_t* __restrict__ bits, uint64_t n_words, uint64_t* __restrict__ counts) {
    for (uint64_t i = gthread(); i < n_words; i += gstride()) counts[i] = (uint64_t)__popcll(bits[i]);
}

// ascending vertex list of a bitmap, given the exclusive prefix of per-word popcounts
__global__ void k_bits_to_list(const uint64_t* __restrict__ bits, const uint64_t* __restrict__ offs,
                               uint64_t n_words, uint32_t* __restrict__ list) {
    for (uint64_t i = gthread(); i < n_words; i += gstride()) {
        uint64_t w = bits[i];
        uint64_t pos = offs[i];
        while (w) {
            const int b = __ffsll((long long)w) - 1;
            w &= w - 1;
            list[pos++] = (uint32_t)(i * 64 + b);
        }
    }
}

__global__ void k_swap_halves(const uint64_t* __restrict__ in, uint64_t* __restrict__ out, uint64_t n) {
    for (uint64_t i = gthread(); i < n; i += gstride()) {
        const uint64_t k = in[i];
        out[i] = (k << 32) | (k >> 32);
    }
}

// ------------------------------------------------------------------------------------------------
// order-preserving compaction of sorted keys: mode 0 keeps the first of each run of equal keys,
// mode 1 additionally keeps only keys with equal halves (pairs (v, v)); with domain bitmaps (or
// null) only keys whose high half is in dhi and whose low half is in dlo
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ bool keep_key(const uint64_t* keys, uint64_t i, int mode, const uint64_t* dhi,
                                         const uint64_t* dlo) {
    const uint64_t k = keys[i];
    if (i > 0 && keys[i - 1] == k) return false;
    const uint32_t hi = (uint32_t)(k >> 32), lo = (uint32_t)k;
    if (mode == 1 && hi != lo) return false;
    if (dhi && !((dhi[hi >> 6] >> (hi & 63)) & 1)) return false;
    if (dlo && !((dlo[lo >> 6] >> (lo & 63)) & 1)) return false;
    return true;
}

__global__ __launch_bounds__(kBlock) void k_tile_count(const uint64_t* __restrict__ keys, uint64_t n, int mode,
                                                       const uint64_t* __restrict__ dhi,
                                                       const uint64_t* __restrict__ dlo,
                                                       uint64_t* __restrict__ counts) {
    __shared__ uint32_t s_sum[kWaves];
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    uint32_t c = 0;
    for (int j = threadIdx.x; j < kTile; j += kBlock) {
        const uint64_t i = base + j;
        if (i < n && keep_key(keys, i, mode, dhi, dlo)) ++c;
    }
    c = (uint32_t)rpqd::wave_sum_u64(c);
    if (__lane_id() == 0) s_sum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kWaves; ++w) t += s_sum[w];
        counts[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_tile_write(const uint64_t* __restrict__ keys, uint64_t n, int mode,
                                                       const uint64_t* __restrict__ dhi,
                                                       const uint64_t* __restrict__ dlo,
                                                       const uint64_t* __restrict__ offs, uint64_t* __restrict__ out) {
    __shared__ uint32_t s_sum[kWaves];
    __shared__ uint64_t s_run;
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    if (threadIdx.x == 0) s_run = offs[blockIdx.x];
    __syncthreads();
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    for (int j0 = 0; j0 < kTile; j0 += kBlock) {
        const uint64_t i = base + j0 + threadIdx.x;
        const bool keep = i < n && keep_key(keys, i, mode, dhi, dlo);
        const uint64_t m = __ballot(keep);
        if (lane == 0) s_sum[wv] = (uint32_t)__popcll(m);
        __syncthreads();
        uint64_t pre = s_run;
        for (int w = 0; w < wv; ++w) pre += s_sum[w];
        if (keep) out[pre + __popcll(m & rpqd::lanemask_lt())] = keys[i];
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t t = 0;
            for (int w = 0; w < kWaves; ++w) t += s_sum[w];
            s_run += t;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------------
// edge scan: every (s, l, t) with s in the source list, l in the atom's label set and t in the
// destination domain; keys s << 32 | t (or t << 32 | s when scanning in-edges)
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_edge_scan(const uint32_t* __restrict__ row_ptr,
                                                      const uint32_t* __restrict__ dst,
                                                      const uint64_t* __restrict__ lmask, uint32_t L, uint64_t lang,
                                                      const uint32_t* __restrict__ srcs, uint64_t n_src,
                                                      const uint64_t* __restrict__ target, int swap,
                                                      uint64_t* __restrict__ out, unsigned long long* __restrict__ cnt,
                                                      uint64_t cap) {
    const int lane = __lane_id();
    for (uint64_t b = gwave_base(); b < n_src; b += gstride()) {
        const uint64_t i = b + lane;
        uint32_t s = 0;
        uint64_t m = 0, deg = 0;
        if (i < n_src) {
            s = srcs[i];
            m = lmask[s] & lang;
            uint64_t mm = m;
            while (mm) {
                const uint32_t l = (uint32_t)(__ffsll((long long)mm) - 1);
                mm &= mm - 1;
                const uint64_t r = (uint64_t)s * L + l;
                deg += row_ptr[r + 1] - row_ptr[r];
            }
        }
        const uint64_t incl = rpqd::wave_incl_scan_u64(deg);
        const uint64_t excl = incl - deg;
        const uint64_t total = __shfl(incl, 63, 64);
        for (uint64_t base = 0; base < total; base += 64) {
            const uint64_t item = base + lane;
            const int c = wave_owner(excl, item);
            const uint32_t cs = __shfl(s, c, 64);
            const uint64_t cm = __shfl(m, c, 64);
            const uint64_t cx = __shfl(excl, c, 64);
            bool keep = false;
            uint32_t t = 0;
            if (item < total) {
                uint64_t off = item - cx;
                uint64_t mm = cm;
                while (mm) {
                    const uint32_t l = (uint32_t)(__ffsll((long long)mm) - 1);
                    mm &= mm - 1;
                    const uint64_t r = (uint64_t)cs * L + l;
                    const uint32_t b0 = row_ptr[r], d = row_ptr[r + 1] - b0;
                    if (off < d) {
                        t = dst[b0 + off];
                        break;
                    }
                    off -= d;
                }
                keep = bit_of(target, t);
            }
            const uint64_t pos = wave_append(keep, cnt);
            if (keep && pos < cap) out[pos] = swap ? (((uint64_t)t << 32) | cs) : (((uint64_t)cs << 32) | t);
        }
    }
}

// ------------------------------------------------------------------------------------------------
// sparse multi-source search: visited set = device hash set of (source index, state, vertex)
// ------------------------------------------------------------------------------------------------
struct SNfa {
    uint32_t Q, L, init, final;
    uint64_t qlab[RPQ_MAX_STATES];
    uint32_t delta[RPQ_MAX_STATES * RPQ_MAX_LABELS];   // compact [q * L + l]
};

struct SArgs {
    const uint32_t* row_ptr;
    const uint32_t* dst;
    const uint64_t* lmask;
    const SNfa* nfa;
    const uint32_t* srcs;        // source vertices (ascending), index = source id in keys
    uint64_t n_src;
    const uint64_t* target;      // destination domain bitmap, or null (every vertex)
    unsigned long long* table;   // hash set, kEmpty = free
    uint64_t mask;               // table size - 1
    const uint64_t* front_in;
    uint64_t n_in;
    uint64_t* front_out;
    uint64_t front_cap;
    uint64_t* pairs;
    uint64_t pair_cap;
    unsigned long long* ctr;     // [0] next frontier length, [1] pairs, [2] error flags, [3] product edges
    uint64_t ins_limit;          // new entries this launch may add before the table counts as full
    uint32_t V;
};

// Flags in ctr[2]: an insert ran out of probes, or the table passed its load limit.  Either one
// ends the run (the host retries with a larger table), so the waves of the launch stop early
// instead of probing an overfull table.
constexpr unsigned long long kFlagProbe = 1, kFlagFull = 2;

__device__ __forceinline__ bool run_over(const SArgs& a) {
    const unsigned long long f = __hip_atomic_load(&a.ctr[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __ballot(f != 0) != 0;
}

// true if key was not in the set (and is now)
__device__ __forceinline__ bool set_insert(const SArgs& a, uint64_t key) {
    uint64_t h = rpqd::mix64(key) & a.mask;
    for (uint32_t p = 0; p < kMaxProbe; ++p) {
        const unsigned long long cur = a.table[h];
        if (cur == key) return false;
        if (cur == kEmpty) {
            const unsigned long long prev = atomicCAS(&a.table[h], kEmpty, (unsigned long long)key);
            if (prev == kEmpty) return true;
            if (prev == key) return false;
        }
        h = (h + 1) & a.mask;
    }
    atomicOr(&a.ctr[2], kFlagProbe);
    return false;
}

__global__ __launch_bounds__(kBlock) void k_sparse_seed(SArgs a) {
    const int lane = __lane_id();
    const uint32_t init = a.nfa->init, fin = a.nfa->final;
    for (uint64_t b = gwave_base(); b < a.n_src; b += gstride()) {
        const uint64_t si = b + lane;
        const bool ok = si < a.n_src;
        const uint32_t s = ok ? a.srcs[si] : 0;
        for (uint32_t q = 0; q < a.nfa->Q; ++q) {
            if (!((init >> q) & 1)) continue;
            const uint64_t key = (si << 32) | ((uint64_t)q * a.V + s);
            const bool ins = ok && set_insert(a, key);
            const uint64_t pos = wave_append(ins, &a.ctr[0]);
            if (ins && pos < a.front_cap) a.front_out[pos] = key;
            if (ins && pos >= a.ins_limit) atomicOr(&a.ctr[2], kFlagFull);
            const bool emit = ins && ((fin >> q) & 1) && (!a.target || bit_of(a.target, s));
            const uint64_t pp = wave_append(emit, &a.ctr[1]);
            if (emit && pp < a.pair_cap) a.pairs[pp] = ((uint64_t)s << 32) | s;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_sparse_level(SArgs a) {
    __shared__ uint32_t s_delta[RPQ_MAX_STATES * RPQ_MAX_LABELS];
    __shared__ uint64_t s_qlab[RPQ_MAX_STATES];
    const uint32_t Q = a.nfa->Q, L = a.nfa->L, fin = a.nfa->final;
    for (uint32_t i = threadIdx.x; i < Q * L; i += kBlock) s_delta[i] = a.nfa->delta[i];
    for (uint32_t i = threadIdx.x; i < Q; i += kBlock) s_qlab[i] = a.nfa->qlab[i];
    __syncthreads();
    const int lane = __lane_id();
    const uint32_t V = a.V;
    for (uint64_t b = gwave_base(); b < a.n_in; b += gstride()) {
        if (run_over(a)) return;
        const uint64_t e = b + lane;
        uint64_t key = 0, m = 0, deg = 0, eprod = 0;
        uint32_t q = 0, v = 0;
        if (e < a.n_in) {
            key = a.front_in[e];
            const uint32_t lo = (uint32_t)(key & 0xFFFFFFFFull);
            q = lo / V;
            v = lo - q * V;
            m = a.lmask[v] & s_qlab[q];
            uint64_t mm = m;
            while (mm) {
                const uint32_t l = (uint32_t)(__ffsll((long long)mm) - 1);
                mm &= mm - 1;
                const uint64_t r = (uint64_t)v * L + l;
                const uint32_t d = a.row_ptr[r + 1] - a.row_ptr[r];
                deg += d;
                eprod += (uint64_t)d * (uint32_t)__popc(s_delta[q * L + l]);
            }
        }
        eprod = rpqd::wave_sum_u64(eprod);
        if (lane == 0 && eprod) atomicAdd(&a.ctr[3], (unsigned long long)eprod);
        const uint64_t incl = rpqd::wave_incl_scan_u64(deg);
        const uint64_t excl = incl - deg;
        const uint64_t total = __shfl(incl, 63, 64);
        for (uint64_t base = 0; base < total; base += 64) {
            if (base && run_over(a)) return;
            const uint64_t item = base + lane;
            const int c = wave_owner(excl, item);
            const uint64_t ckey = __shfl(key, c, 64);
            const uint32_t cq = __shfl(q, c, 64);
            const uint32_t cv = __shfl(v, c, 64);
            const uint64_t cm = __shfl(m, c, 64);
            const uint64_t cx = __shfl(excl, c, 64);
            uint32_t w = 0, succ = 0;
            if (item < total) {
                uint64_t off = item - cx;
                uint64_t mm = cm;
                while (mm) {
                    const uint32_t l = (uint32_t)(__ffsll((long long)mm) - 1);
                    mm &= mm - 1;
                    const uint64_t r = (uint64_t)cv * L + l;
                    const uint32_t b0 = a.row_ptr[r], d = a.row_ptr[r + 1] - b0;
                    if (off < d) {
                        w = a.dst[b0 + off];
                        succ = s_delta[cq * L + l];
                        break;
                    }
                    off -= d;
                }
            }
            const uint64_t si = ckey >> 32;
            // one successor state per round; every lane takes part in every append
            while (__ballot(succ != 0)) {
                bool ins = false;
                uint32_t q2 = 0;
                if (succ) {
                    q2 = __ffs(succ) - 1;
                    succ &= succ - 1;
                    ins = set_insert(a, (si << 32) | ((uint64_t)q2 * V + w));
                }
                const uint64_t pos = wave_append(ins, &a.ctr[0]);
                if (ins && pos < a.front_cap) a.front_out[pos] = (si << 32) | ((uint64_t)q2 * V + w);
                if (ins && pos >= a.ins_limit) atomicOr(&a.ctr[2], kFlagFull);
                const bool emit = ins && ((fin >> q2) & 1) && (!a.target || bit_of(a.target, w));
                const uint64_t pp = wave_append(emit, &a.ctr[1]);
                if (emit && pp < a.pair_cap) a.pairs[pp] = ((uint64_t)a.srcs[si] << 32) | w;
            }
        }
    }
}

// ------------------------------------------------------------------------------------------------
// join step: bind one new variable z
// ------------------------------------------------------------------------------------------------
struct StepArgs {
    const uint32_t* in_cols[CRPQ_MAX_VARS];
    uint32_t* out_cols[CRPQ_MAX_VARS];
    uint64_t n_rows;
    uint32_t n_cols;                        // input columns; z becomes column n_cols
    uint32_t n_conn;
    const uint64_t* conn_keys[kMaxConn];    // sorted (u << 32 | z)
    uint64_t conn_n[kMaxConn];
    uint32_t conn_col[kMaxConn];            // input column of u
    uint32_t n_self;
    uint32_t n_neq;
    const uint64_t* self_keys[kMaxConn];    // relations of atoms z -> z (sorted keys)
    uint64_t self_n[kMaxConn];
    uint32_t neq_col[CRPQ_MAX_VARS];
    const uint64_t* dom_bits;               // z's domain
    const uint32_t* dom_list;               // ascending domain of z (candidates when n_conn == 0)
    uint64_t dom_n;
    uint64_t* row_lo;                       // [n_rows][n_conn]
    uint64_t* row_len;                      // [n_rows][n_conn]
    uint32_t* row_best;                     // [n_rows]
    uint64_t* row_off;                      // [n_rows + 1]: counts, then exclusive prefix
    uint64_t total;                         // candidates over all rows
    uint64_t cap;                           // output rows
    unsigned long long* out_cnt;
    int reduce;                             // count and hash instead of writing rows
    uint32_t n_free;
    uint32_t free_col[CRPQ_MAX_VARS];       // output-row columns of the free variables, declared order
    unsigned long long* acc;                // [count, hash]
};

__global__ __launch_bounds__(kBlock) void k_step_ranges(StepArgs a) {
    for (uint64_t r = gthread(); r < a.n_rows; r += gstride()) {
        uint64_t best_len = a.dom_n;
        uint32_t best = 0;
        for (uint32_t i = 0; i < a.n_conn; ++i) {
            const uint64_t u = a.in_cols[a.conn_col[i]][r];
            const uint64_t lo = lower_bound(a.conn_keys[i], 0, a.conn_n[i], u << 32);
            const uint64_t hi = lower_bound(a.conn_keys[i], lo, a.conn_n[i], (u + 1) << 32);
            a.row_lo[r * a.n_conn + i] = lo;
            a.row_len[r * a.n_conn + i] = hi - lo;
            if (i == 0 || hi - lo < best_len) {
                best_len = hi - lo;
                best = i;
            }
        }
        a.row_best[r] = best;
        a.row_off[r] = best_len;
    }
}

__global__ __launch_bounds__(kBlock) void k_step_expand(StepArgs a) {
    const int lane = __lane_id();
    uint64_t cnt = 0, hsum = 0;
    for (uint64_t b = gwave_base(); b < a.total; b += gstride()) {
        const uint64_t item = b + lane;
        bool keep = false;
        uint64_t r = 0;
        uint32_t z = 0;
        if (item < a.total) {
            // row owning the item: last r with row_off[r] <= item
            uint64_t lo = 0, hi = a.n_rows;
            while (hi - lo > 1) {
                const uint64_t mid = (lo + hi) >> 1;
                if (a.row_off[mid] <= item) lo = mid;
                else hi = mid;
            }
            r = lo;
            const uint64_t idx = item - a.row_off[r];
            uint32_t best = 0;
            if (a.n_conn) {
                best = a.row_best[r];
                z = (uint32_t)(a.conn_keys[best][a.row_lo[r * a.n_conn + best] + idx] & 0xFFFFFFFFull);
            } else {
                z = a.dom_list[idx];
            }
            keep = bit_of(a.dom_bits, z);
            for (uint32_t i = 0; keep && i < a.n_conn; ++i) {
                if (i == best) continue;
                const uint64_t u = a.in_cols[a.conn_col[i]][r];
                const uint64_t l0 = a.row_lo[r * a.n_conn + i];
                keep = contains(a.conn_keys[i], l0, l0 + a.row_len[r * a.n_conn + i], (u << 32) | z);
            }
            for (uint32_t i = 0; keep && i < a.n_self; ++i)
                keep = contains(a.self_keys[i], 0, a.self_n[i], ((uint64_t)z << 32) | z);
            for (uint32_t i = 0; keep && i < a.n_neq; ++i) keep = a.in_cols[a.neq_col[i]][r] != z;
        }
        if (a.reduce) {
            if (keep) {
                ++cnt;
                uint64_t m = 0;
                for (uint32_t j = 0; j < a.n_free; ++j) {
                    const uint32_t c = a.free_col[j];
                    const uint64_t x = c == a.n_cols ? z : a.in_cols[c][r];
                    m = j == 0 ? rpqd::mix64(x) : rpqd::mix64(m ^ x);
                }
                hsum += m;
            }
        } else {
            const uint64_t pos = wave_append(keep, a.out_cnt);
            if (keep && pos < a.cap) {
                for (uint32_t c = 0; c < a.n_cols; ++c) a.out_cols[c][pos] = a.in_cols[c][r];
                a.out_cols[a.n_cols][pos] = z;
            }
        }
    }
    if (a.reduce) {
        cnt = rpqd::wave_sum_u64(cnt);
        hsum = rpqd::wave_sum_u64(hsum);
        if (lane == 0 && cnt) {
            atomicAdd(&a.acc[0], (unsigned long long)cnt);
            atomicAdd(&a.acc[1], (unsigned long long)hsum);
        }
    }
}

// ------------------------------------------------------------------------------------------------
// output
// ------------------------------------------------------------------------------------------------
struct OutArgs {
    const uint32_t* cols[CRPQ_MAX_VARS];   // table columns of the free variables, declared order
    uint32_t n_free;
    uint64_t n_rows;
};

__global__ __launch_bounds__(kBlock) void k_rows_hash(OutArgs a, unsigned long long* __restrict__ acc) {
    uint64_t h = 0;
    for (uint64_t r = gthread(); r < a.n_rows; r += gstride()) {
        uint64_t m = 0;
        for (uint32_t j = 0; j < a.n_free; ++j) m = j == 0 ? rpqd::mix64(a.cols[j][r]) : rpqd::mix64(m ^ a.cols[j][r]);
        h += m;
    }
    h = rpqd::wave_sum_u64(h);
    if (__lane_id() == 0 && h) atomicAdd(&acc[1], (unsigned long long)h);
}

__global__ void k_iota(uint32_t* __restrict__ p, uint64_t n) {
    for (uint64_t i = gthread(); i < n; i += gstride()) p[i] = (uint32_t)i;
}

__global__ void k_sort_keys(const uint32_t* __restrict__ col, const uint32_t* __restrict__ perm, uint64_t n,
                            uint64_t* __restrict__ keys) {
    for (uint64_t i = gthread(); i < n; i += gstride()) keys[i] = ((uint64_t)col[perm[i]] << 32) | i;
}

__global__ void k_perm_apply(const uint64_t* __restrict__ sorted, const uint32_t* __restrict__ perm_in, uint64_t n,
                             uint32_t* __restrict__ perm_out) {
    for (uint64_t i = gthread(); i < n; i += gstride()) perm_out[i] = perm_in[sorted[i] & 0xFFFFFFFFull];
}

__global__ void k_write_tuples(OutArgs a, const uint32_t* __restrict__ perm, uint64_t n_out,
                               uint32_t* __restrict__ out) {
    for (uint64_t i = gthread(); i < n_out * a.n_free; i += gstride()) {
        const uint64_t r = i / a.n_free;
        const uint32_t j = (uint32_t)(i - r * a.n_free);
        out[i] = a.cols[j][perm[r]];
    }
}

// ------------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------------
struct Arena {
    char* base = nullptr;
    uint64_t size = 0, top = 0, need = 0;
    template <class T>
    T* take(uint64_t count) {
        const uint64_t bytes = align256(std::max<uint64_t>(1, count) * sizeof(T));
        if (top + bytes > size) {
            need = std::max(need, top + bytes);
            return nullptr;
        }
        T* p = reinterpret_cast<T*>(base + top);
        top += bytes;
        return p;
    }
    uint64_t free_bytes() const { return size > top ? size - top : 0; }
};

struct Rel {
    uint64_t* fwd = nullptr;   // sorted f(x) << 32 | f(y)
    uint64_t* bwd = nullptr;   // sorted f(y) << 32 | f(x), when needed
    uint64_t n = 0;
    uint32_t x = 0, y = 0;
};

struct Ctx {
    rpq_graph_t g;
    hipStream_t s;
    Arena ar;
    uint64_t* stage;                 // pinned host staging (graph-owned)
    unsigned long long* dctr;        // device counters [8]
    uint64_t n_words;
};

#define CRPQ_TAKE(ptr, T, n)                                                                  \
    do {                                                                                      \
        (ptr) = c.ar.take<T>(n);                                                              \
        if (!(ptr)) {                                                                         \
            rpq::set_error("workspace exhausted (%llu bytes needed so far)",                  \
                           (unsigned long long)c.ar.need);                                    \
            return RPQ_ENOMEM;                                                                \
        }                                                                                     \
    } while (0)

int read_counters(Ctx& c, int n) {
    RPQ_HIP(hipMemcpyAsync(c.stage, c.dctr, (size_t)n * 8, hipMemcpyDeviceToHost, c.s));
    RPQ_HIP(hipStreamSynchronize(c.s));
    return RPQ_OK;
}

int zero_counters(Ctx& c) { return rpq::fill_u64(reinterpret_cast<uint64_t*>(c.dctr), 8, 0, c.s); }

int popcount_bits(Ctx& c, const uint64_t* bits, uint64_t* count) {
    const uint64_t mark = c.ar.top;
    uint64_t* cnt;
    CRPQ_TAKE(cnt, uint64_t, c.n_words + 1);
    uint64_t* tmp;
    CRPQ_TAKE(tmp, uint64_t, rpq::scan_temp_elems(c.n_words));
    hipLaunchKernelGGL(k_word_popc, dim3(grid_for(c.n_words)), dim3(kBlock), 0, c.s, bits, c.n_words, cnt);
    RPQ_LAUNCH_CHECK();
    RPQ_TRY(rpq::exclusive_scan_u64(cnt, cnt, c.n_words, tmp, cnt + c.n_words, c.s));
    RPQ_HIP(hipMemcpyAsync(c.stage, cnt + c.n_words, 8, hipMemcpyDeviceToHost, c.s));
    RPQ_HIP(hipStreamSynchronize(c.s));
    *count = c.stage[0];
    c.ar.top = mark;
    return RPQ_OK;
}

// ascending vertex list of a bitmap (allocated in the arena; *n = its length)
int bits_to_list(Ctx& c, const uint64_t* bits, uint32_t** list, uint64_t* n) {
    uint64_t* cnt;
    CRPQ_TAKE(cnt, uint64_t, c.n_words + 1);
    const uint64_t mark = c.ar.top;
    uint64_t* tmp;
    CRPQ_TAKE(tmp, uint64_t, rpq::scan_temp_elems(c.n_words));
    hipLaunchKernelGGL(k_word_popc, dim3(grid_for(c.n_words)), dim3(kBlock), 0, c.s, bits, c.n_words, cnt);
    RPQ_LAUNCH_CHECK();
    RPQ_TRY(rpq::exclusive_scan_u64(cnt, cnt, c.n_words, tmp, cnt + c.n_words, c.s));
    RPQ_HIP(hipMemcpyAsync(c.stage, cnt + c.n_words, 8, hipMemcpyDeviceToHost, c.s));
    RPQ_HIP(hipStreamSynchronize(c.s));
    c.ar.top = mark;
    *n = c.stage[0];
    CRPQ_TAKE(*list, uint32_t, *n);
    hipLaunchKernelGGL(k_bits_to_list, dim3(grid_for(c.n_words)), dim3(kBlock), 0, c.s, bits, cnt, c.n_words, *list);
    RPQ_LAUNCH_CHECK();
    return RPQ_OK;
}

// sort keys (both halves are vertex ids) and keep distinct ones (mode 1: only (v, v)); result
// replaces *keys (same allocation), *n updated
int sort_unique(Ctx& c, uint64_t* keys, uint64_t* n, bool sorted_already, int mode, const uint64_t* dhi = nullptr,
                const uint64_t* dlo = nullptr) {
    if (*n == 0) return RPQ_OK;
    const uint64_t mark = c.ar.top;
    const int vb = rpq::bits_for(c.g->V ? c.g->V - 1 : 0);
    uint64_t* src = keys;
    if (!sorted_already) {
        uint64_t* alt;
        CRPQ_TAKE(alt, uint64_t, *n);
        void* tmp;
        CRPQ_TAKE(tmp, char, rpq::radix_temp_bytes(*n));
        RPQ_TRY(rpq::radix_sort_u64(keys, alt, *n, vb, vb, tmp, c.s, &src));
    }
    const uint64_t tiles = (*n + kTile - 1) / kTile;
    uint64_t* offs;
    CRPQ_TAKE(offs, uint64_t, tiles + 1);
    uint64_t* stmp;
    CRPQ_TAKE(stmp, uint64_t, rpq::scan_temp_elems(tiles));
    uint64_t* out = keys;
    if (src == keys) CRPQ_TAKE(out, uint64_t, *n);   // compaction needs distinct in/out buffers
    hipLaunchKernelGGL(k_tile_count, dim3((unsigned)tiles), dim3(kBlock), 0, c.s, src, *n, mode, dhi, dlo, offs);
    RPQ_LAUNCH_CHECK();
    RPQ_TRY(rpq::exclusive_scan_u64(offs, offs, tiles, stmp, offs + tiles, c.s));
    hipLaunchKernelGGL(k_tile_write, dim3((unsigned)tiles), dim3(kBlock), 0, c.s, src, *n, mode, dhi, dlo, offs, out);
    RPQ_LAUNCH_CHECK();
    RPQ_HIP(hipMemcpyAsync(c.stage, offs + tiles, 8, hipMemcpyDeviceToHost, c.s));
    RPQ_HIP(hipStreamSynchronize(c.s));
    const uint64_t m = c.stage[0];
    if (out != keys) RPQ_HIP(hipMemcpyAsync(keys, out, m * 8, hipMemcpyDeviceToDevice, c.s));
    *n = m;
    c.ar.top = mark;
    return RPQ_OK;
}

// language of single-label words only: the labels that lead from an initial state to final
// states with no way on, no initial state final
bool single_step_language(const rpq_nfa& n, uint64_t* lang) {
    if (n.initial_mask & n.final_mask) return false;
    uint64_t ls = 0;
    uint32_t targets = 0;
    for (uint32_t q = 0; q < n.n_states; ++q) {
        if (!((n.initial_mask >> q) & 1)) continue;
        for (uint32_t l = 0; l < n.n_labels; ++l) {
            const uint32_t d = n.delta[q * RPQ_MAX_LABELS + l];
            if (d) {
                ls |= 1ull << l;
                targets |= d;
            }
        }
    }
    if (!ls || (targets & n.initial_mask) || (targets & ~n.final_mask)) return false;
    for (uint32_t q = 0; q < n.n_states; ++q) {
        if (!((targets >> q) & 1)) continue;
        for (uint32_t l = 0; l < RPQ_MAX_LABELS; ++l)
            if (n.delta[q * RPQ_MAX_LABELS + l]) return false;
    }
    *lang = ls;
    return true;
}

int check_nfa(const rpq_graph* g, const rpq_nfa& n) {
    if (n.n_states == 0 || n.n_states > RPQ_MAX_STATES || n.n_labels == 0 || n.n_labels > g->L) {
        rpq::set_error("atom automaton has %u states over %u labels (graph: %u labels)", n.n_states, n.n_labels, g->L);
        return RPQ_EINVAL;
    }
    const uint32_t smask = n.n_states == 32 ? 0xFFFFFFFFu : ((1u << n.n_states) - 1);
    if ((n.initial_mask & ~smask) || (n.final_mask & ~smask)) {
        rpq::set_error("atom automaton masks name states >= n_states");
        return RPQ_EINVAL;
    }
    for (uint32_t q = 0; q < RPQ_MAX_STATES; ++q)
        for (uint32_t l = 0; l < RPQ_MAX_LABELS; ++l) {
            const uint32_t d = n.delta[q * RPQ_MAX_LABELS + l];
            if (d && (q >= n.n_states || l >= n.n_labels || (d & ~smask))) {
                rpq::set_error("atom automaton delta[%u][%u] is outside the automaton", q, l);
                return RPQ_EINVAL;
            }
        }
    if ((uint64_t)n.n_states * g->V >= 0xFFFFFFFFull) {
        rpq::set_error("states * vertices must stay below 2^32");
        return RPQ_EUNSUPPORTED;
    }
    return RPQ_OK;
}

void to_snfa(const rpq_nfa& n, uint32_t L, SNfa* d) {
    std::memset(d, 0, sizeof *d);
    d->Q = n.n_states;
    d->L = L;
    d->init = n.initial_mask;
    d->final = n.final_mask;
    for (uint32_t q = 0; q < n.n_states; ++q)
        for (uint32_t l = 0; l < L; ++l) {
            const uint32_t m = l < n.n_labels ? n.delta[q * RPQ_MAX_LABELS + l] : 0;
            d->delta[q * L + l] = m;
            if (m) d->qlab[q] |= 1ull << l;
        }
}

// Evaluate one atom from the source list into keys oriented (source << 32 | destination)
// of the traversal direction.  *keys is allocated in the arena; *sorted tells whether the
// keys come out sorted and distinct.
int eval_edge_scan(Ctx& c, const rpq::Csr& csr, uint64_t lang, const uint32_t* srcs, uint64_t n_src,
                   const uint64_t* target, uint64_t** keys, uint64_t* n) {
    // count first (capacity 0), then write
    RPQ_TRY(zero_counters(c));
    hipLaunchKernelGGL(k_edge_scan, dim3(grid_for(n_src, 16384)), dim3(kBlock), 0, c.s, csr.row_ptr, csr.dst,
                       csr.lmask, c.g->L, lang, srcs, n_src, target, 0, nullptr, c.dctr, (uint64_t)0);
    RPQ_LAUNCH_CHECK();
    RPQ_TRY(read_counters(c, 1));
    const uint64_t m = c.stage[0];
    CRPQ_TAKE(*keys, uint64_t, m);
    RPQ_TRY(zero_counters(c));
    hipLaunchKernelGGL(k_edge_scan, dim3(grid_for(n_src, 16384)), dim3(kBlock), 0, c.s, csr.row_ptr, csr.dst,
                       csr.lmask, c.g->L, lang, srcs, n_src, target, 0, *keys, c.dctr, m);
    RPQ_LAUNCH_CHECK();
    *n = m;
    return RPQ_OK;
}

int eval_dense(Ctx& c, const rpq_nfa& nfa, bool reverse, const uint32_t* srcs, uint64_t n_src,
               const uint64_t* target, uint64_t** keys, uint64_t* n) {
    const uint32_t flags = RPQ_PAIRS | (reverse ? RPQ_REVERSE : 0u);
    rpq_eval_opts o;
    std::memset(&o, 0, sizeof o);
    uint64_t ws = 0;
    RPQ_TRY(rpq_eval_workspace_size(c.g, &nfa, n_src, flags, &o, &ws));
    // leave at least half of the free workspace for the pairs: fewer units in flight if needed
    const uint64_t avail = c.ar.free_bytes();
    uint32_t conc = 1024;
    while (ws + 4096 > avail / 2 && conc > 1) {
        conc /= 2;
        o.concurrency = conc;
        RPQ_TRY(rpq_eval_workspace_size(c.g, &nfa, n_src, flags, &o, &ws));
    }
    if (ws + 4096 > avail) {
        c.ar.need = std::max<uint64_t>(c.ar.need, c.ar.top + 2 * align256(ws) + (1ull << 20));
        rpq::set_error("workspace exhausted (traversal needs %llu bytes)", (unsigned long long)ws);
        return RPQ_ENOMEM;
    }
    const uint64_t mark = c.ar.top;
    const uint64_t cap = (avail - align256(ws) - 512) / 8;
    uint64_t* pairs;
    CRPQ_TAKE(pairs, uint64_t, cap);
    void* wsp;
    CRPQ_TAKE(wsp, char, ws);
    rpq_result r;
    std::memset(&r, 0, sizeof r);
    r.pairs = pairs;
    r.capacity = cap;
    const int rc = rpq::eval_impl(c.g, &nfa, srcs, n_src, flags, &o, target, wsp, ws, &r, c.s);
    if (rc == RPQ_EOVERFLOW) {
        c.ar.need = std::max<uint64_t>(c.ar.need, mark + align256(r.count * 8) + align256(ws) + (1ull << 20));
        rpq::set_error("workspace exhausted (atom has %llu pairs)", (unsigned long long)r.count);
        return RPQ_ENOMEM;
    }
    RPQ_TRY(rc);
    c.ar.top = mark + align256(std::max<uint64_t>(1, r.count) * 8);   // keep the pairs, drop the traversal state
    *keys = pairs;
    *n = r.count;
    return RPQ_OK;
}

// CRPQ_BATCH_ATOMS: the query's forward bit-parallel atoms run together in the batched persistent
// form (Section 4.2's traversal queue feeding one exploration kernel, here across atoms), each from
// its source variable's domain as the constraints fix it.  One run counts their pairs, a second
// writes them into the workspace, where they stay for the join.
struct BatchGuard {
    rpq_batch_t b = nullptr;
    ~BatchGuard() {
        if (b) (void)rpq_batch_destroy(b);
    }
};

int batch_run(Ctx& c, const crpq_atom* atoms, const std::vector<uint32_t>& ids, const std::vector<uint32_t*>& srcs,
              const std::vector<uint64_t>& ns, const std::vector<const uint64_t*>& targets, uint32_t width,
              uint64_t* const* pairs, std::vector<uint64_t>& counts) {
    BatchGuard bg;
    rpq_batch_opts o;
    std::memset(&o, 0, sizeof o);
    o.batch_width = width;
    RPQ_TRY(rpq_batch_create(c.g, &o, &bg.b));
    std::vector<uint32_t> qid(ids.size());
    for (size_t j = 0; j < ids.size(); ++j) {
        RPQ_TRY(rpq_batch_add(bg.b, &atoms[ids[j]].nfa, srcs[j], ns[j], pairs ? RPQ_PAIRS : 0u,
                              pairs ? pairs[j] : nullptr, pairs ? counts[j] : 0, nullptr, &qid[j]));
        // only destinations in the atom's destination domain, as the sequential plan's filter
        RPQ_TRY(rpq::batch_filter_targets(bg.b, qid[j], targets[j]));
    }
    uint64_t ws = 0;
    RPQ_TRY(rpq_batch_workspace_size(bg.b, &ws));
    const uint64_t mark = c.ar.top;
    char* w;
    CRPQ_TAKE(w, char, ws);
    RPQ_TRY(rpq_batch_run(bg.b, w, ws, c.s));
    for (size_t j = 0; j < ids.size(); ++j) {
        rpq_result r;
        RPQ_TRY(rpq_batch_result(bg.b, qid[j], &r));
        if (pairs && r.count != counts[j]) {
            rpq::set_error("batched atom %u: %llu pairs on the second run, %llu on the first", ids[j],
                           (unsigned long long)r.count, (unsigned long long)counts[j]);
            return RPQ_EDEVICE;
        }
        counts[j] = r.count;
    }
    c.ar.top = mark;   // the traversal state goes; the pairs were taken below it
    return RPQ_OK;
}

int batch_atoms(Ctx& c, const crpq_atom* atoms, uint32_t n_atoms, uint32_t flags, const std::vector<uint64_t*>& dom,
                const std::vector<uint64_t>& dom_n, std::vector<bool>& pre, std::vector<uint64_t*>& keys,
                std::vector<uint64_t>& nk) {
    std::vector<uint32_t> ids;
    uint64_t widest = 1;
    for (uint32_t i = 0; i < n_atoms; ++i) {
        const uint32_t x = atoms[i].src_var, y = atoms[i].dst_var;
        uint64_t lang = 0;
        const bool scan = !(flags & CRPQ_NO_EDGE_SCAN) && single_step_language(atoms[i].nfa, &lang);
        const bool reverse = !(flags & CRPQ_NO_REVERSE) && c.g->has_in && x != y && dom_n[y] < dom_n[x];
        const bool dense = (flags & CRPQ_FORCE_DENSE) || (!(flags & CRPQ_FORCE_SPARSE) && dom_n[x] <= kDenseMaxSources);
        if (!scan && !reverse && dense) {
            ids.push_back(i);
            widest = std::max(widest, dom_n[x]);
        }
    }
    if (ids.empty()) return RPQ_OK;
    // units as wide as the largest source set needs, 64 .. 2048
    uint32_t width = 64;
    while (width < 2048 && width < widest) width *= 2;
    std::vector<uint32_t*> srcs(ids.size());
    std::vector<uint64_t> ns(ids.size()), counts(ids.size(), 0);
    std::vector<const uint64_t*> targets(ids.size());
    for (size_t j = 0; j < ids.size(); ++j) {
        RPQ_TRY(bits_to_list(c, dom[atoms[ids[j]].src_var], &srcs[j], &ns[j]));
        targets[j] = dom[atoms[ids[j]].dst_var];
    }
    RPQ_TRY(batch_run(c, atoms, ids, srcs, ns, targets, width, nullptr, counts));
    std::vector<uint64_t*> bufs(ids.size());
    for (size_t j = 0; j < ids.size(); ++j) CRPQ_TAKE(bufs[j], uint64_t, counts[j]);
    RPQ_TRY(batch_run(c, atoms, ids, srcs, ns, targets, width, bufs.data(), counts));
    for (size_t j = 0; j < ids.size(); ++j) {
        pre[ids[j]] = true;
        keys[ids[j]] = bufs[j];
        nk[ids[j]] = counts[j];
    }
    return RPQ_OK;
}

// One run of the sparse search with a hash set of T slots; returns RPQ_ENOMEM (without setting
// the error) when T was too small.
int sparse_run(Ctx& c, const rpq_nfa& nfa, const rpq::Csr& csr, const uint32_t* srcs, uint64_t n_src,
               const uint64_t* target, uint64_t T, uint64_t** keys, uint64_t* n, uint64_t* eprod = nullptr,
               uint64_t* levels = nullptr, uint64_t max_len = ~0ull) {
    SNfa h;
    to_snfa(nfa, c.g->L, &h);
    const uint64_t out_mark = c.ar.top;
    uint64_t* pairs;
    CRPQ_TAKE(pairs, uint64_t, T / 2);
    const uint64_t mark = c.ar.top;
    SNfa* dn;
    CRPQ_TAKE(dn, SNfa, 1);
    unsigned long long* table;
    CRPQ_TAKE(table, unsigned long long, T);
    uint64_t *fa, *fb;
    CRPQ_TAKE(fa, uint64_t, T / 2);
    CRPQ_TAKE(fb, uint64_t, T / 2);
    RPQ_HIP(hipMemcpyAsync(dn, &h, sizeof h, hipMemcpyHostToDevice, c.s));
    RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(table), T, kEmpty, c.s));
    RPQ_TRY(zero_counters(c));
    SArgs a;
    std::memset(&a, 0, sizeof a);
    a.row_ptr = csr.row_ptr;
    a.dst = csr.dst;
    a.lmask = csr.lmask;
    a.nfa = dn;
    a.srcs = srcs;
    a.n_src = n_src;
    a.target = target;
    a.table = table;
    a.mask = T - 1;
    a.front_out = fa;
    a.front_cap = T / 2;
    a.pairs = pairs;
    a.pair_cap = T / 2;
    a.ctr = c.dctr;
    a.ins_limit = T / 2;
    a.V = c.g->V;
    hipLaunchKernelGGL(k_sparse_seed, dim3(grid_for(n_src, 16384)), dim3(kBlock), 0, c.s, a);
    RPQ_LAUNCH_CHECK();
    RPQ_TRY(read_counters(c, 3));
    uint64_t n_front = c.stage[0], inserted = n_front;
    uint64_t* cur = fa;
    uint64_t* nxt = fb;
    bool over = c.stage[2] || n_front > T / 2;
    uint64_t n_levels = n_front ? 1 : 0;
    // a first-reach distance in the product graph is below Q * V
    const uint64_t level_bound = (uint64_t)nfa.n_states * c.g->V + 2;
    // level l expands depth l; a length bound k leaves depth k recorded but unexpanded
    for (uint64_t level = 0; !over && n_front > 0 && level < max_len; ++level) {
        if (level > level_bound) {
            rpq::set_error("sparse search found no fixpoint");
            return RPQ_EDEVICE;
        }
        RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(c.dctr), 1, 0, c.s));
        a.front_in = cur;
        a.n_in = n_front;
        a.front_out = nxt;
        a.ins_limit = T / 2 - inserted;   // inserted <= T / 2 here, or the loop would have ended
        hipLaunchKernelGGL(k_sparse_level, dim3(grid_for(n_front, 16384)), dim3(kBlock), 0, c.s, a);
        RPQ_LAUNCH_CHECK();
        RPQ_TRY(read_counters(c, 3));
        n_front = c.stage[0];
        inserted += n_front;
        over = c.stage[2] || n_front > T / 2 || inserted > T / 2;
        if (n_front) ++n_levels;
        std::swap(cur, nxt);
    }
    RPQ_TRY(read_counters(c, 4));
    if (over || c.stage[1] > T / 2) {
        c.ar.top = out_mark;
        return RPQ_ENOMEM;
    }
    (void)mark;
    const uint64_t np = c.stage[1];
    if (eprod) *eprod = c.stage[3];
    if (levels) *levels = n_levels;
    c.ar.top = out_mark + align256(std::max<uint64_t>(1, np) * 8);   // keep the pairs, drop the search state
    *keys = pairs;
    *n = np;
    return RPQ_OK;
}

// t_cap: largest table to try (0 = no limit); past it the search returns RPQ_EOVERFLOW without
// setting an error, and the caller evaluates the atom bit-parallel instead.
int eval_sparse(Ctx& c, const rpq_nfa& nfa_fwd, bool reverse, const uint32_t* srcs, uint64_t n_src,
                const uint64_t* target, uint64_t t_cap, uint64_t** keys, uint64_t* n) {
    rpq_nfa nfa;
    if (reverse) RPQ_TRY(rpq_nfa_reverse(&nfa_fwd, &nfa));
    else nfa = nfa_fwd;
    const rpq::Csr& csr = reverse ? c.g->in : c.g->out;
    // table of T slots (load <= 1/2), two frontiers and the pairs of T/2 each: 20 bytes per slot.
    // Start near 8 states per source and double while the search overflows and the arena allows.
    constexpr uint64_t kSlack = 1ull << 16;
    uint64_t T = 1ull << 16;
    while (T < 16 * n_src * (uint64_t)nfa.n_states && T < (1ull << 34)) T *= 2;
    if (t_cap) t_cap = std::max(t_cap, T);
    for (;;) {
        if (t_cap && T > t_cap) return RPQ_EOVERFLOW;
        if (T * 20 + kSlack > c.ar.free_bytes()) {
            c.ar.need = std::max<uint64_t>(c.ar.need, c.ar.top + T * 20 + kSlack + (1ull << 20));
            rpq::set_error("workspace exhausted (sparse search with %llu slots)", (unsigned long long)T);
            return RPQ_ENOMEM;
        }
        const int rc = sparse_run(c, nfa, csr, srcs, n_src, target, T, keys, n);
        if (rc != RPQ_ENOMEM) return rc;
        T *= 2;
    }
}

__global__ void k_check_sorted_sources(const uint32_t* __restrict__ s, uint64_t n, uint64_t V,
                                       unsigned long long* __restrict__ err) {
    for (uint64_t i = gthread(); i < n; i += gstride())
        if (s[i] >= V || (i > 0 && s[i - 1] >= s[i])) atomicOr(err, 1ull);
}

// count, checksum and per-source tallies of sorted distinct keys (s << 32 | v)
__global__ __launch_bounds__(kBlock) void k_key_tallies(const uint64_t* __restrict__ keys, uint64_t n,
                                                        const uint32_t* __restrict__ srcs, uint64_t n_src,
                                                        unsigned long long* __restrict__ per_source,
                                                        unsigned long long* __restrict__ acc) {
    uint64_t h = 0;
    for (uint64_t i = gthread(); i < n; i += gstride()) {
        const uint64_t k = keys[i];
        const uint64_t m = rpqd::mix64(k);
        h += m;
        if (per_source) {
            const uint64_t s = k >> 32;
            uint64_t lo = 0, hi = n_src;   // position of s in the ascending source list
            while (lo < hi) {
                const uint64_t mid = (lo + hi) >> 1;
                if (srcs[mid] < s) lo = mid + 1;
                else hi = mid;
            }
            atomicAdd(&per_source[2 * lo], 1ull);
            atomicAdd(&per_source[2 * lo + 1], (unsigned long long)m);
        }
    }
    h = rpqd::wave_sum_u64(h);
    if (__lane_id() == 0 && h) atomicAdd(&acc[0], (unsigned long long)h);
}

// Starting hash-set size: 16 slots per (source, state), at least 2^16, and as large as the free
// workspace allows up to 2^24 slots (filling 2^24 slots costs tens of microseconds, a restart
// after an overflow costs a whole search).
uint64_t sparse_start_slots(uint64_t n_src, uint32_t Q, uint64_t free_bytes = 0) {
    uint64_t T = 1ull << 16;
    while (T < 16 * n_src * (uint64_t)Q && T < (1ull << 34)) T *= 2;
    while (T < (1ull << 24) && (2 * T) * 20 + (2 * T) * 12 + (1ull << 20) <= free_bytes) T *= 2;
    return T;
}

}  // namespace

namespace rpq {

int sparse_workspace_size(rpq_graph_t g, const rpq_nfa* nfa, uint64_t n_sources, uint32_t flags, uint64_t* bytes) {
    if (!g || !nfa) {
        rpq::set_error("graph and automaton must not be NULL");
        return RPQ_EINVAL;
    }
    RPQ_TRY(check_nfa(g, *nfa));
    const uint64_t T = sparse_start_slots(n_sources, nfa->n_states);
    // counters, source list, search (20 B per slot), sort of T/2 pairs, slack
    uint64_t b = 4096 + align256(((flags & RPQ_ALL_SOURCES) ? n_sources : 0) * 4) + T * 20 + (1ull << 16);
    b += align256(T / 2 * 8) + align256(rpq::radix_temp_bytes(T / 2)) + align256((T / 2 / kTile + 2) * 16) + 4096;
    *bytes = b;
    return RPQ_OK;
}

int sparse_eval(rpq_graph_t g, const rpq_nfa* nfa_in, const uint32_t* sources, uint64_t n_sources, uint32_t flags,
                uint64_t max_len, void* workspace, uint64_t workspace_bytes, rpq_result* res, hipStream_t stream) {
    RPQ_TRY(check_nfa(g, *nfa_in));
    const bool reverse = (flags & RPQ_REVERSE) != 0;
    if (reverse && !g->has_in) {
        rpq::set_error("RPQ_REVERSE needs a graph built with RPQ_BUILD_IN_CSR");
        return RPQ_EUNSUPPORTED;
    }
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
        rpq::set_error("workspace must be a non-NULL, 256-byte aligned device buffer");
        return RPQ_EINVAL;
    }
    res->written = res->count = res->hash = res->product_edges = res->levels = res->max_depth = 0;
    if (n_sources == 0) return RPQ_OK;
    if (n_sources >= 0xFFFFFFFFull) {
        rpq::set_error("RPQ_SPARSE supports fewer than 2^32 - 1 sources");
        return RPQ_EUNSUPPORTED;
    }
    rpq_nfa nfa;
    if (reverse) RPQ_TRY(rpq_nfa_reverse(nfa_in, &nfa));
    else nfa = *nfa_in;
    Ctx c;
    c.g = g;
    c.s = stream;
    c.ar.base = reinterpret_cast<char*>(workspace);
    c.ar.size = workspace_bytes;
    c.stage = host_stage();
    c.n_words = (g->V + 63) / 64;
    if (!c.stage) {
        rpq::set_error("pinned host staging memory is unavailable");
        return RPQ_EDEVICE;
    }
    auto nomem = [&](int rc) {
        if (rc == RPQ_ENOMEM)
            res->workspace_needed = std::max<uint64_t>(c.ar.need + c.ar.need / 2, workspace_bytes + 1);
        return rc;
    };
    auto body = [&]() -> int {
        CRPQ_TAKE(c.dctr, unsigned long long, 8);
        const uint32_t* srcs = sources;
        if (!srcs) {
            uint32_t* all;
            CRPQ_TAKE(all, uint32_t, n_sources);
            hipLaunchKernelGGL(k_iota, dim3(grid_for(n_sources, 16384)), dim3(kBlock), 0, c.s, all, n_sources);
            RPQ_LAUNCH_CHECK();
            srcs = all;
        } else {
            RPQ_TRY(zero_counters(c));
            hipLaunchKernelGGL(k_check_sorted_sources, dim3(grid_for(n_sources, 4096)), dim3(kBlock), 0, c.s, srcs,
                               n_sources, (uint64_t)g->V, c.dctr);
            RPQ_LAUNCH_CHECK();
            RPQ_TRY(read_counters(c, 1));
            if (c.stage[0]) {
                rpq::set_error("sources must be strictly ascending vertex ids below n_vertices");
                return RPQ_EINVAL;
            }
        }
        const rpq::Csr& csr = reverse ? g->in : g->out;
        // room for the search and, after it, the sort of up to T/2 pairs (~12 bytes per slot)
        uint64_t T = sparse_start_slots(n_sources, nfa.n_states, c.ar.free_bytes());
        uint64_t* keys = nullptr;
        uint64_t nk = 0, eprod = 0, levels = 0;
        for (;;) {
            if (T * 20 + (1ull << 16) > c.ar.free_bytes()) {
                c.ar.need = std::max<uint64_t>(c.ar.need, c.ar.top + T * 20 + (1ull << 16) + (1ull << 20));
                rpq::set_error("workspace exhausted (sparse search with %llu slots)", (unsigned long long)T);
                return RPQ_ENOMEM;
            }
            const int rc =
                sparse_run(c, nfa, csr, srcs, n_sources, nullptr, T, &keys, &nk, &eprod, &levels, max_len);
            if (rc == RPQ_OK) break;
            if (rc != RPQ_ENOMEM) return rc;
            T *= 2;
        }
        RPQ_TRY(sort_unique(c, keys, &nk, false, 0));
        RPQ_TRY(zero_counters(c));
        if (flags & RPQ_PER_SOURCE) RPQ_TRY(rpq::fill_u64(res->per_source, 2 * n_sources, 0, c.s));
        if (nk) {
            hipLaunchKernelGGL(k_key_tallies, dim3(grid_for(nk, 16384)), dim3(kBlock), 0, c.s, keys, nk, srcs,
                               n_sources,
                               (flags & RPQ_PER_SOURCE) ? reinterpret_cast<unsigned long long*>(res->per_source)
                                                        : nullptr,
                               c.dctr);
            RPQ_LAUNCH_CHECK();
        }
        RPQ_TRY(read_counters(c, 1));
        res->count = nk;
        res->hash = c.stage[0];
        res->product_edges = eprod;
        res->levels = levels;
        res->max_depth = levels ? levels - 1 : 0;
        if ((flags & RPQ_PAIRS) && res->pairs) {
            const uint64_t avail = nk > res->pair_offset ? nk - res->pair_offset : 0;
            const uint64_t w = std::min<uint64_t>(avail, res->capacity);
            if (w) RPQ_HIP(hipMemcpyAsync(res->pairs, keys + res->pair_offset, w * 8, hipMemcpyDeviceToDevice, c.s));
            RPQ_HIP(hipStreamSynchronize(c.s));
            res->written = w;
            if (avail > res->capacity) {
                rpq::set_error("result has %llu keys past offset %llu; capacity is %llu", (unsigned long long)avail,
                               (unsigned long long)res->pair_offset, (unsigned long long)res->capacity);
                return RPQ_EOVERFLOW;
            }
        }
        RPQ_HIP(hipStreamSynchronize(c.s));
        return RPQ_OK;
    };
    return nomem(body());
}

}  // namespace rpq

namespace {

int crpq_eval_body(rpq_graph_t g, const crpq_atom* atoms, uint32_t n_atoms, const crpq_vars* vars, uint32_t flags,
                   void* workspace, uint64_t workspace_bytes, crpq_result* res, hipStream_t stream) {
    if (!g || !res || !vars || (n_atoms && !atoms)) {
        rpq::set_error("graph, result, vars and atoms must not be NULL");
        return RPQ_EINVAL;
    }
    const uint32_t NV = vars->n_vars;
    if (NV == 0 || NV > CRPQ_MAX_VARS || n_atoms > CRPQ_MAX_ATOMS) {
        rpq::set_error("n_vars must be 1..%d and n_atoms at most %d", CRPQ_MAX_VARS, CRPQ_MAX_ATOMS);
        return RPQ_EINVAL;
    }
    if (flags & ~(CRPQ_FORCE_DENSE | CRPQ_FORCE_SPARSE | CRPQ_NO_EDGE_SCAN | CRPQ_NO_REVERSE | CRPQ_BATCH_ATOMS)) {
        rpq::set_error("unknown flags 0x%x", flags);
        return RPQ_EINVAL;
    }
    if ((flags & CRPQ_FORCE_DENSE) && (flags & CRPQ_FORCE_SPARSE)) {
        rpq::set_error("CRPQ_FORCE_DENSE and CRPQ_FORCE_SPARSE exclude each other");
        return RPQ_EINVAL;
    }
    for (uint32_t i = 0; i < n_atoms; ++i) {
        if (atoms[i].src_var >= NV || atoms[i].dst_var >= NV) {
            rpq::set_error("atom %u names a variable >= n_vars", i);
            return RPQ_EINVAL;
        }
        RPQ_TRY(check_nfa(g, atoms[i].nfa));
    }
    for (uint32_t i = 0; i < NV; ++i) {
        if (vars->binding && vars->binding[i] >= 0 && (uint64_t)vars->binding[i] >= g->V) {
            rpq::set_error("variable %u is bound to vertex %lld >= n_vertices", i, (long long)vars->binding[i]);
            return RPQ_EINVAL;
        }
        if (vars->vertex_label && vars->vertex_label[i] >= 0) {
            if (!g->vlabel) {
                rpq::set_error("vertex-label conditions need a graph created with vertex labels");
                return RPQ_EINVAL;
            }
            if (vars->vertex_label[i] > 255) {
                rpq::set_error("vertex label %d of variable %u is not a uint8 label", vars->vertex_label[i], i);
                return RPQ_EINVAL;
            }
        }
        if (vars->domain && vars->domain[i] && !vars->domain_size) {
            rpq::set_error("domain given without domain_size");
            return RPQ_EINVAL;
        }
    }
    if (vars->n_neq && !vars->neq) {
        rpq::set_error("neq is NULL");
        return RPQ_EINVAL;
    }
    for (uint32_t j = 0; j < 2 * vars->n_neq; ++j)
        if (vars->neq[j] >= NV) {
            rpq::set_error("inequality names a variable >= n_vars");
            return RPQ_EINVAL;
        }
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
        rpq::set_error("workspace must be a non-NULL, 256-byte aligned device buffer");
        return RPQ_EINVAL;
    }
    if (res->capacity && !res->tuples) {
        rpq::set_error("capacity > 0 with a NULL tuple buffer");
        return RPQ_EINVAL;
    }

    Ctx c;
    c.g = g;
    c.s = stream;
    c.ar.base = reinterpret_cast<char*>(workspace);
    c.ar.size = workspace_bytes;
    c.stage = rpq::host_stage();
    if (!c.stage) {
        rpq::set_error("pinned host staging memory is unavailable");
        return RPQ_EDEVICE;
    }
    c.n_words = (g->V + 63) / 64;
    res->count = res->hash = res->written = res->join_rows = 0;
    res->workspace_needed = 0;
    for (int i = 0; i < CRPQ_MAX_ATOMS; ++i) {
        res->atom_pairs[i] = 0;
        res->atom_strategy[i] = 0;
    }
    uint32_t free_vars[CRPQ_MAX_VARS];
    uint32_t n_free = 0;
    for (uint32_t i = 0; i < NV; ++i)
        if (!(vars->binding && vars->binding[i] >= 0)) free_vars[n_free++] = i;
    res->n_free = n_free;

    auto fail_nomem = [&](int rc) {
        if (rc == RPQ_ENOMEM) res->workspace_needed = std::max<uint64_t>(c.ar.need + c.ar.need / 2, workspace_bytes + 1);
        return rc;
    };
#define CRPQ_STEP(...)                                  \
    do {                                                \
        const int rc__ = (__VA_ARGS__);                 \
        if (rc__ != RPQ_OK) return fail_nomem(rc__);    \
    } while (0)

    CRPQ_STEP([&]() -> int {
        CRPQ_TAKE(c.dctr, unsigned long long, 8);
        return RPQ_OK;
    }());

    // ---- 1. domains
    std::vector<uint64_t*> dom(NV);
    std::vector<uint64_t> dom_n(NV);
    for (uint32_t i = 0; i < NV; ++i) {
        CRPQ_STEP([&]() -> int {
            CRPQ_TAKE(dom[i], uint64_t, c.n_words);
            const int32_t lab = vars->vertex_label ? vars->vertex_label[i] : -1;
            const int64_t bnd = vars->binding ? vars->binding[i] : -1;
            hipLaunchKernelGGL(k_dom_build, dim3(grid_for(c.n_words * 64, 8192)), dim3(kBlock), 0, c.s, dom[i],
                               (uint64_t)g->V, g->vlabel, lab, bnd);
            RPQ_LAUNCH_CHECK();
            if (vars->domain && vars->domain[i]) {
                const uint64_t mark = c.ar.top;
                uint64_t* tmp;
                CRPQ_TAKE(tmp, uint64_t, c.n_words);
                RPQ_TRY(rpq::fill_u64(tmp, c.n_words, 0, c.s));
                RPQ_TRY(zero_counters(c));
                const uint64_t ds = vars->domain_size[i];
                if (ds) {
                    hipLaunchKernelGGL(k_bits_from_list, dim3(grid_for(ds, 16384)), dim3(kBlock), 0, c.s, tmp,
                                       vars->domain[i], ds, (uint64_t)g->V, c.dctr);
                    RPQ_LAUNCH_CHECK();
                }
                hipLaunchKernelGGL(k_and, dim3(grid_for(c.n_words, 16384)), dim3(kBlock), 0, c.s, dom[i], tmp,
                                   c.n_words);
                RPQ_LAUNCH_CHECK();
                RPQ_TRY(read_counters(c, 1));
                if (c.stage[0]) {
                    rpq::set_error("domain of variable %u holds a vertex id >= n_vertices", i);
                    return RPQ_EINVAL;
                }
                c.ar.top = mark;
            }
            return popcount_bits(c, dom[i], &dom_n[i]);
        }());
    }

    auto empty_result = [&]() {
        res->count = 0;
        res->hash = 0;
        res->written = 0;
        return RPQ_OK;
    };
    for (uint32_t i = 0; i < NV; ++i)
        if (dom_n[i] == 0) return empty_result();

    // ---- 2. atoms, smallest source domain first, with semi-join reduction of the domains
    std::vector<bool> pre(n_atoms, false);
    std::vector<uint64_t*> pre_keys(n_atoms, nullptr);
    std::vector<uint64_t> pre_n(n_atoms, 0);
    if (flags & CRPQ_BATCH_ATOMS) CRPQ_STEP(batch_atoms(c, atoms, n_atoms, flags, dom, dom_n, pre, pre_keys, pre_n));
    std::vector<Rel> rel(n_atoms);
    std::vector<bool> done(n_atoms, false);
    for (uint32_t it = 0; it < n_atoms; ++it) {
        int pick = -1;
        uint64_t best = ~0ull;
        for (uint32_t i = 0; i < n_atoms; ++i) {
            if (done[i]) continue;
            const uint64_t m = std::min(dom_n[atoms[i].src_var], dom_n[atoms[i].dst_var]);
            if (m < best) {
                best = m;
                pick = (int)i;
            }
        }
        const crpq_atom& at = atoms[pick];
        done[pick] = true;
        const uint32_t x = at.src_var, y = at.dst_var;
        const bool batched = pre[pick];
        const bool reverse = !batched && !(flags & CRPQ_NO_REVERSE) && g->has_in && x != y && dom_n[y] < dom_n[x];
        const uint32_t sv = reverse ? y : x, dv = reverse ? x : y;
        uint64_t lang = 0;
        const bool scan = !batched && !(flags & CRPQ_NO_EDGE_SCAN) && single_step_language(at.nfa, &lang);
        uint32_t strategy;
        if (batched) strategy = CRPQ_STRATEGY_DENSE;
        else if (scan) strategy = CRPQ_STRATEGY_EDGE_SCAN;
        else if (flags & CRPQ_FORCE_DENSE) strategy = CRPQ_STRATEGY_DENSE;
        else if (flags & CRPQ_FORCE_SPARSE) strategy = CRPQ_STRATEGY_SPARSE;
        else strategy = dom_n[sv] <= kDenseMaxSources ? CRPQ_STRATEGY_DENSE : CRPQ_STRATEGY_SPARSE;
        res->atom_strategy[pick] = strategy | (reverse ? CRPQ_STRATEGY_REVERSED : 0u) |
                                   (batched ? CRPQ_STRATEGY_BATCHED : 0u);
        Rel& R = rel[pick];
        R.x = x;
        R.y = y;
        CRPQ_STEP([&]() -> int {
            const uint64_t mark = c.ar.top;
            uint32_t* srcs = nullptr;
            uint64_t n_src = 0;
            if (!batched) RPQ_TRY(bits_to_list(c, dom[sv], &srcs, &n_src));
            uint64_t* keys = nullptr;
            uint64_t nk = 0;
            bool sorted = false;
            if (batched) {
                // evaluated from the domains before any reduction: restricted to the current ones below
                keys = pre_keys[pick];
                nk = pre_n[pick];
                sorted = true;
            } else if (strategy == CRPQ_STRATEGY_EDGE_SCAN) {
                RPQ_TRY(eval_edge_scan(c, reverse ? g->in : g->out, lang, srcs, n_src, dom[dv], &keys, &nk));
            } else if (strategy == CRPQ_STRATEGY_DENSE) {
                RPQ_TRY(eval_dense(c, at.nfa, reverse, srcs, n_src, dom[dv], &keys, &nk));
                sorted = true;
            } else {
                // Chosen by source count alone, the hash-set search is capped at about V/256 entries
                // per source (a table of 2 * n_src * V / 256 slots): past that the atom's sources reach
                // enough of the graph for the bit-parallel search to be cheaper, and it takes over.
                const uint64_t cap = (flags & CRPQ_FORCE_SPARSE)
                                         ? 0
                                         : std::max<uint64_t>(1ull << 20, 2 * n_src * std::max<uint64_t>(1, g->V / 256));
                const int rc = eval_sparse(c, at.nfa, reverse, srcs, n_src, dom[dv], cap, &keys, &nk);
                if (rc == RPQ_EOVERFLOW) {
                    strategy = CRPQ_STRATEGY_DENSE;
                    res->atom_strategy[pick] = strategy | (reverse ? CRPQ_STRATEGY_REVERSED : 0u);
                    RPQ_TRY(eval_dense(c, at.nfa, reverse, srcs, n_src, dom[dv], &keys, &nk));
                    sorted = true;
                } else {
                    RPQ_TRY(rc);
                }
            }
            if (nk >= 0xFFFFFFFFull) {
                rpq::set_error("atom %d has %llu pairs; at most 2^32 - 2 are supported", pick, (unsigned long long)nk);
                return RPQ_EUNSUPPORTED;
            }
            if (reverse && nk) {
                hipLaunchKernelGGL(k_swap_halves, dim3(grid_for(nk, 16384)), dim3(kBlock), 0, c.s, keys, keys, nk);
                RPQ_LAUNCH_CHECK();
                sorted = false;
            }
            RPQ_TRY(sort_unique(c, keys, &nk, sorted, x == y ? 1 : 0, batched ? dom[x] : nullptr,
                                batched ? dom[y] : nullptr));
            (void)mark;   // the source list below the relation stays allocated (the arena is a stack)
            R.fwd = keys;
            R.n = nk;
            // semi-join reduction of both domains
            const uint64_t m2 = c.ar.top;
            uint64_t* tmp;
            CRPQ_TAKE(tmp, uint64_t, c.n_words);
            for (int side = 0; side < (x == y ? 1 : 2); ++side) {
                RPQ_TRY(rpq::fill_u64(tmp, c.n_words, 0, c.s));
                if (nk) {
                    hipLaunchKernelGGL(k_bits_from_keys, dim3(grid_for(nk, 16384)), dim3(kBlock), 0, c.s, tmp, R.fwd,
                                       nk, side == 0 ? 1 : 0);
                    RPQ_LAUNCH_CHECK();
                }
                const uint32_t var = side == 0 ? x : y;
                hipLaunchKernelGGL(k_and, dim3(grid_for(c.n_words, 16384)), dim3(kBlock), 0, c.s, dom[var], tmp,
                                   c.n_words);
                RPQ_LAUNCH_CHECK();
                RPQ_TRY(popcount_bits(c, dom[var], &dom_n[var]));
            }
            c.ar.top = m2;
            return RPQ_OK;
        }());
        res->atom_pairs[pick] = R.n;
        if (R.n == 0) return empty_result();
    }

    // ---- 3. matching order
    std::vector<int> order;
    std::vector<bool> bound(NV, false);
    for (uint32_t k = 0; k < NV; ++k) {
        int pick = -1;
        double best_est = 0;
        bool best_conn = false;
        for (uint32_t v = 0; v < NV; ++v) {
            if (bound[v]) continue;
            bool conn = false;
            double est = (double)dom_n[v];
            for (uint32_t i = 0; i < n_atoms; ++i) {
                const uint32_t x = atoms[i].src_var, y = atoms[i].dst_var;
                uint32_t u;
                if (x == v && y != v && bound[y]) u = y;
                else if (y == v && x != v && bound[x]) u = x;
                else continue;
                const double per_row = (double)rel[i].n / (double)std::max<uint64_t>(1, dom_n[u]);
                if (!conn || per_row < est) est = per_row;
                conn = true;
            }
            if (pick < 0 || (conn && !best_conn) || (conn == best_conn && est < best_est)) {
                pick = (int)v;
                best_est = est;
                best_conn = conn;
            }
        }
        order.push_back(pick);
        bound[pick] = true;
    }

    // ---- 4. join, one variable per step
    std::vector<int> col_of(NV, -1);
    std::vector<uint32_t*> cols;   // current table columns
    uint64_t n_rows = 1;           // the empty assignment
    const bool want_tuples = res->tuples != nullptr;
    uint64_t out_count = 0, out_hash = 0;
    bool reduced = false;
    std::vector<bool> used(n_atoms, false);
    for (uint32_t k = 0; k < NV; ++k) {
        const uint32_t z = (uint32_t)order[k];
        StepArgs a;
        std::memset(&a, 0, sizeof a);
        a.n_cols = (uint32_t)cols.size();
        for (uint32_t j = 0; j < a.n_cols; ++j) a.in_cols[j] = cols[j];
        a.n_rows = n_rows;
        // atoms between z and bound variables, self atoms of z
        for (uint32_t i = 0; i < n_atoms; ++i) {
            if (used[i]) continue;
            const uint32_t x = atoms[i].src_var, y = atoms[i].dst_var;
            if (x == z && y == z) {
                a.self_keys[a.n_self] = rel[i].fwd;
                a.self_n[a.n_self] = rel[i].n;
                ++a.n_self;
                used[i] = true;
            } else if (y == z && col_of[x] >= 0) {
                a.conn_keys[a.n_conn] = rel[i].fwd;   // keyed by f(x), candidates f(y)
                a.conn_n[a.n_conn] = rel[i].n;
                a.conn_col[a.n_conn] = (uint32_t)col_of[x];
                ++a.n_conn;
                used[i] = true;
            } else if (x == z && col_of[y] >= 0) {
                Rel& R = rel[i];
                if (!R.bwd) {   // slice transpose: keys by f(y)
                    CRPQ_STEP([&]() -> int {
                        CRPQ_TAKE(R.bwd, uint64_t, R.n);
                        hipLaunchKernelGGL(k_swap_halves, dim3(grid_for(R.n, 16384)), dim3(kBlock), 0, c.s, R.fwd,
                                           R.bwd, R.n);
                        RPQ_LAUNCH_CHECK();
                        uint64_t nn = R.n;
                        RPQ_TRY(sort_unique(c, R.bwd, &nn, false, 0));
                        return RPQ_OK;
                    }());
                }
                a.conn_keys[a.n_conn] = R.bwd;
                a.conn_n[a.n_conn] = R.n;
                a.conn_col[a.n_conn] = (uint32_t)col_of[y];
                ++a.n_conn;
                used[i] = true;
            }
        }
        for (uint32_t j = 0; j < vars->n_neq; ++j) {
            const uint32_t p = vars->neq[2 * j], q = vars->neq[2 * j + 1];
            if (p == z && q == z) return empty_result();   // f(z) != f(z) never holds
            if (p == z && col_of[q] >= 0) a.neq_col[a.n_neq++] = (uint32_t)col_of[q];
            else if (q == z && col_of[p] >= 0) a.neq_col[a.n_neq++] = (uint32_t)col_of[p];
        }
        a.dom_bits = dom[z];
        const bool last = k + 1 == NV;
        a.reduce = (last && !want_tuples) ? 1 : 0;
        a.n_free = n_free;
        std::vector<int> col_after = col_of;
        col_after[z] = (int)a.n_cols;
        for (uint32_t j = 0; j < n_free; ++j) a.free_col[j] = (uint32_t)col_after[free_vars[j]];
        CRPQ_STEP([&]() -> int {
            const uint64_t mark = c.ar.top;
            if (a.n_conn == 0) {
                uint32_t* lst;
                uint64_t nl = 0;
                RPQ_TRY(bits_to_list(c, dom[z], &lst, &nl));
                a.dom_list = lst;
                a.dom_n = nl;
            }
            CRPQ_TAKE(a.row_lo, uint64_t, n_rows * std::max<uint32_t>(1, a.n_conn));
            CRPQ_TAKE(a.row_len, uint64_t, n_rows * std::max<uint32_t>(1, a.n_conn));
            CRPQ_TAKE(a.row_best, uint32_t, n_rows);
            CRPQ_TAKE(a.row_off, uint64_t, n_rows + 1);
            uint64_t* stmp;
            CRPQ_TAKE(stmp, uint64_t, rpq::scan_temp_elems(n_rows));
            hipLaunchKernelGGL(k_step_ranges, dim3(grid_for(n_rows, 16384)), dim3(kBlock), 0, c.s, a);
            RPQ_LAUNCH_CHECK();
            RPQ_TRY(rpq::exclusive_scan_u64(a.row_off, a.row_off, n_rows, stmp, a.row_off + n_rows, c.s));
            RPQ_HIP(hipMemcpyAsync(c.stage, a.row_off + n_rows, 8, hipMemcpyDeviceToHost, c.s));
            RPQ_HIP(hipStreamSynchronize(c.s));
            a.total = c.stage[0];
            RPQ_TRY(zero_counters(c));
            a.out_cnt = c.dctr;
            a.acc = c.dctr + 2;
            std::vector<uint32_t*> out(a.n_cols + 1, nullptr);
            if (!a.reduce) {
                // output rows: at most the candidates; capacity limited by the arena
                const uint64_t row_bytes = 4ull * (a.n_cols + 1);
                const uint64_t fit = c.ar.free_bytes() / row_bytes;
                a.cap = std::min<uint64_t>(a.total, fit > (a.n_cols + 1) * 64 ? fit - (a.n_cols + 1) * 64 : 0);
                for (uint32_t j = 0; j <= a.n_cols; ++j) {
                    CRPQ_TAKE(out[j], uint32_t, a.cap);
                    a.out_cols[j] = out[j];
                }
            }
            if (a.total) {
                hipLaunchKernelGGL(k_step_expand, dim3(grid_for(a.total, 65535)), dim3(kBlock), 0, c.s, a);
                RPQ_LAUNCH_CHECK();
            }
            RPQ_TRY(read_counters(c, 4));
            if (a.reduce) {
                out_count = c.stage[2];
                out_hash = c.stage[3];
                reduced = true;
                return RPQ_OK;
            }
            const uint64_t got = c.stage[0];
            if (got > a.cap) {
                c.ar.need = std::max<uint64_t>(c.ar.need, c.ar.top + got * 4ull * (a.n_cols + 1) * 2 + (1ull << 20));
                rpq::set_error("workspace exhausted (join step has %llu rows)", (unsigned long long)got);
                return RPQ_ENOMEM;
            }
            // the new table stays where it was written; the per-row scratch below it and the previous
            // table stay allocated until the call returns
            (void)mark;
            cols = out;
            n_rows = got;
            res->join_rows = std::max(res->join_rows, got);
            return RPQ_OK;
        }());
        col_of[z] = (int)cols.size() - (reduced ? 0 : 1);
        if (!reduced && n_rows == 0) return empty_result();
    }

    // ---- 5. output
    if (reduced) {
        res->count = out_count;
        res->hash = n_free ? out_hash : 0;
        return RPQ_OK;
    }
    OutArgs o;
    std::memset(&o, 0, sizeof o);
    o.n_free = n_free;
    o.n_rows = n_rows;
    for (uint32_t j = 0; j < n_free; ++j) o.cols[j] = cols[col_of[free_vars[j]]];
    res->count = n_rows;
    CRPQ_STEP([&]() -> int {
        RPQ_TRY(zero_counters(c));
        if (n_free) {
            hipLaunchKernelGGL(k_rows_hash, dim3(grid_for(n_rows, 16384)), dim3(kBlock), 0, c.s, o, c.dctr);
            RPQ_LAUNCH_CHECK();
        }
        RPQ_TRY(read_counters(c, 2));
        res->hash = c.stage[1];
        if (!want_tuples || n_free == 0 || n_rows == 0) return RPQ_OK;
        if (n_rows >= 0xFFFFFFFFull) {
            rpq::set_error("sorting more than 2^32 - 2 tuples is not supported; pass tuples = NULL");
            return RPQ_EUNSUPPORTED;
        }
        // lexicographic order: stable passes from the last free variable to the first
        uint32_t *perm, *perm2;
        CRPQ_TAKE(perm, uint32_t, n_rows);
        CRPQ_TAKE(perm2, uint32_t, n_rows);
        uint64_t *keys, *alt;
        CRPQ_TAKE(keys, uint64_t, n_rows);
        CRPQ_TAKE(alt, uint64_t, n_rows);
        void* tmp;
        CRPQ_TAKE(tmp, char, rpq::radix_temp_bytes(n_rows));
        hipLaunchKernelGGL(k_iota, dim3(grid_for(n_rows, 16384)), dim3(kBlock), 0, c.s, perm, n_rows);
        RPQ_LAUNCH_CHECK();
        const int lo_bits = rpq::bits_for(n_rows - 1), hi_bits = rpq::bits_for(g->V ? g->V - 1 : 0);
        for (int j = (int)n_free - 1; j >= 0; --j) {
            hipLaunchKernelGGL(k_sort_keys, dim3(grid_for(n_rows, 16384)), dim3(kBlock), 0, c.s, o.cols[j], perm,
                               n_rows, keys);
            RPQ_LAUNCH_CHECK();
            uint64_t* sorted = nullptr;
            RPQ_TRY(rpq::radix_sort_u64(keys, alt, n_rows, lo_bits, hi_bits, tmp, c.s, &sorted));
            hipLaunchKernelGGL(k_perm_apply, dim3(grid_for(n_rows, 16384)), dim3(kBlock), 0, c.s, sorted, perm,
                               n_rows, perm2);
            RPQ_LAUNCH_CHECK();
            std::swap(perm, perm2);
        }
        const uint64_t n_out = std::min<uint64_t>(n_rows, res->capacity);
        if (n_out) {
            hipLaunchKernelGGL(k_write_tuples, dim3(grid_for(n_out * n_free, 65535)), dim3(kBlock), 0, c.s, o, perm,
                               n_out, res->tuples);
            RPQ_LAUNCH_CHECK();
        }
        RPQ_HIP(hipStreamSynchronize(c.s));
        res->written = n_out;
        return RPQ_OK;
    }());
    if (want_tuples && n_free && res->count > res->capacity) {
        rpq::set_error("%llu tuples; capacity is %llu", (unsigned long long)res->count,
                       (unsigned long long)res->capacity);
        return RPQ_EOVERFLOW;
    }
    if (want_tuples && n_free == 0) res->written = std::min<uint64_t>(res->count, res->capacity);
    return RPQ_OK;
#undef CRPQ_STEP
}

}  // namespace

extern "C" {

int crpq_eval(rpq_graph_t g, const crpq_atom* atoms, uint32_t n_atoms, const crpq_vars* vars, uint32_t flags,
              void* workspace, uint64_t workspace_bytes, crpq_result* res, hipStream_t stream) {
    rpq::clear_error();
    const int rc = crpq_eval_body(g, atoms, n_atoms, vars, flags, workspace, workspace_bytes, res, stream);
    // a failing call may leave kernels of its own queued on the stream (an intermediate that did
    // not fit is found after earlier steps were launched): drain them, so that the caller may reuse
    // or release the workspace as soon as the call returns
    if (rc != RPQ_OK) (void)hipStreamSynchronize(stream);
    return rc;
}

}  // extern "C"
