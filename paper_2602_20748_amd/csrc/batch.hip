// Batched evaluation: many RPQs (different automata, source sets, result
// modes) advanced together by one persistent kernel, captured in a HIP graph.
//
// The queries are cut into units (a query's sources, at most W per unit; a
// single-source query is one unit).  G slots each own a unit's bitmaps, sized
// for the largest automaton of the batch: Vis/Next [Qmax][V][K] words, a
// touch bitmap, a bitmap of the rows the unit has visited, Ans [V][K] and a
// one-bit-per-vertex summary of non-empty Ans rows.  The persistent kernel
// repeats
//
//   expand -> compact -> decide -> (retire) -> refill/seed -> finalize
//
// with a grid barrier between phases: the level kernels of the plain form,
// for every running slot at once, each slot with its own automaton.  A slot
// whose compaction finds no touched rows has reached its fixpoint (no hop
// bound); it is retired at once -- per-source count and checksum, keys into
// per-query staging, then only the rows it visited are cleared (a log of
// first-visited rows) -- and refilled from the unit queue in the same
// iteration.  Units of one query may run in any order and any slot; results
// do not depend on the schedule (every bit enters Vis exactly once and all
// updates are ORs).
//
// This is the counterpart of the paper's traversal queue feeding TGs to the
// exploration kernel (Section 4.2, Algorithm 1), with the queue held on the
// device and the loop held in one launch.
#include "internal.h"

#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kUnroll = 4;                 // rows per lane group loaded before any is updated
constexpr uint32_t kChunkV = 4096;          // vertices per extraction chunk (64 summary words)
constexpr uint32_t kSeenOrFrom = 1u << 22;   // default visit scheme: seen OR from this many vertices

// S_RETIRE: retiring in this iteration's retire phases (queries with pairs); S_DRAIN: retiring in the
// next iteration, its extraction beside that iteration's expansion and its clear beside its compaction
constexpr uint32_t S_IDLE = 0, S_RUN = 1, S_RETIRE = 2, S_DRAIN = 3;

// A slice [beg, beg + len) of the item space of frontier entry `entry` (entries with more than
// H items are cut into such slices of at most H items; lighter ones are expanded straight from
// the frontier list).
struct Desc {
    uint32_t entry, len;
    uint64_t beg;
};

struct BNfa {
    uint32_t Q, L, init, final;
    uint64_t qlab[RPQ_MAX_STATES];
    uint32_t delta[RPQ_MAX_STATES * RPQ_MAX_LABELS];   // compact [q * L + l]
};

struct BQuery {
    const uint32_t* sources;   // device, ascending; null = implicit ids [0, n)
    uint64_t n_sources;
    uint64_t* per_source;      // device [n][2] or null
    uint64_t* pairs;           // device output or null
    uint64_t capacity;
    uint64_t* stage;           // device: where this query's units put their keys (staging, or the
                               // output itself for a single-unit query of the open form)
    uint32_t first_unit, n_units;
    uint32_t flags;
    uint32_t max_len;          // length bound: the deepest depth recorded (0xFFFFFFFF = none)
    const uint64_t* target;    // device bitmap of V bits, or null: only result vertices with their bit
                               // set are counted, hashed and written
};

struct BQueryOut {
    unsigned long long count, hash, eprod, stage_top, max_depth, overflow, levels, units_done;
};

struct BUnit {
    uint32_t query, n;
    uint64_t src_off;
};

struct BSlot {
    uint32_t state, unit, query, alive;
    uint32_t start_iter, end_iter;   // end_iter: the iteration that found the fixpoint (S_DRAIN)
    unsigned long long log_n;
};

struct BCtl {
    rpqd::GridSync gs;
    unsigned long long list_cnt[2], desc_cnt[2];
    unsigned long long queue_head;      // units handed to slots
    unsigned long long units_tail;      // open form: units published by the host
    unsigned long long n_running, n_retiring, n_pairs_retiring, n_started;
    unsigned long long n_drain[2];      // slots to drain, decided by iterations of each parity
    unsigned long long err, iterations;
    unsigned long long items, descs, wreads, wupds;
    unsigned long long frows, fwords;   // finalize tallies: rows, non-zero next words
    unsigned long long t_begin, t_end;  // constant-clock stamps (100 MHz) at kernel entry and exit
    unsigned long long phase_ticks[8];  // constant-clock ticks per phase (block 0's view)
};

struct BArgs {
    const uint32_t* row_ptr;
    const uint32_t* dst;
    const uint64_t* lmask;
    const BNfa* nfas;
    const BQuery* queries;
    BQueryOut* qout;
    const BUnit* units;
    BSlot* slots;
    BCtl* ctl;
    uint64_t* vis;
    uint64_t* next;
    uint64_t* touch;
    uint64_t* ever;          // [G][slot_stride bits]: row touched at some level of the slot's unit
    uint64_t* ans;
    uint64_t* summ;          // [G][V/64 rounded up]: bit v set when Ans row v is non-empty
    uint32_t* ids0;
    uint32_t* ids1;
    uint64_t* rows0;
    uint64_t* rows1;
    Desc* desc0;
    Desc* desc1;
    uint32_t* logs;          // [G][slot_stride] first-visited rows (slot-local row ids)
    uint32_t* retiring;      // [G] slot ids retiring this iteration
    uint32_t* drain;         // [2][G] slot ids to drain, by the parity of the iteration that decided
    uint32_t* partial;       // [G][W][nchunks] pair counts per (source, chunk)
    uint64_t* srcbase;       // [G][W] first staging index of each source of a retiring unit
    uint64_t* stage;         // staging keys of all queries
    uint64_t* unit_total;    // [n_units] keys per unit
    uint64_t* unit_start;    // [n_units] staging index (query-relative) of each unit's keys
    uint32_t V, L, Qmax, H, G, W, nchunks, n_units, n_queries, n_blocks;
    uint64_t slot_stride, summ_words, list_cap, desc_cap, timeout, deadline;
    uint64_t log_cap;        // first-visit log entries per slot
    // open form (a resident engine fed between launches): the unit queue is a ring of unit_mask + 1
    // entries whose tail the host publishes in ctl->units_tail, and a launch ends after max_iters
    // iterations with its state kept for the next one.  Closed form: unit_mask = ~0, max_iters = 0.
    uint32_t open_form, max_iters;
    uint64_t unit_mask;
    uint32_t seen_or;        // visit scheme of the expansion (as in the plain form): 1 = seen OR
};

__device__ __forceinline__ unsigned long long ld(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st32(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st64(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void or_relaxed(uint64_t* p, uint64_t v) {
    (void)__hip_atomic_fetch_or(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
}


// Loads of data written in an earlier phase of the persistent kernel: plain loads, ordered by the
// grid barrier's release/acquire fences.
__device__ __forceinline__ uint64_t xld(const uint64_t* p) { return *p; }
__device__ __forceinline__ uint32_t xld(const uint32_t* p) { return *p; }

// An empty asm that takes each value as an operand, so that the arithmetic consuming conditionally
// loaded values is not moved into the loads' own conditional blocks, where each would wait for its
// load: the loads then stay in flight together.
template <int N>
__device__ __forceinline__ void keep_in_flight(uint64_t (&x)[N]) {
#pragma unroll
    for (int u = 0; u < N; ++u) asm volatile("" : "+v"(x[u]));
}

__device__ __forceinline__ uint64_t gwave(const BArgs& a) {
    return (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
}
__device__ __forceinline__ uint64_t gwaves(const BArgs& a) { return (uint64_t)a.n_blocks * kWaves; }

// ------------------------------------------------------------------------------------------------
// expand: the level expansion of the plain form with per-slot automata.  Segments (entry, first
// item, item count): light entries of the frontier list whole, then slices of heavy ones.
// Item phase: lane per item (segment by a wave prefix); word phase: groups of K lanes per item,
// lane k on word k of the rows.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ void entry_of(const BArgs& a, uint32_t row, uint32_t* slot, uint32_t* q, uint32_t* v,
                                         const BNfa** nfa) {
    const uint32_t stride = (uint32_t)a.slot_stride;
    *slot = row / stride;
    const uint32_t lrow = row - *slot * stride;
    *q = lrow / a.V;
    *v = lrow - *q * a.V;
    *nfa = a.nfas + ld32(&a.slots[*slot].query);
}

template <int K, bool SEEN>
__device__ __forceinline__ void expand_segments(const BArgs& a, const uint64_t* rows, bool have, uint32_t ent,
                                                uint32_t slot, uint32_t q, uint32_t v, uint64_t m,
                                                const uint32_t* delta, uint64_t beg, uint32_t len,
                                                uint64_t& t_items, uint64_t& t_wread, uint64_t& t_wupd) {
    constexpr int GS = 64 / K;
    const int lane = threadIdx.x & 63;
    const int grp = lane / K, k = lane % K;
    const uint64_t gmask = (K == 64) ? ~0ull : (((1ull << K) - 1) << (grp * K));
    const uint32_t V = a.V;
    const uint32_t stride = (uint32_t)a.slot_stride;
    if (!have) len = 0;
    const uint32_t incl = rpqd::wave_incl_scan_u32(len);
    const uint32_t excl = incl - len;
    const uint32_t total = __shfl(incl, 63, 64);
    if (lane == 0) t_items += total;
    const uint64_t dptr = reinterpret_cast<uint64_t>(delta);
    for (uint32_t base = 0; base < total; base += 64) {
        const uint32_t item = base + lane;
        int c = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const int cand = c + step;
            const uint32_t e = __shfl(excl, cand, 64);
            if (e <= item) c = cand;
        }
        const uint32_t c_ent = __shfl(ent, c, 64);
        const uint32_t c_slot = __shfl(slot, c, 64);
        const uint32_t c_q = __shfl(q, c, 64);
        const uint32_t c_v = __shfl(v, c, 64);
        const uint64_t c_m = __shfl(m, c, 64);
        const uint64_t c_beg = __shfl(beg, c, 64);
        const uint64_t c_delta = __shfl(dptr, c, 64);
        const uint32_t c_ex = __shfl(excl, c, 64);
        uint32_t my_row = 0;
        if (item < total) {
            uint32_t w = 0, q2 = 0;
            rpqd::decode_item(a.row_ptr, a.dst, a.L, reinterpret_cast<const uint32_t*>(c_delta), c_v, c_q, c_m,
                              c_beg + (item - c_ex), &w, &q2);
            my_row = c_slot * stride + q2 * V + w;
        }
        const uint32_t n_here = min(64u, total - base);
        for (uint32_t j = 0; j < n_here; j += GS * kUnroll) {
            uint32_t r[kUnroll];
            uint64_t f[kUnroll], nb[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t idx = j + u * GS + grp;
                r[u] = __shfl(my_row, idx & 63, 64);
                const uint32_t e = __shfl(c_ent, idx & 63, 64);
                f[u] = idx < n_here ? xld(rows + (uint64_t)e * K + k) : 0;
            }
            if constexpr (SEEN) {
                // seen OR (as in the plain form): the visited word already holds every bit of the
                // slot's earlier levels (ORed before the last barrier), so bits not in it are new
                uint64_t sw[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) sw[u] = f[u] ? xld(a.vis + (uint64_t)r[u] * K + k) : ~0ull;
                keep_in_flight<kUnroll>(sw);
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    nb[u] = f[u] & ~sw[u];
                    if (nb[u]) {
                        or_relaxed(a.vis + (uint64_t)r[u] * K + k, nb[u]);
                        or_relaxed(a.next + (uint64_t)r[u] * K + k, nb[u]);
                    }
                }
            } else {
                // visited and Next words together (as in the plain form)
                uint64_t vw[kUnroll], nx[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    vw[u] = f[u] ? xld(a.vis + (uint64_t)r[u] * K + k) : ~0ull;
                    nx[u] = f[u] ? xld(a.next + (uint64_t)r[u] * K + k) : ~0ull;
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    nb[u] = f[u] & ~vw[u] & ~nx[u];
                    if (nb[u]) or_relaxed(a.next + (uint64_t)r[u] * K + k, nb[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                t_wread += f[u] != 0;
                t_wupd += nb[u] != 0;
                const uint64_t hit = __ballot(nb[u] != 0) & gmask;
                if (k == 0 && hit) or_relaxed(&a.touch[r[u] >> 6], 1ull << (r[u] & 63));
            }
        }
    }
}

template <int K, bool SEEN>
__device__ void phase_expand(const BArgs& a, int p, uint64_t& t_items, uint64_t& t_descs, uint64_t& t_wread,
                             uint64_t& t_wupd) {
    const uint64_t n_list = min((uint64_t)ld(&a.ctl->list_cnt[p]), a.list_cap);
    const uint64_t n_desc = min((uint64_t)ld(&a.ctl->desc_cnt[p]), a.desc_cap);
    if (n_list == 0) return;
    const int lane = threadIdx.x & 63;
    const uint32_t* ids = p ? a.ids1 : a.ids0;
    const uint64_t* rows = p ? a.rows1 : a.rows0;
    const Desc* desc = p ? a.desc1 : a.desc0;
    const uint32_t H = a.H;
    const uint64_t n_lb = (n_list + 63) / 64;
    for (uint64_t b = gwave(a); b < n_lb; b += gwaves(a)) {
        const uint64_t e = b * 64 + lane;
        bool have = false;
        uint32_t slot = 0, q = 0, v = 0, len = 0;
        uint64_t m = 0;
        const BNfa* nfa = a.nfas;
        if (e < n_list) {
            entry_of(a, xld(ids + e), &slot, &q, &v, &nfa);
            m = a.lmask[v] & nfa->qlab[q];
            const uint64_t work = m ? rpqd::entry_work(a.row_ptr, a.L, nfa->delta, v, q, m) : 0;
            have = work != 0 && work <= H;
            len = have ? (uint32_t)work : 0;
        }
        const uint64_t hb = __ballot(have);   // every lane takes part
        if (lane == 0) t_descs += __popcll(hb);
        expand_segments<K, SEEN>(a, rows, have, (uint32_t)e, slot, q, v, m, nfa->delta, 0, len, t_items, t_wread, t_wupd);
    }
    const uint64_t n_db = (n_desc + 63) / 64;
    for (uint64_t b = gwave(a); b < n_db; b += gwaves(a)) {
        const uint64_t di = b * 64 + lane;
        bool have = false;
        uint32_t ent = 0, slot = 0, q = 0, v = 0, len = 0;
        uint64_t m = 0, beg = 0;
        const BNfa* nfa = a.nfas;
        if (di < n_desc) {
            const uint32_t* dw = reinterpret_cast<const uint32_t*>(desc + di);
            ent = xld(dw + 0);
            len = xld(dw + 1);
            beg = (uint64_t)xld(dw + 2) | ((uint64_t)xld(dw + 3) << 32);
            entry_of(a, xld(ids + ent), &slot, &q, &v, &nfa);
            m = a.lmask[v] & nfa->qlab[q];
            have = true;
        }
        const uint64_t hb = __ballot(have);   // every lane takes part
        if (lane == 0) t_descs += __popcll(hb);
        expand_segments<K, SEEN>(a, rows, have, ent, slot, q, v, m, nfa->delta, beg, len, t_items, t_wread, t_wupd);
    }
}

// ------------------------------------------------------------------------------------------------
// compact: touched rows -> row-id list p^1; per-slot liveness
// ------------------------------------------------------------------------------------------------
__device__ void phase_compact(const BArgs& a, int p, uint32_t iter) {
    const int np = p ^ 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st64(&a.ctl->list_cnt[p], 0);
        st64(&a.ctl->desc_cnt[p], 0);
    }
    const int lane = threadIdx.x & 63;
    const uint64_t n_words = (uint64_t)a.G * a.slot_stride / 64;
    const uint64_t words_per_slot = a.slot_stride / 64;
    uint32_t* ids = np ? a.ids1 : a.ids0;
    for (uint64_t w0 = gwave(a) * 64; w0 < n_words; w0 += gwaves(a) * 64) {
        const uint64_t wi = w0 + lane;
        uint64_t tw = wi < n_words ? xld(a.touch + wi) : 0;
        const uint64_t tw0 = tw;
        const uint32_t slot = (uint32_t)(wi / words_per_slot);
        uint64_t first = 0;   // rows touched for the first time in their unit
        if (tw) {
            if (ld32(&a.slots[slot].alive) != iter) st32(&a.slots[slot].alive, iter);
            const uint64_t ev = xld(a.ever + wi);
            first = tw & ~ev;
            if (first) a.ever[wi] = ev | tw;
        }
        // first-visit log (the rows whose Vis the slot's retirement clears).  A wave's words
        // usually lie in one slot: then one counter update serves the wave
        const uint32_t fc = (uint32_t)__popcll(first);
        const uint64_t fmask = __ballot(fc != 0);
        if (fmask) {
            const uint32_t s0 = __shfl(slot, __ffsll((long long)fmask) - 1, 64);
            unsigned long long li = 0;
            if (__ballot(fc != 0 && slot != s0) == 0) {
                const uint32_t fincl = rpqd::wave_incl_scan_u32(fc);
                const uint32_t ftot = __shfl(fincl, 63, 64);
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(&a.slots[s0].log_n, (unsigned long long)ftot);
                base = __shfl(base, 0, 64);
                li = base + fincl - fc;
            } else if (fc) {
                li = atomicAdd(&a.slots[slot].log_n, (unsigned long long)fc);
            }
            const uint64_t lbase = (wi - (uint64_t)slot * words_per_slot) * 64;
            uint32_t* log = a.logs + (uint64_t)slot * a.log_cap;
            while (first) {
                const int bt = __ffsll((long long)first) - 1;
                first &= first - 1;
                if (li < a.log_cap) log[li] = (uint32_t)(lbase + bt);   // beyond: the slot is cleared whole
                ++li;
            }
        }
        const uint32_t c = (uint32_t)__popcll(tw);
        const uint32_t incl = rpqd::wave_incl_scan_u32(c);
        const uint32_t tot = __shfl(incl, 63, 64);
        if (tot == 0) continue;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&a.ctl->list_cnt[np], (unsigned long long)tot);
        base = __shfl(base, 0, 64);
        uint64_t pos = base + incl - c;
        uint64_t left = 0;   // rows with no room in the list: they keep their touch bit (and Next)
        while (tw) {
            const int bt = __ffsll((long long)tw) - 1;
            tw &= tw - 1;
            if (pos < a.list_cap) ids[pos] = (uint32_t)(wi * 64 + bt);
            else left |= 1ull << bt;
            ++pos;
        }
        if (tw0) {
            a.touch[wi] = left;
            // a row left for the next iteration reaches its level late: exact depths are lost, so a
            // length-bounded query cannot wait
            if (left && a.queries[ld32(&a.slots[slot].query)].max_len != 0xFFFFFFFFu) atomicOr(&a.ctl->err, 1ull);
        }
    }
}

// ------------------------------------------------------------------------------------------------
// decide (block 0): running slots that produced no touched rows this iteration retire
// ------------------------------------------------------------------------------------------------
// Returns (to every thread of block 0) the number of slots that retire.
__device__ uint32_t phase_decide(const BArgs& a, uint32_t iter) {
    __shared__ uint32_t s_n, s_pairs;
    if (threadIdx.x == 0) {
        s_n = 0;
        s_pairs = 0;
    }
    __syncthreads();
    __shared__ uint32_t s_drain;
    if (threadIdx.x == 0) s_drain = 0;
    __syncthreads();
    uint32_t* drain = a.drain + (uint64_t)(iter & 1) * a.G;
    for (uint32_t s = threadIdx.x; s < a.G; s += kBlock) {
        if (ld32(&a.slots[s].state) == S_RUN && ld32(&a.slots[s].alive) != iter) {
            const uint32_t qid = ld32(&a.slots[s].query);
            if (a.queries[qid].pairs) {
                // keys need a prefix over the unit before they are written: retire now
                st32(&a.slots[s].state, S_RETIRE);
                const uint32_t i = atomicAdd(&s_n, 1u);
                st32(&a.retiring[i], s);
                atomicAdd(&s_pairs, 1u);
            } else {
                st32(&a.slots[s].state, S_DRAIN);
                st32(&a.slots[s].end_iter, iter);
                const uint32_t i = atomicAdd(&s_drain, 1u);
                st32(&drain[i], s);
            }
        }
    }
    __syncthreads();
    const uint32_t n = s_n;
    if (threadIdx.x == 0) {
        st64(&a.ctl->n_retiring, n);
        st64(&a.ctl->n_pairs_retiring, s_pairs);
        st64(&a.ctl->n_drain[iter & 1], s_drain);
    }
    return n;
}

// ------------------------------------------------------------------------------------------------
// retire: extraction over the non-empty Ans rows of each retiring slot
// ------------------------------------------------------------------------------------------------
template <int K, bool WRITE>
__device__ void phase_retire_extract(const BArgs& a, const uint32_t* list, uint32_t n_ret) {
    const int lane = threadIdx.x & 63;
    const uint64_t total = (uint64_t)n_ret * K * a.nchunks;
    for (uint64_t wv = gwave(a); wv < total; wv += gwaves(a)) {
        const uint32_t chunk = (uint32_t)(wv % a.nchunks);
        const uint32_t k = (uint32_t)((wv / a.nchunks) % K);
        const uint32_t slot = ld32(&list[wv / ((uint64_t)a.nchunks * K)]);
        const uint32_t u = ld32(&a.slots[slot].unit);
        const BUnit unit = a.units[u & a.unit_mask];
        const BQuery& Qy = a.queries[unit.query];
        if (WRITE && !Qy.pairs) continue;
        const uint32_t j = k * 64 + lane;
        const bool valid = j < unit.n;
        const uint64_t sidx = unit.src_off + j;
        const uint64_t s = valid ? (Qy.sources ? Qy.sources[sidx] : sidx) : 0;
        const uint32_t vbeg = chunk * kChunkV;
        // the chunk's 64 summary words: bit set = Ans row non-empty
        const uint64_t sw_i = (uint64_t)slot * a.summ_words + vbeg / 64 + lane;
        const uint64_t sw = (vbeg / 64 + lane < a.summ_words) ? xld(a.summ + sw_i) : 0;
        uint64_t cnt = 0, h = 0, cursor = 0;
        const uint64_t pidx = ((uint64_t)slot * a.W + j) * a.nchunks + chunk;
        if (WRITE && valid) cursor = a.srcbase[(uint64_t)slot * a.W + j] + a.partial[pidx];
        // per 64-vertex group with a non-empty summary word: one load per lane (lane = vertex),
        // then the non-zero words in ascending vertex order
        uint64_t any = __ballot(sw != 0);
        while (any) {
            const int wl = __ffsll((long long)any) - 1;
            any &= any - 1;
            uint64_t bits = __shfl(sw, wl, 64);
            const uint32_t vg = vbeg + (uint32_t)wl * 64;
            if (Qy.target) bits &= Qy.target[vg >> 6];   // vg is a multiple of 64
            const uint64_t mine = ((bits >> lane) & 1) ? xld(a.ans + ((uint64_t)slot * a.V + vg + lane) * K + k) : 0;
            uint64_t nz = __ballot(mine != 0);
            while (nz) {
                const int jj = __ffsll((long long)nz) - 1;
                nz &= nz - 1;
                const uint64_t word = __shfl(mine, jj, 64);
                const uint32_t v = vg + (uint32_t)jj;
                if (valid && ((word >> lane) & 1)) {
                    const uint64_t key = (s << 32) | v;
                    if (WRITE) {
                        if (cursor < Qy.capacity) Qy.stage[cursor] = key;
                        ++cursor;
                    } else {
                        ++cnt;
                        h += rpqd::mix64(key);
                    }
                }
            }
        }
        if (!WRITE) {
            if (Qy.pairs && valid) a.partial[pidx] = (uint32_t)cnt;
            if (Qy.per_source && valid && cnt) {
                atomicAdd((unsigned long long*)&Qy.per_source[2 * sidx], (unsigned long long)cnt);
                atomicAdd((unsigned long long*)&Qy.per_source[2 * sidx + 1], (unsigned long long)h);
            }
            const uint64_t wc = rpqd::wave_sum_u64(cnt), wh = rpqd::wave_sum_u64(h);
            if (lane == 0 && wc) {
                atomicAdd(&a.qout[unit.query].count, (unsigned long long)wc);
                atomicAdd(&a.qout[unit.query].hash, (unsigned long long)wh);
            }
        }
    }
}

// one block per retiring slot with pairs: chunk prefixes, source offsets, staging allocation
__device__ void phase_retire_prefix(const BArgs& a, uint32_t n_ret) {
    __shared__ uint64_t s_w[kWaves];
    __shared__ uint64_t s_carry, s_base;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (uint32_t r = blockIdx.x; r < n_ret; r += a.n_blocks) {
        const uint32_t slot = ld32(&a.retiring[r]);
        const uint32_t u = ld32(&a.slots[slot].unit);
        const BUnit unit = a.units[u & a.unit_mask];
        const BQuery& Qy = a.queries[unit.query];
        if (!Qy.pairs) continue;   // uniform per block
        if (t == 0) s_carry = 0;
        __syncthreads();
        // source totals and per-source chunk prefixes (pass 1), unit total
        for (uint32_t j0 = 0; j0 < a.W; j0 += kBlock) {
            const uint32_t j = j0 + t;
            uint64_t c = 0;
            if (j < unit.n) {
                uint32_t* pp = a.partial + ((uint64_t)slot * a.W + j) * a.nchunks;
                uint32_t run = 0;
                for (uint32_t ch = 0; ch < a.nchunks; ++ch) {
                    const uint32_t x = pp[ch];
                    pp[ch] = run;
                    run += x;
                }
                c = run;
            }
            const uint64_t incl = rpqd::wave_incl_scan_u64(c);
            if (lane == 63) s_w[wv] = incl;
            __syncthreads();
            uint64_t pre = s_carry;
            for (int w = 0; w < wv; ++w) pre += s_w[w];
            if (j < unit.n) a.srcbase[(uint64_t)slot * a.W + j] = pre + incl - c;   // unit-relative
            __syncthreads();
            if (t == 0) {
                uint64_t tot = 0;
                for (int w = 0; w < kWaves; ++w) tot += s_w[w];
                s_carry += tot;
            }
            __syncthreads();
        }
        if (t == 0) {
            const uint64_t tot = s_carry;
            const unsigned long long st = atomicAdd(&a.qout[unit.query].stage_top, (unsigned long long)tot);
            a.unit_total[u & a.unit_mask] = tot;
            a.unit_start[u & a.unit_mask] = st;
            if (st + tot > Qy.capacity) atomicOr(&a.qout[unit.query].overflow, 1ull);
            s_base = st;
        }
        __syncthreads();
        for (uint32_t j = t; j < unit.n; j += kBlock) a.srcbase[(uint64_t)slot * a.W + j] += s_base;
        __syncthreads();
    }
}

// clear the rows a retiring unit visited, its Ans rows and summary; the slot becomes idle
template <int K>
__device__ void phase_retire_clear(const BArgs& a, const uint32_t* list, uint32_t n_ret) {
    const int lane = threadIdx.x & 63;
    // Vis rows from the per-slot log, and the slot's first-visit bits
    for (uint32_t r = 0; r < n_ret; ++r) {
        const uint32_t slot = ld32(&list[r]);
        const uint64_t wps = a.slot_stride / 64;
        for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < wps; i += (uint64_t)a.n_blocks * kBlock)
            a.ever[(uint64_t)slot * wps + i] = 0;
        const uint64_t n = ld(&a.slots[slot].log_n);
        if (n > a.log_cap) {
            // the log overflowed: clear every row of the slot
            uint64_t* vs = a.vis + (uint64_t)slot * a.slot_stride * K;
            const uint64_t words = a.slot_stride * K;
            for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < words; i += (uint64_t)a.n_blocks * kBlock)
                vs[i] = 0;
            continue;
        }
        const uint32_t* log = a.logs + (uint64_t)slot * a.log_cap;
        for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)a.n_blocks * kBlock) {
            uint64_t* vs = a.vis + ((uint64_t)slot * a.slot_stride + xld(log + i)) * K;
#pragma unroll
            for (int k = 0; k < K; ++k) vs[k] = 0;
        }
    }
    // Ans rows flagged in the summary, then the summary itself
    for (uint32_t r = 0; r < n_ret; ++r) {
        const uint32_t slot = ld32(&list[r]);
        for (uint64_t w0 = gwave(a) * 64; w0 < a.summ_words; w0 += gwaves(a) * 64) {
            const uint64_t wi = w0 + lane;
            uint64_t sw = wi < a.summ_words ? xld(a.summ + (uint64_t)slot * a.summ_words + wi) : 0;
            if (sw) a.summ[(uint64_t)slot * a.summ_words + wi] = 0;
            while (sw) {
                const int bb = __ffsll((long long)sw) - 1;
                sw &= sw - 1;
                uint64_t* an = a.ans + ((uint64_t)slot * a.V + wi * 64 + bb) * K;
#pragma unroll
                for (int k = 0; k < K; ++k) an[k] = 0;
            }
        }
    }
    // The slot itself (log length, state) is reset in the next phase: other blocks may
    // still be reading log_n in this one.
}

// ------------------------------------------------------------------------------------------------
// refill (block 0 assigns units to idle slots), then every block seeds the new units
// ------------------------------------------------------------------------------------------------
__device__ void phase_assign(const BArgs& a, uint32_t iter) {
    __shared__ uint32_t s_running, s_idle, s_started;
    __shared__ unsigned long long s_head, s_avail;
    if (threadIdx.x == 0) {
        s_running = 0;
        s_idle = 0;
        s_started = 0;
        const unsigned long long head = ld(&a.ctl->queue_head);
        const unsigned long long tail = a.open_form ? ld(&a.ctl->units_tail) : (unsigned long long)a.n_units;
        s_head = head;
        s_avail = tail > head ? tail - head : 0;
    }
    __syncthreads();
    const unsigned long long head = s_head, avail = s_avail;
    for (uint32_t s = threadIdx.x; s < a.G; s += kBlock) {
        uint32_t st = ld32(&a.slots[s].state);
        const bool drained = st == S_DRAIN && ld32(&a.slots[s].end_iter) != iter;
        if (st == S_RETIRE || drained) {
            // retired in this iteration's earlier phases (or drained beside its expansion and
            // compaction): account its depth, free the slot
            const uint32_t qid = a.units[ld32(&a.slots[s].unit) & a.unit_mask].query;
            const uint32_t depth = (drained ? ld32(&a.slots[s].end_iter) : iter) - ld32(&a.slots[s].start_iter);
            atomicMax(&a.qout[qid].max_depth, (unsigned long long)depth);
            atomicAdd(&a.qout[qid].levels, (unsigned long long)depth);
            atomicAdd(&a.qout[qid].units_done, 1ull);
            st64(&a.slots[s].log_n, 0);
            st32(&a.slots[s].state, S_IDLE);
            st = S_IDLE;
        }
        if (st == S_IDLE) {
            // idle slots take the next units in queue order; the head moves by exactly the units
            // taken, so a unit published later is never skipped
            const uint32_t rank = atomicAdd(&s_idle, 1u);
            if (rank < avail) {
                const unsigned long long u = head + rank;
                st32(&a.slots[s].unit, (uint32_t)u);
                st32(&a.slots[s].query, a.units[u & a.unit_mask].query);
                st32(&a.slots[s].alive, iter);
                st32(&a.slots[s].start_iter, iter);
                st32(&a.slots[s].state, S_RUN);
                // seeding happens in phase_seed for slots whose start_iter == iter
                st = S_RUN;
                atomicAdd(&s_started, 1u);
            }
        }
        if (st == S_RUN) atomicAdd(&s_running, 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st64(&a.ctl->n_running, s_running);
        st64(&a.ctl->n_started, s_started);
        st64(&a.ctl->queue_head, head + min((unsigned long long)s_idle, avail));
    }
}

template <int K>
__device__ void phase_seed(const BArgs& a, int p, uint32_t iter) {
    const int np = p ^ 1;
    uint32_t* ids = np ? a.ids1 : a.ids0;
    const int lane = threadIdx.x & 63;
    const uint64_t total = (uint64_t)a.G * a.W;
    const uint64_t stride = (uint64_t)a.n_blocks * kBlock;
    // wave-uniform loop so that list appends can be counted once per wave
    for (uint64_t i0 = (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~63u); i0 < total; i0 += stride) {
        const uint64_t i = i0 + lane;
        bool seed = false;
        uint32_t slot = 0, j = 0, s = 0, init = 0;
        if (i < total) {
            slot = (uint32_t)(i / a.W);
            j = (uint32_t)(i % a.W);
            if (ld32(&a.slots[slot].state) == S_RUN && ld32(&a.slots[slot].start_iter) == iter) {
                const BUnit unit = a.units[ld32(&a.slots[slot].unit) & a.unit_mask];
                if (j < unit.n) {
                    const BQuery& Qy = a.queries[unit.query];
                    const uint64_t sidx = unit.src_off + j;
                    s = Qy.sources ? Qy.sources[sidx] : (uint32_t)sidx;
                    init = a.nfas[unit.query].init;
                    seed = true;
                }
            }
        }
        // one list entry per (slot, q, s): sources are distinct vertices, so every (q, s) row of a
        // slot gets exactly one source bit
        while (__ballot(seed && init != 0)) {
            const bool take = seed && init != 0;
            uint64_t row = 0;
            if (take) {
                const uint32_t q = __ffs(init) - 1;
                init &= init - 1;
                row = (uint64_t)slot * a.slot_stride + (uint64_t)q * a.V + s;
                or_relaxed(&a.next[row * K + (j >> 6)], 1ull << (j & 63));
                if (a.seen_or) or_relaxed(&a.vis[row * K + (j >> 6)], 1ull << (j & 63));
                or_relaxed(&a.ever[row >> 6], 1ull << (row & 63));
            }
            const uint64_t m = __ballot(take);
            unsigned long long base = 0, lbase = 0;
            if (lane == 0) base = atomicAdd(&a.ctl->list_cnt[np], (unsigned long long)__popcll(m));
            // a seeded row is new to its unit: it opens the slot's first-visit log (W is a multiple
            // of 64, so the wave's positions lie in one slot)
            if (lane == 0 && m) lbase = atomicAdd(&a.slots[i0 / a.W].log_n, (unsigned long long)__popcll(m));
            base = __shfl(base, 0, 64);
            lbase = __shfl(lbase, 0, 64);
            const unsigned long long pos = base + __popcll(m & rpqd::lanemask_lt());
            const unsigned long long li = lbase + __popcll(m & rpqd::lanemask_lt());
            if (take) {
                if (pos < a.list_cap) {
                    ids[pos] = (uint32_t)row;
                } else {
                    // no room: the seed waits on its touch bit for the next compaction
                    or_relaxed(&a.touch[row >> 6], 1ull << (row & 63));
                    if (a.queries[ld32(&a.slots[slot].query)].max_len != 0xFFFFFFFFu) atomicOr(&a.ctl->err, 1ull);
                }
                if (li < a.log_cap) a.logs[(uint64_t)slot * a.log_cap + li] = (uint32_t)(row - (uint64_t)slot * a.slot_stride);
            }
        }
    }
}

// ------------------------------------------------------------------------------------------------
// finalize: list p^1 -> frontier rows, Vis, Ans (+ summary), slices of heavy entries.  First visits are
// logged earlier, by the compaction (and the seeding) that put the rows on the list.
// Word phase: groups of K lanes per row; row phase: lane per row (as in the plain form).
// ------------------------------------------------------------------------------------------------
template <int K>
__device__ void phase_finalize(const BArgs& a, int p, uint32_t iter, uint64_t& t_frows, uint64_t& t_fwords) {
    constexpr int GS = 64 / K;
    const int np = p ^ 1;
    const uint64_t n = min((uint64_t)ld(&a.ctl->list_cnt[np]), a.list_cap);
    if (n == 0) return;
    const int lane = threadIdx.x & 63;
    const int grp = lane / K, k = lane % K;
    const uint32_t* ids = np ? a.ids1 : a.ids0;
    uint64_t* rows = np ? a.rows1 : a.rows0;
    Desc* dout = np ? a.desc1 : a.desc0;
    unsigned long long* dcnt = &a.ctl->desc_cnt[np];
    const uint32_t H = a.H, L = a.L, V = a.V;
    const uint32_t stride = (uint32_t)a.slot_stride;
    for (uint64_t e0 = gwave(a) * 64; e0 < n; e0 += gwaves(a) * 64) {
        const uint64_t e = e0 + lane;
        const bool active = e < n;
        uint32_t row32 = 0, slot = 0, lrow = 0, q = 0, v = 0, qid = 0;
        uint64_t eprod = 0, work = 0;
        const BNfa* nfa = a.nfas;
        uint32_t my_ans = 0xFFFFFFFFu;   // Ans row of a final-state entry, else none
        // at the depth bound of a length-bounded query a row is recorded (Vis, Ans) but gets an
        // empty frontier row and no work: it is never expanded
        bool stop = false;
        if (active) {
            row32 = xld(ids + e);
            slot = row32 / stride;
            lrow = row32 - slot * stride;
            q = lrow / V;
            v = lrow - q * V;
            qid = ld32(&a.slots[slot].query);
            nfa = a.nfas + qid;
            if ((nfa->final >> q) & 1) my_ans = slot * V + v;
            stop = iter - ld32(&a.slots[slot].start_iter) >= a.queries[qid].max_len;
        }
        const uint32_t n_here = (uint32_t)min<uint64_t>(64, n - e0);
        // the entry's work (its item count) and slices come first: a wave that finds no room for
        // its slices changes nothing and leaves its rows for the next iteration
        if (active) {
            const uint64_t m = stop ? 0 : (a.lmask[v] & nfa->qlab[q]);
            work = m ? rpqd::entry_work(a.row_ptr, L, nfa->delta, v, q, m) : 0;
        }
        const uint64_t ndesc = work > H ? (work + H - 1) / H : 0;
        const uint64_t dincl = rpqd::wave_incl_scan_u64(ndesc);
        const uint64_t dexcl = dincl - ndesc;
        const uint64_t dtot = __shfl(dincl, 63, 64);
        unsigned long long dbase = 0;
        if (dtot) {
            if (lane == 0) dbase = atomicAdd(dcnt, (unsigned long long)dtot);
            dbase = __shfl(dbase, 0, 64);
        }
        if (dtot && dbase + dtot > a.desc_cap) {
            // no room: empty slices where the wave reserved space inside the buffer (the expansion
            // reads every slice below the count), empty frontier rows, and the rows' touch bits back
            // on so that the next compaction lists them again with their Next bits
            for (uint64_t i = lane; i < dtot && dbase + i < a.desc_cap; i += 64) {
                Desc dd;
                dd.entry = (uint32_t)e0;
                dd.beg = 0;
                dd.len = 0;
                dout[dbase + i] = dd;
            }
            for (uint32_t idx = grp; idx < n_here; idx += GS) rows[(e0 + idx) * K + k] = 0;
            if (active) {
                or_relaxed(&a.touch[row32 >> 6], 1ull << (row32 & 63));
                if (a.queries[qid].max_len != 0xFFFFFFFFu) atomicOr(&a.ctl->err, 2ull);
            }
            continue;
        }
        uint32_t my_pc = 0;   // new source bits of this lane's row
        for (uint32_t j = 0; j < n_here; j += GS * kUnroll) {
            uint32_t r[kUnroll], an[kUnroll], sp[kUnroll];
            uint64_t nk[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t idx = j + u * GS + grp;
                r[u] = __shfl(row32, idx & 63, 64);
                an[u] = __shfl(my_ans, idx & 63, 64);
                sp[u] = __shfl((uint32_t)stop, idx & 63, 64);
                nk[u] = idx < n_here ? xld(a.next + (uint64_t)r[u] * K + k) : 0;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t idx = j + u * GS + grp;
                uint32_t pc = 0;
                if (idx < n_here) {
                    rows[(e0 + idx) * K + k] = sp[u] ? 0 : nk[u];
                    if (nk[u]) {
                        a.next[(uint64_t)r[u] * K + k] = 0;
                        // the row is on the list once and nothing else writes its Vis word in this
                        // phase (with seen OR the expansion has set these bits)
                        if (!a.seen_or) a.vis[(uint64_t)r[u] * K + k] |= nk[u];
                        pc = (uint32_t)__popcll(nk[u]);
                        ++t_fwords;
                        if (an[u] != 0xFFFFFFFFu) or_relaxed(a.ans + (uint64_t)an[u] * K + k, nk[u]);
                    }
                }
#pragma unroll
                for (int o = K / 2; o >= 1; o >>= 1) pc += __shfl_xor(pc, o, 64);
                const uint32_t rel = (uint32_t)lane - (j + u * GS);
                const uint32_t got = __shfl(pc, (rel % GS) * K, 64);
                if (rel < (uint32_t)GS) my_pc = got;
            }
        }
        if (active) {
            const uint32_t pc = my_pc;
            ++t_frows;
            if (my_ans != 0xFFFFFFFFu && pc)
                or_relaxed(&a.summ[(uint64_t)slot * a.summ_words + v / 64], 1ull << (v & 63));
            eprod = (uint64_t)pc * work;
        }
        // product edges per query (one atomic per wave when the wave holds one query)
        const uint32_t q0 = __shfl(qid, __ffsll((long long)__ballot(active)) - 1, 64);
        if (__ballot(active && qid != q0) == 0) {
            const uint64_t ws = rpqd::wave_sum_u64(eprod);
            if (lane == 0 && ws) atomicAdd(&a.qout[q0].eprod, (unsigned long long)ws);
        } else if (active && eprod) {
            atomicAdd(&a.qout[qid].eprod, (unsigned long long)eprod);
        }
        // entries of more than H items are cut into slices of at most H items, written by the whole
        // wave into the room reserved above
        if (dtot) {
            for (uint64_t i0 = 0; i0 < dtot; i0 += 64) {
                const uint64_t i = i0 + lane;
                int c = 0;
#pragma unroll
                for (int step = 32; step >= 1; step >>= 1) {
                    const int cand = c + step;
                    const uint64_t ex = __shfl(dexcl, cand, 64);
                    if (ex <= i) c = cand;
                }
                const uint64_t c_work = __shfl(work, c, 64);
                const uint64_t c_ex = __shfl(dexcl, c, 64);
                if (i < dtot) {
                    const uint64_t pos = dbase + i;
                    if (pos < a.desc_cap) {
                        const uint64_t kk = i - c_ex;
                        Desc dd;
                        dd.entry = (uint32_t)(e0 + c);
                        dd.beg = kk * H;
                        dd.len = (uint32_t)min<uint64_t>(H, c_work - kk * H);
                        dout[pos] = dd;
                    } else {
                        atomicOr(&a.ctl->err, 2ull);
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------------------------------------
// the persistent kernel
// ------------------------------------------------------------------------------------------------
// grid barrier, then block 0 charges the time since the previous barrier to `phase`
#define BAR(phase)                                                                   \
    do {                                                                             \
        if (!rpqd::grid_barrier(&a.ctl->gs, a.n_blocks, a.timeout)) return;          \
        if (blockIdx.x == 0 && threadIdx.x == 0) {                                   \
            const uint64_t now_ = wall_clock64();                                    \
            a.ctl->phase_ticks[phase] += now_ - t_last;                              \
            t_last = now_;                                                           \
        }                                                                            \
    } while (0)

template <int K, bool SEEN>
__global__ __launch_bounds__(kBlock, 4) void k_batch(BArgs a) {
    uint64_t t_items = 0, t_descs = 0, t_wread = 0, t_wupd = 0, t_frows = 0, t_fwords = 0;
    // iterations continue the numbering of earlier launches on the same state (open form); every
    // block reads the count before the first barrier, and it is only written after the last one of
    // an iteration.  Iteration i expands list (i - 1) & 1.
    const uint32_t iter0 = (uint32_t)ld(&a.ctl->iterations) + 1;
    int p = (int)((iter0 - 1) & 1);
    const uint64_t t_start = wall_clock64();
    uint64_t t_last = t_start;
    if (blockIdx.x == 0 && threadIdx.x == 0) st64(&a.ctl->t_begin, t_start);
    for (uint32_t iter = iter0;; ++iter) {
        // whole-kernel deadline: a run that exceeds it is abandoned (every block leaves at its
        // next barrier) and reported as an error
        if (blockIdx.x == 0 && threadIdx.x == 0 && wall_clock64() - t_start > a.deadline)
            __hip_atomic_store(&a.ctl->gs.abort, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // slots that reached their fixpoint in the previous iteration (no pairs to write): their counts
        // and checksums beside this expansion, their clear beside this compaction (a retiring slot
        // has no frontier, so its rows are not the ones these phases touch)
        const uint32_t* drain = a.drain + (uint64_t)((iter - 1) & 1) * a.G;
        const uint32_t n_dr = (uint32_t)ld(&a.ctl->n_drain[(iter - 1) & 1]);
        phase_expand<K, SEEN>(a, p, t_items, t_descs, t_wread, t_wupd);
        if (n_dr) phase_retire_extract<K, false>(a, drain, n_dr);
        BAR(0);
        phase_compact(a, p, iter);
        if (n_dr) phase_retire_clear<K>(a, drain, n_dr);
        BAR(1);
        // block 0 decides which slots retire; when none does, it refills at once (nothing to retire
        // first), which saves the refill's barrier
        if (blockIdx.x == 0 && phase_decide(a, iter) == 0) phase_assign(a, iter);
        BAR(2);
        const uint32_t n_ret = (uint32_t)ld(&a.ctl->n_retiring);
        if (n_ret) {
            phase_retire_extract<K, false>(a, a.retiring, n_ret);
            BAR(3);
            if (ld(&a.ctl->n_pairs_retiring)) {
                phase_retire_prefix(a, n_ret);
                BAR(4);
                phase_retire_extract<K, true>(a, a.retiring, n_ret);
                BAR(4);
            }
            phase_retire_clear<K>(a, a.retiring, n_ret);
            BAR(5);
            if (blockIdx.x == 0) phase_assign(a, iter);
            BAR(6);
        }
        // done when no slot runs and none waits to be drained in the next iteration
        if (ld(&a.ctl->n_running) == 0 && ld(&a.ctl->n_drain[iter & 1]) == 0) break;
        // seeding only when a slot took a unit in this iteration
        if (ld(&a.ctl->n_started)) {
            phase_seed<K>(a, p, iter);
            BAR(6);
        }
        phase_finalize<K>(a, p, iter, t_frows, t_fwords);
        BAR(7);
        p ^= 1;
        if (blockIdx.x == 0 && threadIdx.x == 0) st64(&a.ctl->iterations, iter);
        // open form: the launch ends here with its state intact; the next one resumes at iter + 1
        if (a.max_iters && iter - iter0 + 1 >= a.max_iters) break;
    }
    t_items = rpqd::wave_sum_u64(t_items);
    t_descs = rpqd::wave_sum_u64(t_descs);
    t_wread = rpqd::wave_sum_u64(t_wread);
    t_wupd = rpqd::wave_sum_u64(t_wupd);
    t_frows = rpqd::wave_sum_u64(t_frows);
    t_fwords = rpqd::wave_sum_u64(t_fwords);
    if (blockIdx.x == 0 && threadIdx.x == 0) st64(&a.ctl->t_end, wall_clock64());
    if ((threadIdx.x & 63) == 0) {
        if (t_items) {
            atomicAdd(&a.ctl->items, (unsigned long long)t_items);
            atomicAdd(&a.ctl->descs, (unsigned long long)t_descs);
            atomicAdd(&a.ctl->wreads, (unsigned long long)t_wread);
            atomicAdd(&a.ctl->wupds, (unsigned long long)t_wupd);
        }
        if (t_frows) {
            atomicAdd(&a.ctl->frows, (unsigned long long)t_frows);
            atomicAdd(&a.ctl->fwords, (unsigned long long)t_fwords);
        }
    }
}
#undef BAR

__global__ void k_check_sources(const uint32_t* __restrict__ src, uint64_t n, uint32_t V,
                                unsigned long long* __restrict__ bad) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t x = src[i];
        if (x >= V || (i > 0 && src[i - 1] >= x)) atomicOr(bad, 1ull);
    }
}

// after the persistent kernel: move each query's staged keys into its output in unit order
__global__ void k_gather_pairs(BArgs a, const uint64_t* __restrict__ unit_prefix) {
    for (uint32_t u = blockIdx.x; u < a.n_units; u += gridDim.x) {
        const BUnit unit = a.units[u];
        const BQuery& Qy = a.queries[unit.query];
        if (!Qy.pairs) continue;
        const uint64_t first = unit_prefix[Qy.first_unit];
        const uint64_t dst0 = unit_prefix[u] - first;       // keys of earlier units of this query
        const uint64_t src0 = a.unit_start[u];
        const uint64_t n = a.unit_total[u];
        for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) {
            if (src0 + i < Qy.capacity && dst0 + i < Qy.capacity)
                Qy.pairs[dst0 + i] = Qy.stage[src0 + i];
        }
    }
}

// ------------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------------
struct HostQuery {
    rpq_nfa nfa;
    const uint32_t* sources;
    uint64_t n_sources;
    uint32_t flags;
    uint32_t max_len = 0xFFFFFFFFu;
    uint64_t* pairs;
    uint64_t capacity;
    uint64_t* per_source;
    const uint64_t* target = nullptr;
};

struct Layout {
    uint32_t K, W, G, Qmax, H, nchunks, n_units;
    uint32_t seen_or;   // visit scheme of the expansion (1 = seen OR, 0 = two reads)
    uint64_t slot_stride, summ_words, list_cap, desc_cap, log_cap, stage_keys;
    uint64_t off_ctl, off_nfas, off_queries, off_qout, off_units, off_slots, off_vis, off_next, off_touch, off_ever,
        off_ans,
        off_summ, off_ids[2], off_rows[2], off_desc[2], off_logs, off_retiring, off_drain, off_partial, off_srcbase,
        off_stage,
        off_utotal, off_ustart, off_uprefix, off_scan_tmp, total;
};

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

}  // namespace

struct rpq_batch {
    rpq_graph* g = nullptr;
    rpq_batch_opts opts{};
    std::vector<HostQuery> queries;
    std::vector<BUnit> units;
    bool frozen = false;
    Layout lay{};
    // graph capture
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    void* ws_captured = nullptr;
    hipStream_t cap_stream = nullptr;
    unsigned n_blocks = 0;
    BQueryOut* h_out = nullptr;      // pinned copy of the per-query outputs
    BCtl* h_ctl = nullptr;
    double last_ms = 0;
    uint32_t unit_limit = 0;         // autotuning: run only the first units of the queue (0 = all)
    double last_kernel_ms = 0;
};

namespace {

void to_bnfa(const rpq_nfa& n, uint32_t L, BNfa* d) {
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

// Slot geometry shared by both forms: slice size (auto unless fixed), slices per slot and the device
// bytes of one slot.  x.W, x.K, x.Qmax and (when fixed) x.H are set by the caller.
// share > 1 sizes the frontier lists, slice buffers and first-visit logs for 1/share of the worst
// case (every row of every slot in one level): rows beyond them wait for a later iteration, and a
// slot whose log overflows is cleared whole.
void size_slots(const rpq_graph* g, uint32_t max_succ, bool auto_chunk, uint32_t share, Layout* x,
                uint64_t* desc_per_slot, uint64_t* per_slot) {
    x->slot_stride = ((uint64_t)x->Qmax * g->V + 63) / 64 * 64;
    x->summ_words = (g->V + 63) / 64;
    x->nchunks = (uint32_t)((g->V + kChunkV - 1) / kChunkV);
    // slices of one level and slot: entries with more than H items take ceil(work / H) <= 2 work / H
    // each, and all entries of one state hold at most E * max |delta(q, l)| items
    const uint64_t bitmap_bytes = x->slot_stride * x->K * 8 * 2;   // Vis + Next of one slot
    // default slice size: the smallest that keeps a slot's slice buffers within a quarter of its bitmaps
    while (auto_chunk && x->H < 256 &&
           2 * (2 * (uint64_t)x->Qmax * max_succ * g->E / x->H + 2) * sizeof(Desc) > bitmap_bytes / 4)
        x->H *= 2;
    *desc_per_slot = (2 * (uint64_t)x->Qmax * max_succ * g->E / x->H + 2) / share + 64;
    x->log_cap = std::max<uint64_t>(64, x->slot_stride / share);
    const uint64_t list_per_slot = x->slot_stride / share + 64;
    // per slot: Vis + Next, touch and first-visit bits, Ans, summary, first-visit log, and its share
    // of the two frontier lists (row id + K-word row per entry) and of the two slice buffers
    *per_slot = x->slot_stride * x->K * 8 * 2 + x->slot_stride / 4 + (uint64_t)g->V * x->K * 8 + x->summ_words * 8 +
                x->log_cap * 4 + 2 * list_per_slot * (4 + x->K * 8) + 2 * *desc_per_slot * sizeof(Desc);
}

// Offsets of every array for G slots, nq query-table entries and n_unit_entries unit entries.
void place(const rpq_graph* g, uint32_t nq, uint64_t n_unit_entries, Layout* x) {
    const uint64_t G = x->G;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const uint64_t nu = std::max<uint64_t>(1, n_unit_entries);
    x->off_ctl = take(sizeof(BCtl));
    x->off_nfas = take(sizeof(BNfa) * nq);
    x->off_queries = take(sizeof(BQuery) * nq);
    x->off_qout = take(sizeof(BQueryOut) * nq);
    x->off_units = take(sizeof(BUnit) * nu);
    x->off_slots = take(sizeof(BSlot) * G);
    x->off_vis = take(G * x->slot_stride * x->K * 8);
    x->off_next = take(G * x->slot_stride * x->K * 8);
    x->off_touch = take(G * x->slot_stride / 8);
    x->off_ever = take(G * x->slot_stride / 8);
    x->off_ans = take(G * (uint64_t)g->V * x->K * 8);
    x->off_summ = take(G * x->summ_words * 8);
    for (int p = 0; p < 2; ++p) {
        x->off_ids[p] = take(x->list_cap * 4);
        x->off_rows[p] = take(x->list_cap * x->K * 8);
        x->off_desc[p] = take(x->desc_cap * sizeof(Desc));
    }
    x->off_logs = take(G * x->log_cap * 4);
    x->off_retiring = take(G * 4);
    x->off_drain = take(2 * G * 4);
    x->off_partial = take(G * x->W * (uint64_t)x->nchunks * 4);
    x->off_srcbase = take(G * x->W * 8);
    x->off_stage = take(std::max<uint64_t>(1, x->stage_keys) * 8);
    x->off_utotal = take(nu * 8);
    x->off_ustart = take(nu * 8);
    x->off_uprefix = take((nu + 1) * 8);
    x->off_scan_tmp = take((rpq::scan_temp_elems(nu) + 1) * 8);
    x->total = off;
}

bool valid_width(uint32_t W) {
    return W == 64 || W == 128 || W == 256 || W == 512 || W == 1024 || W == 2048 || W == 4096;
}

int plan(rpq_batch* b) {
    const rpq_graph* g = b->g;
    Layout x;
    std::memset(&x, 0, sizeof x);
    x.W = b->opts.batch_width ? b->opts.batch_width : 512;
    if (!valid_width(x.W)) {
        rpq::set_error("batch_width must be 64 .. 4096, a power of two");
        return RPQ_EINVAL;
    }
    x.K = x.W / 64;
    x.H = b->opts.chunk_edges ? b->opts.chunk_edges : 16;
    if (x.H > 65535) {
        rpq::set_error("chunk_edges must be <= 65535");
        return RPQ_EINVAL;
    }
    if (b->opts.visit > RPQ_VISIT_SEEN_OR) {
        rpq::set_error("visit must be 0, RPQ_VISIT_TWO_READS or RPQ_VISIT_SEEN_OR");
        return RPQ_EINVAL;
    }
    x.seen_or = b->opts.visit ? b->opts.visit == RPQ_VISIT_SEEN_OR : g->V >= kSeenOrFrom;
    x.Qmax = 1;
    for (auto& q : b->queries) x.Qmax = std::max(x.Qmax, q.nfa.n_states);
    // units
    b->units.clear();
    uint32_t qi = 0;
    for (auto& q : b->queries) {
        for (uint64_t off = 0; off < q.n_sources; off += x.W) {
            BUnit u;
            u.query = qi;
            u.n = (uint32_t)std::min<uint64_t>(x.W, q.n_sources - off);
            u.src_off = off;
            b->units.push_back(u);
        }
        ++qi;
    }
    x.n_units = (uint32_t)b->units.size();
    uint32_t max_succ = 1;
    for (auto& q : b->queries)
        for (uint32_t i = 0; i < RPQ_MAX_STATES * RPQ_MAX_LABELS; ++i)
            max_succ = std::max(max_succ, (uint32_t)__builtin_popcount(q.nfa.delta[i]));
    // lists and slices sized for a quarter of the worst case (rows beyond wait a level), except when a
    // query is length-bounded: its rows must be expanded at their exact depth
    bool bounded = false;
    for (auto& q : b->queries) bounded |= q.max_len != 0xFFFFFFFFu;
    const uint32_t share = b->opts.list_share ? b->opts.list_share : (bounded ? 1 : 4);
    if (bounded && share != 1) {
        rpq::set_error("a batch with length-bounded queries needs list_share 1");
        return RPQ_EINVAL;
    }
    uint64_t desc_per_slot = 0, per_slot = 0;
    size_slots(g, max_succ, !b->opts.chunk_edges, share, &x, &desc_per_slot, &per_slot);
    uint64_t G = b->opts.slots;
    if (!G) {
        const uint64_t budget = 64ull << 30;
        G = std::max<uint64_t>(1, std::min<uint64_t>(std::max<uint64_t>(1, 65536 / x.W), budget / per_slot));
    }
    G = std::min<uint64_t>(G, std::max<uint32_t>(1, x.n_units));
    G = std::min<uint64_t>(G, 1024);
    if ((uint64_t)G * x.slot_stride >= 0xFFFFFFFFull || G >= (1u << 19)) {
        rpq::set_error("slots * states * vertices must stay below 2^32; use fewer slots");
        return RPQ_EUNSUPPORTED;
    }
    x.G = (uint32_t)G;
    x.list_cap = (uint64_t)x.G * (x.slot_stride / share + 64);
    x.desc_cap = (uint64_t)x.G * desc_per_slot;
    x.stage_keys = 0;
    for (auto& q : b->queries)
        if (q.pairs) x.stage_keys += q.capacity;
    place(g, (uint32_t)b->queries.size(), x.n_units, &x);
    b->lay = x;
    return RPQ_OK;
}

BArgs args_for(const rpq_graph* g, const Layout& x, char* ws, unsigned n_blocks, uint32_t n_units,
               uint32_t n_queries) {
    BArgs a;
    std::memset(&a, 0, sizeof a);
    a.seen_or = x.seen_or;
    a.row_ptr = g->out.row_ptr;
    a.dst = g->out.dst;
    a.lmask = g->out.lmask;
    a.nfas = reinterpret_cast<const BNfa*>(ws + x.off_nfas);
    a.queries = reinterpret_cast<const BQuery*>(ws + x.off_queries);
    a.qout = reinterpret_cast<BQueryOut*>(ws + x.off_qout);
    a.units = reinterpret_cast<const BUnit*>(ws + x.off_units);
    a.slots = reinterpret_cast<BSlot*>(ws + x.off_slots);
    a.ctl = reinterpret_cast<BCtl*>(ws + x.off_ctl);
    a.vis = reinterpret_cast<uint64_t*>(ws + x.off_vis);
    a.next = reinterpret_cast<uint64_t*>(ws + x.off_next);
    a.touch = reinterpret_cast<uint64_t*>(ws + x.off_touch);
    a.ever = reinterpret_cast<uint64_t*>(ws + x.off_ever);
    a.ans = reinterpret_cast<uint64_t*>(ws + x.off_ans);
    a.summ = reinterpret_cast<uint64_t*>(ws + x.off_summ);
    a.ids0 = reinterpret_cast<uint32_t*>(ws + x.off_ids[0]);
    a.ids1 = reinterpret_cast<uint32_t*>(ws + x.off_ids[1]);
    a.rows0 = reinterpret_cast<uint64_t*>(ws + x.off_rows[0]);
    a.rows1 = reinterpret_cast<uint64_t*>(ws + x.off_rows[1]);
    a.desc0 = reinterpret_cast<Desc*>(ws + x.off_desc[0]);
    a.desc1 = reinterpret_cast<Desc*>(ws + x.off_desc[1]);
    a.logs = reinterpret_cast<uint32_t*>(ws + x.off_logs);
    a.retiring = reinterpret_cast<uint32_t*>(ws + x.off_retiring);
    a.drain = reinterpret_cast<uint32_t*>(ws + x.off_drain);
    a.partial = reinterpret_cast<uint32_t*>(ws + x.off_partial);
    a.srcbase = reinterpret_cast<uint64_t*>(ws + x.off_srcbase);
    a.stage = reinterpret_cast<uint64_t*>(ws + x.off_stage);
    a.unit_total = reinterpret_cast<uint64_t*>(ws + x.off_utotal);
    a.unit_start = reinterpret_cast<uint64_t*>(ws + x.off_ustart);
    a.V = g->V;
    a.L = g->L;
    a.Qmax = x.Qmax;
    a.H = x.H;
    a.G = x.G;
    a.W = x.W;
    a.nchunks = x.nchunks;
    a.n_units = n_units;
    a.n_queries = n_queries;
    a.n_blocks = n_blocks;
    a.slot_stride = x.slot_stride;
    a.summ_words = x.summ_words;
    a.list_cap = x.list_cap;
    a.desc_cap = x.desc_cap;
    a.log_cap = x.log_cap;
    a.timeout = 100ull * 1000 * 1000 * 30;    // one barrier wait: 30 s of the 100 MHz clock
    a.deadline = 100ull * 1000 * 1000 * 300;  // whole run: 300 s
    a.open_form = 0;
    a.max_iters = 0;
    a.unit_mask = ~0ull;
    return a;
}

BArgs make_bargs(const rpq_batch* b, char* ws, unsigned n_blocks) {
    const Layout& x = b->lay;
    return args_for(b->g, x, ws, n_blocks, b->unit_limit ? std::min(x.n_units, b->unit_limit) : x.n_units,
                    (uint32_t)b->queries.size());
}

#define RPQ_BDISPATCH_K(K, CALL)                                 \
    switch (K) {                                                 \
        case 1: { constexpr int KK = 1; CALL; } break;           \
        case 2: { constexpr int KK = 2; CALL; } break;           \
        case 4: { constexpr int KK = 4; CALL; } break;           \
        case 8: { constexpr int KK = 8; CALL; } break;           \
        case 16: { constexpr int KK = 16; CALL; } break;         \
        case 32: { constexpr int KK = 32; CALL; } break;         \
        case 64: { constexpr int KK = 64; CALL; } break;         \
        default: rpq::set_error("bad width"); return RPQ_EINVAL; \
    }
// width K and visit scheme SS (seen OR) of the persistent kernel's instantiation
#define RPQ_BDISPATCH(K, SEEN_OR, CALL)                                                       \
    do {                                                                                      \
        if (SEEN_OR) {                                                                        \
            constexpr bool SS = true;                                                         \
            RPQ_BDISPATCH_K(K, CALL);                                                         \
        } else {                                                                              \
            constexpr bool SS = false;                                                        \
            RPQ_BDISPATCH_K(K, CALL);                                                         \
        }                                                                                     \
    } while (0)

template <int K, bool SEEN>
int launch_batch_kernel(unsigned n_blocks, const BArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_batch<K, SEEN>), dim3(n_blocks), dim3(kBlock), 0, s, a);
    return RPQ_OK;
}

template <int K, bool SEEN>
int co_resident_blocks(unsigned* out, int max_per_cu = 4) {
    int per_cu = 0, dev = 0, n_cu = 0;
    RPQ_HIP(hipGetDevice(&dev));
    RPQ_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    RPQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_batch<K, SEEN>), kBlock, 0));
    if (per_cu <= 0) {
        rpq::set_error("persistent kernel does not fit on a compute unit");
        return RPQ_EUNSUPPORTED;
    }
    // up to four 256-thread blocks per CU: enough waves in flight for the level phases
    // while the grid barrier stays cheap
    *out = (unsigned)std::min<uint64_t>((uint64_t)std::min(per_cu, max_per_cu) * n_cu,
                                        (uint64_t)rpqd::kBarMaxGroups * rpqd::kBarGroup);
    return RPQ_OK;
}

template <int K, bool SEEN>
int enqueue_run(rpq_batch* b, char* ws, hipStream_t s) {
    const Layout& x = b->lay;
    const unsigned nb = b->n_blocks;   // co-resident grid, sized before capture began
    BArgs a = make_bargs(b, ws, nb);
    // reset the mutable state with fill kernels (graph-safe, no memset nodes)
    RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(ws + x.off_ctl), sizeof(BCtl) / 8, 0, s));
    RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(ws + x.off_qout), sizeof(BQueryOut) / 8 * b->queries.size(),
                          0, s));
    RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(ws + x.off_slots), sizeof(BSlot) / 8 * x.G, 0, s));
    RPQ_TRY(rpq::fill_u64(a.vis, (uint64_t)x.G * x.slot_stride * x.K, 0, s));
    RPQ_TRY(rpq::fill_u64(a.next, (uint64_t)x.G * x.slot_stride * x.K, 0, s));
    RPQ_TRY(rpq::fill_u64(a.touch, (uint64_t)x.G * x.slot_stride / 64, 0, s));
    RPQ_TRY(rpq::fill_u64(a.ever, (uint64_t)x.G * x.slot_stride / 64, 0, s));
    RPQ_TRY(rpq::fill_u64(a.ans, (uint64_t)x.G * b->g->V * x.K, 0, s));
    RPQ_TRY(rpq::fill_u64(a.summ, (uint64_t)x.G * x.summ_words, 0, s));
    RPQ_TRY(rpq::fill_u64(a.unit_total, std::max<uint32_t>(1, x.n_units), 0, s));
    for (auto& q : b->queries)
        if (q.per_source) RPQ_TRY(rpq::fill_u64(q.per_source, q.n_sources * 2, 0, s));
    hipLaunchKernelGGL((k_batch<K, SEEN>), dim3(nb), dim3(kBlock), 0, s, a);
    RPQ_LAUNCH_CHECK();
    bool any_pairs = false;
    for (auto& q : b->queries) any_pairs |= q.pairs != nullptr;
    if (any_pairs) {
        uint64_t* prefix = reinterpret_cast<uint64_t*>(ws + x.off_uprefix);
        RPQ_TRY(rpq::exclusive_scan_u64(a.unit_total, prefix, x.n_units, reinterpret_cast<uint64_t*>(ws + x.off_scan_tmp),
                                        prefix + x.n_units, s));
        hipLaunchKernelGGL(k_gather_pairs, dim3(std::min<uint32_t>(x.n_units, 4096)), dim3(256), 0, s, a,
                           (const uint64_t*)prefix);
        RPQ_LAUNCH_CHECK();
    }
    return RPQ_OK;
}

}  // namespace

extern "C" {

int rpq_batch_create(rpq_graph_t g, const rpq_batch_opts* opts, rpq_batch_t* out) {
    rpq::clear_error();
    if (!g || !out) {
        rpq::set_error("NULL argument");
        return RPQ_EINVAL;
    }
    rpq_batch* b = new (std::nothrow) rpq_batch();
    if (!b) {
        rpq::set_error("host allocation failed");
        return RPQ_ENOMEM;
    }
    b->g = g;
    if (opts) b->opts = *opts;
    if (hipHostMalloc(reinterpret_cast<void**>(&b->h_ctl), sizeof(BCtl)) != hipSuccess) {
        delete b;
        rpq::set_error("pinned allocation failed");
        return RPQ_ENOMEM;
    }
    *out = b;
    return RPQ_OK;
}

int rpq_batch_destroy(rpq_batch_t b) {
    if (!b) return RPQ_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->h_out) (void)hipHostFree(b->h_out);
    if (b->h_ctl) (void)hipHostFree(b->h_ctl);
    delete b;
    return RPQ_OK;
}

int rpq_batch_add(rpq_batch_t b, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources, uint32_t flags,
                  uint64_t* pairs, uint64_t capacity, uint64_t* per_source, uint32_t* query_id) {
    rpq::clear_error();
    if (!b || !nfa) {
        rpq::set_error("NULL argument");
        return RPQ_EINVAL;
    }
    if (b->frozen) {
        rpq::set_error("batch already ran; create a new batch to add queries");
        return RPQ_EINVAL;
    }
    if (b->queries.size() >= 65535) {
        rpq::set_error("a batch holds at most 65535 queries");
        return RPQ_EUNSUPPORTED;
    }
    if (flags & ~(RPQ_PAIRS | RPQ_PER_SOURCE | RPQ_ALL_SOURCES)) {
        rpq::set_error("unsupported flags 0x%x for a batched query", flags);
        return RPQ_EINVAL;
    }
    if (nfa->n_states == 0 || nfa->n_states > RPQ_MAX_STATES || nfa->n_labels == 0 || nfa->n_labels > b->g->L) {
        rpq::set_error("invalid automaton for this graph");
        return RPQ_EINVAL;
    }
    const uint32_t smask = nfa->n_states == 32 ? 0xFFFFFFFFu : ((1u << nfa->n_states) - 1);
    for (uint32_t q = 0; q < RPQ_MAX_STATES; ++q)
        for (uint32_t l = 0; l < RPQ_MAX_LABELS; ++l) {
            const uint32_t d = nfa->delta[q * RPQ_MAX_LABELS + l];
            if (d && (q >= nfa->n_states || l >= nfa->n_labels || (d & ~smask))) {
                rpq::set_error("delta[%u][%u] is outside the automaton", q, l);
                return RPQ_EINVAL;
            }
        }
    if ((nfa->initial_mask & ~smask) || (nfa->final_mask & ~smask)) {
        rpq::set_error("initial/final mask names states >= n_states");
        return RPQ_EINVAL;
    }
    if (flags & RPQ_ALL_SOURCES) {
        if (sources) {
            rpq::set_error("RPQ_ALL_SOURCES requires sources == NULL");
            return RPQ_EINVAL;
        }
        n_sources = b->g->V;
    } else if (n_sources && !sources) {
        rpq::set_error("sources is NULL");
        return RPQ_EINVAL;
    }
    if ((flags & RPQ_PAIRS) && !pairs) {
        rpq::set_error("RPQ_PAIRS with a NULL pair buffer");
        return RPQ_EINVAL;
    }
    if ((flags & RPQ_PER_SOURCE) && n_sources && !per_source) {
        rpq::set_error("RPQ_PER_SOURCE with a NULL per_source buffer");
        return RPQ_EINVAL;
    }
    HostQuery q;
    q.nfa = *nfa;
    q.sources = sources;
    q.n_sources = n_sources;
    q.flags = flags;
    q.pairs = (flags & RPQ_PAIRS) ? pairs : nullptr;
    q.capacity = (flags & RPQ_PAIRS) ? capacity : 0;
    q.per_source = (flags & RPQ_PER_SOURCE) ? per_source : nullptr;
    if (query_id) *query_id = (uint32_t)b->queries.size();
    b->queries.push_back(q);
    return RPQ_OK;
}

int rpq_batch_bound_length(rpq_batch_t b, uint32_t query_id, uint32_t max_length) {
    rpq::clear_error();
    if (!b) {
        rpq::set_error("NULL argument");
        return RPQ_EINVAL;
    }
    if (b->frozen) {
        rpq::set_error("batch already ran; create a new batch to bound a query");
        return RPQ_EINVAL;
    }
    if (query_id >= b->queries.size()) {
        rpq::set_error("unknown query %u", query_id);
        return RPQ_EINVAL;
    }
    b->queries[query_id].max_len = max_length;
    return RPQ_OK;
}

}  // extern "C"

namespace rpq {

int batch_filter_targets(rpq_batch_t b, uint32_t query_id, const uint64_t* target) {
    if (!b || query_id >= b->queries.size()) {
        rpq::set_error("unknown batch or query");
        return RPQ_EINVAL;
    }
    if (b->frozen) {
        rpq::set_error("batch already ran; create a new batch to filter a query's results");
        return RPQ_EINVAL;
    }
    b->queries[query_id].target = target;
    return RPQ_OK;
}

}  // namespace rpq

extern "C" {

int rpq_batch_workspace_size(rpq_batch_t b, uint64_t* bytes) {
    rpq::clear_error();
    if (!b || !bytes) {
        rpq::set_error("NULL argument");
        return RPQ_EINVAL;
    }
    if (b->queries.empty()) {
        *bytes = 256;
        return RPQ_OK;
    }
    RPQ_TRY(plan(b));
    *bytes = b->lay.total;
    return RPQ_OK;
}

int rpq_batch_run(rpq_batch_t b, void* workspace, uint64_t workspace_bytes, hipStream_t stream) {
    rpq::clear_error();
    if (!b) {
        rpq::set_error("NULL batch");
        return RPQ_EINVAL;
    }
    if (b->queries.empty()) return RPQ_OK;
    if (!b->frozen) {
        RPQ_TRY(plan(b));
        b->frozen = true;
    }
    const Layout& x = b->lay;
    if (!workspace || workspace_bytes < x.total || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
        rpq::set_error("workspace must be 256-byte aligned and hold %llu bytes", (unsigned long long)x.total);
        return RPQ_ENOMEM;
    }
    char* ws = reinterpret_cast<char*>(workspace);
    if (b->ws_captured != workspace) {
        // sources: strictly ascending and below V, checked on the device before any traversal
        unsigned long long* bad = reinterpret_cast<unsigned long long*>(ws + x.off_ctl);
        RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(bad), 1, 0, stream));
        for (auto& q : b->queries)
            if (q.sources && q.n_sources) {
                hipLaunchKernelGGL(k_check_sources, dim3((unsigned)std::min<uint64_t>((q.n_sources + 255) / 256, 4096)),
                                   dim3(256), 0, stream, q.sources, q.n_sources, b->g->V, bad);
                RPQ_LAUNCH_CHECK();
            }
        unsigned long long hbad = 0;
        RPQ_HIP(hipMemcpyAsync(&hbad, bad, 8, hipMemcpyDeviceToHost, stream));
        RPQ_HIP(hipStreamSynchronize(stream));
        if (hbad) {
            rpq::set_error("batched sources must be strictly ascending vertex ids below n_vertices");
            return RPQ_EINVAL;
        }
    }
    const uint32_t nq = (uint32_t)b->queries.size();
    if (b->ws_captured != workspace) {
        // static tables: automata, queries, units (host -> device once per workspace)
        std::vector<BNfa> nf(nq);
        std::vector<BQuery> qs(nq);
        uint64_t stage_off = 0;
        uint32_t ufirst = 0;
        for (uint32_t i = 0; i < nq; ++i) {
            const HostQuery& h = b->queries[i];
            to_bnfa(h.nfa, b->g->L, &nf[i]);
            BQuery& d = qs[i];
            std::memset(&d, 0, sizeof d);
            d.sources = h.sources;
            d.n_sources = h.n_sources;
            d.per_source = h.per_source;
            d.pairs = h.pairs;
            d.capacity = h.capacity;
            d.stage = reinterpret_cast<uint64_t*>(ws + x.off_stage) + stage_off;
            if (h.pairs) stage_off += h.capacity;
            d.first_unit = ufirst;
            d.n_units = (uint32_t)((h.n_sources + x.W - 1) / x.W);
            ufirst += d.n_units;
            d.flags = h.flags;
            d.max_len = h.max_len;
            d.target = h.target;
        }
        RPQ_HIP(hipMemcpy(ws + x.off_nfas, nf.data(), sizeof(BNfa) * nq, hipMemcpyHostToDevice));
        RPQ_HIP(hipMemcpy(ws + x.off_queries, qs.data(), sizeof(BQuery) * nq, hipMemcpyHostToDevice));
        if (!b->units.empty())
            RPQ_HIP(hipMemcpy(ws + x.off_units, b->units.data(), sizeof(BUnit) * b->units.size(),
                              hipMemcpyHostToDevice));
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        if (b->graph) {
            (void)hipGraphDestroy(b->graph);
            b->graph = nullptr;
        }
        b->ws_captured = workspace;
    }
    if (!b->cap_stream) RPQ_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    if (!b->exec) {
        RPQ_BDISPATCH(x.K, x.seen_or, RPQ_TRY((co_resident_blocks<KK, SS>(&b->n_blocks))));
        RPQ_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        int rc = RPQ_OK;
        RPQ_BDISPATCH(x.K, x.seen_or, (rc = enqueue_run<KK, SS>(b, ws, b->cap_stream)));
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(b->cap_stream, &graph);
        if (rc != RPQ_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        RPQ_HIP(ec);
        b->graph = graph;
        RPQ_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    hipEvent_t e0, e1;
    RPQ_HIP(hipEventCreate(&e0));
    RPQ_HIP(hipEventCreate(&e1));
    RPQ_HIP(hipEventRecord(e0, stream));
    RPQ_HIP(hipGraphLaunch(b->exec, stream));
    RPQ_HIP(hipEventRecord(e1, stream));
    RPQ_HIP(hipStreamSynchronize(stream));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->last_ms = ms;
    RPQ_HIP(hipMemcpy(b->h_ctl, ws + x.off_ctl, sizeof(BCtl), hipMemcpyDeviceToHost));
    // block 0 stamps the constant clock (100 MHz) when it enters and leaves the persistent kernel
    if (b->h_ctl->t_end > b->h_ctl->t_begin) b->last_kernel_ms = (b->h_ctl->t_end - b->h_ctl->t_begin) / 1.0e5;
    if (b->h_ctl->gs.abort) {
        rpq::set_error(b->h_ctl->gs.abort == 2 ? "batched run exceeded its deadline and was abandoned"
                                               : "persistent kernel aborted at a grid barrier (grid not co-resident)");
        return RPQ_EDEVICE;
    }
    if (b->h_ctl->err) {
        rpq::set_error("internal capacity exceeded in the batched kernel (flags 0x%llx)",
                       (unsigned long long)b->h_ctl->err);
        return RPQ_EDEVICE;
    }
    return RPQ_OK;
}

int rpq_batch_result(rpq_batch_t b, uint32_t query_id, rpq_result* out) {
    rpq::clear_error();
    if (!b || !out || query_id >= b->queries.size() || !b->frozen || !b->ws_captured) {
        rpq::set_error("invalid batch, query id, or batch has not run");
        return RPQ_EINVAL;
    }
    BQueryOut o;
    const char* ws = reinterpret_cast<const char*>(b->ws_captured);
    RPQ_HIP(hipMemcpy(&o, ws + b->lay.off_qout + sizeof(BQueryOut) * query_id, sizeof o, hipMemcpyDeviceToHost));
    const HostQuery& h = b->queries[query_id];
    std::memset(out, 0, sizeof *out);
    out->pairs = h.pairs;
    out->capacity = h.capacity;
    out->per_source = h.per_source;
    out->count = o.count;
    out->hash = o.hash;
    out->product_edges = o.eprod;
    out->levels = o.levels;
    out->max_depth = o.max_depth;
    if (h.pairs) {
        out->written = std::min<uint64_t>(o.count, h.capacity);
        if (o.count > h.capacity) {
            rpq::set_error("query %u has %llu keys; capacity %llu", query_id, (unsigned long long)o.count,
                           (unsigned long long)h.capacity);
            return RPQ_EOVERFLOW;
        }
    }
    return RPQ_OK;
}

int rpq_batch_stats(rpq_batch_t b, rpq_batch_info* out) {
    rpq::clear_error();
    if (!b || !out) {
        rpq::set_error("NULL argument");
        return RPQ_EINVAL;
    }
    std::memset(out, 0, sizeof *out);
    out->n_queries = (uint32_t)b->queries.size();
    out->n_units = b->lay.n_units;
    out->slots = b->lay.G;
    out->batch_width = b->lay.W;
    out->blocks = b->n_blocks;
    out->visit = b->lay.seen_or ? RPQ_VISIT_SEEN_OR : RPQ_VISIT_TWO_READS;
    out->workspace_bytes = b->lay.total;
    out->last_run_ms = b->last_ms;
    out->last_kernel_ms = b->last_kernel_ms;
    if (b->h_ctl)
        for (int i = 0; i < 8; ++i) out->phase_ms[i] = b->h_ctl->phase_ticks[i] / 1.0e5;
    out->touch_words = b->lay.G * b->lay.slot_stride / 64;
    out->row_words = b->lay.K;
    if (b->h_ctl) {
        out->finalized_rows = b->h_ctl->frows;
        out->finalized_words = b->h_ctl->fwords;
        out->iterations = b->h_ctl->iterations;
        out->edge_items = b->h_ctl->items;
        out->descriptors = b->h_ctl->descs;
        out->word_reads = b->h_ctl->wreads;
        out->word_updates = b->h_ctl->wupds;
    }
    return RPQ_OK;
}

int rpq_batch_autotune(rpq_batch_t b, const rpq_batch_opts* candidates, uint32_t n_candidates, void* workspace,
                       uint64_t workspace_bytes, hipStream_t stream, rpq_batch_opts* best) {
    rpq::clear_error();
    if (!b || !workspace) {
        rpq::set_error("NULL argument");
        return RPQ_EINVAL;
    }
    if (b->queries.empty()) {
        if (best) *best = b->opts;
        return RPQ_OK;
    }
    std::vector<rpq_batch_opts> cands;
    if (candidates && n_candidates) {
        cands.assign(candidates, candidates + n_candidates);
    } else {
        const uint32_t widths[] = {64, 256, 512, 1024, 2048};
        const uint32_t chunks[] = {16, 64};
        for (uint32_t w : widths)
            for (uint32_t h : chunks) {
                rpq_batch_opts o{};
                o.batch_width = w;
                o.chunk_edges = h;
                cands.push_back(o);
            }
    }
    const rpq_batch_opts saved = b->opts;
    double best_rate = -1.0;
    rpq_batch_opts best_opts = saved;
    for (const rpq_batch_opts& c : cands) {
        b->opts = c;
        if (!b->opts.visit) b->opts.visit = saved.visit;   // the scheme is the batch's, not tuned
        b->frozen = false;
        if (plan(b) != RPQ_OK || b->lay.total > workspace_bytes) continue;
        // time a bounded prefix of the unit queue: enough units for a few refills of every slot
        const uint32_t prefix = std::max<uint32_t>(4 * b->lay.G, b->lay.n_units / 20);
        b->unit_limit = std::min<uint32_t>(b->lay.n_units, prefix);
        uint64_t sources_run = 0;
        for (uint32_t u = 0; u < b->unit_limit; ++u) sources_run += b->units[u].n;
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        if (b->graph) {
            (void)hipGraphDestroy(b->graph);
            b->graph = nullptr;
        }
        b->ws_captured = nullptr;
        int rc = rpq_batch_run(b, workspace, workspace_bytes, stream);
        if (rc == RPQ_OK) rc = rpq_batch_run(b, workspace, workspace_bytes, stream);   // replay: steady state
        if (rc != RPQ_OK) continue;
        const double rate = sources_run / std::max(1e-6, b->last_ms);
        if (rate > best_rate) {
            best_rate = rate;
            best_opts = c;
        }
    }
    // settle on the winner: full queue, fresh plan, capture on the next run
    b->unit_limit = 0;
    b->opts = best_rate > 0 ? best_opts : saved;
    b->frozen = false;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    b->ws_captured = nullptr;
    RPQ_TRY(plan(b));
    if (best) *best = b->opts;
    if (best_rate < 0) {
        rpq::set_error("no autotuning candidate fits the workspace");
        return RPQ_ENOMEM;
    }
    return RPQ_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// Resident engine: the open form of the persistent kernel.  Between launches the host uploads the
// queries that arrived (automaton, query record, zeroed outputs, and their units appended to the
// device ring) and publishes the new tail; the kernel's refill phase hands the new units to slots
// as they free up.  A launch ends after max_iters iterations, or earlier when no slot runs and the
// queue is empty, and leaves slots, lists and counters for the next one.
// ------------------------------------------------------------------------------------------------
namespace {

constexpr uint32_t kResQueries = 4096;       // query-table entries
constexpr uint64_t kResRing = 1ull << 16;    // unit-ring entries (a power of two)
constexpr uint32_t kResMaxStaged = 256;      // queries uploaded per launch
constexpr uint64_t kResMaxStagedUnits = 1ull << 14;
constexpr uint32_t kResShare = 8;            // lists, slices and logs for 1/8 of the worst case

struct ResRecord {
    uint32_t q, pad;
    BNfa nfa;
    BQuery bq;
};

// Install the staged records into their table entries, zero their outputs, publish the unit tail
// and reset the grid barrier for the launch that follows on the same stream.
__global__ void k_res_install(BArgs a, const ResRecord* __restrict__ recs, uint32_t n_recs,
                              unsigned long long units_tail) {
    for (uint32_t i = blockIdx.x; i < n_recs; i += gridDim.x) {
        const ResRecord& r = recs[i];
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&r.nfa);
        uint32_t* dst = reinterpret_cast<uint32_t*>(const_cast<BNfa*>(a.nfas) + r.q);
        for (uint32_t j = threadIdx.x; j < sizeof(BNfa) / 4; j += blockDim.x) dst[j] = src[j];
        const uint32_t* qs = reinterpret_cast<const uint32_t*>(&r.bq);
        uint32_t* qd = reinterpret_cast<uint32_t*>(const_cast<BQuery*>(a.queries) + r.q);
        for (uint32_t j = threadIdx.x; j < sizeof(BQuery) / 4; j += blockDim.x) qd[j] = qs[j];
        unsigned long long* o = reinterpret_cast<unsigned long long*>(a.qout + r.q);
        for (uint32_t j = threadIdx.x; j < sizeof(BQueryOut) / 8; j += blockDim.x) o[j] = 0;
        if (r.bq.per_source)
            for (uint64_t j = threadIdx.x; j < 2 * r.bq.n_sources; j += blockDim.x) r.bq.per_source[j] = 0;
    }
    if (blockIdx.x == 0) {
        unsigned int* g = reinterpret_cast<unsigned int*>(&a.ctl->gs);
        for (uint32_t j = threadIdx.x; j < sizeof(rpqd::GridSync) / 4; j += blockDim.x) g[j] = 0;
        if (threadIdx.x == 0) a.ctl->units_tail = units_tail;
    }
}

}  // namespace

namespace rpq {

struct Resident {
    rpq_graph* g = nullptr;
    Layout x{};
    char* ws = nullptr;
    ResRecord* d_recs = nullptr;        // device upload area
    unsigned long long* d_bad = nullptr;
    unsigned n_blocks = 0;
    uint32_t max_succ = 0;
    bool broken = false;
    struct Entry {
        bool used = false;
        uint64_t token = 0, u0 = 0, n_units = 0, capacity = 0;
        bool pairs = false;
    };
    std::vector<Entry> table;
    std::vector<uint32_t> free_q;
    uint32_t q_hi = 0;                  // table entries [0, q_hi) may be in use
    struct Staged {
        uint64_t token;
        ResidentQuery q;
    };
    std::vector<Staged> staged;
    uint64_t units_tail = 0;            // units published to the device ring
    uint64_t n_active = 0;
    ResRecord* h_recs = nullptr;        // pinned
    BUnit* h_units = nullptr;           // pinned
    BQueryOut* h_out = nullptr;         // pinned
    BCtl* h_ctl = nullptr;              // pinned
    unsigned long long* h_bad = nullptr;   // pinned
};

namespace {

int res_layout(const rpq_graph* g, uint32_t W, uint32_t G, uint32_t Qmax, uint32_t max_succ, Layout* out,
               uint64_t* total) {
    if (!valid_width(W) || G == 0 || G > 1024 || Qmax == 0 || Qmax > RPQ_MAX_STATES || max_succ == 0 ||
        max_succ > RPQ_MAX_STATES) {
        rpq::set_error("resident engine: width 64..4096 (power of two), 1..1024 slots, 1..32 states");
        return RPQ_EINVAL;
    }
    Layout x;
    std::memset(&x, 0, sizeof x);
    x.W = W;
    x.K = W / 64;
    x.H = 16;
    x.Qmax = Qmax;
    x.seen_or = g->V >= kSeenOrFrom;
    x.G = G;
    uint64_t desc_per_slot = 0, per_slot = 0;
    size_slots(g, max_succ, true, kResShare, &x, &desc_per_slot, &per_slot);
    if ((uint64_t)G * x.slot_stride >= 0xFFFFFFFFull) {
        rpq::set_error("slots * states * vertices must stay below 2^32; use fewer slots");
        return RPQ_EUNSUPPORTED;
    }
    x.list_cap = (uint64_t)G * (x.slot_stride / kResShare + 64);
    x.desc_cap = (uint64_t)G * desc_per_slot;
    x.stage_keys = 0;
    x.n_units = 0;
    place(g, kResQueries, kResRing, &x);
    *out = x;
    *total = align256(x.total) + align256(sizeof(ResRecord) * kResMaxStaged) + kResMaxStaged * 8;
    return RPQ_OK;
}

BArgs res_args(const Resident* r, uint32_t max_iters) {
    BArgs a = args_for(r->g, r->x, r->ws, r->n_blocks, 0, kResQueries);
    a.open_form = 1;
    a.max_iters = max_iters;
    a.unit_mask = kResRing - 1;
    return a;
}

// every query staged, queued or running completes with `status`
void res_fail_all(Resident* r, int status, std::vector<ResidentDone>* done) {
    for (uint32_t q = 0; q < r->q_hi; ++q) {
        Resident::Entry& e = r->table[q];
        if (!e.used) continue;
        ResidentDone d{};
        d.token = e.token;
        d.status = status;
        done->push_back(d);
        e.used = false;
        r->free_q.push_back(q);
    }
    for (auto& st : r->staged) {
        ResidentDone d{};
        d.token = st.token;
        d.status = status;
        done->push_back(d);
    }
    r->staged.clear();
    r->n_active = 0;
}

}  // namespace

int resident_bytes(const rpq_graph* g, uint32_t W, uint32_t G, uint32_t Qmax, uint32_t max_succ, uint64_t* bytes) {
    Layout x;
    return res_layout(g, W, G, Qmax, max_succ, &x, bytes);
}

int resident_create(rpq_graph* g, uint32_t W, uint32_t G, uint32_t Qmax, uint32_t max_succ, void* mem,
                    uint64_t bytes, hipStream_t stream, Resident** out) {
    Layout x;
    uint64_t need = 0;
    RPQ_TRY(res_layout(g, W, G, Qmax, max_succ, &x, &need));
    if (!mem || bytes < need || (reinterpret_cast<uintptr_t>(mem) & 255)) {
        rpq::set_error("resident engine needs %llu bytes of 256-byte aligned device memory",
                       (unsigned long long)need);
        return RPQ_ENOMEM;
    }
    std::unique_ptr<Resident> r(new (std::nothrow) Resident());
    if (!r) {
        rpq::set_error("out of host memory");
        return RPQ_ENOMEM;
    }
    r->g = g;
    r->x = x;
    r->ws = reinterpret_cast<char*>(mem);
    r->d_recs = reinterpret_cast<ResRecord*>(r->ws + align256(x.total));
    r->d_bad = reinterpret_cast<unsigned long long*>(r->ws + align256(x.total) +
                                                     align256(sizeof(ResRecord) * kResMaxStaged));
    r->max_succ = max_succ;
    r->table.resize(kResQueries);
    for (uint32_t q = kResQueries; q-- > 0;) r->free_q.push_back(q);
    // half the co-resident occupancy: requests outside the engine keep room on every compute unit
    RPQ_BDISPATCH(x.K, x.seen_or, RPQ_TRY((co_resident_blocks<KK, SS>(&r->n_blocks, 2))));
    RPQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&r->h_recs), sizeof(ResRecord) * kResMaxStaged));
    RPQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&r->h_units), sizeof(BUnit) * kResMaxStagedUnits));
    RPQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&r->h_out), sizeof(BQueryOut) * kResQueries));
    RPQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&r->h_ctl), sizeof(BCtl)));
    RPQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&r->h_bad), 8 * kResMaxStaged));
    // a clean state: no units, idle slots, empty bitmaps
    const BArgs a = res_args(r.get(), 1);
    RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(r->ws + x.off_ctl), sizeof(BCtl) / 8, 0, stream));
    RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(r->ws + x.off_qout), sizeof(BQueryOut) / 8 * kResQueries, 0,
                          stream));
    RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(r->ws + x.off_slots), sizeof(BSlot) / 8 * x.G, 0, stream));
    RPQ_TRY(rpq::fill_u64(a.vis, (uint64_t)x.G * x.slot_stride * x.K, 0, stream));
    RPQ_TRY(rpq::fill_u64(a.next, (uint64_t)x.G * x.slot_stride * x.K, 0, stream));
    RPQ_TRY(rpq::fill_u64(a.touch, (uint64_t)x.G * x.slot_stride / 64, 0, stream));
    RPQ_TRY(rpq::fill_u64(a.ever, (uint64_t)x.G * x.slot_stride / 64, 0, stream));
    RPQ_TRY(rpq::fill_u64(a.ans, (uint64_t)x.G * g->V * x.K, 0, stream));
    RPQ_TRY(rpq::fill_u64(a.summ, (uint64_t)x.G * x.summ_words, 0, stream));
    RPQ_TRY(rpq::fill_u64(a.unit_total, kResRing, 0, stream));
    RPQ_HIP(hipStreamSynchronize(stream));
    *out = r.release();
    return RPQ_OK;
}

void resident_destroy(Resident* r) {
    if (!r) return;
    for (void* p : {static_cast<void*>(r->h_recs), static_cast<void*>(r->h_units), static_cast<void*>(r->h_out),
                    static_cast<void*>(r->h_ctl), static_cast<void*>(r->h_bad)})
        if (p) (void)hipHostFree(p);
    delete r;
}

bool resident_fits(const Resident* r, const ResidentQuery& q) {
    if (q.nfa.n_states == 0 || q.nfa.n_states > r->x.Qmax) return false;
    for (uint32_t i = 0; i < RPQ_MAX_STATES * RPQ_MAX_LABELS; ++i)
        if ((uint32_t)__builtin_popcount(q.nfa.delta[i]) > r->max_succ) return false;
    const uint64_t n_units = (q.n_sources + r->x.W - 1) / r->x.W;
    if (q.pairs && n_units > 1) return false;
    return n_units <= kResMaxStagedUnits;
}

bool resident_broken(const Resident* r) { return r->broken; }

int resident_admit(Resident* r, const ResidentQuery& q, uint64_t token) {
    if (r->broken || !resident_fits(r, q)) {
        rpq::set_error("query does not fit the resident engine");
        return RPQ_EUNSUPPORTED;
    }
    uint64_t staged_units = 0;
    for (auto& s : r->staged) staged_units += (s.q.n_sources + r->x.W - 1) / r->x.W;
    const uint64_t n_units = (q.n_sources + r->x.W - 1) / r->x.W;
    // ring room: units still referenced by active queries start at the oldest active unit
    uint64_t oldest = r->units_tail;
    for (uint32_t i = 0; i < r->q_hi; ++i)
        if (r->table[i].used) oldest = std::min(oldest, r->table[i].u0);
    if (r->staged.size() >= kResMaxStaged || r->free_q.size() <= r->staged.size() ||
        staged_units + n_units > kResMaxStagedUnits ||
        r->units_tail + staged_units + n_units - oldest > kResRing) {
        rpq::set_error("resident engine is full");
        return RPQ_ENOMEM;
    }
    r->staged.push_back({token, q});
    return RPQ_OK;
}

bool resident_idle(const Resident* r) { return r->staged.empty() && r->n_active == 0; }

namespace {

int step_body(Resident* r, uint32_t max_iters, hipStream_t stream, std::vector<ResidentDone>* done) {
    const Layout& x = r->x;
    // 1. sources of the staged queries: strictly ascending ids below V, checked before any unit of
    //    them is published
    const uint32_t n_st = (uint32_t)r->staged.size();
    if (n_st) {
        RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(r->d_bad), n_st, 0, stream));
        for (uint32_t i = 0; i < n_st; ++i) {
            const ResidentQuery& q = r->staged[i].q;
            if (q.sources && q.n_sources) {
                hipLaunchKernelGGL(k_check_sources, dim3((unsigned)std::min<uint64_t>((q.n_sources + 255) / 256, 4096)),
                                   dim3(256), 0, stream, q.sources, q.n_sources, r->g->V, r->d_bad + i);
                RPQ_LAUNCH_CHECK();
            }
        }
        RPQ_HIP(hipMemcpyAsync(r->h_bad, r->d_bad, 8ull * n_st, hipMemcpyDeviceToHost, stream));
        RPQ_HIP(hipStreamSynchronize(stream));
    }
    // 2. table entries, records and units of the valid ones
    uint32_t n_rec = 0;
    uint64_t n_u = 0;
    const uint64_t tail0 = r->units_tail;
    for (uint32_t i = 0; i < n_st; ++i) {
        const ResidentQuery& q = r->staged[i].q;
        const uint64_t token = r->staged[i].token;
        if (r->h_bad[i]) {
            ResidentDone d{};
            d.token = token;
            d.status = RPQ_EINVAL;
            done->push_back(d);
            continue;
        }
        const uint64_t nu = (q.n_sources + x.W - 1) / x.W;
        if (nu == 0) {   // no sources: nothing to run
            ResidentDone d{};
            d.token = token;
            d.status = RPQ_OK;
            done->push_back(d);
            continue;
        }
        const uint32_t qi = r->free_q.back();
        r->free_q.pop_back();
        r->q_hi = std::max(r->q_hi, qi + 1);
        Resident::Entry& e = r->table[qi];
        e.used = true;
        e.token = token;
        e.u0 = tail0 + n_u;
        e.n_units = nu;
        e.pairs = q.pairs != nullptr;
        e.capacity = q.pairs ? q.capacity : 0;
        ResRecord& rec = r->h_recs[n_rec++];
        std::memset(&rec, 0, sizeof rec);
        rec.q = qi;
        to_bnfa(q.nfa, r->g->L, &rec.nfa);
        rec.bq.sources = q.sources;
        rec.bq.n_sources = q.n_sources;
        rec.bq.per_source = q.per_source;
        rec.bq.pairs = q.pairs;
        rec.bq.capacity = q.pairs ? q.capacity : 0;
        rec.bq.stage = q.pairs;   // one unit: its keys are the query's output, in order
        rec.bq.first_unit = (uint32_t)(e.u0 & 0xFFFFFFFFu);
        rec.bq.n_units = (uint32_t)nu;
        rec.bq.flags = (q.pairs ? RPQ_PAIRS : 0) | (q.per_source ? RPQ_PER_SOURCE : 0);
        rec.bq.max_len = q.max_len;
        for (uint64_t k = 0; k < nu; ++k) {
            BUnit& u = r->h_units[n_u++];
            u.query = qi;
            u.n = (uint32_t)std::min<uint64_t>(x.W, q.n_sources - k * x.W);
            u.src_off = k * x.W;
        }
        ++r->n_active;
    }
    r->staged.clear();
    if (r->n_active == 0) return RPQ_OK;
    // 3. upload: records, then the units into the ring (two pieces where it wraps)
    BArgs a = res_args(r, max_iters);
    if (n_rec) RPQ_HIP(hipMemcpyAsync(r->d_recs, r->h_recs, sizeof(ResRecord) * n_rec, hipMemcpyHostToDevice, stream));
    if (n_u) {
        BUnit* ring = reinterpret_cast<BUnit*>(r->ws + x.off_units);
        const uint64_t at = tail0 & (kResRing - 1);
        const uint64_t first = std::min<uint64_t>(n_u, kResRing - at);
        RPQ_HIP(hipMemcpyAsync(ring + at, r->h_units, sizeof(BUnit) * first, hipMemcpyHostToDevice, stream));
        if (first < n_u)
            RPQ_HIP(hipMemcpyAsync(ring, r->h_units + first, sizeof(BUnit) * (n_u - first), hipMemcpyHostToDevice,
                                   stream));
    }
    r->units_tail = tail0 + n_u;
    hipLaunchKernelGGL(k_res_install, dim3(std::max<uint32_t>(1, std::min<uint32_t>(n_rec, 256))), dim3(256), 0,
                       stream, a, r->d_recs, n_rec, (unsigned long long)r->units_tail);
    RPQ_LAUNCH_CHECK();
    // 4. one bounded launch, then the control block and the query outputs
    RPQ_BDISPATCH(x.K, x.seen_or, RPQ_TRY((launch_batch_kernel<KK, SS>(r->n_blocks, a, stream))));
    RPQ_LAUNCH_CHECK();
    RPQ_HIP(hipMemcpyAsync(r->h_ctl, r->ws + x.off_ctl, sizeof(BCtl), hipMemcpyDeviceToHost, stream));
    RPQ_HIP(hipMemcpyAsync(r->h_out, r->ws + x.off_qout, sizeof(BQueryOut) * r->q_hi, hipMemcpyDeviceToHost, stream));
    RPQ_HIP(hipStreamSynchronize(stream));
    if (r->h_ctl->gs.abort || r->h_ctl->err) {
        r->broken = true;
        rpq::set_error(r->h_ctl->gs.abort ? "resident kernel aborted at a grid barrier"
                                          : "internal capacity exceeded in the resident kernel (flags 0x%llx)",
                       (unsigned long long)r->h_ctl->err);
        res_fail_all(r, RPQ_EDEVICE, done);
        return RPQ_EDEVICE;
    }
    // 5. queries whose every unit has retired
    for (uint32_t qi = 0; qi < r->q_hi; ++qi) {
        Resident::Entry& e = r->table[qi];
        if (!e.used) continue;
        const BQueryOut& o = r->h_out[qi];
        if (o.units_done < e.n_units) continue;
        ResidentDone d{};
        d.token = e.token;
        d.count = o.count;
        d.hash = o.hash;
        d.product_edges = o.eprod;
        d.levels = o.levels;
        d.max_depth = o.max_depth;
        d.status = RPQ_OK;
        if (e.pairs) {
            d.written = std::min<uint64_t>(o.count, e.capacity);
            if (o.count > e.capacity) d.status = RPQ_EOVERFLOW;
        }
        done->push_back(d);
        e.used = false;
        r->free_q.push_back(qi);
        --r->n_active;
    }
    while (r->q_hi > 0 && !r->table[r->q_hi - 1].used) --r->q_hi;
    return RPQ_OK;
}

}  // namespace

int resident_step(Resident* r, uint32_t max_iters, hipStream_t stream, std::vector<ResidentDone>* done) {
    if (r->broken) {
        res_fail_all(r, RPQ_EDEVICE, done);
        rpq::set_error("resident engine is out of service after a device error");
        return RPQ_EDEVICE;
    }
    const int rc = step_body(r, max_iters, stream, done);
    if (rc != RPQ_OK && !r->broken) {
        // a failed HIP call leaves the device state unknown: nothing staged or in flight can finish
        (void)hipStreamSynchronize(stream);
        r->broken = true;
        res_fail_all(r, rc, done);
    }
    return rc;
}

}  // namespace rpq
