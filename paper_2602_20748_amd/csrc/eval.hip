// Plain RPQ evaluation: multi-source, level-synchronous search of the product
// of the graph and an epsilon-free NFA, to the fixpoint.
//
// Semantics (Definition 1 with the automata-based evaluation of Section 2.2):
// from each source s the search reaches product vertices (v, q); reaching a
// final q at v puts (s, v) in the result.  A visited set of (vertex, state)
// pairs per source keeps every product vertex expanded once per source.
//
// Bit-parallel layout.  Sources are taken W = 64*K at a time (a "unit", the
// counterpart of the paper's start-vertex batch, Section 4.1).  For a unit,
// every product vertex (q, v) owns a row of K 64-bit words; bit i of word k
// stands for source 64*k + i.  Per unit:
//   Vis [Q][V][K]  bits already reached (the per-source visited sets)
//   Next[Q][V][K]  bits reached in the level being expanded
//   Touch[Q][V]    1 while (q, v) already sits on the next frontier list
//   Ans [V][K]     bits of result pairs (s_i, v)
// G units advance together; their rows are tagged by a slot id.
//
// One level = three kernels:
//   expand    every frontier entry (q, v) owns a flattened item space: its edges over the
//             labels q can follow, each counted once per successor state.  For each item
//             (edge v -l-> w, successor q') it ORs the entry's frontier bits that are new for
//             (q', w) into Next; the first writer of a row sets its touch bit.  Entries with
//             at most H items are expanded straight from the frontier list; larger ones
//             arrive as slices of at most H items (edge-balanced work whatever the degree
//             skew, with slice memory bounded by 2 * items / H).
//   compact   the touched rows become the next frontier list (ballot/popcount prefix).
//   finalize  for each new entry moves Next into a compact frontier row, ORs it into Vis
//             (and into Ans when q' is final), counts the product edges it will examine,
//             and cuts entries of more than H items into slices.
// The fixpoint is reached when a level appends nothing; the host checks the
// list counter every few levels (no hop bound).
//
// Extraction walks Ans: per source its count and checksum, and optionally the
// result keys (s << 32) | v written source-major with ascending v, so the
// output is sorted and distinct by construction.
#include "internal.h"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// counters[] slots (uint64)
constexpr int C_LIST = 0;       // [0..1] list length per parity
constexpr int C_DESC = 2;       // [2..3] slice count per parity
constexpr int C_EPROD = 4;      // product edges examined
constexpr int C_ERR = 6;        // capacity / validation error flags
constexpr int C_PAIRBASE = 7;   // global key index where the current group starts
constexpr int C_COUNT = 8;
constexpr int C_HASH = 9;
constexpr int C_ITEMS = 10;     // expansion work tallies (profiling)
constexpr int C_DESCS = 11;
constexpr int C_ROWW = 12;
constexpr int C_WREAD = 13;
constexpr int C_WUPD = 14;
constexpr int C_LASTLEVEL = 15; // 1 + highest level index whose finalize appended rows (this group)
constexpr int C_FROWS = 16;     // finalize tallies (profiling): rows finalized,
constexpr int C_FWORDS = 17;    //   their non-zero Next words,
constexpr int C_FANS = 18;      //   and those of rows of final states
constexpr int C_NCOUNTERS = 19;

constexpr uint64_t ERR_LIST = 1, ERR_DESC = 2, ERR_SOURCES = 4;

// A slice [beg, beg + len) of the item space of frontier entry `entry` (an entry with more than
// H items is cut into such slices of at most H items).
struct Desc {
    uint32_t entry, len;
    uint64_t beg;
};

struct DevNfa {
    uint32_t Q, L, init, final;
    uint64_t qlab[RPQ_MAX_STATES];                   // labels with a transition out of q
    uint32_t delta[RPQ_MAX_STATES * RPQ_MAX_LABELS]; // compact [q * L + l]
};

struct Args {
    const uint32_t* row_ptr;
    const uint32_t* dst;
    const uint64_t* lmask;
    const DevNfa* nfa;
    uint64_t* vis;          // visited bits (with seen_or: also those found at the current level)
    uint64_t* next;         // two reads: bits found at this level; seen_or: Vis as of the last finalize
    uint64_t* touch;        // one bit per (slot, q, v) row: row has bits new at this level
    uint64_t* ans;
    uint64_t* rows0;
    uint64_t* rows1;
    uint32_t* ids0;         // row ids of the frontier lists (row = (slot * Q + q) * V + v)
    uint32_t* ids1;
    Desc* desc0;
    Desc* desc1;
    unsigned long long* counters;
    const uint64_t* target;   // optional [V / 64] bitmap: only result vertices with their bit set count
    uint32_t V, L, Q, H;
    uint32_t seen_or;         // visit scheme: 0 = two reads, 1 = seen OR (see the expansion)
    uint64_t list_cap, desc_cap;
};

__device__ __forceinline__ uint64_t* rows_of(const Args& a, int p) { return p ? a.rows1 : a.rows0; }
__device__ __forceinline__ uint32_t* ids_of(const Args& a, int p) { return p ? a.ids1 : a.ids0; }
__device__ __forceinline__ Desc* desc_of(const Args& a, int p) { return p ? a.desc1 : a.desc0; }

// relaxed device-scope OR whose result is unused (no-return atomic)
__device__ __forceinline__ void or_relaxed(uint64_t* p, uint64_t v) {
    (void)__hip_atomic_fetch_or(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void load_nfa(const Args& a, uint32_t* s_delta, uint64_t* s_qlab, uint32_t* s_final) {
    const uint32_t QL = a.Q * a.L;
    for (uint32_t i = threadIdx.x; i < QL; i += kBlock) s_delta[i] = a.nfa->delta[i];
    if (s_qlab)
        for (uint32_t i = threadIdx.x; i < a.Q; i += kBlock) s_qlab[i] = a.nfa->qlab[i];
    if (s_final && threadIdx.x == 0) *s_final = a.nfa->final;
    __syncthreads();
}

// ------------------------------------------------------------------------------------------------
// level expansion.  Work comes as segments (entry, first item, item count): first every light
// entry of the frontier list whole, then the slices of the heavy ones.  Per batch of
// segments (one per lane) the work is mapped twice per 64 items:
//   item phase  lane i takes item i: finds its segment (prefix of the wave's segment lengths),
//               decodes the edge target w and successor q', and forms the target row id;
//   word phase  the wave splits into 64/K groups of K lanes; group g takes items g, g + 64/K, ...
//               and lane k of the group handles word k of the rows, so the frontier row, the
//               visited row and the Next row of an item are each read or updated as one
//               contiguous K-word access instead of K scattered ones.
// kUnroll items per group are loaded before any of them is updated (memory-level parallelism).
//
// New bits of a target word (Section 4, the visited check before the atomic update) are found in
// one of two ways, both giving the same frontier:
//   two reads  the visited word and the Next word are read; bits in neither are ORed into Next,
//              and finalize ORs each level's Next into the visited bitmap and clears Next;
//   seen OR    only the visited word is read; bits not in it are ORed into it alone.  The visited
//              bitmap then also holds the bits found so far at this level, so it filters as well as
//              the two reads together.  The second bitmap holds the visited bits as of the last
//              finalize, and finalize takes a listed row's new bits as Vis & ~that, then advances
//              it.  One read and one OR per new word, the method's own accesses; finalize reads one
//              more word per row word, and the second bitmap is cleared with Vis for every group.
//              Faster at both scales measured: R-MAT 23, 3.41 -> 2.91 s a step (expansion 2.11 ms
//              a launch when each new word was also ORed into a Next bitmap, 1.53 ms now); R-MAT
//              18, 603 -> 541 ms (expansion 1.43 -> 1.15 ms).
// ------------------------------------------------------------------------------------------------
constexpr int kUnroll = 8;

// An empty asm that takes each value as an operand.  Without it the compiler moves the arithmetic
// that consumes a conditionally loaded value into the load's own conditional block, where it must
// wait for that load: the kUnroll loads would then complete one at a time instead of together.
template <int N>
__device__ __forceinline__ void keep_in_flight(uint64_t (&x)[N]) {
#pragma unroll
    for (int u = 0; u < N; ++u) asm volatile("" : "+v"(x[u]));
}

template <int K, bool SEEN>
__device__ __forceinline__ void expand_segments(const Args& a, const uint32_t* s_delta, const uint64_t* rows,
                                                bool have, uint32_t ent, uint32_t slot, uint32_t q, uint32_t v,
                                                uint64_t m, uint64_t beg, uint32_t len, uint64_t& t_items,
                                                uint64_t& t_wread, uint64_t& t_wupd) {
    constexpr int GS = 64 / K;
    const int lane = threadIdx.x & 63;
    const int grp = lane / K, k = lane % K;
    const uint64_t gmask = (K == 64) ? ~0ull : (((1ull << K) - 1) << (grp * K));
    const uint32_t Q = a.Q, V = a.V;
    if (!have) len = 0;
    const uint32_t incl = rpqd::wave_incl_scan_u32(len);
    const uint32_t excl = incl - len;
    const uint32_t total = __shfl(incl, 63, 64);
    if (lane == 0) t_items += total;
    for (uint32_t base = 0; base < total; base += 64) {
        // item phase
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
        const uint32_t c_ex = __shfl(excl, c, 64);
        uint32_t my_row = 0;
        if (item < total) {
            uint32_t w = 0, q2 = 0;
            rpqd::decode_item(a.row_ptr, a.dst, a.L, s_delta, c_v, c_q, c_m, c_beg + (item - c_ex), &w, &q2);
            my_row = (c_slot * Q + q2) * V + w;
        }
        const uint32_t n_here = min(64u, total - base);
        // word phase
        for (uint32_t j = 0; j < n_here; j += GS * kUnroll) {
            uint32_t r[kUnroll];
            uint64_t f[kUnroll], nb[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t idx = j + u * GS + grp;
                r[u] = __shfl(my_row, idx & 63, 64);
                const uint32_t e = __shfl(c_ent, idx & 63, 64);
                f[u] = idx < n_here ? rows[(uint64_t)e * K + k] : 0;
            }
            if constexpr (SEEN) {
                // the visited word holds every bit of earlier levels (their ORs completed before
                // this launch): bits not in it as read are new at this level
                uint64_t sw[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) sw[u] = f[u] ? a.vis[(uint64_t)r[u] * K + k] : ~0ull;
                keep_in_flight<kUnroll>(sw);
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    nb[u] = f[u] & ~sw[u];
                    if (nb[u]) {
                        or_relaxed(&a.vis[(uint64_t)r[u] * K + k], nb[u]);
                    }
                }
            } else {
                // the visited word and the Next word together: bits already in Next need no OR, and
                // the OR then finds its line in L2 (Next only gains bits during an expansion, so a
                // stale copy can only let through an OR that is not needed)
                uint64_t vw[kUnroll], nx[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    vw[u] = f[u] ? a.vis[(uint64_t)r[u] * K + k] : ~0ull;
                    nx[u] = f[u] ? a.next[(uint64_t)r[u] * K + k] : ~0ull;
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    nb[u] = f[u] & ~vw[u] & ~nx[u];
                    if (nb[u]) or_relaxed(&a.next[(uint64_t)r[u] * K + k], nb[u]);
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
__global__ __launch_bounds__(kBlock) void k_expand(Args a, int p) {
    __shared__ uint32_t s_delta[RPQ_MAX_STATES * RPQ_MAX_LABELS];
    __shared__ uint64_t s_qlab[RPQ_MAX_STATES];
    load_nfa(a, s_delta, s_qlab, nullptr);
    const uint64_t n_list = min((uint64_t)a.counters[C_LIST + p], a.list_cap);
    const uint64_t n_desc = min((uint64_t)a.counters[C_DESC + p], a.desc_cap);
    if (n_list == 0) return;
    const int lane = threadIdx.x & 63;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWaves;
    const uint64_t wave = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    const uint64_t* rows = rows_of(a, p);
    const uint32_t* ids = ids_of(a, p);
    const uint32_t QV = a.Q * a.V, V = a.V, H = a.H;
    uint64_t t_items = 0, t_segs = 0, t_wread = 0, t_wupd = 0;
    // light entries, straight from the frontier list
    const uint64_t n_lb = (n_list + 63) / 64;
    for (uint64_t b = wave; b < n_lb; b += n_waves) {
        const uint64_t e = b * 64 + lane;
        bool have = false;
        uint32_t slot = 0, q = 0, v = 0, len = 0;
        uint64_t m = 0;
        if (e < n_list) {
            const uint32_t row = ids[e];
            slot = row / QV;
            const uint32_t rem = row - slot * QV;
            q = rem / V;
            v = rem - q * V;
            m = a.lmask[v] & s_qlab[q];
            const uint64_t work = m ? rpqd::entry_work(a.row_ptr, a.L, s_delta, v, q, m) : 0;
            have = work != 0 && work <= H;
            len = have ? (uint32_t)work : 0;
        }
        t_segs += __popcll(__ballot(have)) * (lane == 0);
        expand_segments<K, SEEN>(a, s_delta, rows, have, (uint32_t)e, slot, q, v, m, 0, len, t_items, t_wread, t_wupd);
    }
    // heavy entries, as slices
    const Desc* desc = desc_of(a, p);
    const uint64_t n_db = (n_desc + 63) / 64;
    for (uint64_t b = wave; b < n_db; b += n_waves) {
        const uint64_t di = b * 64 + lane;
        bool have = false;
        uint32_t ent = 0, slot = 0, q = 0, v = 0, len = 0;
        uint64_t m = 0, beg = 0;
        if (di < n_desc) {
            const Desc d = desc[di];
            ent = d.entry;
            beg = d.beg;
            len = d.len;
            const uint32_t row = ids[ent];
            slot = row / QV;
            const uint32_t rem = row - slot * QV;
            q = rem / V;
            v = rem - q * V;
            m = a.lmask[v] & s_qlab[q];
            have = true;
        }
        t_segs += __popcll(__ballot(have)) * (lane == 0);
        expand_segments<K, SEEN>(a, s_delta, rows, have, ent, slot, q, v, m, beg, len, t_items, t_wread, t_wupd);
    }
    t_items = rpqd::wave_sum_u64(t_items);
    t_segs = rpqd::wave_sum_u64(t_segs);
    t_wread = rpqd::wave_sum_u64(t_wread);
    t_wupd = rpqd::wave_sum_u64(t_wupd);
    if (lane == 0 && t_items) {
        atomicAdd(&a.counters[C_ITEMS], (unsigned long long)t_items);
        atomicAdd(&a.counters[C_DESCS], (unsigned long long)t_segs);
        atomicAdd(&a.counters[C_ROWW], (unsigned long long)(t_segs * K));
        atomicAdd(&a.counters[C_WREAD], (unsigned long long)t_wread);
        atomicAdd(&a.counters[C_WUPD], (unsigned long long)t_wupd);
    }
}

// ------------------------------------------------------------------------------------------------
// compaction: the rows touched by the last expansion (or by seeding) become the dense list of
// row ids of the next frontier.  Each wave reads 64 consecutive touch words (one per lane),
// clears them, and places its rows with one counter update (popcount prefix over the wave).
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_compact(Args a, int p, uint64_t n_rows, uint32_t level) {
    const int np = p ^ 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the list and slices of parity p were consumed by the expansion that just ran
        a.counters[C_LIST + p] = 0;
        a.counters[C_DESC + p] = 0;
    }
    const int lane = threadIdx.x & 63;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWaves;
    const uint64_t wave = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    const uint64_t n_words = (n_rows + 63) / 64;
    unsigned long long* lcnt = &a.counters[C_LIST + np];
    uint32_t* ids = ids_of(a, np);
    bool appended = false;
    for (uint64_t w0 = wave * 64; w0 < n_words; w0 += n_waves * 64) {
        const uint64_t wi = w0 + lane;
        uint64_t tw = wi < n_words ? a.touch[wi] : 0;
        if (tw) a.touch[wi] = 0;
        const uint32_t c = (uint32_t)__popcll(tw);
        const uint32_t incl = rpqd::wave_incl_scan_u32(c);
        const uint32_t tot = __shfl(incl, 63, 64);
        if (tot == 0) continue;
        appended = true;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(lcnt, (unsigned long long)tot);
        base = __shfl(base, 0, 64);
        uint64_t pos = base + incl - c;
        while (tw) {
            const int b = __ffsll((long long)tw) - 1;
            tw &= tw - 1;
            if (pos < a.list_cap) ids[pos] = (uint32_t)(wi * 64 + b);
            else atomicOr(&a.counters[C_ERR], (unsigned long long)ERR_LIST);
            ++pos;
        }
    }
    if (lane == 0 && appended) atomicMax(&a.counters[C_LASTLEVEL], (unsigned long long)level + 1);
}

// ------------------------------------------------------------------------------------------------
// finalize.  Per batch of 64 new frontier rows:
//   word phase  groups of K lanes take a row each (lane k, word k): Next moves into the compact
//               frontier row, Vis and (for final states) Ans take the new bits, and the group
//               counts the new source bits of the row;
//   row phase   lane i takes row i: counts the items of its item space (the product edges each of
//               its new source bits will examine); the slices of rows with more than H items are
//               written by the whole wave.  With count_work == 0 (the last depth of a
//               length-bounded search) the rows are recorded but not prepared for expansion.
// ------------------------------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(kBlock) void k_finalize(Args a, int p, int count_work) {
    constexpr int GS = 64 / K;
    __shared__ uint32_t s_delta[RPQ_MAX_STATES * RPQ_MAX_LABELS];
    __shared__ uint64_t s_qlab[RPQ_MAX_STATES];
    __shared__ uint32_t s_final;
    load_nfa(a, s_delta, s_qlab, &s_final);
    const int np = p ^ 1;
    const uint64_t n = min((uint64_t)a.counters[C_LIST + np], a.list_cap);
    if (n == 0) return;
    const int lane = threadIdx.x & 63;
    const int grp = lane / K, k = lane % K;
    const uint32_t* ids = ids_of(a, np);
    uint64_t* rows = rows_of(a, np);
    Desc* dout = desc_of(a, np);
    unsigned long long* dcnt = &a.counters[C_DESC + np];
    const uint32_t H = a.H, V = a.V;
    const uint32_t QV = a.Q * a.V;
    const uint32_t fin = s_final;
    uint64_t eprod = 0, t_rows = 0, t_words = 0, t_ans = 0;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWaves;
    const uint64_t wave = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    for (uint64_t e0 = wave * 64; e0 < n; e0 += n_waves * 64) {
        const uint64_t e = e0 + lane;
        const bool active = e < n;
        const uint32_t my_row = active ? ids[e] : 0;
        const uint32_t slot = my_row / QV;
        const uint32_t rem = my_row - slot * QV;
        const uint32_t q = rem / V;
        const uint32_t v = rem - q * V;
        // Ans row of a final-state entry, else none
        const uint32_t my_ans = ((fin >> q) & 1) ? slot * V + v : 0xFFFFFFFFu;
        const uint32_t n_here = (uint32_t)min<uint64_t>(64, n - e0);
        t_rows += n_here * (lane == 0);
        uint32_t my_pc = 0;
        // word phase
        for (uint32_t j = 0; j < n_here; j += GS * kUnroll) {
            uint32_t r[kUnroll], an[kUnroll];
            uint64_t nk[kUnroll], ov[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t idx = j + u * GS + grp;
                r[u] = __shfl(my_row, idx & 63, 64);
                an[u] = __shfl(my_ans, idx & 63, 64);
                nk[u] = ov[u] = 0;
                if (idx < n_here) {
                    if (a.seen_or) {
                        ov[u] = a.next[(uint64_t)r[u] * K + k];
                        nk[u] = a.vis[(uint64_t)r[u] * K + k];
                    } else {
                        nk[u] = a.next[(uint64_t)r[u] * K + k];
                    }
                }
            }
            if (a.seen_or) {
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) nk[u] &= ~ov[u];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t idx = j + u * GS + grp;
                uint32_t pc = 0;
                if (idx < n_here) {
                    rows[(e0 + idx) * K + k] = nk[u];
                    if (nk[u]) {
                        // seen OR: the snapshot catches up with Vis.  Two reads: Next is cleared.
                        a.next[(uint64_t)r[u] * K + k] = a.seen_or ? (ov[u] | nk[u]) : 0;
                        // a row is on the list once, and nothing else writes its Vis word in this
                        // kernel: a plain read-modify-write (an atomic OR cost 0.82 vs 0.69 ms a
                        // launch).  With seen OR the expansion has already set these bits.
                        if (!a.seen_or) a.vis[(uint64_t)r[u] * K + k] |= nk[u];
                        ++t_words;
                        if (an[u] != 0xFFFFFFFFu) {
                            or_relaxed(&a.ans[(uint64_t)an[u] * K + k], nk[u]);
                            ++t_ans;
                        }
                        pc = (uint32_t)__popcll(nk[u]);
                    }
                }
#pragma unroll
                for (int o = K / 2; o >= 1; o >>= 1) pc += __shfl_xor(pc, o, 64);
                // lane i keeps the count of row i
                const uint32_t rel = (uint32_t)lane - (j + u * GS);
                const uint32_t got = __shfl(pc, (rel % GS) * K, 64);
                if (rel < (uint32_t)GS) my_pc = got;
            }
        }
        // row phase: product edges; entries of more than H items are cut into slices.  At the
        // depth bound of a length-bounded query the entries are recorded but never expanded: no
        // product edges, no slices.
        uint64_t work = 0;
        if (active && count_work) {
            const uint64_t m = a.lmask[v] & s_qlab[q];
            work = m ? rpqd::entry_work(a.row_ptr, a.L, s_delta, v, q, m) : 0;
            eprod += (uint64_t)my_pc * work;
        }
        const uint64_t ndesc = work > H ? (work + H - 1) / H : 0;
        const uint64_t dincl = rpqd::wave_incl_scan_u64(ndesc);
        const uint64_t dexcl = dincl - ndesc;
        const uint64_t dtot = __shfl(dincl, 63, 64);
        if (dtot) {
            unsigned long long dbase = 0;
            if (lane == 0) dbase = atomicAdd(dcnt, (unsigned long long)dtot);
            dbase = __shfl(dbase, 0, 64);
            // the wave writes its slices together: slice i is described by the lane owning it
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
                        const uint64_t k = i - c_ex;
                        Desc dd;
                        dd.entry = (uint32_t)(e0 + c);
                        dd.beg = k * H;
                        dd.len = (uint32_t)min<uint64_t>(H, c_work - k * H);
                        dout[pos] = dd;
                    } else {
                        atomicOr(&a.counters[C_ERR], (unsigned long long)ERR_DESC);
                    }
                }
            }
        }
    }
    eprod = rpqd::wave_sum_u64(eprod);
    t_words = rpqd::wave_sum_u64(t_words);
    t_ans = rpqd::wave_sum_u64(t_ans);
    if (lane == 0 && eprod) atomicAdd(&a.counters[C_EPROD], (unsigned long long)eprod);
    if (lane == 0 && t_rows) {
        atomicAdd(&a.counters[C_FROWS], (unsigned long long)t_rows);
        atomicAdd(&a.counters[C_FWORDS], (unsigned long long)t_words);
        atomicAdd(&a.counters[C_FANS], (unsigned long long)t_ans);
    }
}

// ------------------------------------------------------------------------------------------------
// seeding: (q0, s_i) for every initial state q0 and every source of the group
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_seed(Args a, const uint32_t* __restrict__ sources,
                                                 uint64_t n_sources, uint64_t group_base, uint32_t G,
                                                 uint32_t W, uint32_t K) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (uint64_t)G * W) return;
    const uint64_t gi = group_base + i;
    if (gi >= n_sources) return;
    const uint32_t slot = (uint32_t)(i / W), j = (uint32_t)(i % W);
    const uint32_t s = sources ? sources[gi] : (uint32_t)gi;
    const uint32_t k = j >> 6;
    const uint64_t bit = 1ull << (j & 63);
    uint32_t init = a.nfa->init;
    while (init) {
        const uint32_t q = __ffs(init) - 1;
        init &= init - 1;
        const uint64_t row = ((uint64_t)slot * a.Q + q) * a.V + s;
        if (a.seen_or)
            or_relaxed(&a.vis[row * K + k], bit);
        else
            or_relaxed(&a.next[row * K + k], bit);
        or_relaxed(&a.touch[row >> 6], 1ull << (row & 63));
    }
}

__global__ void k_check_sources(const uint32_t* __restrict__ s, uint64_t n, uint32_t V,
                                unsigned long long* __restrict__ counters) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t x = s[i];
        if (x >= V || (i > 0 && s[i - 1] >= x)) atomicOr(&counters[C_ERR], (unsigned long long)ERR_SOURCES);
    }
}

// ------------------------------------------------------------------------------------------------
// extraction
// ------------------------------------------------------------------------------------------------
// Answer words each lane loads per 64-vertex group: four adjacent words (two 16-byte loads) where K
// allows.  Neighbouring lanes read rows one row (K words) apart, so every lane makes its own memory
// request; loading four words per request instead of one cuts the requests per byte fourfold,
// which is what bounds this kernel when most answer words are zero.
template <int K>
constexpr int kExtractWords() { return K >= 4 ? 4 : (K >= 2 ? 2 : 1); }

// One wave per (slot, block of kExtractWords consecutive words, vertex chunk); for word k of the
// block, lane i owns source 64k + i of the slot and walks the non-zero vertex words in ascending
// vertex order.
template <int K, bool WRITE>
__global__ __launch_bounds__(kBlock) void k_extract(Args a, const uint32_t* __restrict__ sources,
                                                    uint64_t n_sources, uint64_t group_base, uint32_t G,
                                                    uint32_t W, uint32_t nchunks, uint32_t chunk_v,
                                                    unsigned long long* __restrict__ acc,
                                                    uint32_t* __restrict__ partial,
                                                    const uint64_t* __restrict__ srcbase,
                                                    uint64_t* __restrict__ pairs, uint64_t pair_off,
                                                    uint64_t capacity) {
    constexpr int KP = kExtractWords<K>();
    constexpr int NKP = K / KP;
    const int lane = threadIdx.x & 63;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWaves;
    const uint64_t total = (uint64_t)G * NKP * nchunks;
    const uint32_t V = a.V;
    for (uint64_t wv = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); wv < total; wv += n_waves) {
        const uint32_t chunk = (uint32_t)(wv % nchunks);
        const uint32_t kp = (uint32_t)((wv / nchunks) % NKP);
        const uint32_t slot = (uint32_t)(wv / ((uint64_t)nchunks * NKP));
        const uint32_t vbeg = chunk * chunk_v;
        const uint32_t vend = min(V, vbeg + chunk_v);
        bool valid[KP];
        uint64_t skey[KP], cnt[KP], h[KP], cursor[KP];
        bool in_window = !WRITE;
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            const uint64_t si = (uint64_t)slot * W + (uint64_t)(kp * KP + u) * 64 + lane;
            const uint64_t gi = group_base + si;
            valid[u] = gi < n_sources;
            skey[u] = (valid[u] ? (sources ? (uint64_t)sources[gi] : gi) : 0) << 32;
            cnt[u] = h[u] = cursor[u] = 0;
            if (WRITE && valid[u]) {
                // this source's keys in this vertex chunk are [cursor, end): partial holds the
                // source's chunk prefixes, acc its total
                const uint32_t* pp = partial + si * nchunks;
                cursor[u] = srcbase[si] + pp[chunk];
                const uint64_t end = srcbase[si] + (chunk + 1 < nchunks ? (uint64_t)pp[chunk + 1] : acc[2 * si]);
                in_window |= end > pair_off && cursor[u] < pair_off + capacity;
            }
        }
        // a wave none of whose keys fall in the output window has nothing to write
        if (WRITE && __ballot(in_window) == 0) continue;
        for (uint32_t v0 = vbeg; v0 < vend; v0 += 64) {
            const uint32_t vv = v0 + lane;
            uint64_t word[KP];
            if (vv < vend) {
                const uint64_t* p = a.ans + ((uint64_t)slot * V + vv) * K + (uint64_t)kp * KP;
                if constexpr (KP >= 2) {
#pragma unroll
                    for (int u = 0; u < KP; u += 2) {
                        const ulonglong2 w2 = *reinterpret_cast<const ulonglong2*>(p + u);
                        word[u] = w2.x;
                        word[u + 1] = w2.y;
                    }
                } else {
                    word[0] = p[0];
                }
            } else {
#pragma unroll
                for (int u = 0; u < KP; ++u) word[u] = 0;
            }
            if (a.target && vv < vend && !((a.target[vv >> 6] >> (vv & 63)) & 1)) {
#pragma unroll
                for (int u = 0; u < KP; ++u) word[u] = 0;
            }
#pragma unroll
            for (int u = 0; u < KP; ++u) {
                uint64_t any = __ballot(word[u] != 0);
                while (any) {
                    const int jj = __ffsll((long long)any) - 1;
                    any &= any - 1;
                    const uint64_t wj = __shfl(word[u], jj, 64);
                    if (valid[u] && ((wj >> lane) & 1)) {
                        const uint64_t key = skey[u] | (uint64_t)(v0 + jj);
                        if (WRITE) {
                            if (cursor[u] >= pair_off && cursor[u] - pair_off < capacity)
                                pairs[cursor[u] - pair_off] = key;
                            ++cursor[u];
                        } else {
                            ++cnt[u];
                            h[u] += rpqd::mix64(key);
                        }
                    }
                }
            }
        }
        if (!WRITE) {
#pragma unroll
            for (int u = 0; u < KP; ++u) {
                if (!valid[u]) continue;
                const uint64_t si = (uint64_t)slot * W + (uint64_t)(kp * KP + u) * 64 + lane;
                if (partial) partial[si * nchunks + chunk] = (uint32_t)cnt[u];
                if (cnt[u]) {
                    atomicAdd(&acc[2 * si], (unsigned long long)cnt[u]);
                    atomicAdd(&acc[2 * si + 1], (unsigned long long)h[u]);
                }
            }
        }
    }
}

// One block: per-source results of the group, chunk prefixes, source offsets, totals.
__global__ __launch_bounds__(1024) void k_group_finish(unsigned long long* __restrict__ counters,
                                                       const unsigned long long* __restrict__ acc,
                                                       uint32_t* __restrict__ partial, uint64_t* __restrict__ srcbase,
                                                       uint64_t* __restrict__ per_source, uint64_t n_sources,
                                                       uint64_t group_base, uint64_t n_group, uint32_t nchunks) {
    __shared__ uint64_t s_w[16];
    __shared__ uint64_t s_carry;
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    if (t == 0) s_carry = counters[C_PAIRBASE];
    uint64_t csum = 0, hsum = 0;
    __syncthreads();
    for (uint64_t b0 = 0; b0 < n_group; b0 += 1024) {
        const uint64_t i = b0 + t;
        const bool valid = i < n_group && group_base + i < n_sources;
        const uint64_t c = valid ? acc[2 * i] : 0;
        const uint64_t h = valid ? acc[2 * i + 1] : 0;
        csum += c;
        hsum += h;
        if (valid && per_source) {
            per_source[2 * (group_base + i)] = c;
            per_source[2 * (group_base + i) + 1] = h;
        }
        if (srcbase) {
            if (valid) {
                uint32_t run = 0;
                uint32_t* pp = partial + i * nchunks;
                for (uint32_t ch = 0; ch < nchunks; ++ch) {
                    const uint32_t x = pp[ch];
                    pp[ch] = run;
                    run += x;
                }
            }
            const uint64_t incl = rpqd::wave_incl_scan_u64(c);
            if (lane == 63) s_w[wv] = incl;
            __syncthreads();
            uint64_t pre = s_carry;
            for (int w = 0; w < wv; ++w) pre += s_w[w];
            if (valid) srcbase[i] = pre + incl - c;
            __syncthreads();
            if (t == 0) {
                uint64_t tot = 0;
                for (int w = 0; w < 16; ++w) tot += s_w[w];
                s_carry += tot;
            }
            __syncthreads();
        }
    }
    csum = rpqd::wave_sum_u64(csum);
    hsum = rpqd::wave_sum_u64(hsum);
    if (lane == 0) {
        atomicAdd(&counters[C_COUNT], (unsigned long long)csum);
        atomicAdd(&counters[C_HASH], (unsigned long long)hsum);
    }
    if (srcbase && t == 0) counters[C_PAIRBASE] = s_carry;
}

// ------------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------------
struct Layout {
    uint32_t K, W, G, Q, L, V, H, nchunks, chunk_v, sync_every;
    uint32_t seen_or;   // visit scheme of the expansion (1 = seen OR, 0 = two reads)
    uint64_t max_len;   // deepest level finalized: the length bound, or no bound (UINT64_MAX)
    uint64_t list_cap, desc_cap;
    uint64_t off_counters, off_nfa, off_vis, off_next, off_touch, off_ans, off_ans2, off_ids[2], off_rows[2],
        off_desc[2], off_acc, off_partial, off_srcbase, total;
};

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

int popc64(uint64_t x) { return __builtin_popcountll(x); }

int validate_nfa(const rpq_graph* g, const rpq_nfa* nfa) {
    if (!nfa) {
        rpq::set_error("automaton is NULL");
        return RPQ_EINVAL;
    }
    if (nfa->n_states == 0 || nfa->n_states > RPQ_MAX_STATES) {
        rpq::set_error("automaton has %u states; 1..%d supported", nfa->n_states, RPQ_MAX_STATES);
        return nfa->n_states == 0 ? RPQ_EINVAL : RPQ_EUNSUPPORTED;
    }
    if (nfa->n_labels == 0 || nfa->n_labels > g->L) {
        rpq::set_error("automaton has %u labels; the graph has %u", nfa->n_labels, g->L);
        return RPQ_EINVAL;
    }
    const uint32_t smask = nfa->n_states == 32 ? 0xFFFFFFFFu : ((1u << nfa->n_states) - 1);
    if ((nfa->initial_mask & ~smask) || (nfa->final_mask & ~smask)) {
        rpq::set_error("initial/final mask names states >= n_states");
        return RPQ_EINVAL;
    }
    for (uint32_t q = 0; q < RPQ_MAX_STATES; ++q)
        for (uint32_t l = 0; l < RPQ_MAX_LABELS; ++l) {
            const uint32_t d = nfa->delta[q * RPQ_MAX_LABELS + l];
            if (!d) continue;
            if (q >= nfa->n_states || l >= nfa->n_labels || (d & ~smask)) {
                rpq::set_error("delta[%u][%u] is outside the automaton", q, l);
                return RPQ_EINVAL;
            }
        }
    return RPQ_OK;
}

void to_dev_nfa(const rpq_nfa* nfa, uint32_t L, DevNfa* d) {
    std::memset(d, 0, sizeof *d);
    d->Q = nfa->n_states;
    d->L = L;
    d->init = nfa->initial_mask;
    d->final = nfa->final_mask;
    for (uint32_t q = 0; q < nfa->n_states; ++q)
        for (uint32_t l = 0; l < L; ++l) {
            const uint32_t m = l < nfa->n_labels ? nfa->delta[q * RPQ_MAX_LABELS + l] : 0;
            d->delta[q * L + l] = m;
            if (m) d->qlab[q] |= 1ull << l;
        }
}

// Default shape: about 64K sources in flight, in units of up to 2048 sources below 2^22
// vertices and 4096 from there (measured: R-MAT scale 18 all-pairs, where throughput rises with
// the sources advanced per level up to ~64K and 2048-wide units beat 1024 and 4096; R-MAT
// scale 23 from 65,536 sources, where 4096-wide units beat 2048 by 5% and 1024 lost 6%), entries
// of more than 16 items cut into slices (16 beat 32, 64, 128 and 256; raised on graphs where the
// slice buffers would outgrow a quarter of the bitmaps).  Units in flight are sized for 64 GB of
// the 288 GB device, and a unit of the default width may take up to 96 GB alone (at scale 23 one
// 4096-wide unit per group, 3.45 s per step, beat two per group within 96 GB, 3.57 s).
constexpr uint64_t kTargetInFlight = 65536;
constexpr uint64_t kWorkspaceBudget = 64ull << 30;
constexpr uint64_t kUnitBudget = 96ull << 30;
constexpr uint32_t kDefaultChunk = 16;

uint32_t max_default_width(uint32_t V) { return V >= (1u << 22) ? 4096 : 2048; }

uint64_t unit_bytes(uint64_t QV, uint32_t W) {
    // Vis + Next + two frontier lists of rows + row ids
    return QV * (W / 8) * 4 + QV * 8;
}

uint32_t default_width(uint64_t n_sources, uint64_t QV, uint32_t V) {
    uint32_t W = 64;
    while (W < max_default_width(V) && (uint64_t)W * 2 <= std::max<uint64_t>(64, n_sources / 8)) W *= 2;
    while (W > 64 && unit_bytes(QV, W) > kUnitBudget) W /= 2;
    return W;
}

int make_layout(const rpq_graph* g, const DevNfa& dn, uint64_t n_sources, uint32_t flags,
                const rpq_eval_opts* o, bool single_ans, Layout* Lo) {
    Layout x;
    std::memset(&x, 0, sizeof x);
    x.Q = dn.Q;
    x.L = g->L;
    x.V = g->V;
    x.W = (o && o->batch_width) ? o->batch_width : default_width(n_sources, (uint64_t)dn.Q * g->V, g->V);
    if (x.W != 64 && x.W != 128 && x.W != 256 && x.W != 512 && x.W != 1024 && x.W != 2048 && x.W != 4096) {
        rpq::set_error("batch_width must be 64, 128, 256, 512, 1024, 2048 or 4096");
        return RPQ_EINVAL;
    }
    x.K = x.W / 64;
    x.H = (o && o->chunk_edges) ? o->chunk_edges : kDefaultChunk;
    // seen OR unless asked otherwise: the faster scheme on both R-MAT 18 and R-MAT 23 (the
    // expansion's comment has the figures)
    x.seen_or = (o && o->visit) ? o->visit == RPQ_VISIT_SEEN_OR : 1u;
    if (x.H > 65535) {
        rpq::set_error("chunk_edges must be <= 65535");
        return RPQ_EINVAL;
    }
    const bool auto_chunk = !(o && o->chunk_edges);
    x.sync_every = (o && o->sync_every) ? o->sync_every : 4;
    x.max_len = (flags & RPQ_LENGTH_BOUND) ? (uint64_t)o->max_length : ~0ull;
    const uint64_t units = std::max<uint64_t>(1, (n_sources + x.W - 1) / x.W);
    const uint64_t QV = (uint64_t)x.Q * x.V;
    const uint64_t bitmap_bytes = QV * x.K * 8;
    // slices of one level and unit: entries with work > H take ceil(work / H) <= 2 work / H
    // each, and the work of all entries of state q is at most E * max |delta(q, l)|
    uint64_t items = 0;
    for (uint32_t q = 0; q < x.Q; ++q) {
        uint32_t max_succ = 0;
        for (uint32_t l = 0; l < x.L; ++l) max_succ = std::max(max_succ, (uint32_t)__builtin_popcount(dn.delta[q * x.L + l]));
        items += (uint64_t)max_succ * g->E;   // the in-CSR holds the same distinct edges
    }
    // default slice size: the smallest (fastest) that keeps a unit's two slice buffers within a
    // quarter of its bitmaps
    while (auto_chunk && x.H < 256 && 2 * (2 * items / x.H + 2) * sizeof(Desc) > unit_bytes(QV, x.W) / 4) x.H *= 2;
    const uint64_t desc_per_unit = 2 * items / x.H + 2;
    uint64_t G = (o && o->concurrency) ? o->concurrency : 0;
    if (!G) {
        G = std::max<uint64_t>(1, kTargetInFlight / x.W);
        const uint64_t per_unit = unit_bytes(QV, x.W) + 2 * desc_per_unit * sizeof(Desc);
        G = std::min<uint64_t>(G, std::max<uint64_t>(1, kWorkspaceBudget / per_unit));
    }
    G = std::min<uint64_t>(G, units);
    x.G = (uint32_t)G;
    x.list_cap = G * QV;
    if (x.list_cap >= 0xFFFFFFFFull) {
        rpq::set_error("concurrency * states * vertices must stay below 2^32; lower concurrency");
        return RPQ_EUNSUPPORTED;
    }
    x.desc_cap = G * desc_per_unit;
    x.chunk_v = 4096;
    x.nchunks = (uint32_t)((x.V + x.chunk_v - 1) / x.chunk_v);
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o2 = off;
        off = align256(off + bytes);
        return o2;
    };
    x.off_counters = take(C_NCOUNTERS * 8);
    x.off_nfa = take(sizeof(DevNfa));
    x.off_vis = take(G * bitmap_bytes);
    x.off_next = take(G * bitmap_bytes);
    x.off_touch = take((G * QV + 63) / 64 * 8);
    x.off_ans = take(G * (uint64_t)x.V * x.K * 8);
    // a second Ans bitmap when there is more than one group: a group's extraction then runs on a
    // second stream while the next group's levels fill the other bitmap
    x.off_ans2 = units > G && !single_ans ? take(G * (uint64_t)x.V * x.K * 8) : x.off_ans;
    for (int p = 0; p < 2; ++p) {
        x.off_ids[p] = take(x.list_cap * 4);
        x.off_rows[p] = take(x.list_cap * x.K * 8);
        x.off_desc[p] = take(x.desc_cap * sizeof(Desc));
    }
    x.off_acc = take(G * x.W * 16);
    const bool want_pairs = (flags & RPQ_PAIRS) != 0;
    x.off_partial = take(want_pairs ? G * x.W * (uint64_t)x.nchunks * 4 : 0);
    x.off_srcbase = take(want_pairs ? G * x.W * 8 : 0);
    x.total = off;
    *Lo = x;
    return RPQ_OK;
}

Args make_args(const rpq_graph* g, uint32_t flags, const Layout& x, char* ws) {
    const rpq::Csr& csr = (flags & RPQ_REVERSE) ? g->in : g->out;
    Args a;
    a.row_ptr = csr.row_ptr;
    a.dst = csr.dst;
    a.lmask = csr.lmask;
    a.nfa = reinterpret_cast<const DevNfa*>(ws + x.off_nfa);
    a.vis = reinterpret_cast<uint64_t*>(ws + x.off_vis);
    a.next = reinterpret_cast<uint64_t*>(ws + x.off_next);
    a.touch = reinterpret_cast<uint64_t*>(ws + x.off_touch);
    a.ans = reinterpret_cast<uint64_t*>(ws + x.off_ans);
    a.ids0 = reinterpret_cast<uint32_t*>(ws + x.off_ids[0]);
    a.ids1 = reinterpret_cast<uint32_t*>(ws + x.off_ids[1]);
    a.rows0 = reinterpret_cast<uint64_t*>(ws + x.off_rows[0]);
    a.rows1 = reinterpret_cast<uint64_t*>(ws + x.off_rows[1]);
    a.desc0 = reinterpret_cast<Desc*>(ws + x.off_desc[0]);
    a.desc1 = reinterpret_cast<Desc*>(ws + x.off_desc[1]);
    a.counters = reinterpret_cast<unsigned long long*>(ws + x.off_counters);
    a.target = nullptr;
    a.V = x.V;
    a.L = x.L;
    a.Q = x.Q;
    a.H = x.H;
    a.seen_or = x.seen_or;
    a.list_cap = x.list_cap;
    a.desc_cap = x.desc_cap;
    return a;
}

// Grid of a level kernel: as many blocks as the device keeps resident at once (the kernels
// stride over their work, so a grid beyond residency would only add a tail round).
unsigned resident_grid(const void* kernel) {
    int dev = 0, n_cu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || n_cu <= 0 ||
        per_cu <= 0)
        return 2048;
    return (unsigned)(n_cu * per_cu);
}

template <int K>
struct LevelGrids {
    unsigned expand, expand_seen, compact, finalize;
    static const LevelGrids& get() {
        static const LevelGrids g{resident_grid(reinterpret_cast<const void*>(&k_expand<K, false>)),
                                  resident_grid(reinterpret_cast<const void*>(&k_expand<K, true>)),
                                  resident_grid(reinterpret_cast<const void*>(&k_compact)),
                                  resident_grid(reinterpret_cast<const void*>(&k_finalize<K>))};
        return g;
    }
};

// Process-wide profiling state: event pairs around level kernels, resolved at
// the host synchronisation points of rpq_eval.
struct Profiler {
    std::mutex mu;
    bool on = false;
    rpq_profile acc{};
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pend_expand, pend_finalize, pend_extract;

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // caller holds mu and has synchronised the stream(s) the events were recorded on; extraction
    // events (second stream) only when with_extract
    void resolve(bool with_extract = false) {
        if (with_extract) {
            for (auto& pr : pend_extract) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
                    acc.extract_ms += ms;
                    acc.extract_launches++;
                }
                pool.push_back(pr.first);
                pool.push_back(pr.second);
            }
            pend_extract.clear();
        }
        for (int which = 0; which < 2; ++which) {
            auto& v = which ? pend_finalize : pend_expand;
            for (auto& pr : v) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
                    if (which) {
                        acc.finalize_ms += ms;
                        acc.finalize_launches++;
                    } else {
                        acc.expand_ms += ms;
                        acc.expand_launches++;
                    }
                }
                // the expansion's end event is also the finalize's start event:
                // return each event to the pool exactly once
                if (which) {
                    pool.push_back(pr.first);
                    pool.push_back(pr.second);
                } else {
                    pool.push_back(pr.first);
                }
            }
            v.clear();
        }
    }
};

Profiler& profiler() {
    static Profiler* p = new Profiler();
    return *p;
}

template <int K>
int launch_level(const Args& a, int p, uint64_t n_rows, uint32_t level, int count_work, bool may_profile,
                 hipStream_t s) {
    Profiler& pr = profiler();
    const bool on = may_profile && pr.on;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    if (on) {
        std::lock_guard<std::mutex> lk(pr.mu);
        e0 = pr.get();
        e1 = pr.get();
        e2 = pr.get();
    }
    if (e0) RPQ_HIP(hipEventRecord(e0, s));
    if (a.seen_or)
        hipLaunchKernelGGL((k_expand<K, true>), dim3(LevelGrids<K>::get().expand_seen), dim3(kBlock), 0, s, a, p);
    else
        hipLaunchKernelGGL((k_expand<K, false>), dim3(LevelGrids<K>::get().expand), dim3(kBlock), 0, s, a, p);
    RPQ_LAUNCH_CHECK();
    if (e1) RPQ_HIP(hipEventRecord(e1, s));
    hipLaunchKernelGGL(k_compact, dim3(LevelGrids<K>::get().compact), dim3(kBlock), 0, s, a, p, n_rows, level);
    RPQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finalize<K>, dim3(LevelGrids<K>::get().finalize), dim3(kBlock), 0, s, a, p, count_work);
    RPQ_LAUNCH_CHECK();
    if (e2) RPQ_HIP(hipEventRecord(e2, s));
    if (on && e0 && e1 && e2) {
        std::lock_guard<std::mutex> lk(pr.mu);
        pr.pend_expand.emplace_back(e0, e1);
        pr.pend_finalize.emplace_back(e1, e2);
    }
    return RPQ_OK;
}

void profile_resolve() {
    Profiler& pr = profiler();
    std::lock_guard<std::mutex> lk(pr.mu);
    pr.resolve();
}

template <int K>
int launch_finalize(const Args& a, int p, uint64_t n_rows, uint32_t level, int count_work, hipStream_t s) {
    hipLaunchKernelGGL(k_compact, dim3(LevelGrids<K>::get().compact), dim3(kBlock), 0, s, a, p, n_rows, level);
    RPQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finalize<K>, dim3(LevelGrids<K>::get().finalize), dim3(kBlock), 0, s, a, p, count_work);
    RPQ_LAUNCH_CHECK();
    return RPQ_OK;
}

// A second stream for extraction (one per host thread and device, created on first use and kept
// for the thread's lifetime) and the events that order its work against the caller's stream.  The
// destructor drains the side stream, so no work of a call outlives it on any return path.  Without
// a side stream (creation failed) everything runs on the caller's stream, in the same order.
struct SideStream {
    static constexpr int kMaxDevices = 64;
    hipStream_t stream = nullptr;
    hipEvent_t leveled = nullptr;
    hipEvent_t extracted[2] = {nullptr, nullptr};

    explicit SideStream(bool want) {
        if (!want) return;
        static thread_local hipStream_t per_device[kMaxDevices] = {};
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
        if (!per_device[dev] && hipStreamCreateWithFlags(&per_device[dev], hipStreamNonBlocking) != hipSuccess) {
            per_device[dev] = nullptr;
            return;
        }
        if (hipEventCreateWithFlags(&leveled, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&extracted[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&extracted[1], hipEventDisableTiming) != hipSuccess) {
            destroy_events();
            return;
        }
        stream = per_device[dev];
    }
    ~SideStream() {
        if (stream) (void)hipStreamSynchronize(stream);
        destroy_events();
    }
    void destroy_events() {
        if (leveled) (void)hipEventDestroy(leveled);
        for (hipEvent_t& e : extracted)
            if (e) (void)hipEventDestroy(e);
        leveled = nullptr;
        extracted[0] = extracted[1] = nullptr;
    }
    SideStream(const SideStream&) = delete;
    SideStream& operator=(const SideStream&) = delete;
};

template <int K>
int launch_extract(const Args& a, bool write, const uint32_t* sources, uint64_t n_sources, uint64_t group_base,
                   uint32_t G, uint32_t W, uint32_t nchunks, uint32_t chunk_v, unsigned long long* acc,
                   uint32_t* partial, const uint64_t* srcbase, uint64_t* pairs, uint64_t off, uint64_t cap,
                   hipStream_t s) {
    const uint64_t waves = (uint64_t)G * (K / kExtractWords<K>()) * nchunks;
    const unsigned grid = (unsigned)std::min<uint64_t>((waves + kWaves - 1) / kWaves, 16384);
    if (write)
        hipLaunchKernelGGL((k_extract<K, true>), dim3(grid), dim3(kBlock), 0, s, a, sources, n_sources, group_base, G,
                           W, nchunks, chunk_v, acc, partial, srcbase, pairs, off, cap);
    else
        hipLaunchKernelGGL((k_extract<K, false>), dim3(grid), dim3(kBlock), 0, s, a, sources, n_sources, group_base,
                           G, W, nchunks, chunk_v, acc, partial, srcbase, pairs, off, cap);
    RPQ_LAUNCH_CHECK();
    return RPQ_OK;
}

#define RPQ_DISPATCH_K(K, CALL)                                      \
    switch (K) {                                                     \
        case 1: { constexpr int KK = 1; CALL; } break;               \
        case 2: { constexpr int KK = 2; CALL; } break;               \
        case 4: { constexpr int KK = 4; CALL; } break;               \
        case 8: { constexpr int KK = 8; CALL; } break;               \
        case 16: { constexpr int KK = 16; CALL; } break;             \
        case 32: { constexpr int KK = 32; CALL; } break;             \
        case 64: { constexpr int KK = 64; CALL; } break;             \
        default: rpq::set_error("bad batch width"); return RPQ_EINVAL; \
    }

// A copy stream per host thread and device (created on first use, kept for the thread's lifetime).
hipStream_t copy_stream() {
    constexpr int kMaxDevices = 64;
    static thread_local hipStream_t per_device[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    if (!per_device[dev] && hipStreamCreateWithFlags(&per_device[dev], hipStreamNonBlocking) != hipSuccess)
        per_device[dev] = nullptr;
    return per_device[dev];
}

// Host side of rpq_eval_stream.  A counted group's keys [next_key, end_key) are cut into windows of
// at most chunk_keys keys; window i is extracted into device chunk i % 2 on the extraction stream,
// copied to host chunk i % 2 on the copy stream, and handed to the sink once its copy is complete.
// At most two windows are in flight, so a chunk is rewritten only after the sink has returned for
// the window it held.  Windows are issued in key order and delivered in issue order.
struct PairStreamer {
    const rpq_pair_stream* ps = nullptr;
    hipStream_t xs = nullptr, cs = nullptr;
    hipEvent_t ext_done[2] = {nullptr, nullptr}, copied[2] = {nullptr, nullptr}, counted = nullptr;
    uint64_t* gend = nullptr;   // pinned: key index at which the counted group ends
    // the group whose windows are being issued
    bool pending = false, end_known = false;
    uint64_t next_key = 0, end_key = 0;
    hipEvent_t group_done = nullptr;   // recorded on xs after the group's last window
    Args ga;
    const uint32_t* sources = nullptr;
    uint64_t n_sources = 0, gbase = 0;
    uint32_t G_eff = 0, K = 0, W = 0, nchunks = 0, chunk_v = 0;
    unsigned long long* acc = nullptr;
    uint32_t* partial = nullptr;
    const uint64_t* srcbase = nullptr;
    // windows issued and not yet delivered: a ring of two, oldest at head
    int win_buf[2] = {0, 0};
    uint64_t win_n[2] = {0, 0};
    int head = 0, n_inflight = 0, next_buf = 0;
    uint64_t delivered = 0;
    uint64_t* written = nullptr;   // the caller's result->written, kept current

    PairStreamer() = default;
    PairStreamer(const PairStreamer&) = delete;
    PairStreamer& operator=(const PairStreamer&) = delete;

    int init(const rpq_pair_stream* p, hipStream_t extraction, uint64_t* pinned_slot, uint64_t* written_out) {
        ps = p;
        written = written_out;
        xs = extraction;
        cs = copy_stream();
        if (!cs) cs = xs;
        gend = pinned_slot;
        for (int b = 0; b < 2; ++b) {
            RPQ_HIP(hipEventCreateWithFlags(&ext_done[b], hipEventDisableTiming));
            RPQ_HIP(hipEventCreateWithFlags(&copied[b], hipEventDisableTiming));
        }
        RPQ_HIP(hipEventCreateWithFlags(&counted, hipEventDisableTiming));
        return RPQ_OK;
    }
    ~PairStreamer() {
        // no work of the call outlives it, whatever the return path
        if (cs) (void)hipStreamSynchronize(cs);
        if (xs) (void)hipStreamSynchronize(xs);
        for (hipEvent_t e : {ext_done[0], ext_done[1], copied[0], copied[1], counted})
            if (e) (void)hipEventDestroy(e);
    }

    // The keys of a group whose count pass and per-source offsets are enqueued on xs; `done` is
    // recorded on xs once its last window is issued.
    int start_group(const Args& a, hipEvent_t done, const uint32_t* src, uint64_t n_src, uint64_t base, uint32_t G,
                    uint32_t K_, uint32_t W_, uint32_t nch, uint32_t chv, unsigned long long* acc_,
                    uint32_t* partial_, const uint64_t* srcbase_, const unsigned long long* pairbase) {
        RPQ_HIP(hipMemcpyAsync(gend, pairbase, 8, hipMemcpyDeviceToHost, xs));
        RPQ_HIP(hipEventRecord(counted, xs));
        pending = true;
        end_known = false;
        next_key = end_key;   // this group's keys follow the previous group's
        group_done = done;
        ga = a;
        sources = src;
        n_sources = n_src;
        gbase = base;
        G_eff = G;
        K = K_;
        W = W_;
        nchunks = nch;
        chunk_v = chv;
        acc = acc_;
        partial = partial_;
        srcbase = srcbase_;
        return RPQ_OK;
    }

    int deliver_head() {
        const int b = win_buf[head];
        const uint64_t n = win_n[head];
        head ^= 1;
        --n_inflight;
        if (ps->sink(ps->host_chunks + (uint64_t)b * ps->chunk_keys, n, ps->user) != 0) {
            rpq::set_error("the pair sink stopped the evaluation after %llu keys", (unsigned long long)delivered);
            return RPQ_ECANCELED;
        }
        delivered += n;
        if (written) *written = delivered;
        return RPQ_OK;
    }

    // hand every completed window to the sink; with wait, block for the oldest one first
    int deliver(bool wait) {
        while (n_inflight) {
            const hipEvent_t e = copied[win_buf[head]];
            if (wait) {
                RPQ_HIP(hipEventSynchronize(e));
                wait = false;
            } else {
                const hipError_t q = hipEventQuery(e);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) {
                    rpq::set_error("HIP error in hipEventQuery: %s", hipGetErrorString(q));
                    return RPQ_EDEVICE;
                }
            }
            RPQ_TRY(deliver_head());
        }
        return RPQ_OK;
    }

    int issue_window() {
        const int b = next_buf;
        next_buf ^= 1;
        const uint64_t n = std::min<uint64_t>(ps->chunk_keys, end_key - next_key);
        uint64_t* dev = ps->device_chunks + (uint64_t)b * ps->chunk_keys;
        RPQ_DISPATCH_K(K, RPQ_TRY(launch_extract<KK>(ga, true, sources, n_sources, gbase, G_eff, W, nchunks, chunk_v,
                                                     acc, partial, srcbase, dev, next_key, n, xs)));
        RPQ_HIP(hipEventRecord(ext_done[b], xs));
        RPQ_HIP(hipStreamWaitEvent(cs, ext_done[b], 0));
        RPQ_HIP(hipMemcpyAsync(ps->host_chunks + (uint64_t)b * ps->chunk_keys, dev, n * 8, hipMemcpyDeviceToHost, cs));
        RPQ_HIP(hipEventRecord(copied[b], cs));
        const int slot = (head + n_inflight) & 1;
        win_buf[slot] = b;
        win_n[slot] = n;
        ++n_inflight;
        next_key += n;
        return RPQ_OK;
    }

    // Deliver what is complete and issue what fits.  With finish, return only once every window of
    // the pending group is issued: its Ans bitmap and per-source arrays may then be reused by work
    // enqueued on xs after this point (or ordered after group_done).
    int pump(bool finish) {
        for (;;) {
            RPQ_TRY(deliver(false));
            if (!pending) return RPQ_OK;
            if (!end_known) {
                if (finish) {
                    RPQ_HIP(hipEventSynchronize(counted));
                } else {
                    const hipError_t q = hipEventQuery(counted);
                    if (q == hipErrorNotReady) return RPQ_OK;
                    if (q != hipSuccess) {
                        rpq::set_error("HIP error in hipEventQuery: %s", hipGetErrorString(q));
                        return RPQ_EDEVICE;
                    }
                }
                end_key = *gend;
                end_known = true;
            }
            while (n_inflight < 2 && next_key < end_key) RPQ_TRY(issue_window());
            if (next_key == end_key) {
                if (group_done) RPQ_HIP(hipEventRecord(group_done, xs));
                pending = false;
                return RPQ_OK;
            }
            if (!finish) return RPQ_OK;
            RPQ_TRY(deliver(true));
        }
    }

    // every window issued and delivered
    int drain() {
        RPQ_TRY(pump(true));
        while (n_inflight) RPQ_TRY(deliver(true));
        return RPQ_OK;
    }
};

int prepare(rpq_graph_t g, const rpq_nfa* nfa_in, uint64_t n_sources, uint32_t flags, const rpq_eval_opts* opts,
            rpq_nfa* eff, DevNfa* dn, Layout* lay, bool single_ans = false) {
    if (!g) {
        rpq::set_error("graph is NULL");
        return RPQ_EINVAL;
    }
    if (flags & ~(RPQ_PAIRS | RPQ_PER_SOURCE | RPQ_ALL_SOURCES | RPQ_REVERSE | RPQ_SPARSE | RPQ_LENGTH_BOUND)) {
        rpq::set_error("unknown flags 0x%x", flags);
        return RPQ_EINVAL;
    }
    if ((flags & RPQ_LENGTH_BOUND) && !opts) {
        rpq::set_error("RPQ_LENGTH_BOUND needs opts->max_length");
        return RPQ_EINVAL;
    }
    if (opts && opts->visit > RPQ_VISIT_SEEN_OR) {
        rpq::set_error("rpq_eval_opts.visit must be 0, RPQ_VISIT_TWO_READS or RPQ_VISIT_SEEN_OR");
        return RPQ_EINVAL;
    }
    RPQ_TRY(validate_nfa(g, nfa_in));
    if ((flags & RPQ_REVERSE) && !g->has_in) {
        rpq::set_error("RPQ_REVERSE needs a graph built with RPQ_BUILD_IN_CSR");
        return RPQ_EUNSUPPORTED;
    }
    if (flags & RPQ_REVERSE) RPQ_TRY(rpq_nfa_reverse(nfa_in, eff));
    else *eff = *nfa_in;
    to_dev_nfa(eff, g->L, dn);
    return make_layout(g, *dn, n_sources, flags, opts, single_ans, lay);
}

}  // namespace

extern "C" {

int rpq_eval_workspace_size(rpq_graph_t g, const rpq_nfa* nfa, uint64_t n_sources, uint32_t flags,
                            const rpq_eval_opts* opts, uint64_t* bytes) {
    rpq::clear_error();
    if (!bytes) {
        rpq::set_error("bytes is NULL");
        return RPQ_EINVAL;
    }
    if (g && (flags & RPQ_ALL_SOURCES) && n_sources == 0) n_sources = g->V;
    if (flags & RPQ_SPARSE) return rpq::sparse_workspace_size(g, nfa, n_sources, flags, bytes);
    rpq_nfa eff;
    DevNfa dn;
    Layout lay;
    RPQ_TRY(prepare(g, nfa, n_sources, flags, opts, &eff, &dn, &lay));
    *bytes = lay.total;
    return RPQ_OK;
}

int rpq_eval(rpq_graph_t g, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources, uint32_t flags,
             const rpq_eval_opts* opts, void* workspace, uint64_t workspace_bytes, rpq_result* res,
             hipStream_t stream) {
    rpq::clear_error();
    const int rc =
        rpq::eval_impl(g, nfa, sources, n_sources, flags, opts, nullptr, workspace, workspace_bytes, res, stream);
    // a failing call may leave kernels of its own queued on the stream: drain them, so that the
    // caller may reuse or release the workspace as soon as the call returns
    if (rc != RPQ_OK && rc != RPQ_EOVERFLOW) (void)hipStreamSynchronize(stream);
    return rc;
}

}  // extern "C"

namespace {

// The plain evaluation.  With noalloc the call creates nothing: counters are read into a
// pageable stack buffer instead of the thread's pinned staging buffer, extraction stays on the
// caller's stream (the layout then holds a single answer bitmap), and no profiling events are
// recorded.
int eval_core(rpq_graph_t g, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources, uint32_t flags,
              const rpq_eval_opts* opts, const uint64_t* target, void* workspace, uint64_t workspace_bytes,
              rpq_result* res, hipStream_t stream, bool noalloc, const rpq_pair_stream* ps = nullptr) {
    if (!res) {
        rpq::set_error("result is NULL");
        return RPQ_EINVAL;
    }
    if (g && (flags & RPQ_ALL_SOURCES)) {
        if (sources) {
            rpq::set_error("RPQ_ALL_SOURCES requires sources == NULL");
            return RPQ_EINVAL;
        }
        if (n_sources == 0) n_sources = g->V;
        if (n_sources != g->V) {
            rpq::set_error("RPQ_ALL_SOURCES requires n_sources == n_vertices");
            return RPQ_EINVAL;
        }
    } else if (n_sources && !sources) {
        rpq::set_error("sources is NULL");
        return RPQ_EINVAL;
    }
    if (!ps && (flags & RPQ_PAIRS) && res->capacity && !res->pairs) {
        rpq::set_error("RPQ_PAIRS with a NULL pair buffer");
        return RPQ_EINVAL;
    }
    if ((flags & RPQ_PER_SOURCE) && n_sources && !res->per_source) {
        rpq::set_error("RPQ_PER_SOURCE with a NULL per_source buffer");
        return RPQ_EINVAL;
    }
    res->workspace_needed = 0;
    if ((flags & RPQ_LENGTH_BOUND) && !opts) {
        rpq::set_error("RPQ_LENGTH_BOUND needs opts->max_length");
        return RPQ_EINVAL;
    }
    if (flags & RPQ_SPARSE) {
        if (target) {
            rpq::set_error("internal: a result filter is not supported with RPQ_SPARSE");
            return RPQ_EINVAL;
        }
        if (flags & ~(RPQ_PAIRS | RPQ_PER_SOURCE | RPQ_ALL_SOURCES | RPQ_REVERSE | RPQ_SPARSE | RPQ_LENGTH_BOUND)) {
            rpq::set_error("unknown flags 0x%x", flags);
            return RPQ_EINVAL;
        }
        const uint64_t max_len = (flags & RPQ_LENGTH_BOUND) ? (uint64_t)opts->max_length : ~0ull;
        return rpq::sparse_eval(g, nfa, sources, n_sources, flags, max_len, workspace, workspace_bytes, res, stream);
    }
    rpq_nfa eff;
    DevNfa dn;
    Layout x;
    // streamed keys need the per-source offsets of the pairs layout
    if (ps) flags |= RPQ_PAIRS;
    RPQ_TRY(prepare(g, nfa, n_sources, flags, opts, &eff, &dn, &x, noalloc));
    if (!workspace || workspace_bytes < x.total) {
        rpq::set_error("workspace of %llu bytes is smaller than the %llu bytes needed",
                       (unsigned long long)workspace_bytes, (unsigned long long)x.total);
        res->workspace_needed = x.total;
        return RPQ_ENOMEM;
    }
    if (reinterpret_cast<uintptr_t>(workspace) & 255) {
        rpq::set_error("workspace must be 256-byte aligned");
        return RPQ_EINVAL;
    }
    const bool want_pairs = !ps && (flags & RPQ_PAIRS) && res->pairs != nullptr;
    res->written = res->count = res->hash = res->product_edges = res->levels = res->max_depth = 0;
    if (n_sources == 0) return RPQ_OK;

    char* ws = reinterpret_cast<char*>(workspace);
    Args a = make_args(g, flags, x, ws);
    a.target = target;
    uint64_t local_stage[C_NCOUNTERS];
    uint64_t* stage = noalloc ? local_stage : rpq::host_stage();
    if (!stage) {
        rpq::set_error("pinned host staging memory is unavailable");
        return RPQ_EDEVICE;
    }
    RPQ_HIP(hipMemcpyAsync(ws + x.off_nfa, &dn, sizeof dn, hipMemcpyHostToDevice, stream));
    RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(a.counters), C_NCOUNTERS, 0, stream));
    RPQ_TRY(rpq::fill_u64(a.next, (uint64_t)x.G * x.Q * x.V * x.K, 0, stream));
    RPQ_TRY(rpq::fill_u64(a.touch, ((uint64_t)x.G * x.Q * x.V + 63) / 64, 0, stream));
    if (sources) {
        hipLaunchKernelGGL(k_check_sources, dim3((unsigned)std::min<uint64_t>((n_sources + 255) / 256, 4096)),
                           dim3(256), 0, stream, sources, n_sources, x.V, a.counters);
        RPQ_LAUNCH_CHECK();
    }
    RPQ_HIP(hipMemcpyAsync(stage, a.counters, C_NCOUNTERS * 8, hipMemcpyDeviceToHost, stream));
    RPQ_HIP(hipStreamSynchronize(stream));
    if (stage[C_ERR] & ERR_SOURCES) {
        rpq::set_error("sources must be strictly ascending vertex ids below n_vertices");
        return RPQ_EINVAL;
    }

    const uint64_t per_group = (uint64_t)x.G * x.W;
    const uint64_t n_groups = (n_sources + per_group - 1) / per_group;
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(ws + x.off_acc);
    uint32_t* partial = want_pairs || ps ? reinterpret_cast<uint32_t*>(ws + x.off_partial) : nullptr;
    uint64_t* srcbase = want_pairs || ps ? reinterpret_cast<uint64_t*>(ws + x.off_srcbase) : nullptr;
    uint64_t levels_total = 0, max_depth = 0;
    // Extraction of group g runs on a second stream (xs) while the levels of group g + 1 run on
    // `stream` into the other Ans bitmap: the level kernels are bound by memory, extraction by its
    // instruction stream.  Events order each bitmap's reuse and the final join.
    uint64_t* const ans_buf[2] = {reinterpret_cast<uint64_t*>(ws + x.off_ans),
                                  reinterpret_cast<uint64_t*>(ws + x.off_ans2)};
    const bool overlap = n_groups > 1 && x.off_ans2 != x.off_ans && !noalloc;
    SideStream side(overlap);
    hipStream_t xs = side.stream ? side.stream : stream;
    // streamed keys: windows of group g are extracted on xs while group g + 1's levels run; the
    // group-end key index is read through the pinned staging buffer, past the counter words
    PairStreamer st;
    if (ps) RPQ_TRY(st.init(ps, xs, stage + 64, &res->written));
    for (uint64_t grp = 0; grp < n_groups; ++grp) {
        const uint64_t gbase = grp * per_group;
        const uint64_t n_here = std::min<uint64_t>(per_group, n_sources - gbase);
        const uint32_t G_eff = (uint32_t)((n_here + x.W - 1) / x.W);
        const int buf = side.stream ? (int)(grp & 1) : 0;
        a.ans = ans_buf[buf];
        // the bitmap's previous group must be extracted before it is cleared for this one
        if (side.stream && grp >= 2) RPQ_HIP(hipStreamWaitEvent(stream, side.extracted[buf], 0));
        RPQ_TRY(rpq::fill_u64(a.vis, (uint64_t)G_eff * x.Q * x.V * x.K, 0, stream));
        if (x.seen_or) RPQ_TRY(rpq::fill_u64(a.next, (uint64_t)G_eff * x.Q * x.V * x.K, 0, stream));
        RPQ_TRY(rpq::fill_u64(a.ans, (uint64_t)G_eff * x.V * x.K, 0, stream));
        hipLaunchKernelGGL(k_seed, dim3((unsigned)(((uint64_t)G_eff * x.W + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           stream, a, sources, n_sources, gbase, G_eff, x.W, x.K);
        RPQ_LAUNCH_CHECK();
        const uint64_t n_rows = (uint64_t)G_eff * x.Q * x.V;
        RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(a.counters) + C_LASTLEVEL, 1, 0, stream));
        // list and slice counts start at zero (a length-bounded group ends with a frontier left)
        RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(a.counters) + C_LIST, 4, 0, stream));
        RPQ_DISPATCH_K(x.K, RPQ_TRY(launch_finalize<KK>(a, 0, n_rows, 0, x.max_len > 0, stream)));
        uint64_t level = 1;
        int p = 1;
        // a first-reach distance in the product graph is below Q * V, so the
        // fixpoint arrives within Q * V + 1 levels; more means a defect
        const uint64_t level_bound = (uint64_t)x.Q * x.V + 2;
        uint64_t launched = 0;
        // level l expands depth l - 1 and finalizes depth l; a length bound k stops after level k
        while (level <= x.max_len) {
            uint32_t n_launch = 0;
            for (; n_launch < x.sync_every && level <= x.max_len; ++n_launch) {
                RPQ_DISPATCH_K(x.K, RPQ_TRY(launch_level<KK>(a, p, n_rows, (uint32_t)level, level < x.max_len,
                                                              !noalloc, stream)));
                p ^= 1;
                ++level;
            }
            launched += n_launch;
            RPQ_HIP(hipMemcpyAsync(stage, a.counters, C_NCOUNTERS * 8, hipMemcpyDeviceToHost, stream));
            if (ps) RPQ_TRY(st.pump(false));   // the previous group's windows, while these levels run
            RPQ_HIP(hipStreamSynchronize(stream));
            if (!noalloc && profiler().on) profile_resolve();
            if (stage[C_ERR] & (ERR_LIST | ERR_DESC)) {
                rpq::set_error("internal capacity exceeded (flags 0x%llx)", (unsigned long long)stage[C_ERR]);
                return RPQ_EDEVICE;
            }
            if (stage[C_LIST + p] == 0) break;   // the last finalize produced no new entries
            if (launched > level_bound) {
                rpq::set_error("no fixpoint after %llu levels", (unsigned long long)launched);
                return RPQ_EDEVICE;
            }
        }
        if (launched == 0) {   // a bound of 0: only the seeds' zero-length walks
            RPQ_HIP(hipMemcpyAsync(stage, a.counters, C_NCOUNTERS * 8, hipMemcpyDeviceToHost, stream));
            RPQ_HIP(hipStreamSynchronize(stream));
        }
        const uint64_t lv = stage[C_LASTLEVEL];   // levels with a non-empty frontier, seeds included
        levels_total += lv;
        if (lv > 0 && lv - 1 > max_depth) max_depth = lv - 1;
        if (side.stream) {
            RPQ_HIP(hipEventRecord(side.leveled, stream));
            RPQ_HIP(hipStreamWaitEvent(xs, side.leveled, 0));
        }
        // the previous group's windows read acc, partial and srcbase: all of them go on xs before
        // this group's count pass overwrites those arrays
        if (ps) RPQ_TRY(st.pump(true));
        RPQ_TRY(rpq::fill_u64(reinterpret_cast<uint64_t*>(acc), (uint64_t)G_eff * x.W * 2, 0, xs));
        // profiling: the count pass timed on its own stream; it reads every answer word of the group
        hipEvent_t xe0 = nullptr, xe1 = nullptr;
        if (!noalloc && profiler().on) {
            Profiler& pr = profiler();
            std::lock_guard<std::mutex> lk(pr.mu);
            xe0 = pr.get();
            xe1 = pr.get();
            pr.acc.extract_words += (uint64_t)G_eff * x.V * x.K;
        }
        if (xe0) RPQ_HIP(hipEventRecord(xe0, xs));
        RPQ_DISPATCH_K(x.K, RPQ_TRY(launch_extract<KK>(a, false, sources, n_sources, gbase, G_eff, x.W, x.nchunks,
                                                       x.chunk_v, acc, partial, nullptr, nullptr, 0, 0, xs)));
        if (xe0 && xe1) {
            RPQ_HIP(hipEventRecord(xe1, xs));
            Profiler& pr = profiler();
            std::lock_guard<std::mutex> lk(pr.mu);
            pr.pend_extract.emplace_back(xe0, xe1);
        }
        hipLaunchKernelGGL(k_group_finish, dim3(1), dim3(1024), 0, xs, a.counters, acc, partial, srcbase,
                           (flags & RPQ_PER_SOURCE) ? res->per_source : nullptr, n_sources, gbase,
                           (uint64_t)G_eff * x.W, x.nchunks);
        RPQ_LAUNCH_CHECK();
        if (want_pairs) {
            RPQ_DISPATCH_K(x.K, RPQ_TRY(launch_extract<KK>(a, true, sources, n_sources, gbase, G_eff, x.W, x.nchunks,
                                                           x.chunk_v, acc, partial, srcbase, res->pairs,
                                                           res->pair_offset, res->capacity, xs)));
        }
        if (ps) {
            RPQ_TRY(st.start_group(a, side.stream ? side.extracted[buf] : nullptr, sources, n_sources, gbase, G_eff,
                                   x.K, x.W, x.nchunks, x.chunk_v, acc, partial, srcbase, a.counters + C_PAIRBASE));
            RPQ_TRY(st.pump(false));
        } else if (side.stream) {
            RPQ_HIP(hipEventRecord(side.extracted[buf], xs));
        }
    }
    if (ps) RPQ_TRY(st.drain());
    if (side.stream) {
        // join: everything the side stream did happens before the totals are read on `stream`
        RPQ_HIP(hipEventRecord(side.leveled, xs));
        RPQ_HIP(hipStreamWaitEvent(stream, side.leveled, 0));
    }
    RPQ_HIP(hipMemcpyAsync(stage, a.counters, C_NCOUNTERS * 8, hipMemcpyDeviceToHost, stream));
    RPQ_HIP(hipStreamSynchronize(stream));
    if (!noalloc) {
        Profiler& pr = profiler();
        std::lock_guard<std::mutex> lk(pr.mu);
        if (pr.on) {
            pr.resolve(true);   // both streams are drained here
            pr.acc.finalize_rows += stage[C_FROWS];
            pr.acc.finalize_row_words += stage[C_FROWS] * x.K;
            pr.acc.finalize_words += stage[C_FWORDS];
            // 8-byte accesses of finalize to Vis: a read of every row word (seen OR), or a read and
            // a write of every non-zero word (two reads)
            pr.acc.finalize_vis_words += x.seen_or ? stage[C_FROWS] * x.K : 2 * stage[C_FWORDS];
            // beyond the method's bytes: the Next word read beside each visited word (two reads);
            // seen OR makes the method's accesses only
            pr.acc.expand_extra_words += x.seen_or ? 0 : stage[C_WREAD];
            pr.acc.finalize_ans_words += stage[C_FANS];
            pr.acc.edge_items += stage[C_ITEMS];
            pr.acc.descriptors += stage[C_DESCS];
            pr.acc.row_words += stage[C_ROWW];
            pr.acc.word_reads += stage[C_WREAD];
            pr.acc.word_updates += stage[C_WUPD];
        }
    }
    res->count = stage[C_COUNT];
    res->hash = stage[C_HASH];
    if (ps) res->written = st.delivered;
    res->product_edges = stage[C_EPROD];
    res->levels = levels_total;
    res->max_depth = max_depth;
    if (want_pairs) {
        const uint64_t avail = res->count > res->pair_offset ? res->count - res->pair_offset : 0;
        res->written = std::min<uint64_t>(avail, res->capacity);
        if (avail > res->capacity) {
            rpq::set_error("result has %llu keys past offset %llu; capacity is %llu",
                           (unsigned long long)avail, (unsigned long long)res->pair_offset,
                           (unsigned long long)res->capacity);
            return RPQ_EOVERFLOW;
        }
    }
    return RPQ_OK;
}

// Static scratch of the allocation-free entry point: a file-scope device array, one copy per
// device, held until the process ends.  In host code `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress, once per device, and only that address is used.
constexpr uint64_t kScratchBytes = RPQ_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;

void* scratch_address() {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        rpq::set_error("no current HIP device (or device id beyond %d)", kMaxDevices - 1);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            rpq::set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
            return nullptr;
        }
        addr[dev] = p;
    }
    return addr[dev];
}

}  // namespace

namespace rpq {

int eval_impl(rpq_graph_t g, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources, uint32_t flags,
              const rpq_eval_opts* opts, const uint64_t* target, void* workspace, uint64_t workspace_bytes,
              rpq_result* res, hipStream_t stream) {
    return eval_core(g, nfa, sources, n_sources, flags, opts, target, workspace, workspace_bytes, res, stream,
                     false);
}

}  // namespace rpq

extern "C" {

int rpq_eval_noalloc(rpq_graph_t g, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources,
                     uint32_t flags, const rpq_eval_opts* opts, rpq_result* res, hipStream_t stream) {
    rpq::clear_error();
    if (flags & RPQ_SPARSE) {
        rpq::set_error("rpq_eval_noalloc runs the bitmap search only; RPQ_SPARSE is not supported");
        return RPQ_EUNSUPPORTED;
    }
    if (!res) {
        rpq::set_error("result is NULL");
        return RPQ_EINVAL;
    }
    if ((flags & RPQ_LENGTH_BOUND) && !opts) {
        rpq::set_error("RPQ_LENGTH_BOUND needs opts->max_length");
        return RPQ_EINVAL;
    }
    uint64_t n = n_sources;
    if (g && (flags & RPQ_ALL_SOURCES) && n == 0) n = g->V;
    // the plan: the caller's knobs, with the unset ones narrowed until the workspace fits the
    // scratch (fewer units in flight first, then narrower units)
    rpq_eval_opts o{};
    if (opts) o = *opts;
    rpq_nfa eff;
    DevNfa dn;
    Layout lay;
    for (;;) {
        RPQ_TRY(prepare(g, nfa, n, flags, &o, &eff, &dn, &lay, true));
        if (lay.total <= kScratchBytes) break;
        if (!(opts && opts->concurrency) && lay.G > 1) {
            o.batch_width = lay.W;
            o.concurrency = lay.G / 2;
        } else if (!(opts && opts->batch_width) && lay.W > 64) {
            o.batch_width = lay.W / 2;
            o.concurrency = (opts && opts->concurrency) ? opts->concurrency : 0;
        } else {
            rpq::set_error("the evaluation needs %llu bytes of workspace; the static scratch holds %llu",
                           (unsigned long long)lay.total, (unsigned long long)kScratchBytes);
            res->workspace_needed = lay.total;
            return RPQ_ENOMEM;
        }
    }
    void* ws = scratch_address();
    if (!ws) return RPQ_EDEVICE;
    const int rc = eval_core(g, nfa, sources, n_sources, flags, &o, nullptr, ws, kScratchBytes, res, stream, true);
    if (rc != RPQ_OK && rc != RPQ_EOVERFLOW) (void)hipStreamSynchronize(stream);
    return rc;
}

int rpq_eval_stream(rpq_graph_t g, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources,
                    uint32_t flags, const rpq_eval_opts* opts, void* workspace, uint64_t workspace_bytes,
                    const rpq_pair_stream* out, rpq_result* res, hipStream_t stream) {
    rpq::clear_error();
    if (!out || !out->sink || !out->device_chunks || !out->host_chunks || out->chunk_keys == 0) {
        rpq::set_error("the pair stream needs a sink, two device and two host chunks of chunk_keys >= 1 keys");
        return RPQ_EINVAL;
    }
    if (flags & RPQ_SPARSE) {
        rpq::set_error("rpq_eval_stream runs the bitmap search only; RPQ_SPARSE is not supported");
        return RPQ_EUNSUPPORTED;
    }
    const int rc = eval_core(g, nfa, sources, n_sources, flags, opts, nullptr, workspace, workspace_bytes, res,
                             stream, false, out);
    if (rc != RPQ_OK) (void)hipStreamSynchronize(stream);
    return rc;
}

int rpq_profile_enable(int on) {
    Profiler& pr = profiler();
    std::lock_guard<std::mutex> lk(pr.mu);
    pr.on = on != 0;
    return RPQ_OK;
}

int rpq_profile_read(rpq_profile* out, int reset) {
    rpq::clear_error();
    if (!out) {
        rpq::set_error("out is NULL");
        return RPQ_EINVAL;
    }
    Profiler& pr = profiler();
    std::lock_guard<std::mutex> lk(pr.mu);
    *out = pr.acc;
    if (reset) pr.acc = rpq_profile{};
    return RPQ_OK;
}

}  // extern "C"
