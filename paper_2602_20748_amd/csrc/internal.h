// Internal declarations of librpq: error plumbing, the graph object, device
// primitives (fill, scan, radix sort) and wave64 helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <vector>

#include <cstdint>
#include <cstdio>

#include "../../include/rpq.h"

namespace rpq {

void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

#define RPQ_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ::rpq::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),        \
                             __FILE__, __LINE__);                                          \
            return RPQ_EDEVICE;                                                            \
        }                                                                                  \
    } while (0)

#define RPQ_TRY(expr)                 \
    do {                              \
        int rc_ = (expr);             \
        if (rc_ != RPQ_OK) return rc_; \
    } while (0)

#define RPQ_LAUNCH_CHECK() RPQ_HIP(hipGetLastError())

// One direction of the label-partitioned CSR.  Row r = v * n_labels + l holds
// the neighbours of v over label l in dst[row_ptr[r] .. row_ptr[r + 1]),
// ascending.  lmask[v] has bit l set when row (v, l) is non-empty.
struct Csr {
    uint32_t* row_ptr = nullptr;   // [V * L + 1]
    uint32_t* dst = nullptr;       // [E]
    uint64_t* lmask = nullptr;     // [V]
    uint64_t nonempty_rows = 0;
};

}  // namespace rpq

struct rpq_graph {
    uint32_t V = 0, L = 0;
    uint64_t E_in = 0, E = 0;
    uint64_t per_label[RPQ_MAX_LABELS] = {};
    rpq::Csr out, in;
    bool has_in = false;
    uint8_t* vlabel = nullptr;          // [V] or null
    uint64_t device_bytes = 0;
    int device = 0;
    uint64_t* h_stage = nullptr;        // pinned host staging for small device->host reads
};

namespace rpq {

// ---- device primitives (prims.hip) ----
int fill_u64(uint64_t* p, uint64_t n, uint64_t value, hipStream_t s);
int fill_u32(uint32_t* p, uint64_t n, uint32_t value, hipStream_t s);

// Temporary uint64 elements needed by exclusive_scan_u64 for n inputs.
uint64_t scan_temp_elems(uint64_t n);
// out[i] = sum of in[0..i); out may alias in.  If total != nullptr the grand
// total is written to *total (device).
int exclusive_scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* temp,
                       uint64_t* total, hipStream_t s);

// Temporary bytes needed by radix_sort_u64 for n keys.
uint64_t radix_temp_bytes(uint64_t n);
// Stable LSD radix sort of n uint64 keys on bits [0, lo_bits) and [32, 32 + hi_bits)
// (bits outside are assumed zero).  keys and alt are two buffers of n keys;
// *sorted receives whichever holds the result.
int radix_sort_u64(uint64_t* keys, uint64_t* alt, uint64_t n, int lo_bits, int hi_bits,
                   void* temp, hipStream_t s, uint64_t** sorted);

// rpq_eval with an optional result-vertex filter (device bitmap of V bits, or null): the
// traversal is unchanged and only result pairs whose non-source vertex has its bit set are
// counted, hashed and written.
// Batched form: only result pairs whose destination has its bit set in `target` (device bitmap of
// V bits) count, as eval_impl's filter; before the batch's first run.
int batch_filter_targets(rpq_batch_t b, uint32_t query_id, const uint64_t* target);

int eval_impl(rpq_graph_t g, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources, uint32_t flags,
              const rpq_eval_opts* opts, const uint64_t* target, void* workspace, uint64_t workspace_bytes,
              rpq_result* res, hipStream_t stream);

// 4 KB of pinned host memory private to the calling thread (small device-to-host reads of
// counters), so that calls on one graph from several threads do not share a staging buffer.
// Allocated on a thread's first use and kept until the process ends; null if pinning fails.
uint64_t* host_stage();

// The per-source hash-set search (RPQ_SPARSE) behind rpq_eval, and its starting workspace.
// max_len: the length bound of RPQ_LENGTH_BOUND (deepest level recorded), or UINT64_MAX.
int sparse_eval(rpq_graph_t g, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources, uint32_t flags,
                uint64_t max_len, void* workspace, uint64_t workspace_bytes, rpq_result* res, hipStream_t stream);
int sparse_workspace_size(rpq_graph_t g, const rpq_nfa* nfa, uint64_t n_sources, uint32_t flags, uint64_t* bytes);

// ---- resident engine: the persistent batched kernel fed between bounded launches (batch.hip) ----
// The open form of the batched launch.  Its slots (fixed unit width W and automaton size Qmax) live
// in a caller-provided device region for the engine's lifetime; queries are staged on the host,
// uploaded before the next launch and join the device unit queue, whose idle slots take units at
// every iteration's refill.  Each launch runs at most max_iters iterations and keeps the state for
// the next one.
struct ResidentQuery {
    rpq_nfa nfa;
    const uint32_t* sources;     // device, ascending; null = ids [0, n_sources)
    uint64_t n_sources;
    uint64_t* pairs;             // device or null (single-unit queries only)
    uint64_t capacity;
    uint64_t* per_source;        // device [n][2] or null
    uint32_t max_len;            // deepest level recorded (0xFFFFFFFF = no bound)
};
struct ResidentDone {
    uint64_t token;
    int status;
    uint64_t count, hash, product_edges, levels, max_depth, written;
};
struct Resident;
// Device bytes of an engine with G slots of W sources for automata of at most Qmax states and at
// most max_succ successors per (state, label).
int resident_bytes(const rpq_graph* g, uint32_t W, uint32_t G, uint32_t Qmax, uint32_t max_succ, uint64_t* bytes);
int resident_create(rpq_graph* g, uint32_t W, uint32_t G, uint32_t Qmax, uint32_t max_succ, void* mem,
                    uint64_t bytes, hipStream_t stream, Resident** out);
void resident_destroy(Resident* r);
// Whether the engine can run this query (automaton within Qmax / max_succ; pairs only when the
// sources fit one unit).  Reads only what is fixed at creation.
bool resident_fits(const Resident* r, const ResidentQuery& q);
// Stage a query for the next launch; RPQ_ENOMEM while the query table or the unit ring is full.
int resident_admit(Resident* r, const ResidentQuery& q, uint64_t token);
// True when no query is staged, queued or running.
bool resident_idle(const Resident* r);
// True once a device error took the engine out of service (it then accepts nothing).
bool resident_broken(const Resident* r);
// Upload what is staged, run one launch of at most max_iters iterations on `stream`, wait, and
// append the queries that completed.  On a device error every query in flight completes with it.
int resident_step(Resident* r, uint32_t max_iters, hipStream_t stream, std::vector<ResidentDone>* done);

inline int bits_for(uint64_t max_value) {   // bits needed to represent values <= max_value
    int b = 0;
    while (b < 64 && (max_value >> b) != 0) ++b;
    return b;
}

}  // namespace rpq

// ---- wave64 helpers (device) ----
namespace rpqd {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = __lane_id();
    return l == 0 ? 0ull : ((~0ull) >> (64 - l));
}

// One SplitMix64 output for state x: the per-key checksum.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
    const int l = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (l >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
    const int l = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t t = __shfl_up(v, o, 64);
        if (l >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        uint32_t t = __shfl_xor(v, o, 64);
        v = t > v ? t : v;
    }
    return v;
}

// Item space of a frontier entry (state q, vertex v) with label set m (labels of v that q can
// follow): labels in ascending order, within a label its edges in CSR order, within an edge the
// successor states of delta(q, l) in ascending order.  delta is the compact [q * L + l] table.
__device__ __forceinline__ uint64_t entry_work(const uint32_t* __restrict__ row_ptr, uint32_t L,
                                               const uint32_t* delta, uint32_t v, uint32_t q, uint64_t m) {
    uint64_t work = 0;
    while (m) {
        const uint32_t l = (uint32_t)(__ffsll((long long)m) - 1);
        m &= m - 1;
        const uint64_t r = (uint64_t)v * L + l;
        work += (uint64_t)(row_ptr[r + 1] - row_ptr[r]) * (uint32_t)__popc(delta[q * L + l]);
    }
    return work;
}

// Item o of that space: edge target *w and successor state *q2.
__device__ __forceinline__ void decode_item(const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ dst,
                                            uint32_t L, const uint32_t* delta, uint32_t v, uint32_t q, uint64_t m,
                                            uint64_t o, uint32_t* w, uint32_t* q2) {
    while (m) {
        const uint32_t l = (uint32_t)(__ffsll((long long)m) - 1);
        m &= m - 1;
        const uint64_t r = (uint64_t)v * L + l;
        const uint32_t b = row_ptr[r], d = row_ptr[r + 1] - b;
        uint32_t succ = delta[q * L + l];
        const uint32_t ns = (uint32_t)__popc(succ);
        const uint64_t cnt = (uint64_t)d * ns;
        if (o < cnt) {
            uint64_t e = o, k = 0;
            if (ns != 1) {
                e = o / ns;
                k = o - e * ns;
            }
            *w = dst[b + e];
            for (uint64_t i = 0; i < k; ++i) succ &= succ - 1;
            *q2 = (uint32_t)(__ffs(succ) - 1);
            return;
        }
        o -= cnt;
    }
}

}  // namespace rpqd

// ---- grid-wide barrier for persistent kernels (device) ----
// Two-level barrier over all workgroups of a co-resident grid.  Workgroups arrive in groups of
// kBarGroup on counters of their own (one 128-byte line each), and only the last arrival of a
// group goes on to the top-level counter, so no counter takes more than kBarGroup atomics per
// barrier where a flat barrier would serialise one per workgroup.  The counters only grow:
// barrier number g (from 0) completes when a group counter reaches (g + 1) * its group size and
// the top counter (g + 1) * the number of groups; the generation word counts completed barriers
// and is what waiters watch.  Waits are bounded by the 100 MHz constant clock: after
// `timeout_ticks` a waiting workgroup raises abort and every workgroup returns from the barrier
// with false, so a grid that is not fully resident can never hang the device.  All counters start
// at zero (the host clears the block before each launch).
namespace rpqd {

constexpr unsigned int kBarGroup = 32;       // workgroups per arrival group
constexpr unsigned int kBarMaxGroups = 64;   // so at most 2,048 workgroups
constexpr unsigned int kBarLine = 32;        // words per 128-byte line

struct GridSync {
    unsigned int count;        // group completions, summed over barriers
    unsigned int generation;   // completed barriers
    unsigned int abort;
    unsigned int pad[kBarLine - 3];
    unsigned int group[kBarMaxGroups * kBarLine];   // arrivals of group i at group[i * kBarLine]
};

__device__ __forceinline__ bool grid_barrier(GridSync* gs, unsigned int n_blocks, uint64_t timeout_ticks) {
    // The workgroup meets first (its writes happen-before thread 0's release fence); thread 0
    // alone releases, arrives, waits and acquires for the whole workgroup, and the workgroup
    // meets again before any wave reads.  One agent-scope fence pair per workgroup per barrier:
    // on gfx950 each agent-scope fence writes back and invalidates the XCD's L2.
    __syncthreads();
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned int gen = __hip_atomic_load(&gs->generation, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();   // release (also keeps the generation read before the arrival)
        const unsigned int grp = blockIdx.x / kBarGroup;
        const unsigned int in_grp = min(kBarGroup, n_blocks - grp * kBarGroup);
        const unsigned int n_grp = (n_blocks + kBarGroup - 1) / kBarGroup;
        bool last = false;
        const unsigned int a_grp =
            __hip_atomic_fetch_add(&gs->group[grp * kBarLine], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (a_grp == (gen + 1) * in_grp) {
            // the group is complete: its last arrival carries it to the top level
            const unsigned int a_top =
                __hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
            last = a_top == (gen + 1) * n_grp;
        }
        if (last) {
            __hip_atomic_store(&gs->generation, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(&gs->generation, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() - t0 > timeout_ticks) {
                    __hip_atomic_store(&gs->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        __threadfence();   // acquire
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

}  // namespace rpqd
