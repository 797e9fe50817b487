/*
 * rpq.h -- C ABI of the MI355X regular-path-query library (librpq.so).
 *
 * What the library computes (cuRPQ paper, arXiv 2602.20748):
 *
 *   RPQ (Section 2.1, Definition 1): for a labelled directed graph G and a
 *   regular expression rho over its edge labels, the set of distinct vertex
 *   pairs (x, y) joined by a walk x -> ... -> y whose label word is in L(rho).
 *   Walks of any length count, including the zero-length walk (x, x) when the
 *   empty word is in L(rho).  Evaluation follows the automata-based approach
 *   of Section 2.2: a search over the product of G and an automaton for rho,
 *   keeping one visited set of (vertex, state) pairs per source vertex; a pair
 *   is emitted when a final state is reached.
 *
 *   CRPQ (Section 2.1, Definition 2): all homomorphisms f from the query
 *   variables to vertices such that labelled variables map to vertices with
 *   that label and every atom x -rho-> y holds for (f(x), f(y)); the atom
 *   results are computed first and then joined (Section 6.2).
 *
 * Conventions for every entry point:
 *   - Return value: RPQ_OK (0) or a negative rpq_status.  rpq_last_error()
 *     returns a thread-local message for the last failing call.  No C++
 *     exception crosses this boundary.
 *   - "device" pointers are HIP device memory of the current device (for
 *     example torch tensors); "host" pointers are ordinary host memory.  The
 *     library never frees memory it did not allocate.
 *   - Every call that launches work takes the hipStream_t it runs on.
 *     Calls that return values in host structs synchronise that stream
 *     before returning.
 *   - Inputs are validated before any traversal kernel runs; invalid input
 *     yields RPQ_EINVAL and leaves outputs untouched.
 *   - A graph is read-only after rpq_graph_create: calls from several host
 *     threads may use one graph at once (each with its own workspace and
 *     stream; the server does so), but rpq_graph_destroy must follow them all.
 *     A batch handle is used from one host thread at a time; a server's calls
 *     may come from any thread.
 *   - Device memory: only rpq_graph_create allocates it (the graph); every other
 *     call works in caller-owned device buffers (workspaces, outputs), and
 *     rpq_eval_noalloc in the library's static scratch array.  Host-side
 *     runtime objects created after rpq_graph_create: rpq_eval keeps, per host
 *     thread, a 4 KB pinned staging buffer for counter reads and a second stream
 *     for extraction, and rpq_eval_stream a copy stream (all created on the
 *     thread's first use, kept until the process ends); rpq_batch_create pins a
 *     small control block; rpq_batch_run creates a capture stream, two timing
 *     events and the executable graph of its batch; rpq_serve_start creates one
 *     stream per worker thread and, with the resident engine, a driver thread
 *     with its stream and five pinned buffers (freed by rpq_serve_stop).
 */
#ifndef RPQ_H
#define RPQ_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RPQ_ABI_VERSION 2

/* Automata are epsilon-free NFAs with at most this many states, over at most
 * this many edge labels (labels are uint8 ids below n_labels). */
#define RPQ_MAX_STATES 32
#define RPQ_MAX_LABELS 64

typedef enum {
    RPQ_OK = 0,
    RPQ_EINVAL = -1,       /* bad argument: label >= n_labels, vertex >= n_vertices, unsorted sources ... */
    RPQ_ENOMEM = -2,       /* workspace too small, or a device allocation failed */
    RPQ_EOVERFLOW = -3,    /* output capacity too small; see rpq_result */
    RPQ_EDEVICE = -4,      /* a HIP call failed; the message carries the HIP error string */
    RPQ_EUNSUPPORTED = -5, /* valid request the library does not support (e.g. > 32 states) */
    RPQ_ECANCELED = -6     /* the caller's pair sink asked rpq_eval_stream to stop */
} rpq_status;

/* Thread-local message describing the last failure on this thread ("" if none). */
const char* rpq_last_error(void);

/* RPQ_ABI_VERSION of the loaded library. */
int rpq_abi_version(void);

/* ------------------------------------------------------------------------------------------ */
/* Graph                                                                                      */
/* ------------------------------------------------------------------------------------------ */

/* rpq_graph_create flags */
#define RPQ_BUILD_IN_CSR 1u    /* also build the in-edge CSR (reverse traversal, CRPQ atoms
                                  whose target is fixed) */

typedef struct rpq_graph* rpq_graph_t;   /* opaque; owned by the library */

typedef struct {
    uint32_t n_vertices;
    uint32_t n_labels;
    uint64_t n_edges_in;                         /* edges passed to rpq_graph_create */
    uint64_t n_edges;                            /* distinct (src, label, dst) triples kept */
    uint64_t edges_per_label[RPQ_MAX_LABELS];
    uint64_t nonempty_rows;                      /* (vertex, label) pairs with >= 1 out-edge */
    uint64_t device_bytes;                       /* device memory held by the graph */
    uint32_t has_in_csr;
    uint32_t has_vertex_labels;
} rpq_graph_info;

/*
 * Build the label-partitioned CSR of a graph (the per-label adjacency of the
 * paper's Labeled Grid Format, Section 2.4, kept as one CSR whose rows are
 * (vertex, label) pairs).
 *
 * src, label, dst: device arrays of n_edges entries (uint32 vertex ids below
 *   n_vertices, uint8 label ids below n_labels).  Identical triples are
 *   collapsed (the edge relation is a set); self-loops are kept.
 * vertex_label: device array of n_vertices uint8 vertex labels, or NULL.
 * n_vertices: 1 .. 2^31; n_labels: 1 .. RPQ_MAX_LABELS;
 *   n_vertices * n_labels must stay below 2^32 and distinct edges below 2^32.
 * flags: RPQ_BUILD_IN_CSR or 0.
 * On success *out receives a handle that owns its device memory until
 * rpq_graph_destroy.  The input arrays are not retained.  Allocates device
 * memory (the only entry point that does).
 * Errors: RPQ_EINVAL for out-of-range ids or sizes, RPQ_ENOMEM, RPQ_EDEVICE.
 */
int rpq_graph_create(const uint32_t* src, const uint8_t* label, const uint32_t* dst,
                     uint64_t n_edges, uint32_t n_vertices, uint32_t n_labels,
                     const uint8_t* vertex_label, uint32_t flags, hipStream_t stream,
                     rpq_graph_t* out);

/* Release a graph and its device memory (synchronises the device). */
int rpq_graph_destroy(rpq_graph_t g);

/* Sizes of a graph (host struct). */
int rpq_graph_info_get(rpq_graph_t g, rpq_graph_info* out);

/*
 * Copy the CSR out (device buffers supplied by the caller; any may be NULL):
 *   row_ptr[n_vertices * n_labels + 1] (uint32): edges of vertex v with label l
 *     are dst[row_ptr[v * n_labels + l] .. row_ptr[v * n_labels + l + 1]),
 *     ascending;
 *   dst[n_edges] (uint32).
 * reverse != 0 copies the in-edge CSR (row = (dst, label), entries = src).
 */
int rpq_graph_export_csr(rpq_graph_t g, int reverse, uint32_t* row_ptr, uint32_t* dst,
                         hipStream_t stream);

/* ------------------------------------------------------------------------------------------ */
/* Automaton                                                                                  */
/* ------------------------------------------------------------------------------------------ */

/*
 * An epsilon-free NFA.  delta[q * RPQ_MAX_LABELS + l] is the bitmask of
 * states reachable from state q on label l; entries for q >= n_states or
 * l >= n_labels must be 0.  initial_mask and final_mask are state bitmasks.
 * Host memory.  This plays the role of the paper's automata plan
 * (Section 2.2, Figure 2(a)).
 */
typedef struct {
    uint32_t n_states;
    uint32_t n_labels;
    uint32_t initial_mask;
    uint32_t final_mask;
    uint32_t delta[RPQ_MAX_STATES * RPQ_MAX_LABELS];
} rpq_nfa;

/*
 * Compile a query string into the Glushkov position automaton: state 0 plus
 * one state per label occurrence, so a.b.c* has 4 states.  Syntax:
 *   alt := cat ('|' cat)*        (the paper writes alternation as infix '+')
 *   cat := post (('.' | U+00B7)? post)*
 *   post := atom ('*' | '+' | '?')*       ('+' = one or more, '?' = optional)
 *   atom := LABEL | '(' alt ')'
 * Labels are matched longest-first against label_names[0..n_labels), so
 * "abc*" over names {a, b, c} is a.b.c*.
 * regex, label_names: host NUL-terminated strings.  out: host.
 * Errors: RPQ_EINVAL (syntax, unknown label), RPQ_EUNSUPPORTED (> 31 label
 * occurrences).
 */
int rpq_nfa_compile(const char* regex, const char* const* label_names, uint32_t n_labels,
                    rpq_nfa* out);

/* The automaton of the reversed language: transitions flipped, initial and
 * final masks swapped (WavePlan's reverse plan, Section 2.3).  Host. */
int rpq_nfa_reverse(const rpq_nfa* in, rpq_nfa* out);

/* ------------------------------------------------------------------------------------------ */
/* Plain evaluation: one query, one source set                                                */
/* ------------------------------------------------------------------------------------------ */

/* rpq_eval flags */
#define RPQ_PAIRS        1u   /* write result keys (src << 32) | dst, ascending */
#define RPQ_PER_SOURCE   2u   /* write per-source {count, hash} */
#define RPQ_ALL_SOURCES  4u   /* sources == NULL: every vertex 0 .. n_vertices-1 */
#define RPQ_REVERSE      8u   /* walk in-edges with the reversed automaton: for each given
                                 vertex y, the x with (x, y) in R(rho); keys are (y << 32) | x */
#define RPQ_SPARSE      16u   /* per-source search with a device hash set of (source, state,
                                 vertex) instead of per-unit bitmaps: workspace grows with what
                                 the sources reach, not with V * states * sources (for few
                                 sources on a large graph).  Same results; levels counts the
                                 search's non-empty frontiers. */
#define RPQ_LENGTH_BOUND 32u  /* length-bounded RPQ (the extension named in the paper's conclusion,
                                 Section 10: a length constraint enforced by the traversal depth):
                                 only walks of at most opts->max_length edges count.  The search
                                 stops after depth max_length; a product vertex first reached at
                                 depth d has a walk of exactly d edges and none shorter, so (x, y)
                                 is a result iff some final state is reached at y within the bound.
                                 product_edges counts the edges of expanded product vertices only
                                 (those at depth < max_length). */

/* Tuning knobs; zero fields take defaults (the autotuner's choice when one is cached). */
typedef struct {
    uint32_t batch_width;    /* sources per unit: 64, 128, 256, 512, 1024, 2048 or 4096
                                (0 = the widest up to 2048, or 4096 on graphs of 2^22 vertices
                                or more, that n_sources / 8 fills) */
    uint32_t concurrency;    /* units advanced together (0 = ~64K sources in flight within
                                64 GB of workspace, at least one unit) */
    uint32_t sync_every;     /* levels launched between host checks for the fixpoint (0 = 4) */
    uint32_t chunk_edges;    /* items (edge x successor state) per expansion work slice: entries
                                with more items are cut into slices of this size (0 = 16, raised
                                while the slice buffers would exceed a quarter of a unit's bitmaps) */
    uint32_t max_length;     /* with RPQ_LENGTH_BOUND: the longest walk (in edges) that counts;
                                0 keeps only zero-length walks */
    uint32_t visit;          /* how the expansion finds a target word's new bits (Section 4, the
                                visited check before the update); same results either way.
                                RPQ_VISIT_TWO_READS: read the visited and the Next word, OR the
                                rest into Next; finalize adds each level's Next to the visited
                                bitmap.  RPQ_VISIT_SEEN_OR: read only the visited word and OR the
                                rest into it; finalize takes a row's new bits as the visited word
                                minus a copy of it kept from the previous level.  0 = seen OR
                                (faster on every graph measured). */
} rpq_eval_opts;

#define RPQ_VISIT_TWO_READS 1u
#define RPQ_VISIT_SEEN_OR   2u

/*
 * Result of rpq_eval (host struct).
 *   pairs, capacity: device buffer for keys, or NULL for counts only.  Keys
 *     with global index in [pair_offset, pair_offset + capacity) are written
 *     to pairs[index - pair_offset]; keys are sorted ascending by
 *     (source position, dst).
 *   per_source: device uint64 [n_sources][2] = {count, hash}, or NULL.
 * Out fields: written (keys stored), count (= |R|), hash (sum over keys of
 *   SplitMix64-output(key) mod 2^64), product_edges (sum over reached
 *   (vertex, state) pairs of sum_l deg_l(v) * |delta(q, l)|, summed over
 *   sources), levels (expansion rounds run), max_depth (longest first-reach
 *   distance in the product graph).
 * If count > pair_offset + capacity and pairs != NULL the call returns
 * RPQ_EOVERFLOW after filling the buffer; calling again with pair_offset
 * advanced by capacity continues the same sorted sequence.
 */
typedef struct {
    uint64_t* pairs;
    uint64_t capacity;
    uint64_t* per_source;
    uint64_t pair_offset;
    uint64_t written;
    uint64_t count;
    uint64_t hash;
    uint64_t product_edges;
    uint64_t levels;
    uint64_t max_depth;
    uint64_t workspace_needed;   /* out, on RPQ_ENOMEM: a workspace size to retry with */
} rpq_result;

/* Device workspace bytes rpq_eval needs for this query shape. */
int rpq_eval_workspace_size(rpq_graph_t g, const rpq_nfa* nfa, uint64_t n_sources,
                            uint32_t flags, const rpq_eval_opts* opts, uint64_t* bytes);

/*
 * Evaluate one RPQ from a source set (all-pairs when RPQ_ALL_SOURCES, a slice
 * or a single vertex otherwise; Section 1 distinguishes the all-pairs and
 * single-source forms).
 *
 * sources: device uint32 [n_sources], strictly ascending, each < n_vertices;
 *   NULL with RPQ_ALL_SOURCES (then n_sources must equal n_vertices).
 * workspace: device memory of at least rpq_eval_workspace_size bytes, 256-byte
 *   aligned, owned by the caller; its contents on entry do not matter.
 * Sources are processed in units of batch_width sources, concurrency units at a
 * time; every unit runs its level-synchronous search to the fixpoint (no hop
 * bound).  Synchronises the stream before returning.  When the sources take more
 * than one group of units, each group's extraction runs on a second stream the
 * library keeps per host thread (created on first use), ordered against `stream`
 * by events; all of it is complete when the call returns.
 * Errors: RPQ_EINVAL, RPQ_ENOMEM (workspace too small), RPQ_EOVERFLOW,
 * RPQ_EUNSUPPORTED (RPQ_REVERSE on a graph without in-CSR), RPQ_EDEVICE.
 */
int rpq_eval(rpq_graph_t g, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources,
             uint32_t flags, const rpq_eval_opts* opts, void* workspace, uint64_t workspace_bytes,
             rpq_result* result, hipStream_t stream);

/* Size of the static device scratch used by rpq_eval_noalloc (per device, held until the
 * process ends once the library's code is loaded on that device). */
#define RPQ_NOALLOC_SCRATCH_BYTES (256ull << 20)

/*
 * rpq_eval without any allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, flags and
 * results as rpq_eval, minus the workspace: the call works in a file-scope device array of
 * RPQ_NOALLOC_SCRATCH_BYTES bytes (one per device), and makes no hipMalloc, hipFree,
 * hipHostMalloc, stream or event creation (counters are read through a pageable host buffer,
 * extraction stays on `stream`, profiling is skipped).
 * Plan: zero knobs in opts are narrowed until the workspace fits the scratch (fewer units in
 * flight first, then narrower units); knobs the caller set are kept.
 * The scratch keeps the last call's contents; every call clears what it needs.  Calls on one
 * device share that device's scratch, so calls that overlap in time on one device (other host
 * threads, other streams) race and give wrong results: serialise them.
 * Errors: as rpq_eval; RPQ_ENOMEM (with result->workspace_needed) when even the narrowest plan
 * needs more than RPQ_NOALLOC_SCRATCH_BYTES; RPQ_EUNSUPPORTED for RPQ_SPARSE.
 */
int rpq_eval_noalloc(rpq_graph_t g, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources,
                     uint32_t flags, const rpq_eval_opts* opts, rpq_result* result, hipStream_t stream);

/*
 * Streaming result pairs (Section 6.1: the unified result buffer is split into chunks that are
 * drained to host memory while the traversal goes on, alternating between two buffers so that the
 * transfer of one overlaps the exploration that fills the other).
 *
 * Called once per chunk on the thread that called rpq_eval_stream, in ascending key order: the
 * concatenation of every chunk is the sorted, distinct key sequence (src << 32) | dst of the whole
 * result.  `keys` points into host_chunks and is valid only until the sink returns.  A non-zero
 * return stops the evaluation (RPQ_ECANCELED).
 */
typedef int (*rpq_pair_sink)(const uint64_t* keys, uint64_t n_keys, void* user);

typedef struct {
    uint64_t* device_chunks;   /* device, 2 * chunk_keys keys, caller-owned */
    uint64_t* host_chunks;     /* pinned host memory (hipHostMalloc or equivalent), 2 * chunk_keys
                                  keys, caller-owned */
    uint64_t chunk_keys;       /* keys per chunk, >= 1 */
    rpq_pair_sink sink;
    void* user;                /* passed to sink */
} rpq_pair_stream;

/*
 * rpq_eval with the result keys streamed to host memory instead of written to one device
 * buffer: there is no capacity limit and no second traversal.  Per group of units (see rpq_eval)
 * the keys are counted, then written window by window into the two device chunks in turn; each
 * chunk is copied to its host chunk on a copy stream and handed to the sink.  While the sink runs
 * and the copies go on, the next window is extracted and the next group's levels run.
 * Arguments as rpq_eval (RPQ_PAIRS is implied; result->pairs and capacity are ignored); size the
 * workspace with rpq_eval_workspace_size(..., flags | RPQ_PAIRS, ...).  On return result->count,
 * hash, per_source (with RPQ_PER_SOURCE) and written (keys delivered) are set.  Uses the thread's
 * extraction stream (as rpq_eval) and a copy stream created per host thread on first use.
 * Errors: as rpq_eval (RPQ_EOVERFLOW does not occur); RPQ_EINVAL for a NULL or empty stream
 * description; RPQ_EUNSUPPORTED with RPQ_SPARSE; RPQ_ECANCELED when the sink returns non-zero (the
 * keys delivered so far are in result->written; no work of the call is left on any stream).
 */
int rpq_eval_stream(rpq_graph_t g, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources,
                    uint32_t flags, const rpq_eval_opts* opts, void* workspace, uint64_t workspace_bytes,
                    const rpq_pair_stream* out, rpq_result* result, hipStream_t stream);

/* ------------------------------------------------------------------------------------------ */
/* Split plans: a materialized sub-result joined with the rest of the expression              */
/* ------------------------------------------------------------------------------------------ */

/*
 * WavePlan's loop-cache and start-in-the-middle plans (Section 2.3), executed as Section 6
 * describes: one sub-RPQ's result is materialized in one direction and then joined with the rest
 * of the expression.  For rho = head . tail (concatenation), walks split at the boundary, so
 * R(rho) = { (x, y) : (x, m) in R(head) and (m, y) in R(tail) for some m }.  rpq_eval_split runs
 *   1. head from the sources; the distinct targets are the middle vertices M;
 *   2. tail from M (exploration starts in the middle of the expression), its pairs materialized
 *      as edges m -lambda-> y of a new label lambda = n_labels of the graph;
 *   3. head . lambda (rpq_nfa_append_label) over the graph with lambda added, from the sources.
 * A split after a closure's prefix (head = a.b, tail = c*) is the loop-cache plan: the closure is
 * explored once per middle vertex instead of once per unit of sources reaching it.
 *
 * The keys, count, checksum and per-source tallies equal rpq_eval's on the concatenated
 * expression; product_edges, levels and max_depth describe step 3's product graph.
 * flags: RPQ_PAIRS, RPQ_PER_SOURCE, RPQ_ALL_SOURCES only (RPQ_EUNSUPPORTED otherwise); result as
 * for rpq_eval (its buffers are the caller's; RPQ_EOVERFLOW with pair_offset resumes, each call
 * running the whole plan).  The graph needs fewer than RPQ_MAX_LABELS labels and head fewer than
 * RPQ_MAX_STATES states.  Unlike rpq_eval the call allocates device memory for the steps'
 * workspaces, the materialized relation and the derived graph, frees it before returning, and
 * synchronises the stream.  info (host, nullable) receives the sizes of the steps.
 */
typedef struct {
    uint64_t head_pairs;        /* pairs of step 1 */
    uint64_t middle_vertices;   /* |M| */
    uint64_t tail_pairs;        /* pairs of step 2: the lambda edges */
    uint64_t derived_edges;     /* distinct edges of the derived graph */
} rpq_split_info;

int rpq_eval_split(rpq_graph_t g, const rpq_nfa* head, const rpq_nfa* tail, const uint32_t* sources,
                   uint64_t n_sources, uint32_t flags, const rpq_eval_opts* opts, rpq_result* result,
                   rpq_split_info* info, hipStream_t stream);

/* The automaton of L(in) . label: one new state, entered on `label` from every final state of
 * `in`, and the only final state.  Host.  Errors: RPQ_EINVAL for n_states >= RPQ_MAX_STATES or a
 * label id >= RPQ_MAX_LABELS. */
int rpq_nfa_append_label(const rpq_nfa* in, uint32_t label, rpq_nfa* out);

/* ------------------------------------------------------------------------------------------ */
/* Batched evaluation: many queries in one persistent, graph-captured launch                  */
/* ------------------------------------------------------------------------------------------ */

/*
 * A batch holds RPQs over one graph -- each with its own automaton, source set
 * and result mode -- and evaluates all of them with one persistent kernel:
 * queries are cut into units of at most batch_width sources, `slots` units
 * advance level by level together, and a slot whose unit reaches its
 * fixpoint is retired and refilled from the device-side unit queue in the
 * same iteration (the role of the paper's traversal queue feeding the
 * exploration kernel, Section 4.2 and Algorithm 1, without host round trips).
 * The launch sequence is captured once into a hipGraph and replayed by
 * rpq_batch_run.  Results are identical to rpq_eval of each query alone.
 */
typedef struct rpq_batch* rpq_batch_t;

typedef struct {
    uint32_t batch_width;   /* sources per unit: 64 .. 4096, power of two (0 = 512) */
    uint32_t slots;         /* units advanced together (0 = sized for ~64K sources in flight, <= 64 GB) */
    uint32_t chunk_edges;   /* items (edge x successor state) per work slice (0 = 16, raised while the
                               slice buffers would exceed a quarter of a slot's bitmaps) */
    uint32_t list_share;    /* frontier lists, slice buffers and first-visit logs hold 1/list_share of
                               the worst case (every row of every slot in one level); rows beyond wait
                               for the next iteration, which changes no result (0 = 4, or 1 when a
                               query is length-bounded: such queries need exact depths and require 1) */
    uint32_t visit;         /* the expansion's visit scheme, RPQ_VISIT_TWO_READS or RPQ_VISIT_SEEN_OR
                               (0 = seen OR on graphs of 2^22 vertices or more, two reads below).
                               The batched kernel's seen OR ORs each new word into the visited word
                               and into Next */
} rpq_batch_opts;

typedef struct {
    uint32_t n_queries, n_units, slots, batch_width, blocks;
    uint32_t visit;              /* visit scheme of the plan: RPQ_VISIT_TWO_READS or RPQ_VISIT_SEEN_OR */
    uint64_t workspace_bytes;
    uint64_t iterations;         /* level iterations of the last run */
    uint64_t edge_items, descriptors, word_reads, word_updates;   /* expansion tallies, last run */
    uint64_t finalized_rows, finalized_words;   /* finalize tallies: rows, non-zero next words */
    uint64_t touch_words;        /* touch-bitmap words scanned per iteration */
    uint64_t row_words;          /* K: 64-bit words per (state, vertex) row */
    double last_run_ms;          /* device time of the last graph launch */
    double last_kernel_ms;       /* device time of the persistent kernel in it */
    double phase_ms[8];          /* persistent-kernel time per phase: expand, compact, decide,
                                    retire extract, retire keys, retire clear, refill+seed, finalize */
} rpq_batch_info;

/* Create an empty batch over graph g (host object with a small pinned control block; no device
 * memory). opts may be NULL. */
int rpq_batch_create(rpq_graph_t g, const rpq_batch_opts* opts, rpq_batch_t* out);

/* Destroy a batch and its captured graph. */
int rpq_batch_destroy(rpq_batch_t b);

/*
 * Add one query.  nfa: host, copied.  sources: device uint32 [n_sources],
 * strictly ascending (checked on the device at the first run), or NULL with
 * RPQ_ALL_SOURCES.  flags: RPQ_PAIRS (pairs: device uint64 [capacity]; keys
 * sorted as in rpq_eval; capacity must hold the whole result, else the query
 * reports RPQ_EOVERFLOW and the buffer content is unspecified),
 * RPQ_PER_SOURCE (per_source: device uint64 [n_sources][2]), RPQ_ALL_SOURCES.
 * Device buffers must stay valid until the last rpq_batch_run.  *query_id
 * receives the query's index.  Queries cannot be added after the first run.
 */
int rpq_batch_add(rpq_batch_t b, const rpq_nfa* nfa, const uint32_t* sources, uint64_t n_sources,
                  uint32_t flags, uint64_t* pairs, uint64_t capacity, uint64_t* per_source,
                  uint32_t* query_id);

/*
 * Make query query_id of the batch length-bounded (as RPQ_LENGTH_BOUND in rpq_eval): only walks
 * of at most max_length edges count.  Call before the first run.  Errors: RPQ_EINVAL for an
 * unknown query or a batch that already ran.
 */
int rpq_batch_bound_length(rpq_batch_t b, uint32_t query_id, uint32_t max_length);

/* Device workspace bytes the batch needs (fixes the unit/slot plan). */
int rpq_batch_workspace_size(rpq_batch_t b, uint64_t* bytes);

/*
 * Run every query of the batch to its fixpoint: one graph launch (reset
 * kernels, the persistent kernel, the key gather) on `stream`, captured on the
 * first run with this workspace.  Synchronises the stream.  workspace: device,
 * 256-byte aligned, >= rpq_batch_workspace_size bytes, caller-owned; reusing
 * the same workspace replays the captured graph.
 * Errors: RPQ_EINVAL (bad sources), RPQ_ENOMEM, RPQ_EDEVICE (including a grid
 * barrier that timed out because the persistent grid was not co-resident).
 */
int rpq_batch_run(rpq_batch_t b, void* workspace, uint64_t workspace_bytes, hipStream_t stream);

/* Per-query results of the last run (host struct; counts, checksum, product edges, depth). */
int rpq_batch_result(rpq_batch_t b, uint32_t query_id, rpq_result* out);

/* Plan and tallies of the batch (host struct). */
int rpq_batch_stats(rpq_batch_t b, rpq_batch_info* out);

/*
 * Autotune the batch's unit width, slot count and slice size: each
 * candidate (default set: widths 64..2048 x chunk 16/64 items, slots sized
 * automatically) whose plan fits in workspace_bytes runs a bounded prefix of
 * the unit queue twice (capture, then replay), and the candidate with the most
 * sources per millisecond on the replay wins.  The batch is re-planned with the
 * winner (written to *best if non-NULL) and recaptured on its next run.
 * Results of the timing runs are not meaningful; call rpq_batch_run afterwards.
 * candidates: host array or NULL.  Errors: RPQ_ENOMEM if no candidate fits.
 */
int rpq_batch_autotune(rpq_batch_t b, const rpq_batch_opts* candidates, uint32_t n_candidates,
                       void* workspace, uint64_t workspace_bytes, hipStream_t stream,
                       rpq_batch_opts* best);

/* ------------------------------------------------------------------------------------------ */
/* Conjunctive regular path queries                                                           */
/* ------------------------------------------------------------------------------------------ */

#define CRPQ_MAX_VARS 16
#define CRPQ_MAX_ATOMS 16

/* One atom x -rho-> y of a CRPQ (Definition 2): rho as an epsilon-free NFA (host struct). */
typedef struct {
    uint32_t src_var, dst_var;   /* variable ids below n_vars; src_var == dst_var is allowed */
    rpq_nfa nfa;
} crpq_atom;

/* The query's variables (host struct; every pointer may be NULL = no constraint of that kind).
 *   binding[i]       >= 0 fixes variable i to that vertex (a constant of the query); -1 = free
 *   vertex_label[i]  >= 0 requires the vertex label of f(i) to equal it (Definition 2,
 *                    condition 1); -1 = any.  Needs a graph created with vertex labels.
 *   domain[i]        device array of domain_size[i] vertex ids (any order, duplicates allowed):
 *                    f(i) must be one of them (a sample of the vertex set); NULL = any
 *   neq[2 j], neq[2 j + 1]   pairs of variables that must map to different vertices
 * Variables that appear in no atom range over their domain (a cartesian factor). */
typedef struct {
    uint32_t n_vars;
    const int64_t* binding;
    const int32_t* vertex_label;
    const uint32_t* const* domain;
    const uint64_t* domain_size;
    const uint32_t* neq;
    uint32_t n_neq;
} crpq_vars;

/* crpq_eval flags: how atoms are traversed (default: chosen per atom, see crpq_eval) */
#define CRPQ_FORCE_DENSE   1u   /* every multi-step atom by the bit-parallel traversal */
#define CRPQ_FORCE_SPARSE  2u   /* every multi-step atom by the per-source hash-set search */
#define CRPQ_NO_EDGE_SCAN  4u   /* single-label atoms are traversed like the others */
#define CRPQ_NO_REVERSE    8u   /* never traverse an atom backwards */
#define CRPQ_BATCH_ATOMS  16u   /* the atoms that run bit-parallel and forward from their source
                                   variable's domain run together in the batched persistent form
                                   (rpq_batch_*): one run counts their pairs, a second writes them.
                                   They then start from the domains as the constraints fix them,
                                   before the semi-join reductions of the other atoms narrow them;
                                   when the join reaches such an atom its pairs are restricted to the
                                   reduced domains, so the result is the same.  Creates a batch and
                                   its capture stream for the call; device memory from the workspace. */

/* Per-atom strategy codes reported in crpq_result.atom_strategy */
#define CRPQ_STRATEGY_EDGE_SCAN 1u
#define CRPQ_STRATEGY_DENSE     2u
#define CRPQ_STRATEGY_SPARSE    3u
#define CRPQ_STRATEGY_REVERSED  0x100u   /* or-ed in when the atom ran backwards from dst_var */
#define CRPQ_STRATEGY_BATCHED   0x200u   /* or-ed in when the atom ran in the batched form */

/* Result of crpq_eval (host struct).
 *   tuples, capacity: device buffer of capacity rows of n_free uint32 (row-major), or NULL
 *     for count and checksum only.  Rows are the distinct assignments of the free variables
 *     (those without a binding) in declared order, sorted lexicographically.
 *   count: number of distinct rows; hash: sum over rows of the chained mix
 *     m = mix64(v_1), m = mix64(m ^ v_i) for i = 2 .. n_free, modulo 2^64 (order-free).
 *   written: rows written (min(count, capacity)).
 *   workspace_needed: on RPQ_ENOMEM, a workspace size to retry with.
 *   atom_pairs / atom_strategy: per atom, the size of its relation after the domain filters
 *     and how it was evaluated; join_rows: largest intermediate table of the join. */
typedef struct {
    uint32_t* tuples;
    uint64_t capacity;
    uint64_t count, hash, written;
    uint32_t n_free, reserved;
    uint64_t workspace_needed;
    uint64_t atom_pairs[CRPQ_MAX_ATOMS];
    uint32_t atom_strategy[CRPQ_MAX_ATOMS];
    uint64_t join_rows;
} crpq_result;

/*
 * Evaluate a CRPQ (Definition 2): every homomorphism f from the variables to vertices with
 * f(x) -> f(y) joined by a walk whose label word is in L(rho) for every atom, the vertex-label
 * condition, the bindings, domains and inequalities.  The atoms are evaluated first and their
 * results joined (Section 6.2):
 *   1. domains: one bitmap of V bits per variable (binding, label, domain intersected);
 *   2. atoms, smallest source domain first, each traversed from the smaller of its two
 *      domains (backwards on the in-CSR when that is dst_var's), its result restricted to
 *      both domains; after each atom the domains of its variables shrink to the values that
 *      occur in its result (semi-join reduction).  An atom whose language holds only
 *      one-label words is an edge scan; otherwise up to 65,536 sources take the bit-parallel
 *      traversal of rpq_eval and more take a per-source search with a device hash set;
 *   3. join: variables are bound one at a time in a matching order (constants and small
 *      domains first, then the variable most connected to bound ones); for each partial row
 *      the candidates of the new variable come from the shortest list among the atoms that
 *      connect it to bound variables, and are checked against the other atoms, its domain
 *      and the inequalities.  An atom needed in the direction opposite to how it was
 *      materialised is transposed first.  When tuples == NULL the last variable is counted
 *      and hashed without being materialised.
 * graph: created with RPQ_BUILD_IN_CSR for backward traversal (else forward only).
 * workspace: device, 256-byte aligned; every intermediate lives in it.  If it is too small the
 *   call returns RPQ_ENOMEM with res->workspace_needed set: call again with that much.
 * Errors: RPQ_EINVAL (bad variable ids, vertex ids, labels, automata, n_vars == 0 or above
 *   CRPQ_MAX_VARS, n_atoms above CRPQ_MAX_ATOMS, vertex labels without graph labels),
 *   RPQ_EOVERFLOW (count > capacity: the first capacity rows are written, count and hash are
 *   complete), RPQ_ENOMEM, RPQ_EUNSUPPORTED (states * vertices >= 2^32), RPQ_EDEVICE.
 */
int crpq_eval(rpq_graph_t graph, const crpq_atom* atoms, uint32_t n_atoms, const crpq_vars* vars,
              uint32_t flags, void* workspace, uint64_t workspace_bytes, crpq_result* res,
              hipStream_t stream);

/* ------------------------------------------------------------------------------------------ */
/* Serving: continuous admission of requests over one resident graph                          */
/* ------------------------------------------------------------------------------------------ */

/*
 * A server keeps one graph resident and runs requests (RPQs and CRPQs) as they arrive.  Each
 * request needs a workspace: its visited sets (per-unit bitmaps of V * states * unit-width bits,
 * or the hash set of RPQ_SPARSE) and its traversal state.  Workspaces are carved from one device
 * pool that the caller hands over at start (first fit, 256-byte aligned); the server never
 * allocates device memory.  A request is admitted when its workspace fits in the free part of
 * the pool (a request may pass queued ones that do not fit yet, unless the oldest has waited
 * more than 50 ms), and runs at once on one of `workers` host threads, each with its own HIP
 * stream, so the work of admitted requests overlaps on the device.  A dense RPQ larger than the
 * whole pool is split: fewer source units in flight (and narrower units), the same result.  A
 * request that asks for more workspace while running (RPQ_SPARSE, CRPQ) goes back to the front
 * of the queue with the larger size.  This is the counterpart, across requests, of the paper's
 * pooled segment memory (Section 5) and of its temporary reduction of the start-vertex batch when
 * that pool runs short (ablation study, Section 8.4).
 * With the resident engine on, dense RPQs skip the worker streams: a persistent batched kernel
 * (rpq_batch_* form, open-ended) keeps its slots on the device and a driver thread appends each
 * arriving request's units to the kernel's device unit queue between launches of a few
 * iterations; idle slots take them at the next refill, so requests that arrive while others run
 * are admitted as slots free up and their levels advance in the same launches (the counterpart of
 * the paper's traversal queue feeding the exploration kernel, Section 4.2 and Algorithm 1).
 * Results are identical to running each request alone.
 */
typedef struct rpq_server* rpq_server_t;

typedef struct {
    uint32_t workers;          /* requests in flight at once on the worker streams (0 = 4) */
    uint32_t reserved;         /* must be 0 */
    /* Resident engine (0 slots = off): a persistent batched kernel whose slots stay on the
     * device.  Dense RPQ requests it can run (automaton of at most resident_states states and
     * resident_succ successors per (state, label); pairs only when the sources fit one unit) join
     * its device unit queue as they arrive, between bounded launches of resident_iters
     * iterations, and take slots as earlier units retire.  Its slot memory comes from the front
     * of the pool; every other request runs on the worker streams in the rest of it. */
    uint32_t resident_slots;   /* slots (units in flight) */
    uint32_t resident_width;   /* sources per unit: 64 .. 4096, a power of two (0 = 64) */
    uint32_t resident_states;  /* largest automaton (0 = 12) */
    uint32_t resident_succ;    /* largest successor set per (state, label) (0 = 4) */
    uint32_t resident_iters;   /* iterations per launch (0 = 8) */
    uint32_t resident_max_units; /* requests of more units (sources / width, rounded up) go to the
                                  workers, whose units can be wider (0 = no limit) */
} rpq_server_opts;

#define RPQ_REQ_RPQ  1u
#define RPQ_REQ_CRPQ 2u

/* One request (host struct, copied by rpq_serve_submit; device buffers it names must stay
 * valid until the request is done). */
typedef struct {
    uint32_t kind;                /* RPQ_REQ_RPQ or RPQ_REQ_CRPQ */
    uint32_t flags;               /* rpq_eval flags (RPQ_REQ_RPQ) or crpq_eval flags (RPQ_REQ_CRPQ) */
    double arrival_ms;            /* scheduled arrival on the server clock (rpq_serve_clock_ms), or
                                     < 0 for the time of submission; latency is measured from it */
    /* RPQ_REQ_RPQ: as rpq_eval */
    rpq_nfa nfa;
    const uint32_t* sources;      /* device, ascending; NULL with RPQ_ALL_SOURCES */
    uint64_t n_sources;
    uint64_t* pairs;              /* device [capacity] or NULL */
    uint64_t capacity;
    uint64_t* per_source;         /* device [n_sources][2] or NULL */
    /* RPQ_REQ_CRPQ: as crpq_eval (host arrays are copied; domain arrays are device memory) */
    const crpq_atom* atoms;
    uint32_t n_atoms;
    crpq_vars vars;
    uint32_t* tuples;             /* device [tuple_capacity][n_free] or NULL */
    uint64_t tuple_capacity;
} rpq_request;

/* State of one request (host struct). */
typedef struct {
    int32_t status;               /* rpq_status once done (RPQ_EOVERFLOW: outputs truncated) */
    uint32_t done;                /* 0 while queued or running */
    uint64_t count, hash, product_edges, written;
    uint64_t workspace_bytes;     /* pool bytes the request ran with (one slot's share on the
                                     resident engine) */
    double arrival_ms, start_ms, end_ms;   /* server clock; start = admitted to a worker or to the
                                     resident engine's queue */
    uint32_t resident;            /* 1 when the resident engine ran the request */
    uint32_t reserved;
} rpq_ticket;

typedef struct {
    uint64_t submitted, completed, failed, queued, running;
    uint64_t pool_bytes, pool_in_use, pool_peak;
    uint64_t product_edges;       /* over completed requests */
    uint64_t resident_completed;  /* requests the resident engine completed */
    uint64_t resident_launches;   /* launches of the resident kernel */
    uint64_t resident_bytes;      /* pool bytes held by the resident engine */
} rpq_server_stats;

/* Start a server on graph g with the device pool [pool, pool + pool_bytes) (256-byte aligned). */
int rpq_serve_start(rpq_graph_t g, const rpq_server_opts* opts, void* pool, uint64_t pool_bytes,
                    rpq_server_t* out);
/* Queue a request; *ticket identifies it.  RPQ_ENOMEM if it can never fit in the pool,
 * RPQ_EINVAL for a malformed request (checked before queueing). */
int rpq_serve_submit(rpq_server_t s, const rpq_request* req, uint64_t* ticket);
/* Current state of a request (done = 0 while pending). */
int rpq_serve_poll(rpq_server_t s, uint64_t ticket, rpq_ticket* out);
/* Block until the request is done, then as rpq_serve_poll. */
int rpq_serve_wait(rpq_server_t s, uint64_t ticket, rpq_ticket* out);
/* Milliseconds since rpq_serve_start on the server's monotonic clock. */
int rpq_serve_clock_ms(rpq_server_t s, double* out);
int rpq_serve_stats(rpq_server_t s, rpq_server_stats* out);
/* Finish every queued and running request, join the workers and free the server. */
int rpq_serve_stop(rpq_server_t s);

/* ------------------------------------------------------------------------------------------ */
/* Profiling of the traversal kernels                                                         */
/* ------------------------------------------------------------------------------------------ */

/*
 * Process-wide counters of the level kernels, accumulated over rpq_eval
 * calls while enabled (host struct).  Durations come from HIP events
 * recorded on the caller's stream around each launch; the work counts are
 * exact device-side tallies of the expansion kernel:
 *   edge_items    items expanded: (frontier entry, edge, successor state), each reading one
 *                 4-byte neighbour id
 *   descriptors   work segments: light frontier entries taken whole from the list and 16-byte
 *                 slices of heavy ones
 *   row_words     8-byte frontier words read (K per segment)
 *   word_reads    8-byte visited words read, each with the 8-byte next-frontier word beside it
 *                 (frontier word != 0)
 *   word_updates  8-byte atomic ORs into the next-frontier bitmap (bits not yet there)
 * and of finalize (finalize_*) and of the extraction's count passes (extract_*).
 */
typedef struct {
    uint64_t expand_launches;
    double expand_ms;
    uint64_t finalize_launches;
    double finalize_ms;
    uint64_t edge_items;
    uint64_t descriptors;
    uint64_t row_words;
    uint64_t word_reads;
    uint64_t word_updates;
    uint64_t finalize_rows;      /* rows moved from Next to the frontier by finalize */
    uint64_t finalize_row_words; /* their 8-byte words (each read from Next, written to the frontier) */
    uint64_t finalize_words;     /* their non-zero 8-byte Next words (each cleared) */
    uint64_t finalize_vis_words; /* 8-byte accesses of finalize to Vis: with two reads a read and a
                                    write of each non-zero word; with seen OR a read of each row
                                    word (its new bits are Vis minus the previous level's copy) */
    uint64_t finalize_ans_words; /* those of final-state rows (each also ORed into Ans) */
    uint64_t extract_launches;   /* extraction count passes, timed on the extraction stream */
    double extract_ms;
    uint64_t extract_words;      /* 8-byte answer words those passes read */
    uint64_t expand_extra_words; /* 8-byte accesses of the expansion beyond the method's: the Next
                                    word read beside each visited word (two reads); none with
                                    seen OR */
} rpq_profile;

/* Turn event timing of the level kernels on (1) or off (0).  Process-wide. */
int rpq_profile_enable(int on);

/* Copy the accumulated counters to *out (host); reset them when reset != 0. */
int rpq_profile_read(rpq_profile* out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* RPQ_H */
