// Graph ingest: edge list -> label-partitioned CSR on the device.
//
// The paper keeps one adjacency per edge label (Labeled Grid Format,
// Section 2.4) so a traversal can follow exactly the edges an automaton
// transition asks for.  Here every (vertex, label) pair is one CSR row, rows
// ordered vertex-major so all label rows of a vertex share cache lines, and a
// per-vertex label bitmask lets the traversal skip labels with no edges.
//
// Steps (all on the device): pack (row, neighbour) into a uint64 key, stable
// radix sort, drop repeated keys (the edge relation is a set), then derive
// row pointers by binary search over the sorted keys and the label masks
// from non-empty rows.  The in-edge CSR is the same construction with source
// and destination swapped.
#include "internal.h"

#include <cstring>
#include <new>

namespace {

constexpr int kThreads = 256;

unsigned grid_for(uint64_t n, uint64_t cap = 65535) {
    uint64_t b = (n + kThreads - 1) / kThreads;
    if (b > cap) b = cap;
    return (unsigned)(b ? b : 1);
}

__global__ void k_make_keys(const uint32_t* __restrict__ a, const uint8_t* __restrict__ lab,
                            const uint32_t* __restrict__ b, uint64_t n, uint32_t V, uint32_t L,
                            uint64_t* __restrict__ keys, unsigned long long* __restrict__ err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t x = a[i], y = b[i], l = lab[i];
        if (x >= V || y >= V || l >= L) {
            atomicOr(err, 1ull);
            keys[i] = 0;
            continue;
        }
        keys[i] = ((uint64_t)(x * L + l) << 32) | y;
    }
}

__global__ void k_mark_first(const uint64_t* __restrict__ keys, uint64_t n, uint64_t* __restrict__ flag) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__global__ void k_compact(const uint64_t* __restrict__ keys, const uint64_t* __restrict__ pos, uint64_t n,
                          uint64_t* __restrict__ ukeys, uint32_t* __restrict__ dst, uint32_t L,
                          unsigned long long* __restrict__ per_label) {
    __shared__ unsigned long long cnt[RPQ_MAX_LABELS];
    for (int i = threadIdx.x; i < RPQ_MAX_LABELS; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t k = keys[i];
        if (i == 0 || k != keys[i - 1]) {
            const uint64_t p = pos[i];
            ukeys[p] = k;
            dst[p] = (uint32_t)k;
            atomicAdd(&cnt[(uint32_t)(k >> 32) % L], 1ull);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (int)L; i += blockDim.x)
        if (cnt[i]) atomicAdd(&per_label[i], cnt[i]);
}

// row_ptr[r] = first index whose row id (upper key word) is >= r, r in [0, R]
__global__ void k_row_ptr(const uint64_t* __restrict__ ukeys, uint64_t m, uint64_t R,
                          uint32_t* __restrict__ row_ptr) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= R; r += stride) {
        uint64_t lo = 0, hi = m;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if ((ukeys[mid] >> 32) < r) lo = mid + 1;
            else hi = mid;
        }
        row_ptr[r] = (uint32_t)lo;
    }
}

__global__ void k_label_mask(const uint32_t* __restrict__ row_ptr, uint32_t V, uint32_t L,
                             uint64_t* __restrict__ lmask, unsigned long long* __restrict__ nonempty) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t local = 0;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += stride) {
        uint64_t m = 0;
        const uint32_t* r = row_ptr + v * L;
        for (uint32_t l = 0; l < L; ++l)
            if (r[l + 1] > r[l]) m |= 1ull << l;
        lmask[v] = m;
        local += __popcll(m);
    }
    local = rpqd::wave_sum_u64(local);
    if ((threadIdx.x & 63) == 0 && local) atomicAdd(nonempty, (unsigned long long)local);
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

int dev_alloc(void** p, uint64_t bytes) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 8);
    if (e != hipSuccess) {
        *p = nullptr;
        rpq::set_error("hipMalloc(%llu) failed: %s", (unsigned long long)bytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? RPQ_ENOMEM : RPQ_EDEVICE;
    }
    return RPQ_OK;
}

// Build one CSR direction.  a/b: row-side and neighbour-side endpoint arrays.
int build_csr(const uint32_t* a, const uint8_t* lab, const uint32_t* b, uint64_t n_edges, uint32_t V,
              uint32_t L, rpq::Csr* out, uint64_t* E_out, uint64_t* per_label, uint64_t* stage,
              hipStream_t s) {
    using namespace rpq;
    const uint64_t R = (uint64_t)V * L;
    const uint64_t ne = n_edges ? n_edges : 1;
    DevBuf keys, alt, flag, sort_tmp, ctr, uk;
    RPQ_TRY(dev_alloc(&keys.p, ne * 8));
    RPQ_TRY(dev_alloc(&alt.p, ne * 8));
    RPQ_TRY(dev_alloc(&flag.p, (ne + scan_temp_elems(ne) + 1) * 8));
    RPQ_TRY(dev_alloc(&sort_tmp.p, radix_temp_bytes(ne)));
    RPQ_TRY(dev_alloc(&ctr.p, (4 + RPQ_MAX_LABELS) * 8));
    unsigned long long* c = reinterpret_cast<unsigned long long*>(ctr.p);   // [0] err [1] total [2] nonempty
    unsigned long long* pl = c + 4;
    RPQ_TRY(fill_u64(reinterpret_cast<uint64_t*>(c), 4 + RPQ_MAX_LABELS, 0, s));
    uint64_t* k = reinterpret_cast<uint64_t*>(keys.p);
    if (n_edges) {
        hipLaunchKernelGGL(k_make_keys, dim3(grid_for(n_edges)), dim3(kThreads), 0, s, a, lab, b, n_edges, V, L,
                           k, c);
        RPQ_LAUNCH_CHECK();
    }
    RPQ_HIP(hipMemcpyAsync(stage, c, 8, hipMemcpyDeviceToHost, s));
    RPQ_HIP(hipStreamSynchronize(s));
    if (stage[0]) {
        set_error("edge list holds a vertex id >= n_vertices or a label id >= n_labels");
        return RPQ_EINVAL;
    }
    uint64_t* sorted = k;
    RPQ_TRY(radix_sort_u64(k, reinterpret_cast<uint64_t*>(alt.p), n_edges, bits_for(V ? V - 1 : 0),
                           bits_for(R ? R - 1 : 0), sort_tmp.p, s, &sorted));
    uint64_t* other = sorted == k ? reinterpret_cast<uint64_t*>(alt.p) : k;
    uint64_t* fl = reinterpret_cast<uint64_t*>(flag.p);
    uint64_t E = 0;
    if (n_edges) {
        hipLaunchKernelGGL(k_mark_first, dim3(grid_for(n_edges)), dim3(kThreads), 0, s, sorted, n_edges, fl);
        RPQ_LAUNCH_CHECK();
        RPQ_TRY(exclusive_scan_u64(fl, fl, n_edges, fl + ne + 1, reinterpret_cast<uint64_t*>(c + 1), s));
        RPQ_HIP(hipMemcpyAsync(stage, c + 1, 8, hipMemcpyDeviceToHost, s));
        RPQ_HIP(hipStreamSynchronize(s));
        E = stage[0];
    }
    if (E >= 0xFFFFFFFFull) {
        set_error("more than 2^32-1 distinct edges");
        return RPQ_EUNSUPPORTED;
    }
    RPQ_TRY(dev_alloc(reinterpret_cast<void**>(&out->dst), (E ? E : 1) * 4));
    RPQ_TRY(dev_alloc(reinterpret_cast<void**>(&out->row_ptr), (R + 1) * 4));
    RPQ_TRY(dev_alloc(reinterpret_cast<void**>(&out->lmask), (uint64_t)V * 8));
    if (n_edges) {
        hipLaunchKernelGGL(k_compact, dim3(grid_for(n_edges, 8192)), dim3(kThreads), 0, s, sorted, fl, n_edges,
                           other, out->dst, L, pl);
        RPQ_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_row_ptr, dim3(grid_for(R + 1)), dim3(kThreads), 0, s, other, E, R, out->row_ptr);
    RPQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_label_mask, dim3(grid_for(V, 8192)), dim3(kThreads), 0, s, out->row_ptr, V, L,
                       out->lmask, c + 2);
    RPQ_LAUNCH_CHECK();
    RPQ_HIP(hipMemcpyAsync(stage, c, (4 + RPQ_MAX_LABELS) * 8, hipMemcpyDeviceToHost, s));
    RPQ_HIP(hipStreamSynchronize(s));
    out->nonempty_rows = stage[2];
    if (per_label)
        for (uint32_t l = 0; l < L; ++l) per_label[l] = stage[4 + l];
    *E_out = E;
    return RPQ_OK;
}

void free_csr(rpq::Csr* c) {
    if (c->row_ptr) (void)hipFree(c->row_ptr);
    if (c->dst) (void)hipFree(c->dst);
    if (c->lmask) (void)hipFree(c->lmask);
    *c = rpq::Csr();
}

void free_graph(rpq_graph* g) {
    if (!g) return;
    free_csr(&g->out);
    free_csr(&g->in);
    if (g->vlabel) (void)hipFree(g->vlabel);
    if (g->h_stage) (void)hipHostFree(g->h_stage);
    delete g;
}

}  // namespace

extern "C" {

int rpq_graph_create(const uint32_t* src, const uint8_t* label, const uint32_t* dst, uint64_t n_edges,
                     uint32_t n_vertices, uint32_t n_labels, const uint8_t* vertex_label, uint32_t flags,
                     hipStream_t stream, rpq_graph_t* out) {
    rpq::clear_error();
    if (!out) {
        rpq::set_error("out is NULL");
        return RPQ_EINVAL;
    }
    *out = nullptr;
    if (n_vertices == 0 || n_vertices > (1u << 31)) {
        rpq::set_error("n_vertices must be in [1, 2^31]");
        return RPQ_EINVAL;
    }
    if (n_labels == 0 || n_labels > RPQ_MAX_LABELS) {
        rpq::set_error("n_labels must be in [1, %d]", RPQ_MAX_LABELS);
        return RPQ_EINVAL;
    }
    if ((uint64_t)n_vertices * n_labels >= 0xFFFFFFFFull) {
        rpq::set_error("n_vertices * n_labels must be below 2^32");
        return RPQ_EINVAL;
    }
    if (n_edges && (!src || !label || !dst)) {
        rpq::set_error("edge arrays are NULL");
        return RPQ_EINVAL;
    }
    if (flags & ~RPQ_BUILD_IN_CSR) {
        rpq::set_error("unknown flags 0x%x", flags);
        return RPQ_EINVAL;
    }
    rpq_graph* g = new (std::nothrow) rpq_graph();
    if (!g) {
        rpq::set_error("host allocation failed");
        return RPQ_ENOMEM;
    }
    g->V = n_vertices;
    g->L = n_labels;
    g->E_in = n_edges;
    if (hipGetDevice(&g->device) != hipSuccess || hipHostMalloc(reinterpret_cast<void**>(&g->h_stage), 4096) !=
                                                      hipSuccess) {
        rpq::set_error("HIP device or pinned staging unavailable");
        free_graph(g);
        return RPQ_EDEVICE;
    }
    int rc = build_csr(src, label, dst, n_edges, n_vertices, n_labels, &g->out, &g->E, g->per_label, g->h_stage,
                       stream);
    if (rc == RPQ_OK && (flags & RPQ_BUILD_IN_CSR)) {
        uint64_t e_in = 0;
        rc = build_csr(dst, label, src, n_edges, n_vertices, n_labels, &g->in, &e_in, nullptr, g->h_stage, stream);
        g->has_in = rc == RPQ_OK;
    }
    if (rc == RPQ_OK && vertex_label) {
        void* p = nullptr;
        rc = dev_alloc(&p, n_vertices);
        if (rc == RPQ_OK) {
            g->vlabel = reinterpret_cast<uint8_t*>(p);
            if (hipMemcpyAsync(g->vlabel, vertex_label, n_vertices, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess) {
                rpq::set_error("copying vertex labels failed");
                rc = RPQ_EDEVICE;
            }
        }
    }
    if (rc != RPQ_OK) {
        free_graph(g);
        return rc;
    }
    const uint64_t R = (uint64_t)n_vertices * n_labels;
    g->device_bytes = (R + 1) * 4 + g->E * 4 + (uint64_t)n_vertices * 8;
    if (g->has_in) g->device_bytes *= 2;
    if (g->vlabel) g->device_bytes += n_vertices;
    *out = g;
    return RPQ_OK;
}

int rpq_graph_destroy(rpq_graph_t g) {
    if (!g) return RPQ_OK;
    (void)hipDeviceSynchronize();
    free_graph(g);
    return RPQ_OK;
}

int rpq_graph_info_get(rpq_graph_t g, rpq_graph_info* out) {
    rpq::clear_error();
    if (!g || !out) {
        rpq::set_error("NULL argument");
        return RPQ_EINVAL;
    }
    std::memset(out, 0, sizeof *out);
    out->n_vertices = g->V;
    out->n_labels = g->L;
    out->n_edges_in = g->E_in;
    out->n_edges = g->E;
    for (uint32_t l = 0; l < g->L; ++l) out->edges_per_label[l] = g->per_label[l];
    out->nonempty_rows = g->out.nonempty_rows;
    out->device_bytes = g->device_bytes;
    out->has_in_csr = g->has_in ? 1 : 0;
    out->has_vertex_labels = g->vlabel ? 1 : 0;
    return RPQ_OK;
}

int rpq_graph_export_csr(rpq_graph_t g, int reverse, uint32_t* row_ptr, uint32_t* dst, hipStream_t stream) {
    rpq::clear_error();
    if (!g) {
        rpq::set_error("NULL graph");
        return RPQ_EINVAL;
    }
    const rpq::Csr& c = reverse ? g->in : g->out;
    if (reverse && !g->has_in) {
        rpq::set_error("graph has no in-edge CSR");
        return RPQ_EUNSUPPORTED;
    }
    const uint64_t R = (uint64_t)g->V * g->L;
    if (row_ptr) RPQ_HIP(hipMemcpyAsync(row_ptr, c.row_ptr, (R + 1) * 4, hipMemcpyDeviceToDevice, stream));
    if (dst && g->E) RPQ_HIP(hipMemcpyAsync(dst, c.dst, g->E * 4, hipMemcpyDeviceToDevice, stream));
    RPQ_HIP(hipStreamSynchronize(stream));
    return RPQ_OK;
}

}  // extern "C"
