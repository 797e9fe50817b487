// Device-wide primitives used by graph ingest and the join: fills, an
// exclusive scan over uint64 and a stable LSD radix sort of uint64 keys.
//
// The sort ranks equal digits inside a wave64 by matching the 8 digit bits
// with 8 ballots (lanes whose digit agrees on every bit form a group), so a
// 256-thread block scatters 256 keys per step with three barriers and no
// global atomics; blocks take contiguous tiles so the order of equal digits
// is preserved across the grid.
#include "internal.h"

#include <cstdarg>
#include <cstring>
#include <string>

namespace rpq {

// ------------------------------------------------------------------------------------------------
// errors (thread-local message)
// ------------------------------------------------------------------------------------------------
static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

const char* last_error_cstr() { return g_last_error.c_str(); }

// ------------------------------------------------------------------------------------------------
// fills
// ------------------------------------------------------------------------------------------------
__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t value) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // two-word stores where the pointer allows it
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
        ulonglong2* p2 = reinterpret_cast<ulonglong2*>(p);
        const uint64_t n2 = n / 2;
        for (uint64_t j = i; j < n2; j += stride) p2[j] = make_ulonglong2(value, value);
        if (i == 0 && (n & 1)) p[n - 1] = value;
    } else {
        for (uint64_t j = i; j < n; j += stride) p[j] = value;
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t value) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = value;
}

static unsigned fill_grid(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b == 0) b = 1;
    return (unsigned)b;
}

int fill_u64(uint64_t* p, uint64_t n, uint64_t value, hipStream_t s) {
    if (n == 0) return RPQ_OK;
    hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(n / 2 + 1)), dim3(256), 0, s, p, n, value);
    RPQ_LAUNCH_CHECK();
    return RPQ_OK;
}

int fill_u32(uint32_t* p, uint64_t n, uint32_t value, hipStream_t s) {
    if (n == 0) return RPQ_OK;
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, s, p, n, value);
    RPQ_LAUNCH_CHECK();
    return RPQ_OK;
}

// ------------------------------------------------------------------------------------------------
// exclusive scan (uint64), 1024 elements per 256-thread block, recursive over block sums
// ------------------------------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr uint64_t kScanTile = kScanThreads * kScanItems;

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint64_t* __restrict__ in, uint64_t n,
                                                              uint64_t* __restrict__ sums) {
    __shared__ uint64_t s_w[kScanThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint64_t t = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) t += in[base + i];
    t = rpqd::wave_sum_u64(t);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) s += s_w[w];
        sums[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const uint64_t* in, uint64_t* out, uint64_t n,
                                                             const uint64_t* __restrict__ offsets,
                                                             uint64_t* __restrict__ total) {
    __shared__ uint64_t s_w[kScanThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t t = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        t += v[i];
    }
    const uint64_t incl = rpqd::wave_incl_scan_u64(t);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) s_w[wv] = incl;
    __syncthreads();
    uint64_t pre = offsets ? offsets[blockIdx.x] : 0;
    for (int w = 0; w < wv; ++w) pre += s_w[w];
    uint64_t run = pre + incl - t;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) *total = run;
}

uint64_t scan_temp_elems(uint64_t n) {
    const uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 1) return 0;
    return nb + scan_temp_elems(nb);
}

int exclusive_scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* temp, uint64_t* total,
                       hipStream_t s) {
    if (n == 0) {
        if (total) RPQ_TRY(fill_u64(total, 1, 0, s));
        return RPQ_OK;
    }
    const uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanThreads), 0, s, in, out, n, nullptr, total);
        RPQ_LAUNCH_CHECK();
        return RPQ_OK;
    }
    uint64_t* sums = temp;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, sums);
    RPQ_LAUNCH_CHECK();
    RPQ_TRY(exclusive_scan_u64(sums, sums, nb, temp + nb, nullptr, s));
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, sums, total);
    RPQ_LAUNCH_CHECK();
    return RPQ_OK;
}

// ------------------------------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits
// ------------------------------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortChunks = 16;                         // 256-key steps per block
constexpr uint64_t kSortTile = (uint64_t)kSortThreads * kSortChunks;

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys, uint64_t n,
                                                             int shift, uint64_t* __restrict__ hist,
                                                             uint32_t nb) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    for (int c = 0; c < kSortChunks; ++c) {
        const uint64_t i = base + (uint64_t)c * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t* __restrict__ in,
                                                                uint64_t* __restrict__ out, uint64_t n,
                                                                int shift,
                                                                const uint64_t* __restrict__ offsets,
                                                                uint32_t nb) {
    __shared__ uint64_t run[256];
    __shared__ uint32_t wcnt[kSortThreads / 64][256];
    const int t = threadIdx.x;
    const int wv = t >> 6;
    run[t] = offsets[(uint64_t)t * nb + blockIdx.x];
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    for (int c = 0; c < kSortChunks; ++c) {
#pragma unroll
        for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][t] = 0;
        __syncthreads();
        const uint64_t i = base + (uint64_t)c * kSortThreads + t;
        const bool valid = i < n;
        const uint64_t key = valid ? in[i] : 0;
        const uint32_t d = valid ? (uint32_t)((key >> shift) & 0xFF) : 0;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & rpqd::lanemask_lt());
        if (valid && rank == 0) wcnt[wv][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint64_t off = run[d] + rank;
            for (int w = 0; w < wv; ++w) off += wcnt[w][d];
            out[off] = key;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kSortThreads / 64; ++w) add += wcnt[w][t];
        run[t] += add;
        __syncthreads();
    }
}

uint64_t radix_temp_bytes(uint64_t n) {
    const uint64_t nb = (n + kSortTile - 1) / kSortTile;
    const uint64_t h = 256 * (nb ? nb : 1);
    return (h + scan_temp_elems(h) + 1) * sizeof(uint64_t);
}

int radix_sort_u64(uint64_t* keys, uint64_t* alt, uint64_t n, int lo_bits, int hi_bits, void* temp,
                   hipStream_t s, uint64_t** sorted) {
    *sorted = keys;
    if (n <= 1) return RPQ_OK;
    const uint64_t nb = (n + kSortTile - 1) / kSortTile;
    if (nb > 0xFFFFFFFFull) {
        set_error("radix sort input too large");
        return RPQ_EUNSUPPORTED;
    }
    uint64_t* hist = reinterpret_cast<uint64_t*>(temp);
    uint64_t* stemp = hist + 256 * nb;
    uint64_t* a = keys;
    uint64_t* b = alt;
    int shifts[16];
    int ns = 0;
    for (int sh = 0; sh < lo_bits && sh < 32; sh += 8) shifts[ns++] = sh;
    for (int sh = 32; sh < 32 + hi_bits && sh < 64; sh += 8) shifts[ns++] = sh;
    for (int i = 0; i < ns; ++i) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, s, a, n, shifts[i], hist,
                           (uint32_t)nb);
        RPQ_LAUNCH_CHECK();
        RPQ_TRY(exclusive_scan_u64(hist, hist, 256 * nb, stemp, nullptr, s));
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, s, a, b, n, shifts[i],
                           hist, (uint32_t)nb);
        RPQ_LAUNCH_CHECK();
        uint64_t* t = a;
        a = b;
        b = t;
    }
    *sorted = a;
    return RPQ_OK;
}

}  // namespace rpq

namespace rpq {

uint64_t* host_stage() {
    thread_local uint64_t* stage = nullptr;
    if (!stage) {
        void* p = nullptr;
        if (hipHostMalloc(&p, 4096) == hipSuccess) stage = static_cast<uint64_t*>(p);
    }
    return stage;
}

}  // namespace rpq
