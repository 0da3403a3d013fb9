// lv_scan.hip -- exclusive prefix sums and fills used by bucketing,
// community renumbering (prefix scan of used flags) and CSR construction.
#include "lv_internal.h"

namespace lv {

namespace {

constexpr int SCAN_TPB = 256;
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = SCAN_TPB * SCAN_IPT;

// Inclusive scan across the 256 threads of a block; returns the thread's
// exclusive prefix and writes the block total to *total.
template <typename T>
__device__ T block_exclusive_scan(T v, T* total) {
    __shared__ T wave_sums[SCAN_TPB / WAVE];
    const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
    T x = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T y = __shfl_up(x, d, WAVE);
        if (lane >= d) x += y;
    }
    if (lane == WAVE - 1) wave_sums[wid] = x;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < SCAN_TPB / WAVE; k++) {
        T ws = wave_sums[k];
        if (k < wid) before += ws;
        all += ws;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

template <typename InT, typename OutT>
__global__ void __launch_bounds__(SCAN_TPB) k_tile_reduce(const InT* __restrict__ in, int64_t n,
                                                          OutT* __restrict__ partial) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    OutT s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; k++)
        if (base + k < n) s += (OutT)in[base + k];
    OutT total;
    block_exclusive_scan<OutT>(s, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

template <typename InT, typename OutT>
__global__ void __launch_bounds__(SCAN_TPB) k_tile_scan(const InT* __restrict__ in, int64_t n,
                                                        const OutT* __restrict__ partial_excl,
                                                        OutT* __restrict__ out) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    OutT v[SCAN_IPT];
    OutT s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; k++) {
        v[k] = (base + k < n) ? (OutT)in[base + k] : (OutT)0;
        s += v[k];
    }
    OutT total;
    OutT run = block_exclusive_scan<OutT>(s, &total) + (partial_excl ? partial_excl[blockIdx.x] : (OutT)0);
#pragma unroll
    for (int k = 0; k < SCAN_IPT; k++) {
        if (base + k < n) {
            out[base + k] = run;
            run += v[k];
            if (base + k == n - 1) out[n] = run;
        }
    }
}

template <typename T>
__global__ void k_set_one(T* p, T v) { *p = v; }

template <typename InT, typename OutT>
void scan_impl(const InT* in, OutT* out, int64_t n, char* scratch, hipStream_t s) {
    if (n <= 0) {
        k_set_one<OutT><<<1, 1, 0, s>>>(out, (OutT)0);
        return;
    }
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles == 1) {
        k_tile_scan<InT, OutT><<<1, SCAN_TPB, 0, s>>>(in, n, nullptr, out);
        return;
    }
    OutT* partial = (OutT*)scratch;
    OutT* partial_excl = partial + (tiles + 1);
    char* next = (char*)(partial_excl + (tiles + 1));
    next = (char*)(((uintptr_t)next + 255) & ~(uintptr_t)255);
    k_tile_reduce<InT, OutT><<<(unsigned)tiles, SCAN_TPB, 0, s>>>(in, n, partial);
    scan_impl<OutT, OutT>(partial, partial_excl, tiles, next, s);
    k_tile_scan<InT, OutT><<<(unsigned)tiles, SCAN_TPB, 0, s>>>(in, n, partial_excl, out);
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_iota_i32(int32_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
    size_t total = 0;
    int64_t m = n;
    while (m > SCAN_TILE) {
        int64_t tiles = (m + SCAN_TILE - 1) / SCAN_TILE;
        total += 2 * (size_t)(tiles + 1) * sizeof(int64_t) + 256;
        m = tiles;
    }
    return total + 1024;
}

void scan_i32_to_i32(const int32_t* in, int32_t* out, int64_t n, void* scratch, hipStream_t s) {
    scan_impl<int32_t, int32_t>(in, out, n, (char*)scratch, s);
}
void scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* scratch, hipStream_t s) {
    scan_impl<int32_t, int64_t>(in, out, n, (char*)scratch, s);
}
void scan_i64_to_i64(const int64_t* in, int64_t* out, int64_t n, void* scratch, hipStream_t s) {
    scan_impl<int64_t, int64_t>(in, out, n, (char*)scratch, s);
}

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
}
void iota_i32(int32_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_iota_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
}

}  // namespace lv
