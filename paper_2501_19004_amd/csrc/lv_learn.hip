// lv_learn.hip -- the learned move-pruner: per-vertex features, the FP32 MLP
// filter of the flagged queue, training-sample recording, and the MLP's
// stand-alone kernels (initialisation, inference, loss gradient, Adam).
//
// The pruner generalises the paper's vertex pruning (Section 4.1): a vertex
// flagged by a moving neighbour is evaluated only if an MLP over eight
// integer-derived features expects it to move.  The features and the MLP
// follow a fixed FP32 recipe -- correctly rounded conversions and divisions,
// every neuron summed from its bias in index order with fused multiply-adds --
// so the keep decision is reproducible bit for bit.
//
// The MLP is ~1.3K FMAs per flagged vertex against ~40 bytes of per-vertex
// state: vector ALU work, one thread per vertex, weights staged in LDS
// (every lane reads the same word: an LDS broadcast).
#include "lv_internal.h"

namespace lv {
namespace {

constexpr int MLP_IN = 8;
constexpr int MLP_H = 32;
constexpr int P_W1 = 0;
constexpr int P_B1 = P_W1 + MLP_H * MLP_IN;
constexpr int P_W2 = P_B1 + MLP_H;
constexpr int P_B2 = P_W2 + MLP_H * MLP_H;
constexpr int P_W3 = P_B2 + MLP_H;
constexpr int P_B3 = P_W3 + MLP_H;
static_assert(P_B3 + 1 == MLP_PARAMS, "parameter layout");
constexpr u64 GOLDEN = 0x9E3779B97F4A7C15ull;

// SplitMix64 output function (Steele, Lea and Flood, 2014) of one counter value.
__device__ __forceinline__ u64 splitmix64(u64 x) {
    u64 z = x + GOLDEN;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ bool sample_selected(int64_t v, int32_t pass, int32_t t, int32_t per_mille) {
    const u64 key = (u64)v + ((u64)((uint32_t)pass * 65536u + (uint32_t)t) << 32);
    return (int32_t)(splitmix64(key) % 1000ull) < per_mille;
}

// Mitchell's piecewise-linear log2 of an integer x >= 1: e + (x - 2^e) / 2^e.
__device__ __forceinline__ float mlog2(int64_t x) {
    const int e = 63 - __clzll((long long)x);
    const int64_t p = (int64_t)1 << e;
    const float frac = (float)(x - p) / (float)p;
    return (float)e + frac;
}

__device__ __forceinline__ float ratio(int64_t a, int64_t b) { return b != 0 ? (float)a / (float)b : 0.0f; }

// Output logit; P points at the weights (LDS).
__device__ __forceinline__ float mlp_logit(const float* P, const float (&x)[MLP_IN]) {
    float h1[MLP_H];
#pragma unroll
    for (int k = 0; k < MLP_H; k++) {
        float a = P[P_B1 + k];
#pragma unroll
        for (int j = 0; j < MLP_IN; j++) a = __builtin_fmaf(P[P_W1 + k * MLP_IN + j], x[j], a);
        h1[k] = a > 0.0f ? a : 0.0f;
    }
    float z = P[P_B3];
    for (int k = 0; k < MLP_H; k++) {
        float a = P[P_B2 + k];
#pragma unroll
        for (int j = 0; j < MLP_H; j++) a = __builtin_fmaf(P[P_W2 + k * MLP_H + j], h1[j], a);
        z = __builtin_fmaf(P[P_W3 + k], a > 0.0f ? a : 0.0f, z);
    }
    return z;
}

__device__ __forceinline__ void stage_weights(float* s_w, const float* w) {
    for (int k = threadIdx.x; k < MLP_PARAMS; k += blockDim.x) s_w[k] = w[k];
    __syncthreads();
}

// Filter of the next iteration's flagged vertices (flags[v] set, or every
// vertex with an arc when all = 1): features, MLP keep decision (a dropped
// vertex is unflagged), sample recording.  In a batch, the vertices of a
// graph whose next iteration is its sweep are all kept (and flagged), and
// every graph with a kept vertex is marked in gany.
template <typename OffT>
__global__ void __launch_bounds__(256) k_learn_filter(FilterArgs f) {
    __shared__ float s_w[MLP_PARAMS];
    __shared__ u64 s_pruned;
    if (threadIdx.x == 0) s_pruned = 0;
    if (f.learned) stage_weights(s_w, f.weights);
    else __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool dropped = false;
    if (v < f.n) {
        const OffT* off = (const OffT*)f.off;
        const int32_t gv = f.gid ? f.gid[v] : -1;
        const bool gsw = f.gsweep && gv >= 0 && f.gsweep[gv];
        bool flagged = f.all || gsw || f.flags[v];
        const int64_t deg = flagged ? (int64_t)off[v + 1] - (int64_t)off[v] : 0;
        flagged = flagged && deg > 0;
        if (gsw && flagged) f.flags[v] = 1;
        const bool selected = flagged && !gsw && f.per_mille > 0 && sample_selected(v, f.pass, f.t, f.per_mille);
        bool keep = flagged;
        if (flagged && !gsw && (f.learned || selected)) {
            const i64 Kv = f.K[v];
            const int32_t m = f.nm[v];
            float x[MLP_IN];
            x[0] = mlog2(1 + deg) / 16.0f;
            x[1] = ratio(f.own[v], Kv);
            x[2] = mlog2(1 + (int64_t)m) / 16.0f;
            x[3] = ratio(m, deg);
            x[4] = f.moved[v] == f.itag_prev ? 1.0f : 0.0f;
            x[5] = (float)f.pass / 10.0f;
            x[6] = (float)f.t / 20.0f;
            x[7] = ratio(f.adv[v], Kv);
            if (f.learned) {
                keep = mlp_logit(s_w, x) >= f.zt;
                if (!keep) {
                    f.flags[v] = 0;
                    dropped = true;
                }
            }
            if (keep && selected) {
                const u64 slot = atomicAdd(&f.ctl->nsamples, 1ull);
                if ((int64_t)slot < f.cap) {
                    float* o = f.samples + slot * SAMPLE_FLOATS;
#pragma unroll
                    for (int j = 0; j < MLP_IN; j++) o[j] = x[j];
                    o[MLP_IN] = __int_as_float((int32_t)v);  // vertex id until the label is known
                }
            }
        }
        if (keep && f.gany && gv >= 0) f.gany[gv] = 1;
    }
    const u64 nd = __ballot(dropped);
    if ((threadIdx.x % WAVE) == 0 && nd) atomicAdd(&s_pruned, (u64)__popcll(nd));
    __syncthreads();
    if (threadIdx.x == 0 && s_pruned) atomicAdd(&f.ctl->pruned, s_pruned);
}

// Label of the samples of one iteration: 1 if the vertex moved in it.
__global__ void __launch_bounds__(256) k_learn_label(float* samples, int64_t lo, int64_t hi,
                                                     const uint32_t* moved, uint32_t itag) {
    const int64_t k = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= hi) return;
    float* o = samples + k * SAMPLE_FLOATS + MLP_IN;
    const int32_t v = __float_as_int(*o);
    *o = moved[v] == itag ? 1.0f : 0.0f;
}

// ------------------------------------------------------------ stand-alone MLP

__global__ void __launch_bounds__(256) k_mlp_init(float* w, u64 seed) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_PARAMS) return;
    int fan = 0;
    if (k < P_B1) fan = MLP_IN + MLP_H;
    else if (k >= P_W2 && k < P_B2) fan = MLP_H + MLP_H;
    else if (k >= P_W3 && k < P_B3) fan = MLP_H + 1;
    if (!fan) { w[k] = 0.0f; return; }
    const float lim = sqrtf(6.0f / (float)fan);
    const float u = (float)(splitmix64(seed + (u64)k * GOLDEN) >> 40) * 0x1p-24f;
    w[k] = (2.0f * u - 1.0f) * lim;
}

__global__ void __launch_bounds__(256) k_mlp_predict(const float* w, const float* X, int64_t count, float* out) {
    __shared__ float s_w[MLP_PARAMS];
    stage_weights(s_w, w);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    float x[MLP_IN];
#pragma unroll
    for (int j = 0; j < MLP_IN; j++) x[j] = X[k * MLP_IN + j];
    out[k] = mlp_logit(s_w, x);
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, WAVE);
    return x;
}

// Adds v (one value per lane) summed over the wave into s_g[p].
__device__ __forceinline__ void acc_param(float* s_g, int p, float v) {
    v = wave_sum(v);
    if ((threadIdx.x % WAVE) == 0 && v != 0.0f) atomicAdd(&s_g[p], v);
}

// Gradient of the mean weighted binary cross-entropy.  One thread per
// sample: forward, backward, per-parameter wave sums into an LDS gradient,
// then one global atomic per parameter and block.  Batch mode (batch > 0):
// slot k of step `step` uses sample splitmix64(seed + (step*batch + k)*gamma)
// mod count; otherwise slot k is sample k.
__global__ void __launch_bounds__(256) k_mlp_loss_grad(const float* w, const float* S, int64_t count, int64_t slots,
                                                       int32_t batch, u64 seed, int64_t step, float pos_weight,
                                                       float* grad, double* loss) {
    __shared__ float s_w[MLP_PARAMS];
    __shared__ float s_g[MLP_PARAMS];
    for (int k = threadIdx.x; k < MLP_PARAMS; k += blockDim.x) s_g[k] = 0.0f;
    stage_weights(s_w, w);
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool on = slot < slots;
    int64_t idx = slot;
    if (on && batch > 0) idx = (int64_t)(splitmix64(seed + (u64)(step * batch + slot) * GOLDEN) % (u64)count);
    float x[MLP_IN], y = 0.0f;
#pragma unroll
    for (int j = 0; j < MLP_IN; j++) x[j] = on ? S[idx * SAMPLE_FLOATS + j] : 0.0f;
    if (on) y = S[idx * SAMPLE_FLOATS + MLP_IN];
    // forward
    float a1[MLP_H], a2[MLP_H];
#pragma unroll
    for (int k = 0; k < MLP_H; k++) {
        float a = s_w[P_B1 + k];
#pragma unroll
        for (int j = 0; j < MLP_IN; j++) a = __builtin_fmaf(s_w[P_W1 + k * MLP_IN + j], x[j], a);
        a1[k] = a;
    }
    float z = s_w[P_B3];
    for (int k = 0; k < MLP_H; k++) {
        float a = s_w[P_B2 + k];
#pragma unroll
        for (int j = 0; j < MLP_H; j++) a = __builtin_fmaf(s_w[P_W2 + k * MLP_H + j], fmaxf(a1[j], 0.0f), a);
        a2[k] = a;
        z = __builtin_fmaf(s_w[P_W3 + k], fmaxf(a, 0.0f), z);
    }
    const float c = y > 0.5f ? pos_weight : 1.0f;
    const float inv_n = 1.0f / (float)slots;
    const float l = on ? c * (fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))) - y * z) : 0.0f;
    const float dz = on ? c * (1.0f / (1.0f + expf(-z)) - y) * inv_n : 0.0f;
    // backward
    acc_param(s_g, P_B3, dz);
    float d2[MLP_H];
    for (int k = 0; k < MLP_H; k++) {
        acc_param(s_g, P_W3 + k, dz * fmaxf(a2[k], 0.0f));
        d2[k] = a2[k] > 0.0f ? dz * s_w[P_W3 + k] : 0.0f;
        acc_param(s_g, P_B2 + k, d2[k]);
    }
    for (int k = 0; k < MLP_H; k++)
        for (int j = 0; j < MLP_H; j++) acc_param(s_g, P_W2 + k * MLP_H + j, d2[k] * fmaxf(a1[j], 0.0f));
    for (int j = 0; j < MLP_H; j++) {
        float d1 = 0.0f;
        for (int k = 0; k < MLP_H; k++) d1 = __builtin_fmaf(d2[k], s_w[P_W2 + k * MLP_H + j], d1);
        d1 = a1[j] > 0.0f ? d1 : 0.0f;
        acc_param(s_g, P_B1 + j, d1);
#pragma unroll
        for (int i = 0; i < MLP_IN; i++) acc_param(s_g, P_W1 + j * MLP_IN + i, d1 * x[i]);
    }
    const float lw = wave_sum(l);
    if ((threadIdx.x % WAVE) == 0 && lw != 0.0f) atomicAdd(loss, (double)lw * (double)inv_n);
    __syncthreads();
    for (int k = threadIdx.x; k < MLP_PARAMS; k += blockDim.x)
        if (s_g[k] != 0.0f) atomicAdd(&grad[k], s_g[k]);
}

__global__ void __launch_bounds__(256) k_mlp_zero(float* p, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0.0f;
}

__global__ void __launch_bounds__(256) k_adam(float* w, const float* g, float* m, float* v, float lr, float bc1,
                                              float bc2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_PARAMS) return;
    const float gk = g[k];
    const float mk = 0.9f * m[k] + 0.1f * gk;
    const float vk = 0.999f * v[k] + 0.001f * gk * gk;
    m[k] = mk;
    v[k] = vk;
    w[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + 1e-8f);
}

}  // namespace

void launch_learn_filter(const FilterArgs& f, int off64, hipStream_t s) {
    if (f.n <= 0) return;
    const unsigned nb = (unsigned)((f.n + 255) / 256);
    if (off64) k_learn_filter<int64_t><<<nb, 256, 0, s>>>(f);
    else k_learn_filter<int32_t><<<nb, 256, 0, s>>>(f);
}

void launch_learn_label(float* samples, int64_t lo, int64_t hi, const uint32_t* moved, uint32_t itag,
                        hipStream_t s) {
    if (hi <= lo) return;
    k_learn_label<<<(unsigned)((hi - lo + 255) / 256), 256, 0, s>>>(samples, lo, hi, moved, itag);
}

void launch_mlp_init(float* w, u64 seed, hipStream_t s) {
    k_mlp_init<<<(MLP_PARAMS + 255) / 256, 256, 0, s>>>(w, seed);
}

void launch_mlp_predict(const float* w, const float* X, int64_t count, float* out, hipStream_t s) {
    if (count <= 0) return;
    k_mlp_predict<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(w, X, count, out);
}

void launch_mlp_zero(float* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_mlp_zero<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
}

void launch_mlp_loss_grad(const float* w, const float* S, int64_t count, int64_t slots, int32_t batch, u64 seed,
                          int64_t step, float pos_weight, float* grad, double* loss, hipStream_t s) {
    if (slots <= 0) return;
    k_mlp_loss_grad<<<(unsigned)((slots + 255) / 256), 256, 0, s>>>(w, S, count, slots, batch, seed, step,
                                                                      pos_weight, grad, loss);
}

void launch_adam(float* w, const float* g, float* m, float* v, float lr, float bc1, float bc2, hipStream_t s) {
    k_adam<<<(MLP_PARAMS + 255) / 256, 256, 0, s>>>(w, g, m, v, lr, bc1, bc2);
}

}  // namespace lv
