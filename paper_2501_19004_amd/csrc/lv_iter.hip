// lv_iter.hip -- device-driven local-moving iterations.
//
// With louvain_params.device_loop the host does not wait for each iteration
// of a pass: it enqueues the iterations in chunks and reads the pass's state
// back once per chunk.  What the host loop decides between two iterations is
// decided here, on the device, by k_iter_end, which runs after every
// iteration's move, apply and queue launches:
//
// * the tolerance test of Alg. 1 on the iteration's exact 128-bit gain sum
//   (per graph in a batch: a converged graph stops moving for the rest of
//   the pass), not in an ASYNC Pick-Less iteration (whose refused moves say
//   nothing about convergence);
// * with vertex pruning, the next queue's sizes per bucket; an empty queue
//   means the next iteration would move nothing (S = 0, converged), which is
//   counted without running it;
// * the pass ends when every graph has converged.
//
// Launches after the end see dit->halt and return at once.
#include "lv_internal.h"

namespace lv {
namespace {

__global__ void __launch_bounds__(256) k_zero_ranges(const DevIter* __restrict__ dit, ZeroRanges z) {
    if (dit && dit->halt) return;
    const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int r = 0; r < 4; r++) {
        char* p = (char*)z.p[r];
        const int64_t nb = z.bytes[r];
        if (!p || nb <= 0) continue;
        const int64_t head = min(nb, (int64_t)((16 - ((uintptr_t)p & 15)) & 15));
        const int64_t nq = (nb - head) / 16;
        for (int64_t i = tid; i < head; i += stride) p[i] = 0;
        uint4* q = (uint4*)(p + head);
        for (int64_t i = tid; i < nq; i += stride) q[i] = make_uint4(0, 0, 0, 0);
        for (int64_t i = head + nq * 16 + tid; i < nb; i += stride) p[i] = 0;
    }
}

// Slice table of a queue whose bucket sizes are cnt (starts seg): one thread
// per (slice, bucket) pair.
__device__ void write_shares(const int32_t* cnt, const int32_t* seg, int32_t* dshare, int ns, int interleave) {
    for (int x = threadIdx.x; x < ns * NB_MOVE; x += blockDim.x) {
        const int k = x / NB_MOVE, b = x % NB_MOVE;
        const int64_t tot = cnt[b];
        int64_t lo = 0, num;
        if (interleave) {
            num = tot > k ? (tot - k + ns - 1) / ns : 0;
        } else {
            lo = tot * k / ns;
            num = tot * (k + 1) / ns - lo;
        }
        dshare[2 * x] = seg[b] + (int32_t)lo;
        dshare[2 * x + 1] = (int32_t)num;
    }
}

__global__ void __launch_bounds__(256) k_iter_setup(DevIter* __restrict__ dit, const int32_t* __restrict__ bcount,
                                                    int nbt, int32_t max_iterations, int32_t* __restrict__ dshare,
                                                    int ns, int interleave) {
    __shared__ int32_t s_cnt[MAX_BUCKETS], s_seg[MAX_BUCKETS + 1];
    if (threadIdx.x == 0) {
        dit->halt = 0;
        dit->li = max_iterations;
        dit->ran = 0;
        dit->extra = 0;
        dit->moves = 0;
        int32_t acc = 0;
        for (int b = 0; b < MAX_BUCKETS; b++) {
            const int32_t c = b < nbt ? bcount[b] : 0;
            dit->cnt[b] = s_cnt[b] = c;
            dit->seg[b] = s_seg[b] = acc;
            acc += c;
        }
        dit->seg[MAX_BUCKETS] = s_seg[MAX_BUCKETS] = acc;
    }
    __syncthreads();
    write_shares(s_cnt, s_seg, dshare, ns, interleave);
}

// The tolerance test of a pass, exactly: 2 S tol_den drop^pass <= tol_num W^2
// (the same 128-bit evaluation as the host loop's).
__device__ bool converged_dev(unsigned __int128 S, i64 W, int64_t tn, int64_t td, int64_t drop, int pass) {
    const unsigned __int128 rhs = (unsigned __int128)tn * ((unsigned __int128)W * (unsigned __int128)W);
    unsigned __int128 lhs = 2 * S * (unsigned __int128)td;
    for (int k = 0; k < pass; k++) {
        if (lhs > rhs) return false;
        lhs *= (unsigned __int128)drop;
    }
    return lhs <= rhs;
}

constexpr int ET = 1024;

__global__ void __launch_bounds__(ET) k_iter_end(IterEndArgs e) {
    DevIter* dit = e.dit;
    if (dit->halt) return;  // uniform: nothing else writes it during this launch
    __shared__ int s_end;
    const int tid = threadIdx.x;
    if (tid == 0) {
        unsigned __int128 S = 0;
        u64 moves = 0;
        for (int k = 0; k < STRIPES; k++) {
            S += ((unsigned __int128)e.ctl->s_hi[k] << 64) + ((unsigned __int128)e.ctl->s_mid[k] << 32) +
                 (unsigned __int128)e.ctl->s_lo[k];
            moves += e.ctl->moves[k];
        }
        dit->ran += 1;
        dit->moves += moves;
        s_end = (e.nbg == 0 && e.may_end &&
                 converged_dev(S, e.W, e.tol_num, e.tol_den, e.tol_drop, e.pass)) ? 1 : 0;
    }
    __syncthreads();
    if (e.nbg > 0) {
        // per-graph tests; the pass ends when no graph is left moving
        int any = 0;
        for (int64_t g = tid; g < e.nbg; g += ET) {
            if (!e.gact[g]) continue;
            const unsigned __int128 Sg = ((unsigned __int128)e.Sg[2 * g + 1] << 64) + (unsigned __int128)e.Sg[2 * g];
            if (e.may_end && converged_dev(Sg, (i64)e.Wg[g], e.tol_num, e.tol_den, e.tol_drop, e.pass)) {
                e.gact[g] = 0;
                e.lig[g] = e.t + 1;
            } else {
                any = 1;
            }
        }
        any = __syncthreads_or(any);
        if (tid == 0 && !any) s_end = 1;
        __syncthreads();
    }
    if (s_end) {
        if (tid == 0) {
            dit->li = e.t + 1;
            dit->halt = 1;
        }
        return;
    }
    __shared__ int32_t s_total, s_cnt[MAX_BUCKETS], s_seg[MAX_BUCKETS + 1];
    if (tid == 0) {
        // with pruning the next queue is the flagged vertices, else it stays
        // every vertex with an arc
        int32_t acc = 0;
        for (int b = 0; b < MAX_BUCKETS; b++) {
            const int32_t c = e.prune ? (b < e.nbt ? e.ctl->qcount[b] : 0) : dit->cnt[b];
            dit->cnt[b] = s_cnt[b] = c;
            dit->seg[b] = s_seg[b] = acc;
            acc += c;
        }
        dit->seg[MAX_BUCKETS] = s_seg[MAX_BUCKETS] = acc;
        s_total = acc;
    }
    __syncthreads();
    write_shares(s_cnt, s_seg, e.dshare, e.ns_next, e.interleave);
    if (!e.prune || s_total != 0) return;
    // nothing flagged: the next iteration moves nothing and converges; it is
    // counted (if the pass allows it) without running
    if (e.t + 1 >= e.max_iterations) {
        if (tid == 0) dit->halt = 1;  // li stays max_iterations
        return;
    }
    for (int64_t g = tid; g < e.nbg; g += ET)
        if (e.gact[g]) e.lig[g] = e.t + 2;
    if (tid == 0) {
        dit->extra += 1;
        dit->li = e.t + 2;
        dit->halt = 1;
    }
}

}  // namespace

void launch_zero_ranges(const DevIter* dit, const ZeroRanges& z, hipStream_t s) {
    int64_t most = 0;
    for (int r = 0; r < 4; r++)
        if (z.p[r]) most = std::max(most, z.bytes[r]);
    if (most <= 0) return;
    const int64_t blocks = std::min<int64_t>(2048, (most / 16 + 255) / 256 + 1);
    k_zero_ranges<<<(unsigned)blocks, 256, 0, s>>>(dit, z);
}

void launch_iter_setup(DevIter* dit, const int32_t* bcount, int nbt, int32_t max_iterations, int32_t* dshare,
                       int ns, int interleave, hipStream_t s) {
    k_iter_setup<<<1, 256, 0, s>>>(dit, bcount, nbt, max_iterations, dshare, ns, interleave);
}

void launch_iter_end(const IterEndArgs& e, hipStream_t s) { k_iter_end<<<1, ET, 0, s>>>(e); }

}  // namespace lv
