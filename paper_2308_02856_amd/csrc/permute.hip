// Keyed permutation of 0..n-1 on the device: Durstenfeld's form of the
// Fisher-Yates shuffle (CACM 7(7), 1964, Algorithm 235) driven by the
// SplitMix64 stream of a key.  Not in the paper (which draws V_i i.i.d.,
// Sec. III.B step 1); it defines the permute-split sampling of the small and
// contraction workloads.
//
// Sequential definition: start from the identity; for k = n-1 down to 1
// exchange entries k and j_k, with j_k = high word of r_t * (k + 1), r_t the
// SplitMix64 output t = n-1-k (Lemire's multiply-shift map without
// rejection; bias below (k+1)/2^64).
//
// The loop is sequential, but its result has a closed form that parallel
// passes can evaluate.  Iteration k touches positions k and j_k <= k, and
// position k never changes after iteration k.  Let G_p = {k > p : j_k = p}
// be the later-index iterations that swap with position p (they run before
// iteration p, in descending k), and
//     pre(p) = the value at position p just before iteration p.
// The last of G_p in time is its smallest element g_1, which leaves at p
// what position g_1 held before its own iteration, so pre(p) = pre(g_1), or
// p when G_p is empty: pre(p) is the end of the chain p -> min G_p -> ...
// (indices strictly increase).  The result is then
//     pi[k] = pre(k)                      if j_k = k (k >= 1), and pi[0] = pre(0);
//     pi[g_s] = pre(g_{s+1})              for g_1 < ... < g_r the sorted G_p, s < r;
//     pi[g_r] = p                         (the first exchange with p moves p).
// Passes: count |G_p| (atomics), exclusive scan -> group starts, fill the
// groups (atomics; unordered), sort each group, chain ends by walking with
// path compression, then write pi.  Scratch: three uint32 arrays of n.
#include <algorithm>

#include "ssbh_internal.hpp"

namespace ssbh {
namespace {

constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kScanPer = 16;                       // elements per thread
constexpr uint32_t kScanChunk = kScanThreads * kScanPer;  // 4096 per block

// j_k of the keyed shuffle (1 <= k < n).
__device__ __forceinline__ uint64_t shuffle_choice(uint64_t key, uint64_t n,
                                                   uint64_t k) {
    const uint64_t r = splitmix64_at(key, n - 1 - k);
    return __umul64hi(r, k + 1);
}

__global__ __launch_bounds__(256) void k_pc_fill_u32(uint32_t *a, uint64_t n,
                                                     uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride)
        a[i] = v;
}

// cnt[p] = |G_p|.
__global__ __launch_bounds__(256) void k_pc_count(uint64_t key, uint64_t n,
                                                  uint32_t *cnt) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = 1 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
         k < n; k += stride) {
        const uint64_t j = shuffle_choice(key, n, k);
        if (j < k) atomicAdd(&cnt[j], 1u);
    }
}

// ---- exclusive scan of uint32 (sums below 2^32) ----

// Sum of thread t's kScanPer consecutive elements of the block's chunk.
__device__ __forceinline__ uint32_t thread_sum(const uint32_t *in, uint64_t n,
                                               uint64_t base, uint32_t *v) {
    uint32_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; ++k) {
        const uint64_t i = base + k;
        v[k] = i < n ? in[i] : 0u;
        s += v[k];
    }
    return s;
}

// Exclusive scan over the block's threads of x; also the block total.
__device__ __forceinline__ uint32_t block_excl(uint32_t x, uint32_t *total) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = x;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int k = 0; k < (int)(kScanThreads / 64); ++k) {
        if (k < w) before += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return before + incl - x;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(
        const uint32_t *in, uint64_t n, uint32_t *sums) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanChunk +
                          (uint64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    const uint32_t s = thread_sum(in, n, base, v);
    uint32_t tot;
    (void)block_excl(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// out[i] = offs[block] + exclusive prefix of in inside the block's chunk
// (offs == nullptr: no block offsets, the single-block case).
__global__ __launch_bounds__(kScanThreads) void k_scan_down(
        const uint32_t *in, uint64_t n, const uint32_t *offs, uint32_t *out) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanChunk +
                          (uint64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    const uint32_t s = thread_sum(in, n, base, v);
    uint32_t tot;
    uint32_t run = block_excl(s, &tot) + (offs ? offs[blockIdx.x] : 0u);
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; ++k) {
        const uint64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

// Group p = list[ends[p-1] .. ends[p]) (ends[-1] = 0): sort it ascending and
// set nx[p] = its smallest element, or p when it is empty.
__global__ __launch_bounds__(256) void k_pc_sort(uint64_t n,
                                                 const uint32_t *ends,
                                                 uint32_t *list, uint32_t *nx) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += stride) {
        const uint32_t b = p ? ends[p - 1] : 0u, e = ends[p];
        for (uint32_t s = b + 1; s < e; ++s) {   // insertion sort (groups are short)
            const uint32_t x = list[s];
            uint32_t t = s;
            while (t > b && list[t - 1] > x) {
                list[t] = list[t - 1];
                --t;
            }
            list[t] = x;
        }
        nx[p] = e > b ? list[b] : (uint32_t)p;
    }
}

// a[p] = end of the chain p -> a[p] -> ... (a[r] = r at the end).  Threads
// overwrite a[p] with the chain end while others walk through p; either value
// lies on the same chain, so every walk still ends at the same place.
__global__ __launch_bounds__(256) void k_pc_walk(uint64_t n, uint32_t *a) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += stride) {
        uint32_t r = (uint32_t)p;
        for (uint32_t nxt = a[r]; nxt != r; nxt = a[r]) r = nxt;
        a[p] = r;
    }
}

// pi over the groups: pi[g_s] = pre(g_{s+1}), pi[g_r] = p.
__global__ __launch_bounds__(256) void k_pc_place(uint64_t n,
                                                  const uint32_t *ends,
                                                  const uint32_t *list,
                                                  const uint32_t *pre,
                                                  uint32_t *perm) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += stride) {
        const uint32_t b = p ? ends[p - 1] : 0u, e = ends[p];
        for (uint32_t s = b; s < e; ++s)
            perm[list[s]] = s + 1 < e ? pre[list[s + 1]] : (uint32_t)p;
    }
}

// pi[k] = pre(k) where the exchange of iteration k is with itself, and
// pi[0] = pre(0).
__global__ __launch_bounds__(256) void k_pc_self(uint64_t key, uint64_t n,
                                                 const uint32_t *pre,
                                                 uint32_t *perm) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += stride)
        if (k == 0 || shuffle_choice(key, n, k) == k) perm[k] = pre[k];
}

// fill: slot = atomicAdd(&ends[j_k], 1) over the exclusive starts, so that
// afterwards ends[p] is where group p ends.
__global__ __launch_bounds__(256) void k_pc_group(uint64_t key, uint64_t n,
                                                  uint32_t *ends,
                                                  uint32_t *list) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = 1 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
         k < n; k += stride) {
        const uint64_t j = shuffle_choice(key, n, k);
        if (j < k) list[atomicAdd(&ends[j], 1u)] = (uint32_t)k;
    }
}

uint32_t grid_for(uint64_t n, int num_cus) {
    const uint64_t want = (n + 255) / 256;
    return (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>(want, (uint64_t)std::max(num_cus, 1) * 32));
}

}  // namespace

// Words of the block-sum levels of a scan over n elements.
static uint64_t scan_level_words(uint64_t n) {
    uint64_t w = 0;
    while (n > kScanChunk) {
        n = (n + kScanChunk - 1) / kScanChunk;
        w += n;
    }
    return w;
}

size_t permutation_scratch(uint64_t n) {
    return (size_t)(3 * n + scan_level_words(n) + 64) * sizeof(uint32_t);
}

// Exclusive scan in -> out (n elements), levels = scan_level_words(n) words.
static ssbh_status scan_u32(const uint32_t *in, uint32_t *out, uint64_t n,
                            uint32_t *levels, hipStream_t stream) {
    const uint64_t nb = (n + kScanChunk - 1) / kScanChunk;
    if (nb <= 1) {
        hipLaunchKernelGGL(k_scan_down, dim3(1), dim3(kScanThreads), 0, stream,
                           in, n, (const uint32_t *)nullptr, out);
        SSBH_CHECK_HIP(hipGetLastError());
        return SSBH_OK;
    }
    uint32_t *sums = levels;
    hipLaunchKernelGGL(k_scan_sums, dim3((uint32_t)nb), dim3(kScanThreads), 0,
                       stream, in, n, sums);
    SSBH_CHECK_HIP(hipGetLastError());
    ssbh_status st = scan_u32(sums, sums, nb, levels + nb, stream);
    if (st != SSBH_OK) return st;
    hipLaunchKernelGGL(k_scan_down, dim3((uint32_t)nb), dim3(kScanThreads), 0,
                       stream, in, n, (const uint32_t *)sums, out);
    SSBH_CHECK_HIP(hipGetLastError());
    return SSBH_OK;
}

ssbh_status launch_permutation(ssbh_ctx *ctx, DevBuf &scratch, uint64_t key,
                               uint64_t n, uint32_t *d_perm,
                               hipStream_t stream) {
    if (n > SSBH_MAX_SAMPLE_BITS) {
        set_error("n must be at most %llu", (unsigned long long)SSBH_MAX_SAMPLE_BITS);
        return SSBH_E_UNSUPPORTED;
    }
    if (!n) return SSBH_OK;
    if (!d_perm) SSBH_INVAL("d_perm is null");
    ssbh_status st = scratch.reserve(permutation_scratch(n));
    if (st != SSBH_OK) return st;
    uint32_t *a = scratch.as<uint32_t>();   // counts, then chain links / ends
    uint32_t *ends = a + n;                 // group starts, then group ends
    uint32_t *list = ends + n;              // group members
    uint32_t *levels = list + n;            // scan block sums
    const uint32_t g = grid_for(n, ctx->num_cus);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_pc_fill_u32, dim3(g), dim3(256), 0, stream, a, n, 0u);
    hipLaunchKernelGGL(k_pc_count, dim3(g), dim3(256), 0, stream, key, n, a);
    SSBH_CHECK_HIP(hipGetLastError());
    if ((st = scan_u32(a, ends, n, levels, stream)) != SSBH_OK) return st;
    hipLaunchKernelGGL(k_pc_group, dim3(g), dim3(256), 0, stream, key, n, ends,
                       list);
    hipLaunchKernelGGL(k_pc_sort, dim3(g), dim3(256), 0, stream, n,
                       (const uint32_t *)ends, list, a);
    hipLaunchKernelGGL(k_pc_walk, dim3(g), dim3(256), 0, stream, n, a);
    hipLaunchKernelGGL(k_pc_place, dim3(g), dim3(256), 0, stream, n,
                       (const uint32_t *)ends, (const uint32_t *)list,
                       (const uint32_t *)a, d_perm);
    hipLaunchKernelGGL(k_pc_self, dim3(g), dim3(256), 0, stream, key, n,
                       (const uint32_t *)a, d_perm);
    SSBH_CHECK_HIP(hipGetLastError());
    return SSBH_OK;
}

}  // namespace ssbh
