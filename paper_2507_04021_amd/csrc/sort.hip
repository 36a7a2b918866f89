// Device-wide exclusive scan and LSD radix sort (64-bit keys, 32-bit
// payload), shared by the hierarchy build and the diffuse-record ordering.
#include "common.h"
#include "internal.h"

namespace pcrt {

// LSD, 8-bit digits, 64-bit keys with 32-bit payload. Per pass: tile
// histograms, one exclusive scan in digit-major order, stable scatter with a
// wavefront multisplit (8 ballots per key) for the in-tile rank.
constexpr int kRsBlock = 256;
constexpr int kRsRounds = 8;
constexpr int kRsTile = kRsBlock * kRsRounds;

__global__ void k_rs_hist(const uint64_t *__restrict__ key, uint32_t n, int shift, uint32_t *__restrict__ hist,
                          uint32_t tiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint32_t base = blockIdx.x * kRsTile;
    for (int r = 0; r < kRsRounds; ++r) {
        uint32_t i = base + r * kRsBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of a u32 array in one block of 1024 threads (build only).
__global__ void k_scan_small(uint32_t *__restrict__ a, uint32_t n) {
    __shared__ uint32_t part[1024];
    uint32_t per = (n + 1023) / 1024;
    uint32_t b = threadIdx.x * per, e = min(n, b + per);
    uint32_t s = 0;
    for (uint32_t i = b; i < e; ++i) s += a[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t v = threadIdx.x >= (uint32_t)o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (uint32_t i = b; i < e; ++i) {
        uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

__global__ void k_rs_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                             uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, uint32_t n, int shift,
                             const uint32_t *__restrict__ hist, uint32_t tiles) {
    __shared__ uint32_t base[256], run[256];
    __shared__ uint32_t wcnt[kRsBlock / kWave][256];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    base[threadIdx.x] = hist[threadIdx.x * tiles + blockIdx.x];
    run[threadIdx.x] = 0;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kRsRounds; ++r) {
        for (int w = 0; w < kRsBlock / kWave; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        uint32_t i = blockIdx.x * kRsTile + r * kRsBlock + threadIdx.x;
        bool ok = i < n;
        uint64_t k = ok ? kin[i] : 0;
        uint32_t dg = (uint32_t)(k >> shift) & 255;
        uint64_t peers = __ballot(ok);
        for (int b = 0; b < 8; ++b) {
            bool bit = (dg >> b) & 1;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t rank = __popcll(peers & lt);
        if (ok && rank == 0) wcnt[wave][dg] = __popcll(peers);
        __syncthreads();
        if (ok) {
            uint32_t before = 0;
            for (int w = 0; w < wave; ++w) before += wcnt[w][dg];
            uint32_t dst = base[dg] + run[dg] + before + rank;
            kout[dst] = k;
            vout[dst] = vin[i];
        }
        __syncthreads();
        uint32_t tot = 0;
        for (int w = 0; w < kRsBlock / kWave; ++w) tot += wcnt[w][threadIdx.x];
        run[threadIdx.x] += tot;
        __syncthreads();
    }
}


__global__ __launch_bounds__(1024) void k_scan_block(uint32_t *a, uint32_t n, uint32_t *blk) {
    __shared__ uint32_t s[1024];
    uint32_t i = blockIdx.x * 1024 + threadIdx.x;
    uint32_t v = i < n ? a[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t t = threadIdx.x >= (uint32_t)o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) a[i] = s[threadIdx.x] - v;
    if (threadIdx.x == 1023) blk[blockIdx.x] = s[1023];
    if (blockIdx.x == 0 && threadIdx.x == 0) blk[gridDim.x] = 0;  // becomes the total after the block-sum scan
}

__global__ __launch_bounds__(1024) void k_scan_add(uint32_t *a, uint32_t n, const uint32_t *blk) {
    uint32_t i = blockIdx.x * 1024 + threadIdx.x;
    if (i < n) a[i] += blk[blockIdx.x];
}

uint32_t scan_blk_words(uint32_t n) { return (n + 1023) / 1024 + 1; }
uint32_t radix_hist_words(uint32_t n) { return 256u * ((n + kRsTile - 1) / kRsTile); }

// In-place exclusive scan; the total lands in blk[ceil(n / 1024)].
void exclusive_scan(uint32_t *a, uint32_t n, uint32_t *blk, hipStream_t s) {
    const uint32_t nb = (n + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(1024), 0, s, a, n, blk);
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, blk, nb + 1);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, s, a, n, blk);
}

// Sorts (key, value) by key bits [bit_lo, bit_hi) with 8-bit passes; returns
// true if the sorted data ended in (k1, v1), false if in (k0, v0).
bool radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, uint32_t n, int bit_lo, int bit_hi,
                    uint32_t *hist, uint32_t *blk, hipStream_t s) {
    const uint32_t tiles = (n + kRsTile - 1) / kRsTile;
    bool flip = false;
    for (int shift = bit_lo; shift < bit_hi; shift += 8) {
        uint64_t *ki = flip ? k1 : k0, *ko = flip ? k0 : k1;
        uint32_t *vi = flip ? v1 : v0, *vo = flip ? v0 : v1;
        hipLaunchKernelGGL(k_rs_hist, dim3(tiles), dim3(kRsBlock), 0, s, ki, n, shift, hist, tiles);
        exclusive_scan(hist, 256 * tiles, blk, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(tiles), dim3(kRsBlock), 0, s, ki, vi, ko, vo, n, shift, hist, tiles);
        flip = !flip;
    }
    return flip;
}

}  // namespace pcrt
