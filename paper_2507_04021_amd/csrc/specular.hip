// Specular paths (Sec. II-B.2, II-B.4).
//
// Keys: every prefix (s_1..s_k) of a traced ray's surface labels. The hash
// set built during tracing holds, per key, the smallest ray id having it
// (the representative). Here:
//   1. mark each record that is its key's representative,
//   2. exclusive-scan the marks and compact them: the key list comes out in
//      (transmitter, ray, k) order, independent of hash-slot placement,
//   3. per transmitter, split its keys into fixed chunks (deterministic
//      FP64 reduction units),
//   4. per (key, receiver): minimise the path length of Eq. (1) on the
//      representative's disk planes -- on infinite planes its minimiser is
//      the image-method point set -- then validate every interaction with a
//      ray from the previous point (surface label, angle t_a, plane distance
//      t_d), retrying up to kappa times with the plane of the disk actually
//      hit, check the last segment for occlusion and evaluate the field.
#include "common.h"
#include "internal.h"
#include "refine.h"

namespace pcrt {

__device__ __forceinline__ uint32_t ray_id_of(const LaunchArgs &A, uint32_t g, int *item_out) {
    int it = find_item(A.items, A.D.n_items, g);
    *item_out = it;
    uint32_t local = g - A.items[it].ray_off;
    return A.subset ? A.subset[local] : local;
}

// flag[r] = record r is the representative of its key.
__global__ void k_mark(LaunchArgs A, uint32_t n_rec) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rec) return;
    uint32_t f = 0;
    int id = A.rb.id[r];
    uint32_t slot = A.rb.slot[r];
    if (id >= 0 && slot != 0xffffffffu) {
        int it;
        uint32_t j = ray_id_of(A, r / A.D.K, &it);
        f = A.hb.rep[(size_t)it * A.hb.cap + slot] == j;
    }
    A.scan[r] = f;
}

// keylist[scan[r]] = r for every marked record (mark = scan[r+1] - scan[r]).
__global__ void k_compact(LaunchArgs A, uint32_t n_rec, const uint32_t *total) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rec) return;
    uint32_t nxt = r + 1 < n_rec ? A.scan[r + 1] : *total;
    uint32_t cur = A.scan[r];
    if (nxt != cur) A.keylist[cur] = r;
}

// Per transmitter: key range and reduction chunks (one block).
__global__ void k_plan(LaunchArgs A, const uint32_t *total) {
    __shared__ uint32_t chunks[1024];
    const uint32_t n_items = A.D.n_items;
    const uint32_t n_rec = A.D.T * A.D.K;
    uint32_t per = (n_items + 1023) / 1024;
    uint32_t b = threadIdx.x * per, e = min(n_items, b + per);
    uint32_t s = 0;
    for (uint32_t i = b; i < e; ++i) {
        uint32_t r0 = A.items[i].ray_off * A.D.K;
        uint32_t r1 = i + 1 < n_items ? A.items[i + 1].ray_off * A.D.K : n_rec;
        uint32_t k0 = r0 < n_rec ? A.scan[r0] : *total;
        uint32_t k1 = r1 < n_rec ? A.scan[r1] : *total;
        A.key_off[i] = k0;
        s += (k1 - k0 + kKeyChunk - 1) / kKeyChunk;
    }
    chunks[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t v = threadIdx.x >= (uint32_t)o ? chunks[threadIdx.x - o] : 0;
        __syncthreads();
        chunks[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = chunks[threadIdx.x] - s;
    for (uint32_t i = b; i < e; ++i) {
        A.chunk_off[i] = run;
        uint32_t r1 = i + 1 < n_items ? A.items[i + 1].ray_off * A.D.K : n_rec;
        uint32_t k1 = r1 < n_rec ? A.scan[r1] : *total;
        run += (k1 - A.key_off[i] + kKeyChunk - 1) / kKeyChunk;
    }
    if (threadIdx.x == 1023) {
        A.chunk_off[n_items] = chunks[1023];
        A.key_off[n_items] = *total;
        A.counters[3] = *total;
    }
}

void launch_keys(const LaunchArgs &A, hipStream_t s) {
    const uint32_t n_rec = A.D.T * A.D.K;
    const uint32_t blk = (n_rec + 255) / 256;
    hipLaunchKernelGGL(k_mark, dim3(blk), dim3(256), 0, s, A, n_rec);
    const uint32_t nb = (n_rec + 1023) / 1024;
    uint32_t *total = A.scan_blk + nb;
    exclusive_scan(A.scan, n_rec, A.scan_blk, s);
    hipLaunchKernelGGL(k_compact, dim3(blk), dim3(256), 0, s, A, n_rec, total);
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, s, A, total);
}

template <int KM, int W>
uint32_t refine_cap() {
    static const uint32_t cap = resident_blocks((const void *)k_refine<KM, W, false, false>, kWave);
    return cap;
}

template <int W>
uint32_t refine_cap_k(uint32_t K) {
    switch (K) {
        case 1: return refine_cap<1, W>();
        case 2: return refine_cap<2, W>();
        case 3: return refine_cap<3, W>();
        case 4: return refine_cap<4, W>();
        case 5: return refine_cap<5, W>();
        case 6: return refine_cap<6, W>();
        case 7: return refine_cap<7, W>();
        default: return refine_cap<8, W>();
    }
}

uint32_t refine_grid(const SolveDims &D) {
    const uint32_t cap = D.width == 8 ? refine_cap_k<8>(D.K) : D.width == 4 ? refine_cap_k<4>(D.K) : refine_cap_k<2>(D.K);
    const uint32_t units = D.max_key_chunks * ((D.n_rx + kRefineRxSlice - 1) / kRefineRxSlice);
    return std::max<uint32_t>(1, std::min(cap, units));
}

// Point-set averaging and the polarised field have kernels of their own, so
// that the plain refinement keeps its register allocation.
template <int W>
void launch_refine_w(const LaunchArgs &A, dim3 grid, hipStream_t s) {
    if (A.rb.nk) launch_refine_wa<W, true, false>(A, grid, s);
    else launch_refine_wa<W, false, false>(A, grid, s);
}

void launch_refine(const LaunchArgs &A, hipStream_t s) {
    const dim3 grid(refine_grid(A.D));
    if (A.flags & PCRT_POLARIZED) {
        launch_refine_pol(A, grid, s);
        return;
    }
    switch (A.D.width) {
        case 8: launch_refine_w<8>(A, grid, s); break;
        case 4: launch_refine_w<4>(A, grid, s); break;
        default: launch_refine_w<2>(A, grid, s); break;
    }
}

// Copy of the key list and per-(key, RX) results of a RECORD solve.
__global__ void k_paths_copy(LaunchArgs A, uint32_t cap, uint32_t *key_ray, uint8_t *key_len, int32_t *key_seq,
                             uint8_t *valid, float *length, float *amp, int32_t *hit) {
    const uint32_t n_keys = A.key_off[A.D.n_items];
    const uint32_t K = A.D.K, n_rx = A.D.n_rx;
    const uint32_t lim = min(min(n_keys, cap), A.D.rec_keys);
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < lim; q += gridDim.x * blockDim.x) {
        uint32_t rec = A.keylist[q];
        uint32_t g = rec / K;
        int it;
        uint32_t j = ray_id_of(A, g, &it);
        uint32_t k = rec % K + 1;
        if (key_ray) key_ray[q] = j;
        if (key_len) key_len[q] = (uint8_t)k;
        if (key_seq)
            for (uint32_t m = 0; m < K; ++m) key_seq[(size_t)q * K + m] = m < k ? A.rb.id[(size_t)g * K + m] : -1;
        for (uint32_t r = 0; r < n_rx; ++r) {
            size_t p = (size_t)q * n_rx + r;
            bool v = A.sb.valid[p];
            if (valid) valid[p] = v;
            if (length) length[p] = A.sb.len[p];
            if (amp) {
                float4 a = A.sb.amp[p];
                amp[4 * p] = a.x;
                amp[4 * p + 1] = a.y;
                amp[4 * p + 2] = a.z;
                amp[4 * p + 3] = a.w;
            }
            if (hit)
                for (uint32_t m = 0; m < K; ++m) hit[p * K + m] = (v && m < k) ? A.sb.hit[p * K + m] : -1;
        }
    }
}

void launch_paths_copy(const LaunchArgs &A, uint32_t cap, uint32_t *key_ray, uint8_t *key_len, int32_t *key_seq,
                       uint8_t *valid, float *length, float *amp, int32_t *hit, hipStream_t s) {
    hipLaunchKernelGGL(k_paths_copy, dim3(256), dim3(256), 0, s, A, cap, key_ray, key_len, key_seq, valid, length,
                       amp, hit);
}

}  // namespace pcrt
