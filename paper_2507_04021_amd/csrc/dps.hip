// Discretised point sets (Sec. II-A): the point centres are binned into
// voxels of edge rho and every non-empty voxel is one set. The members of a
// set are stored together (centre and id, normal), so the weighted-average
// intersection (Sec. II-C) reads a set as one contiguous run.
//
// Steps: a 63-bit key per point (21 bits per axis, biased voxel index, x
// major), a stable radix sort of (key, id), set heads where the key changes,
// an exclusive scan of the heads, then one pass that writes the members, the
// set offsets and the set of every id. Members of a set keep increasing id
// order (the sort is stable and starts from ids in order).
#include "common.h"
#include "internal.h"

namespace pcrt {

constexpr int kVoxBits = 21;
constexpr int64_t kVoxBias = 1ll << 20;  // voxel indices in [-2^20, 2^20)

__global__ void k_voxel_keys(const float4 *__restrict__ pos, uint32_t n, double rho, uint64_t *__restrict__ key,
                             uint32_t *__restrict__ val, uint32_t *__restrict__ stat) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float4 p = pos[i];
        const double c[3] = {p.x, p.y, p.z};
        uint64_t k = 0;
        bool bad = false;
        for (int a = 0; a < 3; ++a) {
            const double v = floor(c[a] / rho);  // FP64, correctly rounded division
            const bool in = v >= -(double)kVoxBias && v < (double)kVoxBias;
            bad |= !in;
            k = k << kVoxBits | (in ? (uint64_t)((int64_t)v + kVoxBias) : 0ull);
        }
        if (bad) atomicOr(stat, 1u);
        key[i] = k;
        val[i] = i;
    }
}

__global__ void k_set_heads(const uint64_t *__restrict__ key, uint32_t n, uint32_t *__restrict__ head) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        head[j] = (j == 0 || key[j] != key[j - 1]) ? 1u : 0u;
}

// scan: exclusive scan of the heads (sets that start before j).
__global__ void k_set_fill(const uint64_t *__restrict__ key, const uint32_t *__restrict__ id,
                           const uint32_t *__restrict__ scan, uint32_t n, const float4 *__restrict__ pos,
                           const float4 *__restrict__ nrm, float4 *__restrict__ pt, uint32_t *__restrict__ off,
                           uint32_t *__restrict__ of, uint32_t *__restrict__ stat) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const bool head = j == 0 || key[j] != key[j - 1];
        const uint32_t g = scan[j] + (head ? 1u : 0u) - 1u;
        const uint32_t i = id[j];
        of[i] = g;
        if (head) off[g] = j;
        const float4 p = pos[i], q = nrm[i];
        pt[2 * (size_t)j] = make_float4(p.x, p.y, p.z, __int_as_float((int)i));
        pt[2 * (size_t)j + 1] = make_float4(q.x, q.y, q.z, 0.f);
        if (j == n - 1) {
            off[g + 1] = n;
            stat[1] = g + 1;
        }
    }
}

// Reception point of each set (Sec. II-A): the mean of its members' centres,
// summed in FP64 in member order and rounded to FP32.
__global__ void k_set_recv(const float4 *__restrict__ pt, const uint32_t *__restrict__ off,
                           const uint32_t *__restrict__ stat, float4 *__restrict__ recv) {
    const uint32_t n_sets = stat[1];
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < n_sets; g += gridDim.x * blockDim.x) {
        double x = 0.0, y = 0.0, z = 0.0;
        const uint32_t b = off[g], e = off[g + 1];
        for (uint32_t m = b; m < e; ++m) {
            const float4 p = pt[2 * (size_t)m];
            x += p.x;
            y += p.y;
            z += p.z;
        }
        const double c = (double)(e - b);
        recv[g] = make_float4((float)(x / c), (float)(y / c), (float)(z / c), 0.f);
    }
}

// The set of every leaf-ordered disk goes into the spare word of its normal,
// so walks that must ignore one set test it without another load.
__global__ void k_disk_sets(float4 *__restrict__ disk, uint32_t n, const uint32_t *__restrict__ of) {
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int id = __float_as_int(disk[2 * (size_t)k].w);
        disk[2 * (size_t)k + 1].w = __int_as_float((int)of[id]);
    }
}

hipError_t build_point_sets(const SceneLayout &L, char *ws, uint32_t n, float rho, hipStream_t s) {
    auto P = [&](size_t o) { return ws + o; };
    uint64_t *k0 = (uint64_t *)P(L.code0), *k1 = (uint64_t *)P(L.code1);
    uint32_t *v0 = (uint32_t *)P(L.idx0), *v1 = (uint32_t *)P(L.idx1);
    uint32_t *stat = (uint32_t *)P(L.dps_stat), *flag = (uint32_t *)P(L.dps_flag);
    const dim3 g(std::min<uint32_t>((n + 255) / 256, 8192)), b(256);
    fill_u32(stat, 0u, 2, s);
    hipLaunchKernelGGL(k_voxel_keys, g, b, 0, s, (const float4 *)P(L.pos_id), n, (double)rho, k0, v0, stat);
    const bool in1 = radix_sort_u64(k0, v0, k1, v1, n, 0, 3 * kVoxBits, (uint32_t *)P(L.hist),
                                    (uint32_t *)P(L.scan_blk), s);
    const uint64_t *key = in1 ? k1 : k0;
    const uint32_t *id = in1 ? v1 : v0;
    hipLaunchKernelGGL(k_set_heads, g, b, 0, s, key, n, flag);
    exclusive_scan(flag, n, (uint32_t *)P(L.dps_blk), s);
    hipLaunchKernelGGL(k_set_fill, g, b, 0, s, key, id, flag, n, (const float4 *)P(L.pos_id),
                       (const float4 *)P(L.nrm_id), (float4 *)P(L.dps_pt), (uint32_t *)P(L.dps_off),
                       (uint32_t *)P(L.dps_of), stat);
    hipLaunchKernelGGL(k_set_recv, g, b, 0, s, (const float4 *)P(L.dps_pt), (const uint32_t *)P(L.dps_off),
                       (const uint32_t *)stat, (float4 *)P(L.dps_recv));
    hipLaunchKernelGGL(k_disk_sets, g, b, 0, s, (float4 *)P(L.disk), n, (const uint32_t *)P(L.dps_of));
    return hipGetLastError();
}

}  // namespace pcrt
