// Visibility matrix (Sec. II-A, II-B): whether each receiver sees each point
// set's reception point. Receiver r sees reception point j when the open
// segment between them meets no disk outside set j farther than eps_self
// from both ends (the set's own disks surround its reception point).
//
// Mapping, as for the diffuse connections: a wavefront takes 64 consecutive
// sets (voxel-key order, so neighbouring voxels) against one receiver, and
// every lane walks from the receiver, so the 64 walks share their start and
// their path through the upper tree. Persistent single-wavefront blocks; the
// blocks of XCD x work through the x-th eighth of the (set chunk, receiver)
// units, receiver-minor, so one XCD's L2 serves one region of the scene.
#include "common.h"
#include "internal.h"

namespace pcrt {

template <int W>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(W == 8 ? 4 : 6, 8))) void k_visibility(
    DevScene S, const float *__restrict__ rx, uint32_t n_rx, const float4 *__restrict__ recv, uint32_t n_sets,
    float eps_self, uint8_t *__restrict__ out, uint32_t share) {
    __shared__ int lds_stack[kStackLds * kWave];
    const int lane = threadIdx.x;
    const uint32_t glane = blockIdx.x * kWave + lane;
    Stack stk{lds_stack + lane, S.spill + glane, S.spill_lanes};
    const uint32_t n_units = (n_sets + kWave - 1) / kWave * n_rx;
    const uint32_t xcd = blockIdx.x % kXcds, nb = gridDim.x / kXcds, i = blockIdx.x / kXcds;
    for (uint32_t k = i; k < share; k += nb) {
        const uint32_t u = xcd * share + k;
        if (u >= n_units) break;
        const uint32_t c = u / n_rx, r = u % n_rx;
        const uint32_t j = c * kWave + lane;
        if (j < n_sets) {
            const f3 a = mk(rx[3 * r], rx[3 * r + 1], rx[3 * r + 2]);
            const bool vis = !occluded<W, true>(S, a, xyz(recv[j]), (int)j, eps_self, stk);
            out[(size_t)r * n_sets + j] = vis ? 1 : 0;
        }
    }
}

template <int W>
uint32_t visibility_cap() {
    static const uint32_t cap = resident_blocks((const void *)k_visibility<W>, kWave);
    return cap;
}

uint32_t visibility_grid(uint32_t width) {
    const uint32_t cap = width == 8 ? visibility_cap<8>() : width == 4 ? visibility_cap<4>() : visibility_cap<2>();
    return std::max<uint32_t>(kXcds, cap / kXcds * kXcds);  // a multiple of the XCD count
}

void launch_visibility(const DevScene &S, const float *rx, uint32_t n_rx, const float4 *recv, uint32_t n_sets,
                       float eps_self, uint8_t *out, hipStream_t s) {
    const uint32_t grid = visibility_grid((uint32_t)S.width);
    const uint32_t n_units = (n_sets + kWave - 1) / kWave * n_rx;
    const uint32_t share = (n_units + kXcds - 1) / kXcds;
    switch (S.width) {
        case 8: hipLaunchKernelGGL(k_visibility<8>, dim3(grid), dim3(kWave), 0, s, S, rx, n_rx, recv, n_sets, eps_self,
                                   out, share); break;
        case 4: hipLaunchKernelGGL(k_visibility<4>, dim3(grid), dim3(kWave), 0, s, S, rx, n_rx, recv, n_sets, eps_self,
                                   out, share); break;
        default: hipLaunchKernelGGL(k_visibility<2>, dim3(grid), dim3(kWave), 0, s, S, rx, n_rx, recv, n_sets,
                                    eps_self, out, share); break;
    }
}

__global__ void k_recv_copy(const float4 *__restrict__ recv, uint32_t n, float *__restrict__ out) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const float4 c = recv[j];
        out[3 * (size_t)j] = c.x;
        out[3 * (size_t)j + 1] = c.y;
        out[3 * (size_t)j + 2] = c.z;
    }
}

void launch_recv_copy(const float4 *recv, uint32_t n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_recv_copy, dim3(std::min<uint32_t>((n + 255) / 256, 8192)), dim3(256), 0, s, recv, n, out);
}

}  // namespace pcrt
