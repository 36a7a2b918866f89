// Visibility matrix (Sec. II-A, II-B): whether each receiver sees each point
// set's reception point. Receiver r sees reception point j when the open
// segment between them meets no disk outside set j farther than eps_self
// from both ends (the set's own disks surround its reception point).
//
// Mapping, as for the diffuse connections: a wavefront takes a chunk of
// kVisChunk consecutive sets (voxel-key order, so neighbouring voxels)
// against one receiver, and every lane walks from the receiver, so walks
// started together share their start and their path through the upper tree.
// Walks are resumable with ballot-compacted refill, as in the diffuse
// connections: the wavefront steps its walking lanes until at most a quarter
// of its busy lanes still walk, then hands the idle lanes the chunk's next
// sets in lane order. Each output byte is written by the lane that decided
// it, so the result does not depend on the schedule. On the office's 64 x
// 181 523 matrix: 2.65 ms with one 64-set batch per unit and no refill,
// 1.7 ms with refill over 1024-set units. Persistent
// single-wavefront blocks; the blocks of XCD x work through the x-th eighth
// of the (set chunk, receiver) units, receiver-minor, so one XCD's L2 serves
// one region of the scene.
#include "common.h"
#include "internal.h"

namespace pcrt {

constexpr uint32_t kVisChunk = 1024;  // sets per work unit (office: 128 / 256 / 512 / 1024 / 2048 ->
                                      // 2.65 / 2.16 / 2.0 / 1.7 / 1.89 ms)
constexpr int kVisRefillShift = 2;    // refill once at most busy / 4 lanes still walk

template <int W>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(W == 8 ? 4 : 6, 8))) void k_visibility(
    DevScene S, const float *__restrict__ rx, uint32_t n_rx, const float4 *__restrict__ recv, uint32_t n_sets,
    float eps_self, uint8_t *__restrict__ out, uint32_t share) {
    __shared__ int lds_stack[kStackLds * kWave];
    const int lane = threadIdx.x;
    const uint32_t glane = blockIdx.x * kWave + lane;
    Stack stk{lds_stack + lane, S.spill + glane, S.spill_lanes};
    const uint32_t n_units = (n_sets + kVisChunk - 1) / kVisChunk * n_rx;
    const uint32_t xcd = blockIdx.x % kXcds, nb = gridDim.x / kXcds, i = blockIdx.x / kXcds;
    for (uint32_t k = i; k < share; k += nb) {
        const uint32_t u = xcd * share + k;
        if (u >= n_units) break;
        const uint32_t c = u / n_rx, r = u % n_rx;
        const f3 a = mk(rx[3 * r], rx[3 * r + 1], rx[3 * r + 2]);
        const uint32_t j0 = c * kVisChunk, j1 = min(n_sets, j0 + kVisChunk);
        uint32_t next = j0;                   // next set of the chunk to hand out (wave-uniform)
        bool walking = false, hit = false;
        uint32_t j = 0;
        int ref = kNoRef, sp = 0, park = kNoRef;  // kNoRef / kNoRef whenever the lane is not walking
        f3 d = mk(0.f, 0.f, 1.f), inv = mk(1.f, 1.f, 1.f), oi = mk(0.f, 0.f, 0.f);
        float t_hi = 0.f;
        Octant oq = octant<W>(inv);
        for (;;) {
            const uint64_t idle = __ballot(!walking);
            const uint32_t avail = min(j1 - next, (uint32_t)__popcll(idle));
            if (!walking && mbcnt(idle) < avail) {
                j = next + mbcnt(idle);
                // the set-up of occluded(a, recv[j]), walked from the receiver
                const f3 dv = xyz(recv[j]) - a;
                const float L = len(dv);
                d = (1.0f / L) * dv;
                inv = safe_inv(d);
                oi = times(a, inv);
                oq = octant<W>(inv);
                t_hi = L - eps_self;
                ref = t_hi > eps_self ? S.root : kNoRef;
                sp = 0;
                park = kNoRef;
                hit = false;
                walking = true;
            }
            next += avail;
            const uint32_t n_busy = (uint32_t)__popcll(__ballot(walking));
            if (n_busy == 0) break;  // the chunk's sets are all decided
            uint32_t n_walk = n_busy;
            for (;;) {
                for (;;) {
                    if (ref < 0 && ref != kNoRef && park == kNoRef) {
                        park = ref;
                        ref = sp > 0 ? stk.get(--sp) : kNoRef;
                    }
                    const uint32_t n_park = (uint32_t)__popcll(__ballot(park != kNoRef));
                    if (!__ballot(ref >= 0) || 2 * n_park >= n_walk) break;
                    if (ref >= 0) {
                        stk.visit();
                        if (!step_any<W>(S, ref, sp, oq, inv, oi, eps_self, t_hi, stk))
                            ref = sp > 0 ? stk.get(--sp) : kNoRef;
                    }
                }
                if (park != kNoRef) {
                    const int v = -1 - park;
                    const int first = v >> 3, cnt = (v & 7) + 1;
                    stk.test(cnt);
                    for (int q = 0; q < cnt; ++q) {
                        const float4 dp = ld4(S.disk, (uint32_t)(first + q) * 32u);
                        const float4 dn = ld4(S.disk, (uint32_t)(first + q) * 32u + 16u);
                        float t, d2;
                        const bool h = disk_hit(a, d, xyz(dp), xyz(dn), S.r2, t, d2);
                        if (h & (__float_as_int(dn.w) != (int)j) & (t > eps_self) & (t < t_hi)) {
                            hit = true;
                            break;
                        }
                    }
                    park = kNoRef;
                    if (hit) ref = kNoRef;
                }
                const bool done = walking && ref == kNoRef && park == kNoRef;
                if (done) {
                    out[(size_t)r * n_sets + j] = hit ? 0 : 1;
                    walking = false;
                }
                n_walk = (uint32_t)__popcll(__ballot(walking));
                if (n_walk == 0 || (n_walk << kVisRefillShift) <= n_busy) break;
            }
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
    const uint32_t n_units = (n_sets + kVisChunk - 1) / kVisChunk * n_rx;
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
