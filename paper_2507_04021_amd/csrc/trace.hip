// Ray launch and the constant-count bounce loop (Sec. II-B): every ray keeps
// bouncing specularly for up to K interactions; each interaction is recorded,
// its specular prefix key (surface-label sequence, Sec. II-B.4) is inserted
// into a per-transmitter hash set, and -- for diffuse scattering -- the
// Fresnel-weighted coefficient of the chain up to this point is stored.
//
// Persistent grid of one-wave blocks; each wave takes 64 consecutive ray
// slots from an atomic counter until the rays run out.
#include "common.h"
#include "internal.h"

namespace pcrt {

__device__ __forceinline__ uint32_t key_insert(const HashBufs &hb, uint32_t base, uint64_t enc, uint32_t j,
                                               uint64_t *status) {
    const uint32_t mask = hb.cap - 1;
    uint32_t slot = (uint32_t)mix64(enc) & mask;
    for (uint32_t probe = 0; probe < hb.cap; ++probe) {
        unsigned long long *kp = hb.key + base + slot;
        unsigned long long cur = __hip_atomic_load(kp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == 0ull) cur = atomicCAS(kp, 0ull, (unsigned long long)enc);
        if (cur == 0ull || cur == enc) {
            uint32_t *rp = hb.rep + base + slot;
            if (__hip_atomic_load(rp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > j) atomicMin(rp, j);
            return slot;
        }
        slot = (slot + 1) & mask;
    }
    atomicOr((unsigned long long *)status, 1ull);
    return 0xffffffffu;
}

// One ray slot g: launch direction, up to K closest hits, records.
template <int W>
__device__ __forceinline__ void trace_one(const LaunchArgs &A, uint32_t g, Stack &stk, uint32_t &n_int,
                                          uint32_t &n_ray, uint32_t &n_spill) {
    const uint32_t K = A.D.K;
    const bool want_diff = A.flags & 4, want_spec = A.flags & 2;
    const bool want_geom = A.flags & (4 | 8 | 32);  // points/lengths/cosines: diffuse, tape, averaged planes
    const bool avg = A.flags & 32;             // weighted-average intersection over point sets
    const int it = find_item(A.items, A.D.n_items, g);
    const Item I = A.items[it];
    const uint32_t local = g - I.ray_off;
    const size_t rb = (size_t)g * K;
    if (local >= I.n_rays) {
        for (uint32_t k = 0; k < K; ++k) A.rb.id[rb + k] = -1;
        return;
    }
    const uint32_t j = A.subset ? A.subset[local] : local;
    f3 d;
    if (A.flags & 64) {  // towards reception point j (Sec. II-B): FP64 direction, rounded to FP32
        if (j >= A.S.n_sets) {
            for (uint32_t k = 0; k < K; ++k) A.rb.id[rb + k] = -1;
            n_ray += 1;
            return;
        }
        d = normalize(aim_dir(I.tx, A.S.dps_recv[j]));
    } else {
        d = normalize(fib_dir(j, I.budget));
    }
    f3 o = mk(I.tx[0], I.tx[1], I.tx[2]);
    float L = 0.f;
    int excl = -1;
    c32 pte = {1.f, 0.f}, ptm = {1.f, 0.f};
    uint64_t enc = 0;
    uint32_t k = 0;
    for (; k < K; ++k) {
        float t;
        bool sp;
        int h = closest_hit<W>(A.S, o, d, excl, A.thr.eps_self, A.thr.eps_tie, stk, t, sp);
        n_spill += sp;
        if (h < 0) break;
        const float4 pn = A.S.nrm[h];
        f3 n = xyz(pn);
        if (avg) {  // the point set's weighted average replaces the disk's point and normal
            dps_average(A.S, o, d, excl, A.thr.eps_self, A.thr.lambda_d, h, t, n);
            A.rb.nk[rb + k] = make_float4(n.x, n.y, n.z, 0.f);
        }
        float dn = dot(d, n);
        float sgn = dn > 0.f ? -1.f : 1.f;
        float cosi = fabsf(dn);
        f3 q = o + t * d;
        L += t;
        A.rb.id[rb + k] = h;
        if (want_geom) {
            A.rb.xl[rb + k] = make_float4(q.x, q.y, q.z, L);
            A.rb.cs[rb + k] = sgn * cosi;
        }
        if (want_diff) {
            uint32_t lab = __float_as_uint(pn.w);
            if (lab >= A.n_labels) {
                atomicOr((unsigned long long *)&A.counters[6], 2ull);
                lab = 0;
            }
            float er = A.mats[3 * lab], sg = A.mats[3 * lab + 1], sc = A.mats[3 * lab + 2];
            c32 te, tm;
            fresnel(er, sg * A.fc.inv_we0, cosi, te, tm);
            c32 cte = cmul(pte, te), ctm = cmul(ptm, tm);
            float w = A.fc.amp_iso * sc;
            A.rb.coef[rb + k] = make_float4(w * cte.re, w * cte.im, w * ctm.re, w * ctm.im);
            float R = sqrtf(fmaxf(0.f, 1.f - sc * sc));
            pte = {R * cte.re, R * cte.im};
            ptm = {R * ctm.re, R * ctm.im};
        }
        if (A.rb.dslot) {  // voxel diffuse key: labels before this interaction, then this point set
            const uint64_t encd = enc * (uint64_t)A.S.n_sets + (uint64_t)A.S.dps_of[h] + 1ull;
            A.rb.dslot[rb + k] = key_insert(A.dhb, 0u, encd, j, A.counters + 6);
        }
        if (want_spec || A.rb.dslot) {
            uint32_t su = __float_as_uint(A.S.pos[h].w);
            enc = enc * (uint64_t)A.n_surf1 + (uint64_t)(su + 1);
            if (want_spec) A.rb.slot[rb + k] = key_insert(A.hb, (uint32_t)it * A.hb.cap, enc, j, A.counters + 6);
        }
        d = normalize(d - (2.f * dn) * n);
        o = q;
        excl = h;
    }
    for (uint32_t kk = k; kk < K; ++kk) A.rb.id[rb + kk] = -1;
    n_int += k;
    n_ray += 1;
}

// Persistent wavefronts take wave_rays consecutive ray slots per atomic
// fetch; each lane traces wave_rays / 64 of them in turn. Five wavefronts
// per SIMD for the 2- and 4-wide walks (four without the register cap):
// 3.62 -> 3.32 ms on the office.
template <int W>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(W == 8 ? 3 : 5, 8))) void k_trace(
    LaunchArgs A) {
    __shared__ int lds_stack[kStackLds * kWave];
    const int lane = threadIdx.x;
    const uint32_t glane = blockIdx.x * kWave + lane;
    Stack stk{lds_stack + lane, A.S.spill + glane, A.S.spill_lanes};
    const uint32_t T = A.D.T;
    const uint32_t U = A.wave_rays / kWave;
    const uint32_t n_units = (T + A.wave_rays - 1) / A.wave_rays;
    uint32_t n_int = 0, n_ray = 0, n_spill = 0;
    for (;;) {
        uint32_t unit = 0;
        if (lane == 0) unit = atomicAdd(&A.work[0], 1u);
        unit = __shfl(unit, 0, kWave);
        if (unit >= n_units) break;
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t g = unit * A.wave_rays + u * kWave + lane;
            if (g < T) trace_one<W>(A, g, stk, n_int, n_ray, n_spill);
        }
    }
    flush_visits(stk, A.counters, 9);
    n_int = warp_sum_u(n_int);
    n_ray = warp_sum_u(n_ray);
    n_spill = warp_sum_u(n_spill);
    if (lane == 0) {
        atomicAdd((unsigned long long *)&A.counters[0], (unsigned long long)n_int);
        atomicAdd((unsigned long long *)&A.counters[1], (unsigned long long)n_ray);
        atomicAdd((unsigned long long *)&A.counters[8], (unsigned long long)n_spill);
    }
}

uint32_t resident_blocks(const void *kernel, int block_threads) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block_threads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 2048;  // no device to ask: an upper bound for 256 compute units
    }
    return (uint32_t)std::max(per_cu, 1) * (uint32_t)std::max(cus, 1);
}

template <int W>
uint32_t trace_cap() {
    static const uint32_t cap = resident_blocks((const void *)k_trace<W>, kWave);
    return cap;
}

uint32_t trace_grid(const SolveDims &D, uint32_t wave_rays) {
    const uint32_t cap = D.width == 8 ? trace_cap<8>() : D.width == 4 ? trace_cap<4>() : trace_cap<2>();
    const uint32_t units = (D.T + wave_rays - 1) / wave_rays;
    return std::max<uint32_t>(1, std::min(cap, units));
}

void launch_trace(const LaunchArgs &A, hipStream_t s) {
    uint32_t grid = trace_grid(A.D, A.wave_rays);
    switch (A.D.width) {
        case 8: hipLaunchKernelGGL(k_trace<8>, dim3(grid), dim3(kWave), 0, s, A); break;
        case 4: hipLaunchKernelGGL(k_trace<4>, dim3(grid), dim3(kWave), 0, s, A); break;
        default: hipLaunchKernelGGL(k_trace<2>, dim3(grid), dim3(kWave), 0, s, A); break;
    }
}

__global__ void k_raygen(uint32_t n_budget, const uint32_t *ids, uint32_t n, float *out) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    f3 d = fib_dir(ids ? ids[i] : i, n_budget);
    out[3 * i] = d.x;
    out[3 * i + 1] = d.y;
    out[3 * i + 2] = d.z;
}

void launch_raygen(uint32_t n_budget, const uint32_t *ids, uint32_t n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_raygen, dim3((n + 255) / 256), dim3(256), 0, s, n_budget, ids, n, out);
}

}  // namespace pcrt
