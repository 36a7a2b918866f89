// Ray launch and the constant-count bounce loop (Sec. II-B): every ray keeps
// bouncing specularly for up to K interactions; each interaction is recorded,
// its specular prefix key (surface-label sequence, Sec. II-B.4) is inserted
// into a per-transmitter hash set, and -- for diffuse scattering -- the
// Fresnel-weighted coefficient of the chain up to this point is stored.
//
// Persistent grid of one-wave blocks; each wave reserves wave_rays
// consecutive ray slots per atomic fetch and hands them to its idle lanes.
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

// Resumable closest-hit walk of one lane: the walk of closest_hit (near
// child first, tie window, candidate list with its exact second pass), its
// state kept across the bounce loop's iterations; park holds a leaf reached
// but not yet tested.
struct Walk {
    f3 inv, oi;
    int ref, sp, park;
    float tmin;
    Cand c[kTieList];
    bool spill, pass2;  // candidate list overflowed; second (exact) pass running
    float t_win, bd2, bt;
    int bid;
};

__device__ __forceinline__ void walk_start(Walk &w, int root, f3 o, f3 d) {
    w.inv = safe_inv(d);
    w.oi = times(o, w.inv);
    w.ref = root;
    w.sp = 0;
    w.park = kNoRef;
    w.tmin = INFINITY;
#pragma unroll
    for (int q = 0; q < kTieList; ++q) w.c[q] = {INFINITY, INFINITY, -1};
    w.spill = w.pass2 = false;
    w.t_win = 0.f;
    w.bd2 = w.bt = INFINITY;
    w.bid = 0x7fffffff;
}

// One node of the walk: true if a child was entered (ref is then that child,
// the other entered children are on the stack).
template <int W>
__device__ __forceinline__ bool node_step(const DevScene &S, Walk &w, float t_lo, float tc, Stack &stk) {
    if constexpr (W > 2) {
        return wide_step<W>(S, w.ref, w.sp, w.inv, w.oi, t_lo, tc, stk);
    } else {
        const uint32_t nb = (uint32_t)w.ref * 64u;
        const float4 a = ld4(S.node, nb), b = ld4(S.node, nb + 16u), e = ld4(S.node, nb + 32u), r = ld4(S.node, nb + 48u);
        float n0, n1;
        const bool h0 = box_hit(a.x, a.y, a.z, a.w, b.x, b.y, w.inv, w.oi, t_lo, tc, n0);
        const bool h1 = box_hit(b.z, b.w, e.x, e.y, e.z, e.w, w.inv, w.oi, t_lo, tc, n1);
        const int r0 = __float_as_int(r.x), r1 = __float_as_int(r.y);
        if (h0 && h1) {
            const bool f0 = n0 <= n1;
            stk.put(w.sp++, f0 ? r1 : r0);
            w.ref = f0 ? r0 : r1;
            return true;
        }
        if (h0 | h1) {
            w.ref = h0 ? r0 : r1;
            return true;
        }
        return false;
    }
}

// The bounce loop (Sec. II-B) with ballot-compacted ray refill. Every lane
// keeps one ray's state -- its bounce, origin, direction, unfolded length,
// chain coefficients and key -- and the state of its current closest-hit
// walk, which resumes from one iteration to the next. The wavefront steps
// its walking lanes until at most half of its busy lanes are still walking;
// the lanes whose walks ended then finish their bounce together (record the
// interaction, reflect) and start the next bounce's walk, and lanes whose
// rays ended are refilled, compacted in lane order by a ballot, from the ray
// slots the wavefront reserved (wave_rays per atomic fetch). Within the
// walking, a lane that reaches a leaf parks it and keeps taking node steps
// (the next stack entry) until half of the walking lanes hold a leaf; the
// parked leaves are then tested together, so node and leaf steps rarely
// share an iteration. A lane never waits for the wavefront's longest walk.
// Parking only delays when a leaf's disks are tested; the nearest hit and its
// tie rule do not depend on the visiting order, so the results are those of
// closest_hit (bitwise, tested). Measured on the 1M-point office (4-wide
// tree, leaf 2): 3.11 ms -> 2.46 ms; without parking the refill alone gave
// 3.26 ms (node and leaf steps in the same iterations), and half / half
// thresholds beat one third or two thirds for either.
template <int W>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(W == 8 ? 3 : 4, 8))) void k_trace(
    LaunchArgs A) {
    __shared__ int lds_stack[kStackLds * kWave];
    const int lane = threadIdx.x;
    const uint32_t glane = blockIdx.x * kWave + lane;
    Stack stk{lds_stack + lane, A.S.spill + glane, A.S.spill_lanes};
    const uint32_t T = A.D.T, K = A.D.K;
    const bool want_diff = A.flags & 4, want_spec = A.flags & 2;
    const bool want_geom = A.flags & (4 | 8 | 32);  // points/lengths/cosines: diffuse, tape, averaged planes
    const bool avg = A.flags & 32;                  // weighted-average intersection over point sets
    const float eps_self = A.thr.eps_self, eps_tie = A.thr.eps_tie;
    enum { kIdle = 0, kWalk = 1, kDone = 2 };
    int phase = kIdle;
    uint32_t g = 0, j = 0, k = 0;
    int it = 0, excl = -1;
    f3 o = mk(0.f, 0.f, 0.f), d = mk(0.f, 0.f, 1.f);
    float L = 0.f;
    c32 pte = {1.f, 0.f}, ptm = {1.f, 0.f};
    uint64_t enc = 0;
    Walk w;
    walk_start(w, A.S.root, o, d);
    uint32_t q_next = 0, q_end = 0;  // this wavefront's reserved ray slots [q_next, q_end)
    bool q_dry = false;
    uint32_t n_int = 0, n_ray = 0, n_spill = 0;
    for (;;) {
        // refill idle lanes, in lane order, from the reserved slots
        for (;;) {
            const uint64_t idle = __ballot(phase == kIdle);
            if (!idle || q_dry) break;
            if (q_next >= q_end) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(&A.work[0], A.wave_rays);
                base = __builtin_amdgcn_readfirstlane(base);
                if (base >= T) {
                    q_dry = true;
                    break;
                }
                q_next = base;
                q_end = min(base + A.wave_rays, T);
            }
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
            const uint32_t avail = q_end - q_next;
            if (phase == kIdle && rank < avail) {
                g = q_next + rank;
                it = find_item(A.items, A.D.n_items, g);
                const Item &I = A.items[it];
                const uint32_t local = g - I.ray_off;
                const size_t rb = (size_t)g * K;
                if (local >= I.n_rays) {  // padding slot of the item
                    for (uint32_t kk = 0; kk < K; ++kk) A.rb.id[rb + kk] = -1;
                } else {
                    j = A.subset ? A.subset[local] : local;
                    bool live = true;
                    if (A.flags & 64) {  // towards reception point j (Sec. II-B): FP64 direction, rounded to FP32
                        if (j >= A.S.n_sets) {
                            for (uint32_t kk = 0; kk < K; ++kk) A.rb.id[rb + kk] = -1;
                            n_ray += 1;
                            live = false;
                        } else {
                            d = normalize(aim_dir(I.tx, A.S.dps_recv[j]));
                        }
                    } else {
                        d = normalize(fib_dir(j, I.budget));
                    }
                    if (live) {
                        o = mk(I.tx[0], I.tx[1], I.tx[2]);
                        L = 0.f;
                        excl = -1;
                        pte = ptm = {1.f, 0.f};
                        enc = 0;
                        k = 0;
                        walk_start(w, A.S.root, o, d);
                        phase = kWalk;
                    }
                }
            }
            q_next += min((uint32_t)__popcll(idle), avail);
        }
        const uint32_t n_busy = (uint32_t)__popcll(__ballot(phase != kIdle));
        if (n_busy == 0) break;  // the slots are used up and every ray has ended
        // walk until at most half of the busy lanes are still walking; node steps
        // run until half of the walking lanes hold a leaf (parked), then the
        // parked leaves are tested together
        for (;;) {
            for (;;) {
                if (phase == kWalk && w.ref < 0 && w.ref != kNoRef && w.park == kNoRef) {
                    w.park = w.ref;
                    w.ref = w.sp > 0 ? stk.get(--w.sp) : kNoRef;
                }
                const uint32_t n_walk = (uint32_t)__popcll(__ballot(phase == kWalk));
                const uint32_t n_park = (uint32_t)__popcll(__ballot(phase == kWalk && w.park != kNoRef));
                if (!__ballot(phase == kWalk && w.ref >= 0) || 2 * n_park >= n_walk) break;
                if (phase == kWalk && w.ref >= 0) {
                    stk.visit();
                    const float tc = w.pass2 ? w.t_win : w.tmin + eps_tie;
                    if (!node_step<W>(A.S, w, eps_self, tc, stk)) w.ref = w.sp > 0 ? stk.get(--w.sp) : kNoRef;
                }
            }
            if (phase == kWalk && w.park != kNoRef) {
                const int v = -1 - w.park;
                const int first = v >> 3, cnt = (v & 7) + 1;
                stk.test(cnt);
                for (int i = 0; i < cnt; ++i) {
                    if (w.pass2)
                        visit_disk<true>(A.S, first + i, o, d, excl, eps_self, eps_tie, w.tmin, w.c, w.spill, w.t_win,
                                         w.bd2, w.bid, w.bt);
                    else
                        visit_disk<false>(A.S, first + i, o, d, excl, eps_self, eps_tie, w.tmin, w.c, w.spill,
                                          w.t_win, w.bd2, w.bid, w.bt);
                }
                w.park = kNoRef;
            }
            if (phase == kWalk && w.ref == kNoRef) phase = kDone;
            const uint32_t n_walk = (uint32_t)__popcll(__ballot(phase == kWalk));
            if (n_walk == 0 || 2 * n_walk <= n_busy) break;
        }
        if (phase != kDone) continue;
        // this lane's walk ended: the second, exact pass if the tie list overflowed, else the bounce
        if (w.spill && !w.pass2 && w.tmin < INFINITY) {
            n_spill += 1;
            w.pass2 = true;
            w.t_win = w.tmin + eps_tie;
            w.ref = A.S.root;
            w.sp = 0;
            w.park = kNoRef;
            phase = kWalk;
            continue;
        }
        int h = -1;
        float t = INFINITY;
        if (w.tmin < INFINITY) {
            if (w.pass2) {
                h = w.bid;
                t = w.bt;
            } else {
#pragma unroll
                for (int q = 0; q < kTieList; ++q)
                    if (w.c[q].id >= 0 && (w.c[q].d2 < w.bd2 || (w.c[q].d2 == w.bd2 && w.c[q].id < w.bid))) {
                        w.bd2 = w.c[q].d2;
                        w.bid = w.c[q].id;
                        w.bt = w.c[q].t;
                    }
                h = w.bid;
                t = w.bt;
            }
        }
        const size_t rb = (size_t)g * K;
        if (h < 0) {  // the ray leaves the scene
            for (uint32_t kk = k; kk < K; ++kk) A.rb.id[rb + kk] = -1;
            n_int += k;
            n_ray += 1;
            phase = kIdle;
            continue;
        }
        const float4 pn = A.S.nrm[h];
        f3 n = xyz(pn);
        if (avg) {  // the point set's weighted average replaces the disk's point and normal
            dps_average(A.S, o, d, excl, eps_self, A.thr.lambda_d, h, t, n);
            A.rb.nk[rb + k] = make_float4(n.x, n.y, n.z, 0.f);
        }
        const float dn = dot(d, n);
        const float sgn = dn > 0.f ? -1.f : 1.f;
        const float cosi = fabsf(dn);
        const f3 q = fma3(t, d, o);
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
            const float er = A.mats[3 * lab], sg = A.mats[3 * lab + 1], sc = A.mats[3 * lab + 2];
            c32 te, tm;
            fresnel(er, sg * A.fc.inv_we0, cosi, te, tm);
            const c32 cte = cmul(pte, te), ctm = cmul(ptm, tm);
            const float wgt = A.fc.amp_iso * sc;
            A.rb.coef[rb + k] = make_float4(wgt * cte.re, wgt * cte.im, wgt * ctm.re, wgt * ctm.im);
            const float R = sqrtf(fmaxf(0.f, 1.f - sc * sc));
            pte = {R * cte.re, R * cte.im};
            ptm = {R * ctm.re, R * ctm.im};
        }
        if (A.rb.dslot) {  // voxel diffuse key: labels before this interaction, then this point set
            const uint64_t encd = enc * (uint64_t)A.S.n_sets + (uint64_t)A.S.dps_of[h] + 1ull;
            A.rb.dslot[rb + k] = key_insert(A.dhb, 0u, encd, j, A.counters + 6);
        }
        if (want_spec || A.rb.dslot) {
            const uint32_t su = __float_as_uint(A.S.pos[h].w);
            enc = enc * (uint64_t)A.n_surf1 + (uint64_t)(su + 1);
            if (want_spec) A.rb.slot[rb + k] = key_insert(A.hb, (uint32_t)it * A.hb.cap, enc, j, A.counters + 6);
        }
        d = normalize(fma3(-2.f * dn, n, d));
        o = q;
        excl = h;
        k += 1;
        if (k == K) {
            n_int += K;
            n_ray += 1;
            phase = kIdle;
        } else {
            walk_start(w, A.S.root, o, d);
            phase = kWalk;
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
