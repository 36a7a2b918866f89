// Diffuse connections, line of sight and the per-receiver reduction.
//
// Diffuse scattering is the last interaction of a path (Sec. II-B.1): every
// recorded interaction is connected to every receiver on its lit side by a
// validation segment; visible connections contribute a Lambertian ray-tube
// amplitude. Line of sight is one segment per receiver (Sec. II-B).
//
// All sums are FP64 and deterministic: partial sums are indexed by fixed
// chunks of rays / keys, never by the block that happened to compute them.
#include "common.h"
#include "internal.h"

namespace pcrt {

// Diffuse connections (Sec. II-B.1): each interaction point is joined to
// every receiver on its lit side; a connection counts if nothing lies on the
// open segment between them (any-hit, two-sided disks, the point's own disk
// excluded, eps_self trimmed at both ends).
//
// Mapping. The records are first put in Morton order of their hit points,
// with the transmitter index as the high key bits: a transmitter's records
// keep their range of chunks and only their order inside it changes, so the
// per-chunk partial sums still add up per transmitter. A wavefront takes a
// chunk of spatially adjacent interaction points and one receiver at a time,
// and each lane walks its segment FROM THE RECEIVER towards its interaction
// point (the test is symmetric in the two end points). Walks started together
// then leave the same point with nearly the same direction, make the same
// near-child choices through the upper tree and only part near their own end
// points, which keeps the lanes of a wavefront on the same nodes for most of
// the walk.
//
// Sums: the chunk's visible records for a receiver are listed in record
// order and lane l adds the contributions of list entries l, l + 64, ...; one
// fixed xor-butterfly over the lanes then gives the chunk's partial sum for
// that receiver. The result does
// not depend on timing, on which lane walked which segment, or on the
// hierarchy.
__global__ void k_diffuse_keys(LaunchArgs A) {
    const uint32_t n_rec = A.D.T * A.D.K;
    const float *B = A.S.bounds;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n_rec; r += gridDim.x * blockDim.x) {
        const uint32_t it = (uint32_t)find_item(A.items, A.D.n_items, r / A.D.K);
        uint32_t code = 0xffffffffu;
        if (A.rb.id[r] >= 0) {
            const float4 x = A.rb.xl[r];
            const float c[3] = {x.x, x.y, x.z};
            uint32_t q[3];
            for (int a = 0; a < 3; ++a) {
                const float ext = B[3 + a] - B[a];
                float u = ext > 0.f ? (c[a] - B[a]) / ext : 0.5f;
                u = fminf(fmaxf(u, 0.f), 1.f);
                uint32_t v = (uint32_t)(u * 1023.f);
                v = (v | v << 16) & 0x030000ffu;
                v = (v | v << 8) & 0x0300f00fu;
                v = (v | v << 4) & 0x030c30c3u;
                v = (v | v << 2) & 0x09249249u;
                q[a] = v;
            }
            code = q[0] << 2 | q[1] << 1 | q[2];
        }
        A.dsort.key0[r] = (uint64_t)it << 32 | code;
        A.dsort.val0[r] = r;
    }
}

// Lambertian ray-tube amplitude of one visible connection, from the packed
// record (hit point x, lit-side normal n, unfolded length w from the TX).
__device__ __forceinline__ void diffuse_amplitude(const LaunchArgs &A, uint32_t ri, f3 x, f3 n, float w, f3 rx,
                                                  float budget, double *v5) {
    const f3 v = rx - x;
    const float rs = len(v);
    const float cos_s = dot(v, n) / rs;
    const float a0 = sqrtf(4.f * cos_s / budget) / rs;
    const c32 ph = propagate(w + rs, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
    const float4 cf = A.rb.coef[ri];
    const c32 te = cmul({a0 * cf.x, a0 * cf.y}, ph);
    const c32 tm = cmul({a0 * cf.z, a0 * cf.w}, ph);
    const double tr = te.re, ti = te.im, mr = tm.re, mi = tm.im;
    v5[0] = 0.5 * (tr * tr + ti * ti + mr * mr + mi * mi);
    v5[1] = tr;
    v5[2] = ti;
    v5[3] = mr;
    v5[4] = mi;
}

// The records in Morton order, packed: the connection loop below reads each
// record once per receiver, and the packed copy makes those reads contiguous
// across the lanes and independent of each other (no id -> normal chain).
// Measured on the 1M-point office: 34.0 -> 32.5 ms for the connections, for
// 0.24 ms of packing.
__global__ void k_diffuse_pack(LaunchArgs A, const uint32_t *order) {
    const uint32_t n_rec = A.D.T * A.D.K;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_rec; j += gridDim.x * blockDim.x) {
        const uint32_t ri = order[j];
        const int id = A.rb.id[ri];
        float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f), p1 = make_float4(0.f, 0.f, 1.f, __int_as_float(-1));
        if (id >= 0) {
            p0 = A.rb.xl[ri];
            const f3 nn = record_normal(A, ri);
            p1 = make_float4(nn.x, nn.y, nn.z, __int_as_float(id));
        }
        A.dsort.pack[2 * (size_t)j] = p0;
        A.dsort.pack[2 * (size_t)j + 1] = p1;
    }
}

// Persistent single-wavefront blocks. A work unit is (ray chunk, receiver):
// the wavefront tests the chunk's records against the receiver and writes the
// chunk's partial sums of that receiver itself, so no block barrier ever makes
// it wait for another wavefront. One receiver per unit balanced best on the
// 1M-point office (receivers per unit 32 / 16 / 8 / 4 / 2 / 1: 58.9 / 51.9 /
// 47.8 / 45.7 / 44.4 / 43.5 ms), and the units of one chunk (consecutive
// counter values) then run at the same time on one XCD and share its L2.
//
// Lit compaction. The wavefront classifies the chunk's records 64 at a time
// and queues the offsets of those on the receiver's lit side in LDS, in
// record order, so no lane ever walks a record that is dark or empty for the
// receiver (a fifth of them on the office).
//
// Resumable walks with ballot-compacted refill. Each lane keeps one
// connection's any-hit walk (the walk of occluded(): node, stack, parked
// leaf) across rounds. The wavefront steps its walking lanes until at most a
// quarter of its busy lanes still walk, then hands the lanes whose walks
// ended the next queued records, in lane order (classifying further groups as
// the queue runs low). A lane no longer waits for the longest walk of a
// batch of 64, and the lanes refilled together start from the receiver
// together, on the same upper nodes. Measured on the office (4-wide tree):
// batches of 64 walks 28.7 ms (with grazing and steep connections queued
// apart; 29.1 in one queue); refill when at most half / a quarter / an eighth
// of the busy lanes walk 29.1 / 27.05 / 27.05 ms (at half, the lanes part
// too early to share nodes); grazing and steep queues under refill 0.45 ms
// slower. Parked leaves are tested once half of the walking lanes hold one
// (a third or two thirds: 27.2 and 27.4 ms).
//
// Sums. The walks only decide visibility, kept as one bit per record of the
// chunk in LDS; once the chunk's walks have ended, the visible records are
// listed in record order, lane l adds list entries l, l + 64, ... and one
// fixed butterfly adds the lanes. The sums do not depend on which lane walked
// which connection, nor on the hierarchy. (Groups of 64 records with one lane
// per record, half of them idle, took 0.3 ms more on the office.)
//
// Occupancy: the 6.25 KiB of LDS per wavefront let 25 wavefronts share a
// compute unit's 160 KiB; the 2- and 4-wide walks stay within the register
// budget of six per SIMD (at 80 registers, six beat five by 2-3 % on the
// office; seven and eight spilled and lost). A second queue of 256 B took the
// LDS to 6.5 KiB and the kernel lost 0.6 ms.
constexpr uint32_t kLitQueue = 2 * kWave;  // < 64 queued before a classification + 64 added
constexpr int kRefillShift = 2;            // refill once at most busy / 2^kRefillShift lanes still walk

template <int W>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(W == 8 ? 4 : 6, 8))) void k_diffuse(
    LaunchArgs A) {
    __shared__ int lds_stack[kStackLds * kWave];
    __shared__ uint16_t lit_q[kLitQueue];                 // chunk-relative offsets of lit records
    __shared__ uint32_t vis_bits[kRayChunk * kMaxK / 32];  // visible connections of the chunk
    static_assert(kRayChunk * kMaxK * sizeof(uint16_t) <= sizeof(lds_stack), "the visible list fits the stacks");
    const int lane = threadIdx.x;
    const uint32_t glane = blockIdx.x * kWave + lane;
    Stack stk{lds_stack + lane, A.S.spill + glane, A.S.spill_lanes};
    const uint32_t K = A.D.K, n_rx = A.D.n_rx;
    const uint32_t n_chunks = A.D.n_ray_chunks;
    const bool rec = A.flags & 8;
    const float eps = A.thr.eps_self;
    const uint32_t n_groups = kRayChunk * K / kWave;  // groups of 64 records per chunk
    uint32_t n_seg = 0, n_vis = 0;
    uint64_t n_occ_visits = 0;  // instrumented builds: node visits of occluded segments
    // Workgroups are dealt to the XCDs round robin, and each XCD has its own
    // L2: the wavefronts of XCD x take chunks from the x-th eighth of the
    // (Morton-ordered) chunk range first, so one XCD's L2 serves one region
    // of the scene, then help the other ranges in turn. Within a range, units
    // are receiver-minor, so consecutive units reuse a chunk's records.
    const uint32_t xcd = blockIdx.x % kXcds;
    enum { kIdle = 0, kWalk = 1, kDone = 2 };
    for (;;) {
        uint32_t u = 0xffffffffu;
        if (lane == 0) {
            for (uint32_t k = 0; k < kXcds; ++k) {
                const uint32_t x = (xcd + k) % kXcds;
                const uint32_t lo = (uint32_t)((uint64_t)x * n_chunks / kXcds) * n_rx;
                const uint32_t hi = (uint32_t)((uint64_t)(x + 1) * n_chunks / kXcds) * n_rx;
                const uint32_t uu = lo + atomicAdd(&A.work[8 + x], 1u);
                if (uu < hi) {
                    u = uu;
                    break;
                }
            }
        }
        u = __builtin_amdgcn_readfirstlane(u);
        if (u == 0xffffffffu) break;
        const uint32_t c = u / n_rx, r = u % n_rx;
        const uint32_t g0 = c * kRayChunk;
        const f3 rx = mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]);
        for (uint32_t i = lane; i < 2 * n_groups; i += kWave) vis_bits[i] = 0u;
        uint32_t q = 0, head = 0, tail = 0;  // next group to classify; queue positions (wave-uniform)
        int phase = kIdle;
        uint32_t mo = 0;  // this lane's record, chunk-relative
        int excl = -1, ref = kNoRef, sp = 0, park = kNoRef;
        bool hit = false;
        f3 d = mk(0.f, 0.f, 1.f), inv = mk(1.f, 1.f, 1.f), oi = mk(0.f, 0.f, 0.f);
        float t_hi = 0.f;
        Octant oq = octant<W>(inv);
        uint32_t nv0 = 0;
        for (;;) {
            const uint64_t idle = __ballot(phase == kIdle);
            const uint32_t n_idle = (uint32_t)__popcll(idle);
            while (tail - head < n_idle && q < n_groups) {
                const uint32_t o = q * kWave + lane;
                const uint32_t j = g0 * K + o;
                const float4 p0 = A.dsort.pack[2 * (size_t)j], p1 = A.dsort.pack[2 * (size_t)j + 1];
                const float vn = dot(rx - xyz(p0), xyz(p1));
                const bool lit = __float_as_int(p1.w) >= 0 && vn > 0.f;
                if (rec && !lit) A.dvis[(size_t)A.dsort.order[j] * n_rx + r] = 0;
                const uint64_t m = __ballot(lit);
                if (lit) lit_q[(tail + mbcnt(m)) % kLitQueue] = (uint16_t)o;
                tail += (uint32_t)__popcll(m);
                ++q;
            }
            __syncthreads();
            const uint32_t avail = min(tail - head, n_idle);
            if (phase == kIdle && mbcnt(idle) < avail) {
                mo = lit_q[(head + mbcnt(idle)) % kLitQueue];
                const uint32_t j = g0 * K + mo;
                const float4 p0 = A.dsort.pack[2 * (size_t)j], p1 = A.dsort.pack[2 * (size_t)j + 1];
                excl = __float_as_int(p1.w);
                // the set-up of occluded(rx, x): walked from the receiver
                const f3 dv = xyz(p0) - rx;
                const float L = len(dv);
                d = (1.0f / L) * dv;
                inv = safe_inv(d);
                oi = times(rx, inv);
                oq = octant<W>(inv);
                t_hi = L - eps;
                ref = t_hi > eps ? A.S.root : kNoRef;
                sp = 0;
                park = kNoRef;
                hit = false;
                phase = kWalk;
                ++n_seg;
                nv0 = stk.nv;
            }
            head += avail;
            __syncthreads();  // the taken queue slots may be refilled next round
            const uint32_t n_busy = (uint32_t)__popcll(__ballot(phase != kIdle));
            if (n_busy == 0) break;  // the chunk's lit records are all walked
            // A lane that is not walking holds ref = park = kNoRef, so the node
            // and leaf conditions below need no phase test; the count of walking
            // lanes only changes when walks end, between the rounds of node steps.
            uint32_t n_walk = (uint32_t)__popcll(__ballot(phase == kWalk));
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
                        if (!step_any<W>(A.S, ref, sp, oq, inv, oi, eps, t_hi, stk))
                            ref = sp > 0 ? stk.get(--sp) : kNoRef;
                    }
                }
                if (park != kNoRef) {
                    const int v = -1 - park;
                    const int first = v >> 3, cnt = (v & 7) + 1;
                    stk.test(cnt);
                    for (int i = 0; i < cnt; ++i) {
                        const float4 dp = ld4(A.S.disk, (uint32_t)(first + i) * 32u);
                        const float4 dn = ld4(A.S.disk, (uint32_t)(first + i) * 32u + 16u);
                        float t, d2;
                        const bool h = disk_hit(rx, d, xyz(dp), xyz(dn), A.S.r2, t, d2);
                        if (h & (__float_as_int(dp.w) != excl) & (t > eps) & (t < t_hi)) {
                            hit = true;
                            break;
                        }
                    }
                    park = kNoRef;
                    if (hit) ref = kNoRef;
                }
                if (phase == kWalk && ref == kNoRef && park == kNoRef) phase = kDone;
                n_walk = (uint32_t)__popcll(__ballot(phase == kWalk));
                if (n_walk == 0 || (n_walk << kRefillShift) <= n_busy) break;
            }
            if (phase == kDone) {
                if (kCountVisits && hit) n_occ_visits += stk.nv - nv0;
                if (rec) A.dvis[(size_t)A.dsort.order[g0 * K + mo] * n_rx + r] = !hit;
                if (!hit) {
                    atomicOr(&vis_bits[mo >> 5], 1u << (mo & 31));
                    ++n_vis;
                }
                phase = kIdle;
            }
        }
        __syncthreads();
        // The visible records in record order, listed in the LDS of the walks'
        // stacks (every walk has ended: at most 2 KiB of offsets); lane l then
        // adds list entries l, l + 64, ..., so every lane computes amplitudes
        // (not only those whose own record of a group is visible).
        uint16_t *vlist = (uint16_t *)lds_stack;
        uint32_t n_list = 0;
        for (uint32_t g = 0; g < n_groups; ++g) {
            const uint64_t m = (uint64_t)vis_bits[2 * g] | ((uint64_t)vis_bits[2 * g + 1] << 32);
            if ((m >> lane) & 1u) vlist[n_list + mbcnt(m)] = (uint16_t)(g * kWave + lane);
            n_list += (uint32_t)__popcll(m);
        }
        __syncthreads();
        const Item I = A.items[find_item(A.items, A.D.n_items, g0)];
        const float budget = (float)I.budget;
        double acc[5] = {};
        for (uint32_t i = (uint32_t)lane; i < n_list; i += kWave) {
            const uint32_t j = g0 * K + vlist[i];
            const float4 p0 = A.dsort.pack[2 * (size_t)j], p1 = A.dsort.pack[2 * (size_t)j + 1];
            double v5[5];
            diffuse_amplitude(A, A.dsort.order[j], xyz(p0), xyz(p1), p0.w, rx, budget, v5);
            for (int a = 0; a < 5; ++a) acc[a] += v5[a];
        }
        double sv[5];
        for (int a = 0; a < 5; ++a) sv[a] = wave_sum_d(acc[a]);
        if (lane == 0) {
            double *o = A.diff_part + ((size_t)c * n_rx + r) * 5;
            for (int a = 0; a < 5; ++a) o[a] = sv[a];
        }
        __syncthreads();  // the visibility bits are cleared and the stacks reused by the next unit
    }
    flush_visits(stk, A.counters, 13);
    n_seg = warp_sum_u(n_seg);
    n_vis = warp_sum_u(n_vis);
    if (kCountVisits)
        for (int o = 32; o > 0; o >>= 1) n_occ_visits += __shfl_xor(n_occ_visits, o, kWave);
    if (lane == 0) {
        atomicAdd((unsigned long long *)&A.counters[2], (unsigned long long)n_seg);
        atomicAdd((unsigned long long *)&A.counters[5], (unsigned long long)n_vis);
        if (kCountVisits) atomicAdd((unsigned long long *)&A.counters[15], (unsigned long long)n_occ_visits);
    }
}

template <int W>
uint32_t diffuse_cap() {
    static const uint32_t cap = resident_blocks((const void *)k_diffuse<W>, kWave);
    return cap;
}

uint32_t diffuse_grid(const SolveDims &D) {
    const uint32_t cap = D.width == 8 ? diffuse_cap<8>() : D.width == 4 ? diffuse_cap<4>() : diffuse_cap<2>();
    const uint32_t units = D.n_ray_chunks * D.n_rx;
    return std::max<uint32_t>(1, std::min(cap, units));
}

const uint32_t *launch_diffuse_order(const LaunchArgs &A, hipStream_t s) {
    const uint32_t n_rec = A.D.T * A.D.K;
    hipLaunchKernelGGL(k_diffuse_keys, dim3(std::min<uint32_t>((n_rec + 255) / 256, 8192)), dim3(256), 0, s, A);
    int item_bits = 0;
    while ((1u << item_bits) < A.D.n_items) ++item_bits;
    const int hi = 32 + 8 * ((item_bits + 7) / 8);  // 30 Morton bits, then the transmitter index
    const bool in1 = radix_sort_u64(A.dsort.key0, A.dsort.val0, A.dsort.key1, A.dsort.val1, n_rec, 0, hi,
                                    A.dsort.hist, A.dsort.blk, s);
    const uint32_t *order = in1 ? A.dsort.val1 : A.dsort.val0;
    hipLaunchKernelGGL(k_diffuse_pack, dim3(std::min<uint32_t>((n_rec + 255) / 256, 8192)), dim3(256), 0, s, A, order);
    return order;
}

void launch_diffuse(const LaunchArgs &A, hipStream_t s) {
    const dim3 g(diffuse_grid(A.D));
    switch (A.D.width) {
        case 8: hipLaunchKernelGGL(k_diffuse<8>, g, dim3(kWave), 0, s, A); break;
        case 4: hipLaunchKernelGGL(k_diffuse<4>, g, dim3(kWave), 0, s, A); break;
        default: hipLaunchKernelGGL(k_diffuse<2>, g, dim3(kWave), 0, s, A); break;
    }
}

// Diffuse paths of the reception-point launch (Sec. II-B.1, II-B.4): one per
// unique voxel diffuse key (surface labels before the last interaction, point
// set of the last), its representative's record giving the geometry. A path
// reaches receiver r when r sees the set's reception point (the visibility
// matrix) and lies on the lit side of the interaction; it stands for the field
// scattered by an area rho^2 there, a Lambertian patch lit from the (image)
// transmitter at the unfolded length L:
//   a0 = sqrt(rho^2 cos_i cos_s / pi) / (L r_s)   (times lambda/4pi S and the chain, in coef)
// Block: a share of the keys x 64 receivers (dps_key_range); each thread adds
// its receiver's paths over its part in key order (keys are in record order),
// FP64.
__global__ __launch_bounds__(kDpsWaves * kWave) void k_dps_diffuse(LaunchArgs A, float area) {
    __shared__ double red[kDpsWaves][kWave][5];
    const uint32_t n_rx = A.D.n_rx;
    const uint32_t n_keys = A.dkey_off[A.D.n_items];
    const uint32_t w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const uint32_t c = blockIdx.x, r = blockIdx.y * kWave + lane;
    const float inv_pi = (float)(1.0 / kPi);
    double acc[5] = {0, 0, 0, 0, 0};
    uint32_t n_vis = 0;
    if (r < n_rx) {
        const f3 rx = mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]);
        uint32_t q0, k1;
        dps_key_range(n_keys, c, A.D.n_ray_chunks, w, q0, k1);
        for (uint32_t q = q0; q < k1; ++q) {
            const uint32_t ri = A.dkeylist[q];
            const int id = A.rb.id[ri];
            if (!A.dps_vis[(size_t)r * A.S.n_sets + A.S.dps_of[id]]) continue;
            const float4 xl = A.rb.xl[ri];
            const f3 v = rx - xyz(xl);
            const float vn = dot(v, record_normal(A, ri));
            if (!(vn > 0.f)) continue;
            const float rs = len(v);
            const float a0 = sqrtf(area * fabsf(A.rb.cs[ri]) * (vn / rs) * inv_pi) / (xl.w * rs);
            const c32 ph = propagate(xl.w + rs, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
            const float4 cf = A.rb.coef[ri];
            const c32 te = cmul({a0 * cf.x, a0 * cf.y}, ph);
            const c32 tm = cmul({a0 * cf.z, a0 * cf.w}, ph);
            const double tr = te.re, ti = te.im, mr = tm.re, mi = tm.im;
            acc[0] += 0.5 * (tr * tr + ti * ti + mr * mr + mi * mi);
            acc[1] += tr;
            acc[2] += ti;
            acc[3] += mr;
            acc[4] += mi;
            ++n_vis;
        }
    }
    dps_block_sum(red, w, lane, acc, r < n_rx ? A.diff_part + ((size_t)c * n_rx + r) * 5 : nullptr);
    n_vis = warp_sum_u(n_vis);
    if (lane == 0 && n_vis) atomicAdd((unsigned long long *)&A.counters[5], (unsigned long long)n_vis);
}

uint32_t dps_key_cap(const SolveDims &D) {  // twice the records, a power of two
    const uint64_t want = 2ull * D.T * D.K + 1;
    uint32_t cap = 1;
    while (cap < want && cap < (1u << 31)) cap <<= 1;
    return cap;
}

void launch_dps_diffuse(const LaunchArgs &A, float area, hipStream_t s) {
    // compact the voxel diffuse keys with the specular key machinery on the other table
    LaunchArgs B = A;
    B.hb = A.dhb;
    B.rb.slot = A.rb.dslot;
    B.keylist = A.dkeylist;
    B.key_off = A.dkey_off;
    B.chunk_off = A.dchunk_off;
    B.counters = A.dcnt;
    fill_u32(B.key_off, 0, A.D.n_items + 1, s);
    fill_u32(B.chunk_off, 0, A.D.n_items + 1, s);
    launch_keys(B, s);
    const dim3 g(A.D.n_ray_chunks, (A.D.n_rx + kWave - 1) / kWave);
    hipLaunchKernelGGL(k_dps_diffuse, g, dim3(kDpsWaves * kWave), 0, s, A, area);
}

template <int W>
__global__ __launch_bounds__(kWave) void k_los(LaunchArgs A) {
    __shared__ int lds_stack[kStackLds * kWave];
    const int lane = threadIdx.x;
    const uint32_t glane = blockIdx.x * kWave + lane;
    Stack stk{lds_stack + lane, A.S.spill + glane, A.S.spill_lanes};
    const uint32_t n = A.D.n_items * A.D.n_rx;
    const uint32_t p = glane;
    if (p >= n) return;
    const uint32_t it = p / A.D.n_rx, r = p % A.D.n_rx;
    const Item I = A.items[it];
    const f3 tx = mk(I.tx[0], I.tx[1], I.tx[2]);
    const f3 rx = mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]);
    double *o = A.los_part + (size_t)p * 5;
    if (occluded<W>(A.S, tx, rx, -1, A.thr.eps_self, stk)) {
        for (int a = 0; a < 5; ++a) o[a] = 0.0;
        return;
    }
    const float d = len(rx - tx);
    const c32 ph = propagate(d, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
    float a0 = A.fc.amp_iso / d;
    if (A.flags & PCRT_POLARIZED) {  // the two dipoles' transverse parts
        const f3 u = (1.0f / d) * (rx - tx);
        a0 *= dot(transverse(A.pol_tx, u), transverse(A.pol_rx, u));
    }
    const double ar = a0 * ph.re, ai = a0 * ph.im;
    o[0] = ar * ar + ai * ai;
    o[1] = ar;
    o[2] = ai;
    o[3] = ar;
    o[4] = ai;
}

// Per (transmitter, receiver), one 256-lane block: LOS + specular chunks +
// diffuse chunks. Lane t sums chunks t, t+256, ... in order; the lanes are
// then combined by a fixed pairwise tree, so the result is bitwise repeatable.
__global__ __launch_bounds__(256) void k_combine(LaunchArgs A, double *gain, double *h_te, double *h_tm,
                                                 double *parts) {
    __shared__ double red[256][10];
    const uint32_t p = blockIdx.x;
    const uint32_t it = p / A.D.n_rx, r = p % A.D.n_rx;
    const uint32_t n_rx = A.D.n_rx;
    const int t = threadIdx.x;
    double sp[5] = {0, 0, 0, 0, 0}, df[5] = {0, 0, 0, 0, 0};
    if (A.flags & 2) {
        for (uint32_t c = A.chunk_off[it] + t; c < A.chunk_off[it + 1]; c += 256)
            for (int a = 0; a < 5; ++a) sp[a] += A.spec_part[((size_t)c * n_rx + r) * 5 + a];
    }
    if (A.flags & 4) {
        const Item I = A.items[it];
        const uint32_t c0 = I.ray_off / kRayChunk;
        const uint32_t c1 = c0 + (I.n_rays + kRayChunk - 1) / kRayChunk;
        for (uint32_t c = c0 + t; c < c1; c += 256)
            for (int a = 0; a < 5; ++a) df[a] += A.diff_part[((size_t)c * n_rx + r) * 5 + a];
    }
    for (int a = 0; a < 5; ++a) {
        red[t][a] = sp[a];
        red[t][5 + a] = df[a];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s)
            for (int a = 0; a < 10; ++a) red[t][a] += red[t + s][a];
        __syncthreads();
    }
    if (t != 0) return;
    double los[5] = {0, 0, 0, 0, 0};
    if (A.flags & 1)
        for (int a = 0; a < 5; ++a) los[a] = A.los_part[(size_t)p * 5 + a];
    double *S = red[0];
    gain[p] = los[0] + S[0] + S[5];
    if (h_te) {
        h_te[2 * p] = los[1] + S[1] + S[6];
        h_te[2 * p + 1] = los[2] + S[2] + S[7];
    }
    if (h_tm) {
        h_tm[2 * p] = los[3] + S[3] + S[8];
        h_tm[2 * p + 1] = los[4] + S[4] + S[9];
    }
    if (parts) {
        parts[3 * p] = los[0];
        parts[3 * p + 1] = S[0];
        parts[3 * p + 2] = S[5];
    }
}

void launch_los_and_combine(const LaunchArgs &A, double *gain, double *h_te, double *h_tm, double *parts,
                            hipStream_t s) {
    const uint32_t n = A.D.n_items * A.D.n_rx;
    if (A.flags & 1) {
        const dim3 g((n + kWave - 1) / kWave);
        switch (A.D.width) {
            case 8: hipLaunchKernelGGL(k_los<8>, g, dim3(kWave), 0, s, A); break;
            case 4: hipLaunchKernelGGL(k_los<4>, g, dim3(kWave), 0, s, A); break;
            default: hipLaunchKernelGGL(k_los<2>, g, dim3(kWave), 0, s, A); break;
        }
    }
    launch_combine(A, gain, h_te, h_tm, parts, s);
}

void launch_combine(const LaunchArgs &A, double *gain, double *h_te, double *h_tm, double *parts, hipStream_t s) {
    const uint32_t n = A.D.n_items * A.D.n_rx;
    hipLaunchKernelGGL(k_combine, dim3(n), dim3(256), 0, s, A, gain, h_te, h_tm, parts);
}

}  // namespace pcrt
