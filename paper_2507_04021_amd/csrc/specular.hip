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

// Image method on k planes (exact minimiser of Eq. (1) restricted to them):
// images I_m of the TX, back-trace from the RX; every segment must cross its
// plane strictly inside, and both neighbours of x_m must lie strictly on the
// same side of plane m, farther than eps_self (a reflection, not a
// transmission).
template <int KM>
__device__ __forceinline__ bool refine_planes(int k, f3 tx, f3 rx, const f3 *pp, const f3 *pn, float eps_self,
                                              f3 *x) {
    f3 img[KM + 1];
    img[0] = tx;
#pragma unroll
    for (int m = 1; m <= KM; ++m)
        if (m <= k) img[m] = img[m - 1] - (2.f * dot(img[m - 1] - pp[m - 1], pn[m - 1])) * pn[m - 1];
    x[0] = tx;
    f3 cur = rx;
#pragma unroll
    for (int m = KM; m >= 1; --m) {
        if (m > k) continue;
        f3 seg = img[m] - cur;
        float den = dot(seg, pn[m - 1]);
        if (den == 0.f) return false;
        float s = dot(pp[m - 1] - cur, pn[m - 1]) / den;
        if (!(s > 0.f && s < 1.f)) return false;
        cur = cur + s * seg;
        x[m] = cur;
    }
#pragma unroll
    for (int m = 1; m <= KM; ++m) {
        if (m > k) continue;
        f3 nb = (m == k) ? rx : x[m + 1];
        float da = dot(x[m - 1] - pp[m - 1], pn[m - 1]);
        float db = dot(nb - pp[m - 1], pn[m - 1]);
        if (!(da * db > 0.f && fabsf(da) > eps_self && fabsf(db) > eps_self)) return false;
    }
    return true;
}

struct PairOut {
    bool valid;
    float len;
    c32 te, tm;
};

// The representative's interaction planes of key q: its first k hit disks'
// planes, or with point-set averaging its first k averaged interactions
// (point and normal from the records).
template <int KM>
struct KeyPlanes {
    f3 pp[KM], pn[KM];
    uint32_t ks[KM];  // surface labels
    int k;
};

template <int KM, bool AVG>
__device__ __forceinline__ void load_planes(const LaunchArgs &A, uint32_t q, KeyPlanes<KM> &kp) {
    const uint32_t K = A.D.K;
    const uint32_t rec = A.keylist[q];
    const uint32_t g = rec / K;
    kp.k = (int)(rec % K) + 1;
#pragma unroll
    for (int m = 0; m < KM; ++m)
        if (m < kp.k) {
            const size_t ri = (size_t)g * K + m;
            const int id = A.rb.id[ri];
            const float4 p4 = A.S.pos[id];
            kp.ks[m] = __float_as_uint(p4.w);
            if (AVG) {
                kp.pp[m] = xyz(A.rb.xl[ri]);
                kp.pn[m] = xyz(A.rb.nk[ri]);
            } else {
                kp.pp[m] = xyz(p4);
                kp.pn[m] = xyz(A.S.nrm[id]);
            }
        }
}

__device__ __forceinline__ f3 rx_point(const LaunchArgs &A, uint32_t r) {
    return mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]);
}

// One validation pass of a (key, receiver) candidate on its current planes
// (the key's disk planes, some replaced after earlier passes): a ray from each
// image point to the next must hit a disk of the expected surface, close in
// angle (t_a) and plane distance (t_d). The first interaction that fails
// those two tests asks for another pass with that plane replaced by the hit
// disk's (kPassRetry: slot, disk), unless retries already equals kappa; any
// other failure ends the candidate. If every interaction holds, the last
// point must see the receiver, and the path's field is evaluated. With
// point-set averaging the validation hit is averaged over its set first
// (Sec. II-C): its point and normal are tested, and a retry takes them as the
// new plane (rp, rn).
enum { kPassDone = 0, kPassRetry = 1 };

template <int KM, int W, bool AVG>
__device__ int validate_pass(const LaunchArgs &A, uint32_t q, uint32_t r, f3 tx, const KeyPlanes<KM> &kp,
                             int retries, Stack &stk, PairOut &po, int &slot, int &disk, f3 &rp, f3 &rn) {
    po.valid = false;
    const uint32_t K = A.D.K;
    const int k = kp.k;
    const f3 rx = rx_point(A, r);
    f3 x[KM + 1];
    int hid[KM];
    if (!refine_planes<KM>(k, tx, rx, kp.pp, kp.pn, A.thr.eps_self, x)) return kPassDone;
    int prev = -1;
    bool retry = false, fail = false;
#pragma unroll
    for (int m = 1; m <= KM; ++m) {
        if (m > k || retry || fail) continue;
        f3 u = normalize(x[m] - x[m - 1]);
        float t;
        bool sp;
        int h = closest_hit<W>(A.S, x[m - 1], u, prev, A.thr.eps_self, A.thr.eps_tie, stk, t, sp);
        if (h < 0) { fail = true; continue; }
        float4 hp = A.S.pos[h];
        if (__float_as_uint(hp.w) != kp.ks[m - 1]) { fail = true; continue; }
        f3 hn = xyz(A.S.nrm[h]);
        if (AVG) dps_average(A.S, x[m - 1], u, prev, A.thr.eps_self, A.thr.lambda_d, h, t, hn);
        f3 qh = x[m - 1] + t * u;
        bool ang_ok = fabsf(dot(hn, kp.pn[m - 1])) >= A.thr.cos_ta;
        bool dist_ok = fabsf(dot(qh - kp.pp[m - 1], kp.pn[m - 1])) <= A.thr.t_d;
        if (!(ang_ok && dist_ok)) {
            if (retries >= A.thr.kappa) { fail = true; continue; }
            slot = m - 1;
            disk = h;
            if (AVG) {
                rp = qh;
                rn = hn;
            }
            retry = true;
            continue;
        }
        hid[m - 1] = h;
        prev = h;
    }
    if (fail) return kPassDone;
    if (retry) return kPassRetry;
    f3 xk = x[1];
    int hk = hid[0];
#pragma unroll
    for (int m = 1; m <= KM; ++m)
        if (m == k) {
            xk = x[m];
            hk = hid[m - 1];
        }
    if (occluded<W>(A.S, xk, rx, hk, A.thr.eps_self, stk)) return kPassDone;
    float L = 0.f;
    c32 pte = {1.f, 0.f}, ptm = {1.f, 0.f};
    float csv[KM];
#pragma unroll
    for (int m = 1; m <= KM; ++m) {
        if (m > k) continue;
        f3 seg = x[m] - x[m - 1];
        float sl = len(seg);
        L += sl;
        float c = fabsf(dot((1.0f / sl) * seg, kp.pn[m - 1]));
        csv[m - 1] = c;
        uint32_t lab = __float_as_uint(A.S.nrm[hid[m - 1]].w);
        if (lab >= A.n_labels) lab = 0;
        float er = A.mats[3 * lab], sg = A.mats[3 * lab + 1], sc = A.mats[3 * lab + 2];
        c32 te, tm;
        fresnel(er, sg * A.fc.inv_we0, c, te, tm);
        float R = sqrtf(fmaxf(0.f, 1.f - sc * sc));
        pte = cmul(pte, {R * te.re, R * te.im});
        ptm = cmul(ptm, {R * tm.re, R * tm.im});
    }
    L += len(rx - xk);
    c32 ph = propagate(L, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
    float a0 = A.fc.amp_iso / L;
    po.te = cmul({a0 * pte.re, a0 * pte.im}, ph);
    po.tm = cmul({a0 * ptm.re, a0 * ptm.im}, ph);
    po.len = L;
    po.valid = true;
    if ((A.flags & 8) && q < A.D.rec_keys) {
        size_t p = (size_t)q * A.D.n_rx + r;
#pragma unroll
        for (int m = 0; m < KM; ++m)
            if (m < k) {
                A.sb.hit[p * K + m] = hid[m];
                A.sb.cs[p * K + m] = csv[m];
            }
    }
    return kPassDone;
}

// Persistent single-wavefront blocks. A work unit is (key chunk, slice of up
// to kRefineRxSlice receivers); units are handed out by an atomic counter,
// slice-minor so that consecutive units reuse a chunk's key planes.
//
// The wavefront deals a unit's (key, receiver) pairs to its lanes in tiles
// of 64 and solves the image method for each pair (cheap, no traversal);
// pairs with a solution join a queue in LDS. Whenever 64 are queued, or no
// tile is left to run, every lane takes one queued candidate through ONE
// validation pass. A pass that asks for a plane replacement puts the
// candidate back at the end of the queue with that replacement recorded
// (the disk whose plane it takes), so a candidate that needs many passes
// holds one lane for one pass at a time. Up to two units are open at once:
// while the last candidates of one unit still cycle through the queue, the
// tiles of the next unit refill it, so the batches stay full.
//
// Sums: a path's amplitudes go to this block's result slots, indexed by the
// open unit and the pair within it, with a bit in LDS. When a unit is done,
// lane r adds the paths of receiver r in increasing key order and writes the
// unit's partial sum of receiver r0 + r for chunk c. The result does not
// depend on timing or on the order in which passes ran.
constexpr int kRefineOpen = 2;          // units open at once per wavefront

template <int KM>
struct QEntry {
    uint32_t e;   // pair within its unit: key * nr + receiver
    int slot;     // open-unit slot
    int retries;  // passes so far that ended in a plane replacement
    int ovr[KM];  // per interaction: the disk whose plane replaced the key's, -1 if none
};

struct RefUnit {  // an open unit (wavefront-uniform)
    uint32_t c, r0, nr, q0, ne, t, pending;  // pending: candidates queued or in a pass
    f3 tx;
    bool open;
};

// Global-memory writes of some lanes of a single-wavefront block are visible
// to its other lanes after this.
__device__ __forceinline__ void block_sync_global() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Occupancy: four wavefronts per SIMD up to K = 5 (a 128-register budget,
// with a few spills): on the office two gave 6.1 ms, three 4.8, four 4.7.
template <int KM, int W, bool AVG>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(KM <= 5 ? 4 : 2, 8))) void k_refine(
    LaunchArgs A) {
    constexpr uint32_t kUnitPairs = kKeyChunk * kRefineRxSlice;
    static_assert(kRefineOpen == 2 && kRefineOpen * kUnitPairs == kRefineResPerBlock, "two open units");
    __shared__ int lds_stack[kStackLds * kWave];
    __shared__ QEntry<KM> queue[kRefineQueue];
    __shared__ uint32_t vbits[kRefineOpen][kUnitPairs / 32];  // pairs of an open unit that are paths
    const int lane = threadIdx.x;
    const uint64_t below = (1ull << lane) - 1;
    const uint32_t glane = blockIdx.x * kWave + lane;
    Stack stk{lds_stack + lane, A.S.spill + glane, A.S.spill_lanes};
    float4 *res = A.spec_res + (size_t)blockIdx.x * kRefineOpen * kUnitPairs;
    // point-set averaging: the current planes of a queued candidate with
    // retries sit at its ring position, (point, normal) per interaction
    constexpr bool avg = AVG;
    float4 *qpl = avg ? A.spec_ovr + (size_t)blockIdx.x * kRefineQueue * KM * 2 : nullptr;
    const uint32_t n_rx = A.D.n_rx, n_items = A.D.n_items;
    const uint32_t n_chunks = A.chunk_off[n_items];
    const uint32_t n_slices = (n_rx + kRefineRxSlice - 1) / kRefineRxSlice;
    const uint32_t n_units = n_chunks * n_slices;
    const bool rec = A.flags & 8;
    uint32_t n_cand = 0, n_valid = 0;
    RefUnit U[kRefineOpen];
#pragma unroll
    for (int k = 0; k < kRefineOpen; ++k) U[k] = RefUnit{0, 0, 0, 0, 0, 0, 0, mk(0.f, 0.f, 0.f), false};
    bool exhausted = false;       // the unit counter has run out
    uint32_t head = 0, tail = 0;  // queue ring positions (wavefront-uniform)
    for (;;) {
        // close the units whose tiles are done and whose candidates have all ended
#pragma unroll
        for (int k = 0; k < kRefineOpen; ++k) {
            if (!(U[k].open && U[k].t * kWave >= U[k].ne && U[k].pending == 0)) continue;
            block_sync_global();  // result slots written by other lanes are visible
            if ((uint32_t)lane < U[k].nr) {
                double acc[5] = {0, 0, 0, 0, 0};
                for (uint32_t e = (uint32_t)lane; e < U[k].ne; e += U[k].nr)  // increasing key
                    if ((vbits[k][e >> 5] >> (e & 31)) & 1u) {
                        const float4 v = res[k * kUnitPairs + e];
                        const double tr = v.x, ti = v.y, mr = v.z, mi = v.w;
                        acc[0] += 0.5 * (tr * tr + ti * ti + mr * mr + mi * mi);
                        acc[1] += tr;
                        acc[2] += ti;
                        acc[3] += mr;
                        acc[4] += mi;
                    }
                double *o = A.spec_part + ((size_t)U[k].c * n_rx + U[k].r0 + lane) * 5;
                for (int a = 0; a < 5; ++a) o[a] = acc[a];
            }
            block_sync_global();  // sums read before the slot is reused
            U[k].open = false;
        }
        const uint32_t live = tail - head;
        if (live < (uint32_t)kWave) {
            // image-test tile of an open unit with tiles left, else of a newly opened one
            int s = -1;
#pragma unroll
            for (int k = 0; k < kRefineOpen; ++k)
                if (s < 0 && U[k].open && U[k].t * kWave < U[k].ne) s = k;
            if (s < 0 && !exhausted) {
#pragma unroll
                for (int k = 0; k < kRefineOpen; ++k) {
                    if (s >= 0 || U[k].open) continue;
                    uint32_t u = 0;
                    if (lane == 0) u = atomicAdd(&A.work[1], 1u);
                    u = __builtin_amdgcn_readfirstlane(u);
                    if (u >= n_units) {
                        exhausted = true;
                        break;
                    }
                    const uint32_t c = u / n_slices;
                    int lo = 0, hi = (int)n_items - 1;  // item of this chunk
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (A.chunk_off[mid] <= c) lo = mid;
                        else hi = mid - 1;
                    }
                    const Item I = A.items[lo];
                    U[k].c = c;
                    U[k].r0 = (u % n_slices) * kRefineRxSlice;
                    U[k].nr = min((uint32_t)kRefineRxSlice, n_rx - U[k].r0);
                    U[k].q0 = A.key_off[lo] + (c - A.chunk_off[lo]) * kKeyChunk;
                    const uint32_t q1 = min(U[k].q0 + kKeyChunk, A.key_off[lo + 1]);
                    U[k].ne = (q1 - U[k].q0) * U[k].nr;
                    U[k].t = 0;
                    U[k].pending = 0;
                    U[k].tx = mk(I.tx[0], I.tx[1], I.tx[2]);
                    U[k].open = true;
                    if ((uint32_t)lane < kUnitPairs / 32) vbits[k][lane] = 0u;
                    wave_sync();
                    s = k;
                }
            }
            auto tile = [&](RefUnit &R, int slot) {
                const uint32_t e = R.t * kWave + lane;
                bool cand = false;
                if (e < R.ne) {
                    const uint32_t q = R.q0 + e / R.nr, r = R.r0 + e % R.nr;
                    KeyPlanes<KM> kp;
                    load_planes<KM, AVG>(A, q, kp);
                    f3 x[KM + 1];
                    cand = refine_planes<KM>(kp.k, R.tx, rx_point(A, r), kp.pp, kp.pn, A.thr.eps_self, x);
                    // launch at the reception points: only where the receiver sees the reception
                    // point of the set the representative ray ends in (the visibility matrix)
                    if (cand && A.dps_vis)
                        cand = A.dps_vis[(size_t)r * A.S.n_sets + A.S.dps_of[A.rb.id[A.keylist[q]]]] != 0;
                    if (rec) {
                        if (q >= A.D.rec_keys) {
                            atomicOr((unsigned long long *)&A.counters[6], 4ull);  // tape capacity exceeded
                        } else if (!cand) {
                            const size_t p = (size_t)q * n_rx + r;
                            A.sb.valid[p] = 0;
                            A.sb.len[p] = 0.f;
                            A.sb.amp[p] = make_float4(0.f, 0.f, 0.f, 0.f);
                        }
                    }
                }
                n_cand += cand;
                const uint64_t m = __ballot(cand);
                if (cand) {
                    QEntry<KM> &qe = queue[(tail + (uint32_t)__popcll(m & below)) % kRefineQueue];
                    qe.e = e;
                    qe.slot = slot;
                    qe.retries = 0;
#pragma unroll
                    for (int j = 0; j < KM; ++j) qe.ovr[j] = -1;
                }
                tail += (uint32_t)__popcll(m);
                R.pending += (uint32_t)__popcll(m);
                ++R.t;
                wave_sync();
            };
            if (s == 0) {
                tile(U[0], 0);
                continue;
            }
            if (s == 1) {
                tile(U[1], 1);
                continue;
            }
        }
        if (live == 0) break;  // no tile to run, nothing queued, every unit closed
        // one validation pass for up to 64 queued candidates
        const uint32_t nb = min(live, (uint32_t)kWave);
        const bool have = (uint32_t)lane < nb;
        QEntry<KM> me;
        const uint32_t at = (head + lane) % kRefineQueue;
        if (have) me = queue[at];
        head += nb;
        wave_sync();  // taken entries are read before their ring slots are reused
        bool again = false, ended = false;
        KeyPlanes<KM> kp;
        if (have) {
            const bool s1 = me.slot == 1;
            const uint32_t nr = s1 ? U[1].nr : U[0].nr;
            const uint32_t q = (s1 ? U[1].q0 : U[0].q0) + me.e / nr;
            const uint32_t r = (s1 ? U[1].r0 : U[0].r0) + me.e % nr;
            const f3 tx = s1 ? U[1].tx : U[0].tx;
            load_planes<KM, AVG>(A, q, kp);
#pragma unroll
            for (int j = 0; j < KM; ++j)
                if (j < kp.k && me.ovr[j] >= 0) {
                    if (avg) {
                        kp.pp[j] = xyz(qpl[((size_t)at * KM + j) * 2]);
                        kp.pn[j] = xyz(qpl[((size_t)at * KM + j) * 2 + 1]);
                    } else {
                        kp.pp[j] = xyz(A.S.pos[me.ovr[j]]);
                        kp.pn[j] = xyz(A.S.nrm[me.ovr[j]]);
                    }
                }
            PairOut po;
            int slot = 0, disk = -1;
            f3 rp = mk(0.f, 0.f, 0.f), rn = mk(0.f, 0.f, 1.f);
            const int out = validate_pass<KM, W, AVG>(A, q, r, tx, kp, me.retries, stk, po, slot, disk, rp, rn);
            if (out == kPassRetry) {
                again = true;
                me.retries += 1;
#pragma unroll
                for (int j = 0; j < KM; ++j)
                    if (j == slot) {
                        me.ovr[j] = disk;
                        if (AVG) {
                            kp.pp[j] = rp;
                            kp.pn[j] = rn;
                        }
                    }
            } else {
                ended = true;
                if (rec && q < A.D.rec_keys) {
                    const size_t p = (size_t)q * n_rx + r;
                    A.sb.valid[p] = po.valid;
                    A.sb.len[p] = po.valid ? po.len : 0.f;
                    A.sb.amp[p] = po.valid ? make_float4(po.te.re, po.te.im, po.tm.re, po.tm.im)
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
                }
                if (po.valid) {
                    ++n_valid;
                    res[me.slot * kUnitPairs + me.e] = make_float4(po.te.re, po.te.im, po.tm.re, po.tm.im);
                    atomicOr(&vbits[me.slot][me.e >> 5], 1u << (me.e & 31));
                }
            }
        }
        U[0].pending -= (uint32_t)__popcll(__ballot(ended && me.slot == 0));
        U[1].pending -= (uint32_t)__popcll(__ballot(ended && me.slot == 1));
        const uint64_t m = __ballot(again);
        if (again) {
            const uint32_t to = (tail + (uint32_t)__popcll(m & below)) % kRefineQueue;
            queue[to] = me;
            if (avg) {  // the replaced planes travel with the candidate
#pragma unroll
                for (int j = 0; j < KM; ++j)
                    if (me.ovr[j] >= 0) {
                        qpl[((size_t)to * KM + j) * 2] = make_float4(kp.pp[j].x, kp.pp[j].y, kp.pp[j].z, 0.f);
                        qpl[((size_t)to * KM + j) * 2 + 1] = make_float4(kp.pn[j].x, kp.pn[j].y, kp.pn[j].z, 0.f);
                    }
            }
        }
        tail += (uint32_t)__popcll(m);
        if (avg) block_sync_global();  // plane rows written by some lanes are read by others later
        else wave_sync();
    }
    flush_visits(stk, A.counters, 11);
    n_cand = warp_sum_u(n_cand);
    n_valid = warp_sum_u(n_valid);
    if (lane == 0) {
        atomicAdd((unsigned long long *)&A.counters[7], (unsigned long long)n_cand);
        atomicAdd((unsigned long long *)&A.counters[4], (unsigned long long)n_valid);
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
    static const uint32_t cap = resident_blocks((const void *)k_refine<KM, W, false>, kWave);
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

template <int W, bool AVG>
void launch_refine_wa(const LaunchArgs &A, dim3 grid, hipStream_t s) {
    switch (A.D.K) {
        case 1: hipLaunchKernelGGL((k_refine<1, W, AVG>), grid, dim3(kWave), 0, s, A); break;
        case 2: hipLaunchKernelGGL((k_refine<2, W, AVG>), grid, dim3(kWave), 0, s, A); break;
        case 3: hipLaunchKernelGGL((k_refine<3, W, AVG>), grid, dim3(kWave), 0, s, A); break;
        case 4: hipLaunchKernelGGL((k_refine<4, W, AVG>), grid, dim3(kWave), 0, s, A); break;
        case 5: hipLaunchKernelGGL((k_refine<5, W, AVG>), grid, dim3(kWave), 0, s, A); break;
        case 6: hipLaunchKernelGGL((k_refine<6, W, AVG>), grid, dim3(kWave), 0, s, A); break;
        case 7: hipLaunchKernelGGL((k_refine<7, W, AVG>), grid, dim3(kWave), 0, s, A); break;
        default: hipLaunchKernelGGL((k_refine<8, W, AVG>), grid, dim3(kWave), 0, s, A); break;
    }
}

// Point-set averaging has kernels of its own, so that the plain refinement
// keeps its register allocation.
template <int W>
void launch_refine_w(const LaunchArgs &A, dim3 grid, hipStream_t s) {
    if (A.rb.nk) launch_refine_wa<W, true>(A, grid, s);
    else launch_refine_wa<W, false>(A, grid, s);
}

void launch_refine(const LaunchArgs &A, hipStream_t s) {
    const dim3 grid(refine_grid(A.D));
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
