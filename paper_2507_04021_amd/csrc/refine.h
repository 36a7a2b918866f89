// The specular refinement kernel (Sec. II-B.2): image-method minimiser,
// validation passes with plane replacements, final occlusion test and the
// path field. A template shared by the translation units that instantiate
// it: specular.hip (the scalar TE/TM field) and specular_pol.hip (the
// polarised field), compiled in parallel.
#pragma once

#include "common.h"
#include "internal.h"

namespace pcrt {

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

template <int KM, int W, bool AVG, bool POL>
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
    constexpr bool pol = POL;
    cv3 ev = {};
    if (pol) ev = pol_launch(A.pol_tx, normalize(x[1] - x[0]));
#pragma unroll
    for (int m = 1; m <= KM; ++m) {
        if (m > k) continue;
        f3 seg = x[m] - x[m - 1];
        float sl = len(seg);
        L += sl;
        const f3 di = (1.0f / sl) * seg;
        float c = fabsf(dot(di, kp.pn[m - 1]));
        csv[m - 1] = c;
        uint32_t lab = __float_as_uint(A.S.nrm[hid[m - 1]].w);
        if (lab >= A.n_labels) lab = 0;
        float er = A.mats[3 * lab], sg = A.mats[3 * lab + 1], sc = A.mats[3 * lab + 2];
        c32 te, tm;
        fresnel(er, sg * A.fc.inv_we0, c, te, tm);
        float R = sqrtf(fmaxf(0.f, 1.f - sc * sc));
        if (pol) {
            const f3 nxt = m < k ? x[m < KM ? m + 1 : m] : rx;
            pol_reflect(ev, di, normalize(nxt - x[m]), kp.pn[m - 1], te, tm, R);
        } else {
            pte = cmul(pte, {R * te.re, R * te.im});
            ptm = cmul(ptm, {R * tm.re, R * tm.im});
        }
    }
    L += len(rx - xk);
    c32 ph = propagate(L, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
    float a0 = A.fc.amp_iso / L;
    if (pol) pte = ptm = pol_receive(ev, A.pol_rx, normalize(rx - xk));
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
// POL: the polarised field (its own instances, so that the scalar ones keep
// their register allocation).
template <int KM, int W, bool AVG, bool POL>
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
            const int out = validate_pass<KM, W, AVG, POL>(A, q, r, tx, kp, me.retries, stk, po, slot, disk, rp, rn);
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


template <int W, bool AVG, bool POL>
void launch_refine_wa(const LaunchArgs &A, dim3 grid, hipStream_t s) {
    switch (A.D.K) {
        case 1: hipLaunchKernelGGL((k_refine<1, W, AVG, POL>), grid, dim3(kWave), 0, s, A); break;
        case 2: hipLaunchKernelGGL((k_refine<2, W, AVG, POL>), grid, dim3(kWave), 0, s, A); break;
        case 3: hipLaunchKernelGGL((k_refine<3, W, AVG, POL>), grid, dim3(kWave), 0, s, A); break;
        case 4: hipLaunchKernelGGL((k_refine<4, W, AVG, POL>), grid, dim3(kWave), 0, s, A); break;
        case 5: hipLaunchKernelGGL((k_refine<5, W, AVG, POL>), grid, dim3(kWave), 0, s, A); break;
        case 6: hipLaunchKernelGGL((k_refine<6, W, AVG, POL>), grid, dim3(kWave), 0, s, A); break;
        case 7: hipLaunchKernelGGL((k_refine<7, W, AVG, POL>), grid, dim3(kWave), 0, s, A); break;
        default: hipLaunchKernelGGL((k_refine<8, W, AVG, POL>), grid, dim3(kWave), 0, s, A); break;
    }
}

}  // namespace pcrt
