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

// Device-wide exclusive scan: per-1024-element block scan, scan of the block
// sums, add-back.
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
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t *a, uint32_t n, uint32_t *total) {
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
    if (threadIdx.x == 1023) *total = part[1023];
}

__global__ __launch_bounds__(1024) void k_scan_add(uint32_t *a, uint32_t n, const uint32_t *blk) {
    uint32_t i = blockIdx.x * 1024 + threadIdx.x;
    if (i < n) a[i] += blk[blockIdx.x];
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

template <int KM>
__device__ void solve_pair(const LaunchArgs &A, uint32_t q, uint32_t r, const Item &I, Stack &stk, PairOut &po,
                           uint32_t &n_cand) {
    po.valid = false;
    const uint32_t K = A.D.K;
    const uint32_t rec = A.keylist[q];
    const uint32_t g = rec / K;
    const int k = (int)(rec % K) + 1;
    f3 pp[KM], pn[KM];
    uint32_t ks[KM];
#pragma unroll
    for (int m = 0; m < KM; ++m)
        if (m < k) {
            int id = A.rb.id[(size_t)g * K + m];
            float4 p4 = A.S.pos[id];
            pp[m] = xyz(p4);
            ks[m] = __float_as_uint(p4.w);
            pn[m] = xyz(A.S.nrm[id]);
        }
    const f3 tx = mk(I.tx[0], I.tx[1], I.tx[2]);
    const f3 rx = mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]);
    f3 x[KM + 1];
    int hid[KM];
    int retries = 0;
    bool counted = false;
    for (;;) {
        if (!refine_planes<KM>(k, tx, rx, pp, pn, A.thr.eps_self, x)) return;
        if (!counted) {
            ++n_cand;
            counted = true;
        }
        int prev = -1;
        bool retry = false, fail = false;
#pragma unroll
        for (int m = 1; m <= KM; ++m) {
            if (m > k || retry || fail) continue;
            f3 u = normalize(x[m] - x[m - 1]);
            float t;
            bool sp;
            int h = closest_hit(A.S, x[m - 1], u, prev, A.thr.eps_self, A.thr.eps_tie, stk, t, sp);
            if (h < 0) { fail = true; continue; }
            float4 hp = A.S.pos[h];
            if (__float_as_uint(hp.w) != ks[m - 1]) { fail = true; continue; }
            f3 hn = xyz(A.S.nrm[h]);
            f3 qh = x[m - 1] + t * u;
            bool ang_ok = fabsf(dot(hn, pn[m - 1])) >= A.thr.cos_ta;
            bool dist_ok = fabsf(dot(qh - pp[m - 1], pn[m - 1])) <= A.thr.t_d;
            if (!(ang_ok && dist_ok)) {
                if (retries >= A.thr.kappa) { fail = true; continue; }
                ++retries;
                pp[m - 1] = xyz(hp);
                pn[m - 1] = hn;
                retry = true;
                continue;
            }
            hid[m - 1] = h;
            prev = h;
        }
        if (fail) return;
        if (retry) continue;
        break;
    }
    f3 xk = x[1];
    int hk = hid[0];
#pragma unroll
    for (int m = 1; m <= KM; ++m)
        if (m == k) {
            xk = x[m];
            hk = hid[m - 1];
        }
    if (occluded(A.S, xk, rx, hk, A.thr.eps_self, stk)) return;
    float L = 0.f;
    c32 pte = {1.f, 0.f}, ptm = {1.f, 0.f};
    float csv[KM];
#pragma unroll
    for (int m = 1; m <= KM; ++m) {
        if (m > k) continue;
        f3 seg = x[m] - x[m - 1];
        float sl = len(seg);
        L += sl;
        float c = fabsf(dot((1.0f / sl) * seg, pn[m - 1]));
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
}

// Persistent blocks of 256 lanes; each takes a key chunk and evaluates all
// (key, RX) pairs of it, accumulating FP64 sums per RX in a fixed order.
template <int KM>
__global__ __launch_bounds__(256) void k_refine(LaunchArgs A) {
    // traversal stacks and the FP64 reduction buffer share LDS (never live together)
    __shared__ union {
        int stack[4][kStackLds * kWave];
        double red[256][5];
    } sm;
    auto &lds_stack = sm.stack;
    auto &red = sm.red;
    __shared__ uint32_t s_chunk;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t glane = blockIdx.x * 256 + tid;
    Stack stk{lds_stack[wave] + lane, A.S.spill + glane, A.S.spill_lanes};
    const uint32_t n_rx = A.D.n_rx, n_items = A.D.n_items;
    const uint32_t n_chunks = A.chunk_off[n_items];
    uint32_t n_cand = 0, n_valid = 0;
    for (;;) {
        if (tid == 0) s_chunk = atomicAdd(&A.work[1], 1u);
        __syncthreads();
        const uint32_t c = s_chunk;
        __syncthreads();
        if (c >= n_chunks) break;
        // item of this chunk
        int lo = 0, hi = (int)n_items - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (A.chunk_off[mid] <= c) lo = mid;
            else hi = mid - 1;
        }
        const int it = lo;
        const Item I = A.items[it];
        const uint32_t q0 = A.key_off[it] + (c - A.chunk_off[it]) * kKeyChunk;
        const uint32_t q1 = min(q0 + kKeyChunk, A.key_off[it + 1]);
        for (uint32_t r0 = 0; r0 < n_rx; r0 += 256) {
            const uint32_t nr = min(256u, n_rx - r0);
            const uint32_t G = 256 / nr;
            const uint32_t grp = tid / nr, r = r0 + tid % nr;
            double acc[5] = {0, 0, 0, 0, 0};
            if (grp < G) {
                for (uint32_t q = q0 + grp; q < q1; q += G) {
                    PairOut po;
                    solve_pair<KM>(A, q, r, I, stk, po, n_cand);
                    if ((A.flags & 8) && q >= A.D.rec_keys) {
                        atomicOr((unsigned long long *)&A.counters[6], 4ull);  // tape capacity exceeded
                    } else if (A.flags & 8) {
                        size_t p = (size_t)q * n_rx + r;
                        A.sb.valid[p] = po.valid;
                        A.sb.len[p] = po.valid ? po.len : 0.f;
                        A.sb.amp[p] = po.valid ? make_float4(po.te.re, po.te.im, po.tm.re, po.tm.im)
                                               : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                    if (!po.valid) continue;
                    ++n_valid;
                    double tr = po.te.re, ti = po.te.im, mr = po.tm.re, mi = po.tm.im;
                    acc[0] += 0.5 * (tr * tr + ti * ti + mr * mr + mi * mi);
                    acc[1] += tr;
                    acc[2] += ti;
                    acc[3] += mr;
                    acc[4] += mi;
                }
            }
            __syncthreads();  // every wave is done with its stack
            for (int a = 0; a < 5; ++a) red[tid][a] = acc[a];
            __syncthreads();
            if ((uint32_t)tid < nr) {
                double s[5] = {0, 0, 0, 0, 0};
                for (uint32_t gg = 0; gg < G; ++gg)
                    for (int a = 0; a < 5; ++a) s[a] += red[gg * nr + tid][a];
                double *o = A.spec_part + ((size_t)c * n_rx + r0 + tid) * 5;
                for (int a = 0; a < 5; ++a) o[a] = s[a];
            }
            __syncthreads();
        }
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
    hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(1024), 0, s, A.scan, n_rec, A.scan_blk);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, A.scan_blk, nb, total);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, s, A.scan, n_rec, A.scan_blk);
    hipLaunchKernelGGL(k_compact, dim3(blk), dim3(256), 0, s, A, n_rec, total);
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, s, A, total);
}

void launch_refine(const LaunchArgs &A, hipStream_t s) {
    const uint32_t grid = wide_grid(A.D.max_key_chunks);
    switch (A.D.K) {
#define PCRT_REFINE_CASE(KK) \
    case KK: hipLaunchKernelGGL(k_refine<KK>, dim3(grid), dim3(256), 0, s, A); break;
        PCRT_REFINE_CASE(1)
        PCRT_REFINE_CASE(2)
        PCRT_REFINE_CASE(3)
        PCRT_REFINE_CASE(4)
        PCRT_REFINE_CASE(5)
        PCRT_REFINE_CASE(6)
        PCRT_REFINE_CASE(7)
        PCRT_REFINE_CASE(8)
#undef PCRT_REFINE_CASE
        default: break;
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
