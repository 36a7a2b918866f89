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

// Blocks of 256 lanes take one chunk of kRayChunk rays at a time. Lane t
// serves receiver r0 + t % nr for group t / nr; the records of the chunk are
// dealt to the groups round robin. For 64 receivers a wavefront handles one
// interaction point against all receivers (one origin, coherent traversal).
__global__ __launch_bounds__(256) void k_diffuse(LaunchArgs A) {
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
    const uint32_t K = A.D.K, n_rx = A.D.n_rx;
    const uint32_t n_chunks = A.D.n_ray_chunks;
    const bool rec = A.flags & 8;
    uint32_t n_seg = 0, n_vis = 0;
    for (;;) {
        if (tid == 0) s_chunk = atomicAdd(&A.work[2], 1u);
        __syncthreads();
        const uint32_t c = s_chunk;
        __syncthreads();
        if (c >= n_chunks) break;
        const uint32_t g0 = c * kRayChunk;
        const Item I = A.items[find_item(A.items, A.D.n_items, g0)];
        const float budget = (float)I.budget;
        const uint32_t rec0 = g0 * K, nrec = kRayChunk * K;
        for (uint32_t r0 = 0; r0 < n_rx; r0 += 256) {
            const uint32_t nr = min(256u, n_rx - r0);
            const uint32_t G = 256 / nr;
            const uint32_t grp = tid / nr, r = r0 + tid % nr;
            double acc[5] = {0, 0, 0, 0, 0};
            if (grp < G) {
                const f3 rx = mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]);
                for (uint32_t e = grp; e < nrec; e += G) {
                    const uint32_t ri = rec0 + e;
                    const int id = A.rb.id[ri];
                    bool vis = false;
                    if (id >= 0) {
                        const float4 xl = A.rb.xl[ri];
                        const float cs = A.rb.cs[ri];
                        const f3 x = xyz(xl);
                        f3 n = xyz(A.S.nrm[id]);
                        if (cs < 0.f) n = (-1.f) * n;
                        const f3 v = rx - x;
                        const float vn = dot(v, n);
                        if (vn > 0.f) {
                            ++n_seg;
                            if (!occluded(A.S, x, rx, id, A.thr.eps_self, stk)) {
                                vis = true;
                                ++n_vis;
                                const float rs = len(v);
                                const float cos_s = vn / rs;
                                const float a0 = sqrtf(4.f * cos_s / budget) / rs;
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
                            }
                        }
                    }
                    if (rec) A.dvis[(size_t)ri * n_rx + r] = vis;
                }
            }
            __syncthreads();  // every wave is done with its stack
            for (int a = 0; a < 5; ++a) red[tid][a] = acc[a];
            __syncthreads();
            if ((uint32_t)tid < nr) {
                double s[5] = {0, 0, 0, 0, 0};
                for (uint32_t gg = 0; gg < G; ++gg)
                    for (int a = 0; a < 5; ++a) s[a] += red[gg * nr + tid][a];
                double *o = A.diff_part + ((size_t)c * n_rx + r0 + tid) * 5;
                for (int a = 0; a < 5; ++a) o[a] = s[a];
            }
            __syncthreads();
        }
    }
    flush_visits(stk, A.counters, 13);
    n_seg = warp_sum_u(n_seg);
    n_vis = warp_sum_u(n_vis);
    if (lane == 0) {
        atomicAdd((unsigned long long *)&A.counters[2], (unsigned long long)n_seg);
        atomicAdd((unsigned long long *)&A.counters[5], (unsigned long long)n_vis);
    }
}

void launch_diffuse(const LaunchArgs &A, hipStream_t s) {
    hipLaunchKernelGGL(k_diffuse, dim3(wide_grid(A.D.n_ray_chunks)), dim3(256), 0, s, A);
}

// Line of sight per (transmitter, receiver): a_TE = a_TM = lambda/(4 pi d) e^{-j k0 d}.
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
    if (occluded(A.S, tx, rx, -1, A.thr.eps_self, stk)) {
        for (int a = 0; a < 5; ++a) o[a] = 0.0;
        return;
    }
    const float d = len(rx - tx);
    const c32 ph = propagate(d, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
    const float a0 = A.fc.amp_iso / d;
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
    if (A.flags & 1) hipLaunchKernelGGL(k_los, dim3((n + kWave - 1) / kWave), dim3(kWave), 0, s, A);
    launch_combine(A, gain, h_te, h_tm, parts, s);
}

void launch_combine(const LaunchArgs &A, double *gain, double *h_te, double *h_tm, double *parts, hipStream_t s) {
    const uint32_t n = A.D.n_items * A.D.n_rx;
    hipLaunchKernelGGL(k_combine, dim3(n), dim3(256), 0, s, A, gain, h_te, h_tm, parts);
}

}  // namespace pcrt
