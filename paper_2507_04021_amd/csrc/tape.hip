// Differentiable field evaluation on a recorded tape.
//
// A RECORD solve keeps the path geometry: per traced interaction (ray g,
// bounce m) its disk, point, unfolded length and incidence cosine; per
// (key, RX) specular path its validity, length, hit disks and cosines; per
// (interaction, RX) the diffuse visibility. Geometry does not depend on the
// materials, so the field can be re-evaluated for new materials -- or for a
// learned coefficient model -- without tracing again, and differentiated.
//
// Interaction slots: s < T*K are traced interactions (g*K + m); the rest are
// specular-path interactions T*K + (q*n_rx + r)*K + m. Each slot carries
// (Gamma_TE, Gamma_TM, S) in a coefficient table; the backward kernels write
// dL/d of those five reals per slot, and a fixed-order reduction turns them
// into per-label gradients with respect to (eps_r, sigma, S).
#include "common.h"
#include "internal.h"

namespace pcrt {

__device__ __forceinline__ uint32_t n_keys_rec(const LaunchArgs &A) {
    return min(A.key_off[A.D.n_items], A.D.rec_keys);
}

// Label and incidence cosine of every slot; 0xffff marks an empty slot.
__global__ void k_tape_slots(LaunchArgs A) {
    const uint32_t TK = A.D.T * A.D.K, K = A.D.K;
    const uint32_t nk = n_keys_rec(A);
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < A.D.n_slots; s += gridDim.x * blockDim.x) {
        uint16_t lab = 0xffff;
        float c = 0.f;
        if (s < TK) {
            int id = A.rb.id[s];
            if (id >= 0) {
                lab = (uint16_t)__float_as_uint(A.S.nrm[id].w);
                c = fabsf(A.rb.cs[s]);
            }
        } else {
            uint32_t u = s - TK, p = u / K, m = u % K;
            uint32_t q = p / A.D.n_rx;
            if (q < nk && A.sb.valid[p] && m < A.keylist[q] % K + 1) {
                lab = (uint16_t)__float_as_uint(A.S.nrm[A.sb.hit[(size_t)p * K + m]].w);
                c = A.sb.cs[(size_t)p * K + m];
            }
        }
        A.slot_label[s] = lab;
        A.slot_cos[s] = c;
    }
}

void launch_tape_slots(const LaunchArgs &A, hipStream_t s) {
    uint32_t g = std::min<uint32_t>((A.D.n_slots + 255) / 256, 8192);
    hipLaunchKernelGGL(k_tape_slots, dim3(std::max<uint32_t>(g, 1)), dim3(256), 0, s, A);
}

// Coefficients from per-label materials (the paper's per-label Fresnel model).
__global__ void k_tape_fresnel(LaunchArgs A, const float *mats, uint32_t n_labels) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < A.D.n_slots; s += gridDim.x * blockDim.x) {
        uint32_t lab = A.slot_label[s];
        float4 *o = (float4 *)(A.slot_coef + 8 * (size_t)s);
        if (lab == 0xffff || lab >= n_labels) {
            o[0] = make_float4(0.f, 0.f, 0.f, 0.f);
            o[1] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        c32 te, tm;
        fresnel(mats[3 * lab], mats[3 * lab + 1] * A.fc.inv_we0, A.slot_cos[s], te, tm);
        o[0] = make_float4(te.re, te.im, tm.re, tm.im);
        o[1] = make_float4(mats[3 * lab + 2], 0.f, 0.f, 0.f);
    }
}

void launch_tape_fresnel(const LaunchArgs &A, const float *mats, uint32_t n_labels, hipStream_t s) {
    uint32_t g = std::min<uint32_t>((A.D.n_slots + 255) / 256, 8192);
    hipLaunchKernelGGL(k_tape_fresnel, dim3(std::max<uint32_t>(g, 1)), dim3(256), 0, s, A, mats, n_labels);
}

struct SlotCoef {
    c32 te, tm;
    float S;
};
__device__ __forceinline__ SlotCoef load_coef(const float *coef, size_t s) {
    const float4 a = ((const float4 *)(coef + 8 * s))[0];
    const float b = coef[8 * s + 4];
    return {{a.x, a.y}, {a.z, a.w}, b};
}

// Geometry of a diffuse connection (interaction ri to receiver rx): amplitude
// factor a0 = lambda/(4 pi) sqrt(4 cos_s / N) / r_s and the phase length.
__device__ __forceinline__ bool diffuse_geom(const LaunchArgs &A, uint32_t ri, f3 rx, float budget, float &a0,
                                             float &plen) {
    const float4 xl = A.rb.xl[ri];
    const f3 n = record_normal(A, ri);
    const f3 v = rx - xyz(xl);
    const float rs = len(v);
    const float cos_s = dot(v, n) / rs;
    a0 = A.fc.amp_iso * sqrtf(4.f * fmaxf(cos_s, 0.f) / budget) / rs;
    plen = xl.w + rs;
    return true;
}

// Tape forward, diffuse part: same chunking as the solve (kRayChunk rays per
// block iteration, receivers across lanes), visibility from the tape.
__global__ __launch_bounds__(256) void k_tape_diffuse(LaunchArgs A) {
    __shared__ double red[256][5];
    const int tid = threadIdx.x;
    const uint32_t K = A.D.K, n_rx = A.D.n_rx;
    for (uint32_t c = blockIdx.x; c < A.D.n_ray_chunks; c += gridDim.x) {
        const uint32_t g0 = c * kRayChunk;
        const Item I = A.items[find_item(A.items, A.D.n_items, g0)];
        const float budget = (float)I.budget;
        for (uint32_t r0 = 0; r0 < n_rx; r0 += 256) {
            const uint32_t nr = min(256u, n_rx - r0);
            const uint32_t G = 256 / nr;
            const uint32_t grp = tid / nr, r = r0 + tid % nr;
            double acc[5] = {0, 0, 0, 0, 0};
            if (grp < G) {
                const f3 rx = mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]);
                for (uint32_t e = grp; e < kRayChunk * K; e += G) {
                    const uint32_t ri = g0 * K + e;
                    if (A.rb.id[ri] < 0 || !A.dvis[(size_t)ri * n_rx + r]) continue;
                    const uint32_t g = ri / K, k = ri % K;
                    c32 pte = {1.f, 0.f}, ptm = {1.f, 0.f};
                    for (uint32_t m = 0; m <= k; ++m) {
                        SlotCoef cf = load_coef(A.slot_coef, (size_t)g * K + m);
                        float f = m < k ? sqrtf(fmaxf(0.f, 1.f - cf.S * cf.S)) : cf.S;
                        pte = cmul(pte, {f * cf.te.re, f * cf.te.im});
                        ptm = cmul(ptm, {f * cf.tm.re, f * cf.tm.im});
                    }
                    float a0, plen;
                    diffuse_geom(A, ri, rx, budget, a0, plen);
                    const c32 ph = propagate(plen, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
                    const c32 te = cmul({a0 * pte.re, a0 * pte.im}, ph);
                    const c32 tm = cmul({a0 * ptm.re, a0 * ptm.im}, ph);
                    const double tr = te.re, ti = te.im, mr = tm.re, mi = tm.im;
                    acc[0] += 0.5 * (tr * tr + ti * ti + mr * mr + mi * mi);
                    acc[1] += tr;
                    acc[2] += ti;
                    acc[3] += mr;
                    acc[4] += mi;
                }
            }
            for (int a = 0; a < 5; ++a) red[tid][a] = acc[a];
            __syncthreads();
            if ((uint32_t)tid < nr) {
                double sum[5] = {0, 0, 0, 0, 0};
                for (uint32_t gg = 0; gg < G; ++gg)
                    for (int a = 0; a < 5; ++a) sum[a] += red[gg * nr + tid][a];
                double *o = A.diff_part + ((size_t)c * n_rx + r0 + tid) * 5;
                for (int a = 0; a < 5; ++a) o[a] = sum[a];
            }
            __syncthreads();
        }
    }
}

// Geometry of a voxel diffuse path of the reception-point launch
// (representative record ri, receiver r): gated by the visibility matrix and
// the lit side, amplitude factor lambda/(4 pi) sqrt(rho^2 cos_i cos_s / pi)
// / (L r_s) (the solve's k_dps_diffuse) and the phase length.
__device__ __forceinline__ bool voxel_geom(const LaunchArgs &A, uint32_t ri, uint32_t r, f3 rx, float &a0,
                                           float &plen) {
    const int id = A.rb.id[ri];
    if (!A.dps_vis[(size_t)r * A.S.n_sets + A.S.dps_of[id]]) return false;
    const float4 xl = A.rb.xl[ri];
    const f3 v = rx - xyz(xl);
    const float vn = dot(v, record_normal(A, ri));
    if (!(vn > 0.f)) return false;
    const float rs = len(v);
    a0 = A.fc.amp_iso * sqrtf(A.dps_area * fabsf(A.rb.cs[ri]) * (vn / rs) * (float)(1.0 / kPi)) / (xl.w * rs);
    plen = xl.w + rs;
    return true;
}

// Tape forward, voxel diffuse paths of the reception-point launch: the same
// blocks, key shares and sum order as the solve's k_dps_diffuse, the chain's
// coefficients taken from the tape's slots.
__global__ __launch_bounds__(kDpsWaves * kWave) void k_tape_dps_diffuse(LaunchArgs A) {
    __shared__ double red[kDpsWaves][kWave][5];
    const uint32_t n_rx = A.D.n_rx, K = A.D.K;
    const uint32_t n_keys = A.dkey_off[A.D.n_items];
    const uint32_t w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const uint32_t c = blockIdx.x, r = blockIdx.y * kWave + lane;
    double acc[5] = {0, 0, 0, 0, 0};
    const f3 rx = r < n_rx ? mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]) : mk(0.f, 0.f, 0.f);
    uint32_t q0, k1;
    dps_key_range(n_keys, c, A.D.n_ray_chunks, w, q0, k1);
    if (r >= n_rx) k1 = q0;
    for (uint32_t q = q0; q < k1; ++q) {
        const uint32_t ri = A.dkeylist[q];
        float a0, plen;
        if (!voxel_geom(A, ri, r, rx, a0, plen)) continue;
        const uint32_t g = ri / K, k = ri % K;
        c32 pte = {1.f, 0.f}, ptm = {1.f, 0.f};
        for (uint32_t m = 0; m <= k; ++m) {
            SlotCoef cf = load_coef(A.slot_coef, (size_t)g * K + m);
            float f = m < k ? sqrtf(fmaxf(0.f, 1.f - cf.S * cf.S)) : cf.S;
            pte = cmul(pte, {f * cf.te.re, f * cf.te.im});
            ptm = cmul(ptm, {f * cf.tm.re, f * cf.tm.im});
        }
        const c32 ph = propagate(plen, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
        const c32 te = cmul({a0 * pte.re, a0 * pte.im}, ph);
        const c32 tm = cmul({a0 * ptm.re, a0 * ptm.im}, ph);
        const double tr = te.re, ti = te.im, mr = tm.re, mi = tm.im;
        acc[0] += 0.5 * (tr * tr + ti * ti + mr * mr + mi * mi);
        acc[1] += tr;
        acc[2] += ti;
        acc[3] += mr;
        acc[4] += mi;
    }
    dps_block_sum(red, w, lane, acc, r < n_rx ? A.diff_part + ((size_t)c * n_rx + r) * 5 : nullptr);
}

// Tape forward, specular part: per key chunk, receivers across lanes.
__global__ __launch_bounds__(256) void k_tape_specular(LaunchArgs A) {
    __shared__ double red[256][5];
    const int tid = threadIdx.x;
    const uint32_t K = A.D.K, n_rx = A.D.n_rx, n_items = A.D.n_items, TK = A.D.T * A.D.K;
    const uint32_t n_chunks = A.chunk_off[n_items];
    const uint32_t nk = n_keys_rec(A);
    for (uint32_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        int lo = 0, hi = (int)n_items - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (A.chunk_off[mid] <= c) lo = mid;
            else hi = mid - 1;
        }
        const int it = lo;
        const uint32_t q0 = A.key_off[it] + (c - A.chunk_off[it]) * kKeyChunk;
        const uint32_t q1 = min(min(q0 + kKeyChunk, A.key_off[it + 1]), nk);
        for (uint32_t r0 = 0; r0 < n_rx; r0 += 256) {
            const uint32_t nr = min(256u, n_rx - r0);
            const uint32_t G = 256 / nr;
            const uint32_t grp = tid / nr, r = r0 + tid % nr;
            double acc[5] = {0, 0, 0, 0, 0};
            if (grp < G) {
                for (uint32_t q = q0 + grp; q < q1; q += G) {
                    const size_t p = (size_t)q * n_rx + r;
                    if (!A.sb.valid[p]) continue;
                    const uint32_t k = A.keylist[q] % K + 1;
                    c32 pte = {1.f, 0.f}, ptm = {1.f, 0.f};
                    for (uint32_t m = 0; m < k; ++m) {
                        SlotCoef cf = load_coef(A.slot_coef, TK + p * K + m);
                        float f = sqrtf(fmaxf(0.f, 1.f - cf.S * cf.S));
                        pte = cmul(pte, {f * cf.te.re, f * cf.te.im});
                        ptm = cmul(ptm, {f * cf.tm.re, f * cf.tm.im});
                    }
                    const float L = A.sb.len[p];
                    const float a0 = A.fc.amp_iso / L;
                    const c32 ph = propagate(L, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
                    const c32 te = cmul({a0 * pte.re, a0 * pte.im}, ph);
                    const c32 tm = cmul({a0 * ptm.re, a0 * ptm.im}, ph);
                    const double tr = te.re, ti = te.im, mr = tm.re, mi = tm.im;
                    acc[0] += 0.5 * (tr * tr + ti * ti + mr * mr + mi * mi);
                    acc[1] += tr;
                    acc[2] += ti;
                    acc[3] += mr;
                    acc[4] += mi;
                }
            }
            for (int a = 0; a < 5; ++a) red[tid][a] = acc[a];
            __syncthreads();
            if ((uint32_t)tid < nr) {
                double sum[5] = {0, 0, 0, 0, 0};
                for (uint32_t gg = 0; gg < G; ++gg)
                    for (int a = 0; a < 5; ++a) sum[a] += red[gg * nr + tid][a];
                double *o = A.spec_part + ((size_t)c * n_rx + r0 + tid) * 5;
                for (int a = 0; a < 5; ++a) o[a] = sum[a];
            }
            __syncthreads();
        }
    }
}

void launch_tape_forward(const LaunchArgs &A, double *gain, double *h_te, double *h_tm, double *parts,
                         hipStream_t s) {
    if ((A.flags & 4) && A.dps_vis)
        hipLaunchKernelGGL(k_tape_dps_diffuse, dim3(std::max<uint32_t>(A.D.n_ray_chunks, 1), (A.D.n_rx + kWave - 1) / kWave),
                           dim3(kDpsWaves * kWave), 0, s, A);
    else if (A.flags & 4)
        hipLaunchKernelGGL(k_tape_diffuse, dim3(std::min<uint32_t>(std::max<uint32_t>(A.D.n_ray_chunks, 1), 2048)),
                           dim3(256), 0, s, A);
    if (A.flags & 2)
        hipLaunchKernelGGL(k_tape_specular, dim3(std::min<uint32_t>(std::max<uint32_t>(A.D.max_key_chunks, 1), 2048)),
                           dim3(256), 0, s, A);
    // line of sight does not depend on the materials: the solve's values are reused
    launch_combine(A, gain, h_te, h_tm, parts, s);
}

// Adjoint of one path's power 1/2 (|a_TE|^2 + |a_TM|^2) with respect to its
// chain's per-slot coefficients, weighted by w (dL/dG times the geometric
// factor a0^2). f_m = sqrt(1 - S_m^2) for specular interactions, S_m for the
// diffuse end. Products of the other interactions avoid any division by
// Gamma (Gamma_TM vanishes at the Brewster angle).
template <int KM>
__device__ __forceinline__ void chain_adjoint(int k, const SlotCoef *cf, const bool *diff_end, double w,
                                              double (*adj)[5]) {
    double pw_te[KM], pw_tm[KM], f2[KM];
#pragma unroll
    for (int m = 0; m < KM; ++m) {
        if (m >= k) continue;
        const float S = cf[m].S;
        f2[m] = diff_end[m] ? (double)S * S : fmax(0.0, 1.0 - (double)S * S);
        pw_te[m] = (double)cf[m].te.re * cf[m].te.re + (double)cf[m].te.im * cf[m].te.im;
        pw_tm[m] = (double)cf[m].tm.re * cf[m].tm.re + (double)cf[m].tm.im * cf[m].tm.im;
    }
#pragma unroll
    for (int m = 0; m < KM; ++m) {
        if (m >= k) continue;
        double rte = w, rtm = w;
#pragma unroll
        for (int n = 0; n < KM; ++n) {
            if (n >= k || n == m) continue;
            rte *= f2[n] * pw_te[n];
            rtm *= f2[n] * pw_tm[n];
        }
        adj[m][0] += rte * f2[m] * cf[m].te.re;
        adj[m][1] += rte * f2[m] * cf[m].te.im;
        adj[m][2] += rtm * f2[m] * cf[m].tm.re;
        adj[m][3] += rtm * f2[m] * cf[m].tm.im;
        const double S = cf[m].S;
        const double df2 = diff_end[m] ? 2.0 * S : -2.0 * S;
        adj[m][4] += 0.5 * df2 * (rte * pw_te[m] + rtm * pw_tm[m]);
    }
}

// Traced-interaction slots: one thread per ray, all of its diffuse paths.
template <int KM>
__global__ __launch_bounds__(256) void k_tape_adjoint_trace(LaunchArgs A, const double *dldg) {
    const uint32_t K = A.D.K, n_rx = A.D.n_rx;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < A.D.T; g += gridDim.x * blockDim.x) {
        double adj[KM][5];
#pragma unroll
        for (int m = 0; m < KM; ++m)
            for (int a = 0; a < 5; ++a) adj[m][a] = 0.0;
        if ((A.flags & 4) && A.dps_vis) {
            // voxel diffuse paths whose representative is one of this ray's
            // records (the key list is in record order; one transmitter)
            SlotCoef cf[KM];
            bool de[KM];
#pragma unroll
            for (int m = 0; m < KM; ++m)
                if (m < (int)K) cf[m] = load_coef(A.slot_coef, (size_t)g * K + m);
            const uint32_t n_keys = A.dkey_off[A.D.n_items];
            uint32_t lo = 0, hi = n_keys;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) / 2;
                if (A.dkeylist[mid] < g * K) lo = mid + 1;
                else hi = mid;
            }
            for (uint32_t q = lo; q < n_keys && A.dkeylist[q] < (g + 1) * K; ++q) {
                const uint32_t ri = A.dkeylist[q], k = ri % K;
                double W = 0.0;
                for (uint32_t r = 0; r < n_rx; ++r) {
                    float a0, plen;
                    if (voxel_geom(A, ri, r, mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]), a0, plen))
                        W += dldg[r] * (double)a0 * a0;
                }
                if (W == 0.0) continue;
#pragma unroll
                for (int m = 0; m < KM; ++m) de[m] = (m == (int)k);
                chain_adjoint<KM>((int)k + 1, cf, de, W, adj);
            }
        } else if (A.flags & 4) {
            const int it = find_item(A.items, A.D.n_items, g);
            const float budget = (float)A.items[it].budget;
            SlotCoef cf[KM];
            bool de[KM];
#pragma unroll
            for (int m = 0; m < KM; ++m)
                if (m < (int)K) cf[m] = load_coef(A.slot_coef, (size_t)g * K + m);
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (k >= (int)K) continue;
                const uint32_t ri = g * K + k;
                if (A.rb.id[ri] < 0) continue;
                double W = 0.0;
                for (uint32_t r = 0; r < n_rx; ++r) {
                    if (!A.dvis[(size_t)ri * n_rx + r]) continue;
                    float a0, plen;
                    diffuse_geom(A, ri, mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]), budget, a0, plen);
                    W += dldg[(size_t)it * n_rx + r] * (double)a0 * a0;
                }
                if (W == 0.0) continue;
#pragma unroll
                for (int m = 0; m < KM; ++m) de[m] = (m == k);
                chain_adjoint<KM>(k + 1, cf, de, W, adj);
            }
        }
#pragma unroll
        for (int m = 0; m < KM; ++m) {
            if (m >= (int)K) continue;
            float4 *o = (float4 *)(A.slot_adj + 8 * ((size_t)g * K + m));
            o[0] = make_float4((float)adj[m][0], (float)adj[m][1], (float)adj[m][2], (float)adj[m][3]);
            o[1] = make_float4((float)adj[m][4], 0.f, 0.f, 0.f);
        }
    }
}

// Specular-path slots: one thread per (key, RX) pair.
template <int KM>
__global__ __launch_bounds__(256) void k_tape_adjoint_spec(LaunchArgs A, const double *dldg) {
    const uint32_t K = A.D.K, n_rx = A.D.n_rx, TK = A.D.T * A.D.K;
    const uint32_t nk = n_keys_rec(A);
    const size_t n_pairs = (size_t)A.D.rec_keys * n_rx;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n_pairs; p += (size_t)gridDim.x * blockDim.x) {
        double adj[KM][5];
#pragma unroll
        for (int m = 0; m < KM; ++m)
            for (int a = 0; a < 5; ++a) adj[m][a] = 0.0;
        const uint32_t q = (uint32_t)(p / n_rx), r = (uint32_t)(p % n_rx);
        if ((A.flags & 2) && q < nk && A.sb.valid[p]) {
            const uint32_t k = A.keylist[q] % K + 1;
            const int it = find_item(A.items, A.D.n_items, A.keylist[q] / K);
            SlotCoef cf[KM];
            bool de[KM];
#pragma unroll
            for (int m = 0; m < KM; ++m) {
                de[m] = false;
                if (m < (int)k) cf[m] = load_coef(A.slot_coef, TK + p * K + m);
            }
            const double a0 = (double)A.fc.amp_iso / A.sb.len[p];
            chain_adjoint<KM>((int)k, cf, de, dldg[(size_t)it * n_rx + r] * a0 * a0, adj);
        }
#pragma unroll
        for (int m = 0; m < KM; ++m) {
            if (m >= (int)K) continue;
            float4 *o = (float4 *)(A.slot_adj + 8 * (TK + p * K + m));
            o[0] = make_float4((float)adj[m][0], (float)adj[m][1], (float)adj[m][2], (float)adj[m][3]);
            o[1] = make_float4((float)adj[m][4], 0.f, 0.f, 0.f);
        }
    }
}

void launch_tape_backward(const LaunchArgs &A, const double *dldg, hipStream_t s) {
    const uint32_t gt = std::min<uint32_t>((A.D.T + 255) / 256, 4096);
    const size_t np = (size_t)A.D.rec_keys * A.D.n_rx;
    const uint32_t gs = (uint32_t)std::min<size_t>((np + 255) / 256, 4096);
    switch (A.D.K) {
#define PCRT_TB_CASE(KK)                                                                                    \
    case KK:                                                                                                \
        hipLaunchKernelGGL(k_tape_adjoint_trace<KK>, dim3(std::max<uint32_t>(gt, 1)), dim3(256), 0, s, A, dldg); \
        hipLaunchKernelGGL(k_tape_adjoint_spec<KK>, dim3(std::max<uint32_t>(gs, 1)), dim3(256), 0, s, A, dldg);  \
        break;
        PCRT_TB_CASE(1)
        PCRT_TB_CASE(2)
        PCRT_TB_CASE(3)
        PCRT_TB_CASE(4)
        PCRT_TB_CASE(5)
        PCRT_TB_CASE(6)
        PCRT_TB_CASE(7)
        PCRT_TB_CASE(8)
#undef PCRT_TB_CASE
        default: break;
    }
}

// ------------------------------------------- channel frequency response
// H_r(f_n) = sum over the recorded paths of a_p exp(-j 2 pi (f_n - f_c) tau_p)
// with a_p the path's TE / TM amplitudes at the solve's frequency f_c,
// tau_p = L_p / c0 and f_n = f_c + (n - (N - 1) / 2) bw / (N - 1) (Sec. III-B:
// CFR samples over a bandwidth; the CIR is their inverse DFT). Paths per
// receiver in a fixed order: line of sight, the valid specular paths by key,
// the visible diffuse connections by record.
struct cd {
    double re, im;
};
__device__ __forceinline__ cd cdmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cdconj(cd a) { return {a.re, -a.im}; }

struct CfrPath {
    cd te, tm;
    double tau;
};

__device__ __forceinline__ double cfr_df(uint32_t n, uint32_t N, double bw) {
    return N > 1 ? ((double)n - 0.5 * (double)(N - 1)) * bw / (double)(N - 1) : 0.0;
}

// Path j of receiver r: 0 = line of sight, 1..nk = specular key j - 1, then
// diffuse record j - 1 - nk. False if that path does not exist.
__device__ bool cfr_path(const LaunchArgs &A, uint32_t j, uint32_t r, uint32_t nk, CfrPath &out) {
    const uint32_t K = A.D.K, n_rx = A.D.n_rx, TK = A.D.T * A.D.K;
    const f3 rx = mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]);
    if (j == 0) {
        if (!(A.flags & 1)) return false;
        const double *lp = A.los_part + (size_t)r * 5;
        if (!(lp[0] > 0.0)) return false;
        const Item I = A.items[0];
        const float d = len(rx - mk(I.tx[0], I.tx[1], I.tx[2]));
        out.te = {lp[1], lp[2]};
        out.tm = {lp[3], lp[4]};
        out.tau = (double)d / kC0;
        return true;
    }
    if (j <= nk) {
        const uint32_t q = j - 1;
        const size_t p = (size_t)q * n_rx + r;
        if (!A.sb.valid[p]) return false;
        const uint32_t k = A.keylist[q] % K + 1;
        c32 pte = {1.f, 0.f}, ptm = {1.f, 0.f};
        for (uint32_t m = 0; m < k; ++m) {
            SlotCoef cf = load_coef(A.slot_coef, TK + p * K + m);
            float f = sqrtf(fmaxf(0.f, 1.f - cf.S * cf.S));
            pte = cmul(pte, {f * cf.te.re, f * cf.te.im});
            ptm = cmul(ptm, {f * cf.tm.re, f * cf.tm.im});
        }
        const float L = A.sb.len[p];
        const float a0 = A.fc.amp_iso / L;
        const c32 ph = propagate(L, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
        const c32 te = cmul({a0 * pte.re, a0 * pte.im}, ph), tm = cmul({a0 * ptm.re, a0 * ptm.im}, ph);
        out.te = {te.re, te.im};
        out.tm = {tm.re, tm.im};
        out.tau = (double)L / kC0;
        return true;
    }
    const uint32_t ri = j - 1 - nk;
    if (A.rb.id[ri] < 0 || !A.dvis[(size_t)ri * n_rx + r]) return false;
    const uint32_t g = ri / K, k = ri % K;
    c32 pte = {1.f, 0.f}, ptm = {1.f, 0.f};
    for (uint32_t m = 0; m <= k; ++m) {
        SlotCoef cf = load_coef(A.slot_coef, (size_t)g * K + m);
        float f = m < k ? sqrtf(fmaxf(0.f, 1.f - cf.S * cf.S)) : cf.S;
        pte = cmul(pte, {f * cf.te.re, f * cf.te.im});
        ptm = cmul(ptm, {f * cf.tm.re, f * cf.tm.im});
    }
    float a0, plen;
    diffuse_geom(A, ri, rx, (float)A.items[0].budget, a0, plen);
    const c32 ph = propagate(plen, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
    const c32 te = cmul({a0 * pte.re, a0 * pte.im}, ph), tm = cmul({a0 * ptm.re, a0 * ptm.im}, ph);
    out.te = {te.re, te.im};
    out.tm = {tm.re, tm.im};
    out.tau = (double)plen / kC0;
    return true;
}

// Block (receiver r, 16 frequencies), 16 wavefronts: the path list is cut
// into 16 contiguous ranges, one per wavefront. A wavefront's lanes evaluate 64
// paths of its range at a time into LDS; lane l then adds, to frequency l % 16,
// every 4th of them starting at l / 16, in path order (four interleaved
// subsets, so small sample counts still fill the chip). The block adds the
// subsets and then the ranges, both in order. The order of the FP64 sums is
// fixed and independent of the sample count, so results are reproducible.
constexpr int kCfrWaves = 16, kCfrF = 16, kCfrQ = kWave / kCfrF;
__global__ __launch_bounds__(kCfrWaves * kWave) void k_tape_cfr(LaunchArgs A, double bw, uint32_t N, double *cfr) {
    __shared__ CfrPath P[kCfrWaves][kWave];
    __shared__ int ok[kCfrWaves][kWave];
    static_assert(sizeof(P) >= sizeof(double) * kCfrWaves * kWave * 4, "subset sums reuse the path buffer");
    double(*part)[kWave][4] = reinterpret_cast<double(*)[kWave][4]>(&P[0][0]);  // after the last round
    const uint32_t lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const uint32_t sub = lane / kCfrF, r = blockIdx.x, n = blockIdx.y * kCfrF + lane % kCfrF;
    const uint32_t nk = (A.flags & 2) ? n_keys_rec(A) : 0;
    const uint32_t nd = (A.flags & 4) ? A.D.T * A.D.K : 0;
    const uint32_t total = 1 + nk + nd;
    const uint32_t lo = (uint32_t)((uint64_t)total * wv / kCfrWaves);
    const uint32_t hi = (uint32_t)((uint64_t)total * (wv + 1) / kCfrWaves);
    // every wavefront runs the same number of rounds (the longest range), so
    // the block-wide barriers below are reached by all of them
    const uint32_t rounds = (total / kCfrWaves + 1 + kWave - 1) / kWave;
    const double w = -2.0 * M_PI * cfr_df(n, N, bw);
    cd hte = {0.0, 0.0}, htm = {0.0, 0.0};
    for (uint32_t q = 0; q < rounds; ++q) {
        const uint32_t b = lo + q * kWave, j = b + lane;
        CfrPath pp{};
        ok[wv][lane] = j < hi && cfr_path(A, j, r, nk, pp);
        P[wv][lane] = pp;
        __syncthreads();
        const uint32_t cnt = b < hi ? min((uint32_t)kWave, hi - b) : 0u;
        for (uint32_t i = sub; i < cnt; i += kCfrQ) {
            if (!ok[wv][i]) continue;
            double sn, cs;
            sincos(w * P[wv][i].tau, &sn, &cs);
            const cd e = {cs, sn};
            const cd a = cdmul(P[wv][i].te, e), c = cdmul(P[wv][i].tm, e);
            hte.re += a.re;
            hte.im += a.im;
            htm.re += c.re;
            htm.im += c.im;
        }
        __syncthreads();
    }
    part[wv][lane][0] = hte.re;
    part[wv][lane][1] = hte.im;
    part[wv][lane][2] = htm.re;
    part[wv][lane][3] = htm.im;
    __syncthreads();
    if (threadIdx.x < kCfrF * 4) {  // thread (component c, frequency f): subsets, then ranges, in order
        const uint32_t f = threadIdx.x % kCfrF, c = threadIdx.x / kCfrF, nn = blockIdx.y * kCfrF + f;
        double v = 0.0;
        for (int k = 0; k < kCfrWaves; ++k)
            for (int u = 0; u < kCfrQ; ++u) v += part[k][u * kCfrF + f][c];
        if (nn < N) cfr[((size_t)r * N + nn) * 4 + c] = v;
    }
}

void launch_tape_cfr(const LaunchArgs &A, double bw, uint32_t N, double *cfr, hipStream_t s) {
    hipLaunchKernelGGL(k_tape_cfr, dim3(A.D.n_rx, (N + kCfrF - 1) / kCfrF), dim3(kCfrWaves * kWave), 0, s, A, bw, N,
                       cfr);
}

// dL/da_p (as gR + j gI per polarisation) of one path from dL/dH_r:
// sum over n of dL/dH_r(f_n) exp(+j 2 pi (f_n - f_c) tau_p). Called by all
// lanes of a wavefront for the same path: lane l adds samples l, l + 64, ...,
// then a fixed butterfly adds the lanes, so every lane holds the same sums.
__device__ __forceinline__ void cfr_path_grad(const double *dldh, uint32_t r, uint32_t N, double bw, double tau,
                                              uint32_t lane, cd &gte, cd &gtm) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t n = lane; n < N; n += kWave) {
        double sn, cs;
        sincos(2.0 * M_PI * cfr_df(n, N, bw) * tau, &sn, &cs);
        const double *g = dldh + ((size_t)r * N + n) * 4;
        const cd a = cdmul({g[0], g[1]}, {cs, sn}), b = cdmul({g[2], g[3]}, {cs, sn});
        acc[0] += a.re;
        acc[1] += a.im;
        acc[2] += b.re;
        acc[3] += b.im;
    }
    gte = {wave_sum_d(acc[0]), wave_sum_d(acc[1])};
    gtm = {wave_sum_d(acc[2]), wave_sum_d(acc[3])};
}

// Adjoint rows of one chain a = G prod_m f_m Gamma_m (f_m = sqrt(1 - S_m^2)
// for specular interactions, S_m for the diffuse end) from E = g conj(G)
// per polarisation, g = dL/da: dL/dGamma_m = E conj(f_m prod_{n != m} f_n
// Gamma_n), dL/dS_m = Re(E conj(f'_m Gamma_m prod_{n != m} f_n Gamma_n)).
template <int KM>
__device__ __forceinline__ void chain_adjoint_c(int k, const SlotCoef *cf, const bool *diff_end, cd Ete, cd Etm,
                                                double (*adj)[5]) {
    double f[KM], fp[KM];
    cd Fte[KM], Ftm[KM];
#pragma unroll
    for (int m = 0; m < KM; ++m) {
        if (m >= k) continue;
        const double S = cf[m].S;
        if (diff_end[m]) {
            f[m] = S;
            fp[m] = 1.0;
        } else {
            f[m] = sqrt(fmax(0.0, 1.0 - S * S));
            fp[m] = f[m] > 0.0 ? -S / f[m] : 0.0;
        }
        Fte[m] = {f[m] * cf[m].te.re, f[m] * cf[m].te.im};
        Ftm[m] = {f[m] * cf[m].tm.re, f[m] * cf[m].tm.im};
    }
#pragma unroll
    for (int m = 0; m < KM; ++m) {
        if (m >= k) continue;
        cd Pte = {1.0, 0.0}, Ptm = {1.0, 0.0};
#pragma unroll
        for (int n = 0; n < KM; ++n) {
            if (n >= k || n == m) continue;
            Pte = cdmul(Pte, Fte[n]);
            Ptm = cdmul(Ptm, Ftm[n]);
        }
        const cd gte = cdmul(Ete, cdconj({f[m] * Pte.re, f[m] * Pte.im}));
        const cd gtm = cdmul(Etm, cdconj({f[m] * Ptm.re, f[m] * Ptm.im}));
        adj[m][0] += gte.re;
        adj[m][1] += gte.im;
        adj[m][2] += gtm.re;
        adj[m][3] += gtm.im;
        const cd qte = cdmul({fp[m] * cf[m].te.re, fp[m] * cf[m].te.im}, Pte);
        const cd qtm = cdmul({fp[m] * cf[m].tm.re, fp[m] * cf[m].tm.im}, Ptm);
        adj[m][4] += cdmul(Ete, cdconj(qte)).re + cdmul(Etm, cdconj(qtm)).re;
    }
}

// Traced-interaction slots: one wavefront per ray, all of its diffuse paths;
// the lanes share each path's frequency sum, and all of them evaluate the
// (identical) chain; lane 0 writes.
template <int KM>
__global__ __launch_bounds__(256) void k_tape_cfr_adjoint_trace(LaunchArgs A, double bw, uint32_t N,
                                                                const double *dldh) {
    const uint32_t K = A.D.K, n_rx = A.D.n_rx, lane = threadIdx.x % kWave, wpb = blockDim.x / kWave;
    for (uint32_t g = blockIdx.x * wpb + threadIdx.x / kWave; g < A.D.T; g += gridDim.x * wpb) {
        double adj[KM][5];
#pragma unroll
        for (int m = 0; m < KM; ++m)
            for (int a = 0; a < 5; ++a) adj[m][a] = 0.0;
        if (A.flags & 4) {
            const float budget = (float)A.items[0].budget;
            SlotCoef cf[KM];
            bool de[KM];
#pragma unroll
            for (int m = 0; m < KM; ++m)
                if (m < (int)K) cf[m] = load_coef(A.slot_coef, (size_t)g * K + m);
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (k >= (int)K) continue;
                const uint32_t ri = g * K + k;
                if (A.rb.id[ri] < 0) continue;
                cd Ete = {0.0, 0.0}, Etm = {0.0, 0.0};
                bool any = false;
                for (uint32_t r = 0; r < n_rx; ++r) {
                    if (!A.dvis[(size_t)ri * n_rx + r]) continue;
                    float a0, plen;
                    diffuse_geom(A, ri, mk(A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]), budget, a0, plen);
                    const c32 ph = propagate(plen, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
                    const cd G = {(double)a0 * ph.re, (double)a0 * ph.im};
                    cd gte, gtm;
                    cfr_path_grad(dldh, r, N, bw, (double)plen / kC0, lane, gte, gtm);
                    const cd ete = cdmul(gte, cdconj(G)), etm = cdmul(gtm, cdconj(G));
                    Ete.re += ete.re;
                    Ete.im += ete.im;
                    Etm.re += etm.re;
                    Etm.im += etm.im;
                    any = true;
                }
                if (!any) continue;
#pragma unroll
                for (int m = 0; m < KM; ++m) de[m] = (m == k);
                chain_adjoint_c<KM>(k + 1, cf, de, Ete, Etm, adj);
            }
        }
#pragma unroll
        for (int m = 0; m < KM; ++m) {
            if (m >= (int)K || lane != 0) continue;
            float4 *o = (float4 *)(A.slot_adj + 8 * ((size_t)g * K + m));
            o[0] = make_float4((float)adj[m][0], (float)adj[m][1], (float)adj[m][2], (float)adj[m][3]);
            o[1] = make_float4((float)adj[m][4], 0.f, 0.f, 0.f);
        }
    }
}

// Specular-path slots: one wavefront per (key, RX) pair, as above.
template <int KM>
__global__ __launch_bounds__(256) void k_tape_cfr_adjoint_spec(LaunchArgs A, double bw, uint32_t N,
                                                               const double *dldh) {
    const uint32_t K = A.D.K, n_rx = A.D.n_rx, TK = A.D.T * A.D.K;
    const uint32_t nk = n_keys_rec(A), lane = threadIdx.x % kWave, wpb = blockDim.x / kWave;
    const size_t n_pairs = (size_t)A.D.rec_keys * n_rx;
    for (size_t p = blockIdx.x * (size_t)wpb + threadIdx.x / kWave; p < n_pairs; p += (size_t)gridDim.x * wpb) {
        double adj[KM][5];
#pragma unroll
        for (int m = 0; m < KM; ++m)
            for (int a = 0; a < 5; ++a) adj[m][a] = 0.0;
        const uint32_t q = (uint32_t)(p / n_rx), r = (uint32_t)(p % n_rx);
        if ((A.flags & 2) && q < nk && A.sb.valid[p]) {
            const uint32_t k = A.keylist[q] % K + 1;
            SlotCoef cf[KM];
            bool de[KM];
#pragma unroll
            for (int m = 0; m < KM; ++m) {
                de[m] = false;
                if (m < (int)k) cf[m] = load_coef(A.slot_coef, TK + p * K + m);
            }
            const float L = A.sb.len[p];
            const float a0 = A.fc.amp_iso / L;
            const c32 ph = propagate(L, A.fc.inv_lam_hi, A.fc.inv_lam_lo);
            const cd G = {(double)a0 * ph.re, (double)a0 * ph.im};
            cd gte, gtm;
            cfr_path_grad(dldh, r, N, bw, (double)L / kC0, lane, gte, gtm);
            chain_adjoint_c<KM>((int)k, cf, de, cdmul(gte, cdconj(G)), cdmul(gtm, cdconj(G)), adj);
        }
#pragma unroll
        for (int m = 0; m < KM; ++m) {
            if (m >= (int)K || lane != 0) continue;
            float4 *o = (float4 *)(A.slot_adj + 8 * (TK + p * K + m));
            o[0] = make_float4((float)adj[m][0], (float)adj[m][1], (float)adj[m][2], (float)adj[m][3]);
            o[1] = make_float4((float)adj[m][4], 0.f, 0.f, 0.f);
        }
    }
}

void launch_tape_cfr_backward(const LaunchArgs &A, double bw, uint32_t N, const double *dldh, hipStream_t s) {
    const uint32_t gt = std::min<uint32_t>((A.D.T + 3) / 4, 16384);  // four wavefronts per block
    const size_t np = (size_t)A.D.rec_keys * A.D.n_rx;
    const uint32_t gs = (uint32_t)std::min<size_t>((np + 3) / 4, 16384);
    switch (A.D.K) {
#define PCRT_TC_CASE(KK)                                                                                       \
    case KK:                                                                                                   \
        hipLaunchKernelGGL(k_tape_cfr_adjoint_trace<KK>, dim3(std::max<uint32_t>(gt, 1)), dim3(256), 0, s, A, bw, N, \
                           dldh);                                                                              \
        hipLaunchKernelGGL(k_tape_cfr_adjoint_spec<KK>, dim3(std::max<uint32_t>(gs, 1)), dim3(256), 0, s, A, bw, N, \
                           dldh);                                                                              \
        break;
        PCRT_TC_CASE(1)
        PCRT_TC_CASE(2)
        PCRT_TC_CASE(3)
        PCRT_TC_CASE(4)
        PCRT_TC_CASE(5)
        PCRT_TC_CASE(6)
        PCRT_TC_CASE(7)
        PCRT_TC_CASE(8)
#undef PCRT_TC_CASE
        default: break;
    }
}

// Per-label gradient: for each slot, dL/d(eps_r, sigma) = Re(conj(g) dGamma/deta deta/dtheta)
// summed over TE and TM (deta/deps_r = 1, deta/dsigma = -j/(omega eps0)), and
// dL/dS = g_S. One 64-lane block per slot chunk; lane t owns an LDS row of
// per-label sums; rows are combined by a fixed tree.
__global__ __launch_bounds__(64) void k_label_grad(LaunchArgs A, const float *mats, uint32_t n_labels) {
    extern __shared__ double acc[];  // [64][n_labels * 3]
    const int t = threadIdx.x;
    const uint32_t W = n_labels * 3;
    for (uint32_t c = blockIdx.x; c < A.D.n_slot_chunks; c += gridDim.x) {
        for (uint32_t i = 0; i < W; ++i) acc[t * W + i] = 0.0;
        const uint32_t s0 = c * kSlotChunk, s1 = min(s0 + kSlotChunk, A.D.n_slots);
        for (uint32_t s = s0 + t; s < s1; s += 64) {
            const uint32_t lab = A.slot_label[s];
            if (lab >= n_labels) continue;
            const float4 g = ((const float4 *)(A.slot_adj + 8 * (size_t)s))[0];
            const float gS = A.slot_adj[8 * (size_t)s + 4];
            if (g.x == 0.f && g.y == 0.f && g.z == 0.f && g.w == 0.f && gS == 0.f) continue;
            c32 dte, dtm;
            fresnel_deta(mats[3 * lab], mats[3 * lab + 1] * A.fc.inv_we0, A.slot_cos[s], dte, dtm);
            // Re(conj(g) z) = g.re z.re + g.im z.im
            const double de = (double)g.x * dte.re + (double)g.y * dte.im + (double)g.z * dtm.re + (double)g.w * dtm.im;
            // d/dsigma: z * (-j w) with w = 1/(omega eps0): (z.im w, -z.re w)
            const double wv = A.fc.inv_we0;
            const double ds = ((double)g.x * dte.im - (double)g.y * dte.re + (double)g.z * dtm.im -
                               (double)g.w * dtm.re) * wv;
            acc[t * W + 3 * lab] += de;
            acc[t * W + 3 * lab + 1] += ds;
            acc[t * W + 3 * lab + 2] += gS;
        }
        __syncthreads();
        for (int st = 32; st > 0; st >>= 1) {
            if (t < st)
                for (uint32_t i = 0; i < W; ++i) acc[t * W + i] += acc[(t + st) * W + i];
            __syncthreads();
        }
        for (uint32_t i = t; i < W; i += 64) A.grad_part[(size_t)c * kMaxGradLabels * 3 + i] = acc[i];
        __syncthreads();
    }
}

__global__ void k_label_grad_final(LaunchArgs A, uint32_t n_labels, double *out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_labels * 3) return;
    // chunk order; eight loads are issued ahead of their adds
    const uint32_t n = A.D.n_slot_chunks;
    const size_t pitch = (size_t)kMaxGradLabels * 3;
    double s = 0.0;
    uint32_t c = 0;
    for (; c + 8 <= n; c += 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = A.grad_part[(c + k) * pitch + i];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
    }
    for (; c < n; ++c) s += A.grad_part[c * pitch + i];
    out[i] = s;
}

void launch_material_grad(const LaunchArgs &A, const float *mats, uint32_t n_labels, double *out, hipStream_t s) {
    const uint32_t g = std::min<uint32_t>(std::max<uint32_t>(A.D.n_slot_chunks, 1), 4096);
    const size_t lds = sizeof(double) * 64 * n_labels * 3;
    hipLaunchKernelGGL(k_label_grad, dim3(g), dim3(64), lds, s, A, mats, n_labels);
    hipLaunchKernelGGL(k_label_grad_final, dim3((n_labels * 3 + 63) / 64), dim3(64), 0, s, A, n_labels, out);
}

}  // namespace pcrt
