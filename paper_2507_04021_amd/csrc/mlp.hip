// Learned material model: a small MLP that maps (material label, incidence
// cosine, log10 frequency) to (Gamma_TE, Gamma_TM, S) for every interaction
// slot of a tape, in place of the per-label Fresnel model.
//
//   x (32) = [emb[label] (16), cos, log10(f/1 GHz), 0...]
//   h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2), h3 = GELU(W3 h2 + b3)   (64 each)
//   z = W4 h3 + b4 (5 used of 16); Gamma_TE = (z0 + j z1) tanh|.|/|.|,
//   Gamma_TM = (z2 + j z3) tanh|.|/|.|, S = sigmoid(z4)
//
// BF16 operands, FP32 accumulation, on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16). Lane layout of that instruction (one wavefront):
//   A[i][k]: lane l holds i = l % 16, k = 8 (l / 16) + j, j = 0..7
//   B[k][n]: lane l holds n = l % 16, k = 8 (l / 16) + j
//   C[i][n]: lane l holds n = l % 16, i = 4 (l / 16) + r, r = 0..3
//
// Forward: every layer is computed transposed, Y^T = W X^T, with the weights
// as the A operand (held in registers for the wavefront's whole life) and
// 16 rows as the B operand. The result leaves lane (n, g = l / 16) holding
// row n's outputs 16 t + 4 g + r (t = 0..3 output tiles, r = 0..3). A
// contraction does not care in which order its K index runs, so the next
// layer takes its K index in exactly that order: K step ks, element j is
// input 16 (2 ks + j / 4) + 4 g + j % 4, which lane (n, g) already holds. The
// weights are loaded in the same permuted order, and the activations never
// leave the registers between layers.
// Backward: the forward recompute and the gradient chain dH = W^T dZ run the
// same way; the weight gradients dW = dZ^T H contract over rows, so their
// operands are transposed through LDS, and each wavefront accumulates its
// share of every weight gradient in registers, written once as a partial
// that a fixed-order reduction adds up.
//
// GELU: erf by Abramowitz & Stegun 7.1.26 (absolute error below 1.5e-7 in
// erf; GELU within 3.3e-7) in the backward pass; the forward pass
// interpolates linearly in a table of that GELU at 8193 nodes over [-8, 8]
// (spacing 2^-9, built in LDS by every block; beyond the ends the end
// intervals extend linearly), within 1e-6. Both are far below the BF16
// rounding of the activations (2^-8 relative).
#include <cstring>

#include "common.h"
#include "internal.h"
#include "pcrt.h"

namespace pcrt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 32, kHid = 64, kOut = 16, kEmb = 16;
constexpr int kW1 = kHid * kIn, kW2 = kHid * kHid, kW3 = kHid * kHid, kW4 = kOut * kHid;
constexpr int kWAll = kW1 + kW2 + kW3 + kW4;       // 11264 bf16
constexpr int kBAll = kHid * 3 + kOut;             // 208 floats
constexpr int kTileRows = 16;

__device__ __forceinline__ float bf(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }
__device__ __forceinline__ uint16_t to_bf(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ __bf16 as_b(uint16_t u) { return __builtin_bit_cast(__bf16, u); }

// Lanes of one wavefront hand tiles to each other through LDS: order the
// writes before the following reads (wave-scope fence + scheduling barrier).
// GELU(z) = z Phi(z), Phi(z) = (1 + erf(z / sqrt 2)) / 2. With x = |z| / sqrt 2,
// erf(x) = 1 - (a1 t + ... + a5 t^5) exp(-x^2), t = 1 / (1 + p x)
// (Abramowitz & Stegun 7.1.26), so h = (1 - erf(x)) / 2 = Phi(-|z|) and
// GELU(z) = max(z, 0) - |z| h. Returns h; e receives exp(-z^2 / 2).
__device__ __forceinline__ float norm_tail(float z, float &e) {
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, fabsf(z), 1.0f));
    const float poly =  // the coefficients halved
        fmaf(fmaf(fmaf(fmaf(0.5307027145f, t, -0.7265760135f), t, 0.7107068705f), t, -0.142248368f), t, 0.127414796f) *
        t;
    e = __builtin_amdgcn_exp2f(z * z * -0.72134752044448170f);  // 2^(-z^2 log2(e) / 2)
    return poly * e;
}
// max(z, 0) on the bit pattern: a non-negative float is a non-negative int32,
// a negative one a negative int32 (one integer max, no NaN canonicalisation)
__device__ __forceinline__ float relu(float z) { return __int_as_float(max(__float_as_int(z), 0)); }
__device__ __forceinline__ float gelu(float z) {
    float e;
    const float h = norm_tail(z, e);
    return fmaf(-fabsf(z), h, relu(z));
}
// GELU'(z) = Phi(z) + z phi(z), phi(z) = exp(-z^2 / 2) / sqrt(2 pi).
__device__ __forceinline__ float gelu_grad(float z) {
    float e;
    const float h = norm_tail(z, e);
    return fmaf(z * 0.39894228040143268f, e, z >= 0.f ? 1.0f - h : h);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Two floats to two bf16 (round to nearest even), low half first.
__device__ __forceinline__ uint32_t pack_bf2(float a, float b) {
    const bf16x2 v = __builtin_convertvector((f32x2){a, b}, bf16x2);
    return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ bf16x8 bf8_of(u32x4 p) { return __builtin_bit_cast(bf16x8, p); }

// (u + j v) tanh(r)/r and its Jacobian (a = d re/du, b = d re/dv = d im/du, d = d im/dv).
__device__ __forceinline__ void radial(float u, float v, float &re, float &im, float &a, float &b, float &d) {
    float r = sqrtf(u * u + v * v);
    float g, gp;  // g(r) = tanh r / r, gp = g'(r) / r
    if (r < 1e-4f) {
        g = 1.f - r * r / 3.f;
        gp = -2.f / 3.f;
    } else {
        float t = tanhf(r);
        g = t / r;
        gp = (r * (1.f - t * t) - t) / (r * r * r);
    }
    re = u * g;
    im = v * g;
    a = g + u * u * gp;
    b = u * v * gp;
    d = g + v * v * gp;
}

struct MlpArgs {
    const uint16_t *w;   // bf16 bits: W1 [64][32], W2 [64][64], W3 [64][64], W4 [16][64] (row = output)
    const float *b;      // b1 [64], b2 [64], b3 [64], b4 [16]
    const float *emb;    // [n_labels][16] float32
    uint32_t n_labels;
    uint32_t n;          // rows
    const uint16_t *label;
    const float *cosv;
    float logf;
    float *out;          // [n][8]
    const float *gout;   // [n][8]
    float *part;         // per-wavefront gradient partials [kBwdWaves][part_stride]
    uint32_t part_stride;
};

// Per-lane MFMA A fragments of the weights in the transposed formulation
// (lane (i, g): output 16 t + i, K elements j = 0..7 of K step ks), and the
// biases of the outputs the lane holds (16 t + 4 g + r at index 4 t + r).
struct RegNet {
    bf16x8 w1[4], w2[4][2], w3[4][2], w4[2];
    f32x4 b1[4], b2[4], b3[4], b4;  // the MFMA accumulators start from these
};

// Input index of K step ks, element j, lane group g, for the hidden layers
// (the order in which the previous layer's outputs sit in the registers).
__device__ __forceinline__ int perm_k(int ks, int g, int j) { return 16 * (2 * ks + (j >> 2)) + 4 * g + (j & 3); }

__device__ __forceinline__ bf16x8 wfrag(const uint16_t *W, int ld, int row, int ks, int g, bool natural) {
    u32x4 p;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = 2 * q;
        const int k0 = natural ? 8 * g + j : perm_k(ks, g, j), k1 = natural ? 8 * g + j + 1 : perm_k(ks, g, j + 1);
        p[q] = (uint32_t)W[row * ld + k0] | ((uint32_t)W[row * ld + k1] << 16);
    }
    return bf8_of(p);
}

__device__ __forceinline__ void load_regnet(const MlpArgs &M, int lane, RegNet &R) {
    const int i = lane & 15, g = lane >> 4;
    const uint16_t *w1 = M.w, *w2 = w1 + kW1, *w3 = w2 + kW2, *w4 = w3 + kW3;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        R.w1[t] = wfrag(w1, kIn, 16 * t + i, 0, g, true);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            R.w2[t][ks] = wfrag(w2, kHid, 16 * t + i, ks, g, false);
            R.w3[t][ks] = wfrag(w3, kHid, 16 * t + i, ks, g, false);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            R.b1[t][r] = M.b[16 * t + 4 * g + r];
            R.b2[t][r] = M.b[kHid + 16 * t + 4 * g + r];
            R.b3[t][r] = M.b[2 * kHid + 16 * t + 4 * g + r];
        }
    }
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) R.w4[ks] = wfrag(w4, kHid, i, ks, g, false);
#pragma unroll
    for (int r = 0; r < 4; ++r) R.b4[r] = M.b[3 * kHid + 4 * g + r];
}

// Input B fragment of one row for lane group g (natural K order): g = 0, 1
// the embedding's halves, g = 2 (cos, log f, 0, ...), g = 3 zeros; an empty
// slot or a row past the end gives zeros.
__device__ __forceinline__ bf16x8 input_frag(const MlpArgs &M, uint32_t row, uint16_t lab, int g) {
    float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (lab < M.n_labels) {
        if (g < 2) {
            const float4 *e = (const float4 *)(M.emb + (size_t)lab * kEmb + 8 * g);
            const float4 a = e[0], b = e[1];
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
            v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else if (g == 2) {
            v[0] = M.cosv[row];
            v[1] = M.logf;
        }
    }
    return bf8_of(u32x4{pack_bf2(v[0], v[1]), pack_bf2(v[2], v[3]), pack_bf2(v[4], v[5]), pack_bf2(v[6], v[7])});
}

// GELU of one layer's outputs (C layout, bias included) into the next layer's two B
// fragments (K order perm_k).
constexpr int kGeluN = 8192;  // table intervals over [-8, 8): node i at -8 + i / 512
// GELU from the table (value, slope to the next node) of the node below z;
// z outside [-8, 8) uses the end interval's line (GELU(z) = z and 0 there to
// FP32 precision).
__device__ __forceinline__ float gelu_tab(const float2 *tab, float z) {
    const float x = fmaf(z, 512.f, 4096.f);
    const float c = __builtin_amdgcn_fmed3f(floorf(x), 0.f, (float)(kGeluN - 1));
    const float2 e = tab[(int)c];
    return fmaf(x - c, e.y, e.x);
}
__device__ void build_gelu_table(float2 *tab) {  // tab[kGeluN + 1], every thread of the block
    for (int i = threadIdx.x; i <= kGeluN; i += blockDim.x) tab[i].x = gelu(-8.f + (float)i * (1.f / 512.f));
    __syncthreads();
    constexpr int kPer = kGeluN / 256;
    float slope[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int i = threadIdx.x + 256 * k;
        slope[k] = tab[i + 1].x - tab[i].x;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) tab[threadIdx.x + 256 * k].y = slope[k];
    __syncthreads();
}
__device__ __forceinline__ void act_frags(const f32x4 (&acc)[4], bf16x8 (&h)[2], const float2 *tab) {
    float v[16];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) v[4 * t + r] = gelu_tab(tab, acc[t][r]);  // the accumulation started from the bias
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
        h[ks] = bf8_of(u32x4{pack_bf2(v[8 * ks + 0], v[8 * ks + 1]), pack_bf2(v[8 * ks + 2], v[8 * ks + 3]),
                             pack_bf2(v[8 * ks + 4], v[8 * ks + 5]), pack_bf2(v[8 * ks + 6], v[8 * ks + 7])});
}

#define MFMA16(a, b, c) __builtin_amdgcn_mfma_f32_16x16x32_bf16((a), (b), (c), 0, 0, 0)

// The three hidden layers and the output layer of one 16-row tile; x: the
// input fragment. Returns z4 (C layout: lane (n, g) holds outputs 4 g + r).
__device__ __forceinline__ f32x4 net_forward(const RegNet &R, bf16x8 x, const float2 *tab) {
    f32x4 acc[4];
    bf16x8 h[2];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = MFMA16(R.w1[t], x, R.b1[t]);
    act_frags(acc, h, tab);
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = MFMA16(R.w2[t][1], h[1], MFMA16(R.w2[t][0], h[0], R.b2[t]));
    act_frags(acc, h, tab);
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = MFMA16(R.w3[t][1], h[1], MFMA16(R.w3[t][0], h[0], R.b3[t]));
    act_frags(acc, h, tab);
    return MFMA16(R.w4[1], h[1], MFMA16(R.w4[0], h[0], R.b4));
}

constexpr int kFwdTiles = 8;  // 16-row tiles a wavefront carries at once (independent MFMA chains)

// Persistent wavefronts, each holding the whole network in registers; tiles
// are dealt by wavefront index (grid stride), kFwdTiles at a time.
// Output map of the forward pass: (u + j v) tanh(r) / r with tanh r =
// 1 - 2 / (e^{2r} + 1) (relative error near 1e-6 down to r = 0.1), and the
// series 1 - r^2 / 3 + 2 r^4 / 15 below (truncation 6e-8 relative).
__device__ __forceinline__ void radial_fwd(float u, float v, float &re, float &im) {
    const float r2 = u * u + v * v;
    float g;
    if (r2 < 0.01f) {
        g = fmaf(fmaf(0.133333333f, r2, -0.333333333f), r2, 1.0f);
    } else {
        const float rinv = __builtin_amdgcn_rsqf(r2), r = r2 * rinv;
        const float ex = __builtin_amdgcn_exp2f(2.8853900817779268f * r);  // e^{2r}
        g = (1.0f - 2.0f * __builtin_amdgcn_rcpf(ex + 1.0f)) * rinv;
    }
    re = u * g;
    im = v * g;
}

__global__ __launch_bounds__(256) void k_mlp_forward(MlpArgs M) {
    __shared__ float2 tab[kGeluN + 1];
    build_gelu_table(tab);
    const int lane = threadIdx.x & 63, g = lane >> 4, nl = lane & 15;
    RegNet R;
    load_regnet(M, lane, R);
    const uint32_t wave = blockIdx.x * 4 + (threadIdx.x >> 6), n_waves = gridDim.x * 4;
    const uint32_t n_tiles = (M.n + kTileRows - 1) / kTileRows;
    for (uint32_t t0 = wave * kFwdTiles; t0 < n_tiles; t0 += n_waves * kFwdTiles) {
        uint32_t row[kFwdTiles];
        uint16_t lab[kFwdTiles];
        f32x4 z4[kFwdTiles];
#pragma unroll
        for (int tt = 0; tt < kFwdTiles; ++tt) {
            row[tt] = (t0 + tt) * kTileRows + nl;
            lab[tt] = row[tt] < M.n ? M.label[row[tt]] : (uint16_t)0xffff;
        }
#pragma unroll
        for (int tt = 0; tt < kFwdTiles; ++tt) z4[tt] = net_forward(R, input_frag(M, row[tt], lab[tt], g), tab);
#pragma unroll
        for (int tt = 0; tt < kFwdTiles; ++tt) {
            if (row[tt] >= M.n || g > 1) continue;
            float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
            if (lab[tt] < M.n_labels) {
                if (g == 0) {
                    radial_fwd(z4[tt][0], z4[tt][1], o.x, o.y);
                    radial_fwd(z4[tt][2], z4[tt][3], o.z, o.w);
                } else {
                    o.x = 1.f / (1.f + expf(-z4[tt][0]));  // S from output 4
                }
            }
            ((float4 *)(M.out + 8 * (size_t)row[tt]))[g] = o;
        }
    }
}

// ------------------------------------------------------------------ backward
// One kernel: per 16-row tile, the forward recompute (keeping GELU'(z) of
// every hidden unit and the bf16 activations), the output Jacobian, the
// gradient chain dH = W^T dZ, dZ = dH GELU'(z) on the matrix cores
// (transposed formulation, K order as in the forward), and the weight
// gradients dW = dZ^T H over the tile's 16 rows (v_mfma_f32_16x16x16_bf16,
// K = 16 rows). For the last, dZ and H of a layer are written to LDS
// transposed ([feature][row]), so that each operand lane holds one feature
// and 4 rows; the accumulators stay in registers for the wavefront's whole
// life. Bias gradients are per-lane sums of the bf16-rounded dZ, embedding
// gradients an LDS table per wavefront updated row by row. Every wavefront
// writes its partials once; a fixed-order reduction over wavefronts gives
// the gradients. The grid is fixed (kBwdWaves), so the result does not
// depend on the device.
constexpr uint32_t kBwdWaves = 1024;
constexpr int kMaxLabels = 64;
// Weight fragments in LDS, fragment-major (fragment f, lane l at f * 64 + l,
// 16 B each): forward W1 (4), W2 (4 x 2), W3 (4 x 2), W4 (2); then for the
// chain W4^T (4; K = the 16 outputs, lane group g holds outputs 4 g .. 4 g + 3
// and zeros), W3^T (4 x 2), W2^T (4 x 2), W1^T rows 0..15 (2).
constexpr int kFF1 = 0, kFF2 = 4, kFF3 = 12, kFF4 = 20, kFB4 = 22, kFB3 = 26, kFB2 = 34, kFB1 = 42, kFrags = 44;
constexpr int kTrRow = 24;  // bf16 per LDS row of a transposed operand (16 rows + pad: 48 B)
constexpr int kPartW = kWAll + kBAll;  // per-wavefront partial: weights then biases, then the embedding table

typedef short s16x4 __attribute__((ext_vector_type(4)));
#define MFMA16K16(a, b, c) __builtin_amdgcn_mfma_f32_16x16x16bf16_1k((a), (b), (c), 0, 0, 0)

struct BwdShared {
    bf16x8 frag[kFrags * 64];
    float bias[kBAll];
    uint16_t dzt[4][kHid * kTrRow];   // per wavefront: dZ^T of the current layer
    uint16_t ht[4][kHid * kTrRow];    // per wavefront: its input activations H^T
    float emb[4][kMaxLabels * kEmb];  // per wavefront: embedding-gradient table
};

__device__ __forceinline__ bf16x8 gather_frag(const uint16_t *W, int f, int lane) {
    // element j of lane's fragment f is W[base + row * ld + col]
    const int i = lane & 15, g = lane >> 4;
    u32x4 p;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = 2 * q + h;
            int row, col, base;
            bool zero = false;
            if (f < kFF2) { base = 0; row = 16 * (f - kFF1) + i; col = 8 * g + j; }
            else if (f < kFF3) { base = kW1; const int t = (f - kFF2) >> 1, ks = (f - kFF2) & 1; row = 16 * t + i; col = perm_k(ks, g, j); }
            else if (f < kFF4) { base = kW1 + kW2; const int t = (f - kFF3) >> 1, ks = (f - kFF3) & 1; row = 16 * t + i; col = perm_k(ks, g, j); }
            else if (f < kFB4) { base = kW1 + kW2 + kW3; row = i; col = perm_k(f - kFF4, g, j); }
            else if (f < kFB3) { base = kW1 + kW2 + kW3; row = 4 * g + (j & 3); col = 16 * (f - kFB4) + i; zero = j >= 4; }
            else if (f < kFB2) { base = kW1 + kW2; const int t = (f - kFB3) >> 1, ks = (f - kFB3) & 1; row = perm_k(ks, g, j); col = 16 * t + i; }
            else if (f < kFB1) { base = kW1; const int t = (f - kFB2) >> 1, ks = (f - kFB2) & 1; row = perm_k(ks, g, j); col = 16 * t + i; }
            else { base = 0; row = perm_k(f - kFB1, g, j); col = i; }
            const int ldw = base == 0 ? kIn : kHid;
            v[h] = zero ? 0u : (uint32_t)W[base + row * ldw + col];
        }
        p[q] = v[0] | (v[1] << 16);
    }
    return bf8_of(p);
}

__device__ __forceinline__ void unpack8(bf16x8 v, float (&o)[8]) {
    const u32x4 p = __builtin_bit_cast(u32x4, v);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        o[2 * q] = __uint_as_float(p[q] << 16);
        o[2 * q + 1] = __uint_as_float(p[q] & 0xffff0000u);
    }
}

__device__ __forceinline__ uint16_t elem(bf16x8 v, int j) {
    const uint32_t p = __builtin_bit_cast(u32x4, v)[j >> 1];
    return (uint16_t)((j & 1) ? (p >> 16) : (p & 0xffffu));
}

// A layer's 16 values of one row (the two packed fragments, K order perm_k)
// into a transposed LDS operand [feature][row].
__device__ __forceinline__ void put_t(uint16_t *T, const bf16x8 (&h)[2], int lane) {
    const int n = lane & 15, g = lane >> 4;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int j = 0; j < 8; ++j) T[perm_k(ks, g, j) * kTrRow + n] = elem(h[ks], j);
}

// K = 16 operand of a transposed LDS tile: lane (i, g) gets feature
// 16 ft + i, rows 4 g .. 4 g + 3.
__device__ __forceinline__ s16x4 get_t(const uint16_t *T, int ft, int lane) {
    return *(const s16x4 *)(T + (16 * ft + (lane & 15)) * kTrRow + 4 * (lane >> 4));
}

__global__ __launch_bounds__(256) void k_mlp_backward(MlpArgs M) {
    __shared__ BwdShared S;
    for (int e = threadIdx.x; e < kFrags * 64; e += 256) S.frag[e] = gather_frag(M.w, e / 64, e % 64);
    for (int e = threadIdx.x; e < kBAll; e += 256) S.bias[e] = M.b[e];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    for (int e = lane; e < kMaxLabels * kEmb; e += 64) S.emb[wave][e] = 0.f;
    __syncthreads();
    const bf16x8 *F = S.frag + lane;
    auto bias4 = [&](int off, int t) { return *(const f32x4 *)(S.bias + off + 16 * t + 4 * g); };
    uint16_t *DZ = S.dzt[wave], *HT = S.ht[wave];
    float *ET = S.emb[wave];
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    // weight-gradient accumulators (C layout of dW tiles: out tile a, in tile b)
    f32x4 gw1[4][2], gw2[4][4], gw3[4][4], gw4[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gw4[a] = zero;
#pragma unroll
        for (int b = 0; b < 4; ++b) { gw2[a][b] = zero; gw3[a][b] = zero; }
#pragma unroll
        for (int b = 0; b < 2; ++b) gw1[a][b] = zero;
    }
    float gb1[16] = {}, gb2[16] = {}, gb3[16] = {}, gb4[4] = {};  // this lane's bias-gradient sums
    // GELU and GELU' of a layer's outputs (C layout, bias included)
    auto layer = [&](const f32x4 (&acc)[4], bf16x8 (&h)[2], float (&gp)[16]) {
        float v[16];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = acc[t][r];
                float e;
                const float tail = norm_tail(z, e);
                v[4 * t + r] = fmaf(-fabsf(z), tail, relu(z));
                gp[4 * t + r] = fmaf(z * 0.39894228040143268f, e, z >= 0.f ? 1.0f - tail : tail);
            }
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            h[ks] = bf8_of(u32x4{pack_bf2(v[8 * ks + 0], v[8 * ks + 1]), pack_bf2(v[8 * ks + 2], v[8 * ks + 3]),
                                 pack_bf2(v[8 * ks + 4], v[8 * ks + 5]), pack_bf2(v[8 * ks + 6], v[8 * ks + 7])});
    };
    // dZ = (W^T dZ_next) GELU'(z), rounded to bf16 (K order perm_k), and its bias-gradient sums
    auto chain = [&](int fb, const bf16x8 *src, int nks, const float (&gp)[16], bf16x8 (&out)[2], float (&gb)[16]) {
        f32x4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            acc[t] = zero;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                if (ks < nks) acc[t] = MFMA16(F[64 * (fb + nks * t + ks)], src[ks], acc[t]);
        }
        float v[16];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) v[4 * t + r] = acc[t][r] * gp[4 * t + r];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            out[ks] = bf8_of(u32x4{pack_bf2(v[8 * ks + 0], v[8 * ks + 1]), pack_bf2(v[8 * ks + 2], v[8 * ks + 3]),
                                   pack_bf2(v[8 * ks + 4], v[8 * ks + 5]), pack_bf2(v[8 * ks + 6], v[8 * ks + 7])});
            float dr[8];
            unpack8(out[ks], dr);
#pragma unroll
            for (int j = 0; j < 8; ++j) gb[8 * ks + j] += dr[j];  // element j of fragment ks is value 8 ks + j
        }
    };
    // dW (out tiles x in tiles) += dZ^T H over the tile's rows, from the transposed LDS copies
    auto wgrad = [&](f32x4 (*gw)[4], int n_out, int n_in) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            if (a >= n_out) continue;
            const s16x4 av = get_t(DZ, a, lane);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (b < n_in) gw[a][b] = MFMA16K16(av, get_t(HT, b, lane), gw[a][b]);
        }
    };
    const uint32_t wid = blockIdx.x * 4 + wave;
    const uint32_t n_tiles = (M.n + kTileRows - 1) / kTileRows;
    for (uint32_t tile = wid; tile < n_tiles; tile += kBwdWaves) {
        const uint32_t row = tile * kTileRows + n;
        const uint16_t lab = row < M.n ? M.label[row] : (uint16_t)0xffff;
        const bool live = row < M.n && lab < M.n_labels;
        const bf16x8 x = input_frag(M, row, lab, g);
        bf16x8 h1[2], h2[2], h3[2];
        float gp1[16], gp2[16], gp3[16];
        f32x4 acc[4];
        // forward recompute
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = MFMA16(F[64 * (kFF1 + t)], x, bias4(0, t));
        layer(acc, h1, gp1);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = MFMA16(F[64 * (kFF2 + 2 * t + 1)], h1[1], MFMA16(F[64 * (kFF2 + 2 * t)], h1[0], bias4(kHid, t)));
        layer(acc, h2, gp2);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = MFMA16(F[64 * (kFF3 + 2 * t + 1)], h2[1], MFMA16(F[64 * (kFF3 + 2 * t)], h2[0], bias4(2 * kHid, t)));
        layer(acc, h3, gp3);
        const f32x4 z4 = MFMA16(F[64 * (kFF4 + 1)], h3[1],
                                MFMA16(F[64 * kFF4], h3[0], *(const f32x4 *)(S.bias + 3 * kHid + 4 * g)));
        // output Jacobian: lanes g = 0 (outputs 0..3) and g = 1 (output 4) of live rows
        float dz[4] = {0.f, 0.f, 0.f, 0.f};
        if (live && g < 2) {
            const float *go = M.gout + 8 * (size_t)row;
            if (g == 0) {
                float re, im, a, b, d;
                radial(z4[0], z4[1], re, im, a, b, d);
                dz[0] = go[0] * a + go[1] * b;
                dz[1] = go[0] * b + go[1] * d;
                radial(z4[2], z4[3], re, im, a, b, d);
                dz[2] = go[2] * a + go[3] * b;
                dz[3] = go[2] * b + go[3] * d;
            } else {
                const float s4 = 1.f / (1.f + expf(-z4[0]));
                dz[0] = go[4] * s4 * (1.f - s4);
            }
        }
        const bf16x8 d4 = bf8_of(u32x4{pack_bf2(dz[0], dz[1]), pack_bf2(dz[2], dz[3]), 0u, 0u});
        {
            float dr[8];
            unpack8(d4, dr);
#pragma unroll
            for (int r = 0; r < 4; ++r) gb4[r] += dr[r];
        }
        // layer 4: dZ4^T (rows 4 g + r) and H3^T, then dW4
#pragma unroll
        for (int r = 0; r < 4; ++r) DZ[(4 * g + r) * kTrRow + n] = elem(d4, r);
        put_t(HT, h3, lane);
        wave_sync();
        wgrad(&gw4, 1, 4);  // gw4 as one out tile x four in tiles
        wave_sync();
        // layer 3
        bf16x8 dz3[2], dz2[2], dz1[2];
        chain(kFB4, &d4, 1, gp3, dz3, gb3);
        put_t(DZ, dz3, lane);
        put_t(HT, h2, lane);
        wave_sync();
        wgrad(gw3, 4, 4);
        wave_sync();
        // layer 2
        chain(kFB3, dz3, 2, gp2, dz2, gb2);
        put_t(DZ, dz2, lane);
        put_t(HT, h1, lane);
        wave_sync();
        wgrad(gw2, 4, 4);
        wave_sync();
        // layer 1 (H = the input: 32 features in natural order, element j of lane group g is feature 8 g + j)
        chain(kFB2, dz2, 2, gp1, dz1, gb1);
        put_t(DZ, dz1, lane);
#pragma unroll
        for (int j = 0; j < 8; ++j) HT[(8 * g + j) * kTrRow + n] = elem(x, j);
        const f32x4 dx = MFMA16(F[64 * (kFB1 + 1)], dz1[1], MFMA16(F[64 * kFB1], dz1[0], zero));
        wave_sync();
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const s16x4 av = get_t(DZ, a, lane);
#pragma unroll
            for (int b = 0; b < 2; ++b) gw1[a][b] = MFMA16K16(av, get_t(HT, b, lane), gw1[a][b]);
        }
        // embedding gradient: row by row in order, the four lanes of a row add dims 4 g .. 4 g + 3
        for (int s = 0; s < 16; ++s) {
            if (n == s && live) {
                float *e = ET + lab * kEmb + 4 * g;
#pragma unroll
                for (int r = 0; r < 4; ++r) e[r] += dx[r];
            }
            wave_sync();
        }
    }
    // partials: the weight gradients from the accumulators (C layout: lane
    // holds in-feature 16 b + n, out-features 16 a + 4 g + r), the bias sums
    // reduced over the 16 row lanes in a fixed butterfly, the embedding table
    float *P = M.part + (size_t)wid * M.part_stride;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 16 * a + 4 * g + r;
#pragma unroll
            for (int b = 0; b < 2; ++b) P[o * kIn + 16 * b + n] = gw1[a][b][r];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                P[kW1 + o * kHid + 16 * b + n] = gw2[a][b][r];
                P[kW1 + kW2 + o * kHid + 16 * b + n] = gw3[a][b][r];
            }
        }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int b = 0; b < 4; ++b) P[kW1 + kW2 + kW3 + (4 * g + r) * kHid + 16 * b + n] = gw4[b][r];
    auto lane_sum16 = [&](float v) {  // over the 16 lanes of a lane group, fixed order
        for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
        return v;
    };
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // element 4 t + r of the sums is feature 16 t + 4 g + r
            const float s1 = lane_sum16(gb1[4 * t + r]), s2 = lane_sum16(gb2[4 * t + r]),
                        s3 = lane_sum16(gb3[4 * t + r]);
            if (n == 0) {
                P[kWAll + 16 * t + 4 * g + r] = s1;
                P[kWAll + kHid + 16 * t + 4 * g + r] = s2;
                P[kWAll + 2 * kHid + 16 * t + 4 * g + r] = s3;
            }
        }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float s4 = lane_sum16(gb4[r]);
        if (n == 0) P[kWAll + 3 * kHid + 4 * g + r] = s4;
    }
    wave_sync();
    for (uint32_t e = lane; e < M.n_labels * kEmb; e += 64) P[kPartW + e] = ET[e];
}

// Fixed-order sum of per-block partials, first stage: block (x, y) adds, for
// columns 64 x .. 64 x + 63, the partials of split y (kSumSplits contiguous
// ranges) -- each of its four wavefronts a quarter of the range in order,
// then the four in wavefront order -- into part2[y][column].
constexpr uint32_t kSumSplits = 16;
__global__ __launch_bounds__(256) void k_sum_parts_split(const float *part, uint32_t n_parts, uint32_t width,
                                                         uint32_t stride, float *part2) {
    __shared__ float red[4][64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t i = blockIdx.x * 64 + lane;
    const uint32_t p0 = (uint32_t)((uint64_t)blockIdx.y * n_parts / kSumSplits);
    const uint32_t p1 = (uint32_t)((uint64_t)(blockIdx.y + 1) * n_parts / kSumSplits);
    const uint32_t b0 = p0 + (uint32_t)((uint64_t)wave * (p1 - p0) / 4);
    const uint32_t b1 = p0 + (uint32_t)((uint64_t)(wave + 1) * (p1 - p0) / 4);
    float s = 0.f;
    if (i < width)
        for (uint32_t b = b0; b < b1; ++b) s += part[(size_t)b * stride + i];
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && i < width)
        part2[(size_t)blockIdx.y * width + i] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Second stage: out[i] = sum over the splits in order.
__global__ void k_sum_parts(const float *part2, uint32_t width, float *out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= width) return;
    float s = 0.f;
    for (uint32_t y = 0; y < kSumSplits; ++y) s += part2[(size_t)y * width + i];
    out[i] = s;
}

void sum_parts(const float *part, uint32_t n_parts, uint32_t width, uint32_t stride, float *part2, float *out,
               hipStream_t s) {
    hipLaunchKernelGGL(k_sum_parts_split, dim3((width + 63) / 64, kSumSplits), dim3(256), 0, s, part, n_parts, width,
                       stride, part2);
    hipLaunchKernelGGL(k_sum_parts, dim3((width + 255) / 256), dim3(256), 0, s, part2, width, out);
}

}  // namespace pcrt

using namespace pcrt;

namespace {
struct MlpLayout {
    size_t part, part2, total;
    uint32_t stride;
};
// Per-wavefront partials of the backward kernel (weights, biases, embedding
// table), then the first-stage sums of the fixed-order reduction.
MlpLayout mlp_layout(uint32_t n_labels) {
    Bump b;
    MlpLayout L;
    L.stride = kPartW + n_labels * kEmb;
    L.part = b.take(4ull * kBwdWaves * L.stride);
    L.part2 = b.take(4ull * kSumSplits * L.stride);
    L.total = b.off;
    return L;
}
}  // namespace

extern "C" {

pcrt_status pcrt_mlp_workspace_size(uint32_t n, uint32_t n_labels, size_t *bytes) {
    if (!bytes) return PCRT_EINVAL;
    (void)n;  // the partials are per wavefront of a fixed grid, not per row
    *bytes = mlp_layout(std::max<uint32_t>(n_labels, 1)).total;
    return PCRT_OK;
}

pcrt_status pcrt_mlp_forward(const pcrt_mlp *net, uint32_t n, const uint16_t *label, const float *cosv, float log_f,
                             float *out, void *stream) {
    if (!net || !net->w || !net->b || !net->emb || !label || !cosv || !out) return PCRT_EINVAL;
    if (n == 0) return PCRT_OK;
    MlpArgs M;
    memset(&M, 0, sizeof M);
    M.w = net->w;
    M.b = net->b;
    M.emb = net->emb;
    M.n_labels = net->n_labels;
    M.n = n;
    M.label = label;
    M.cosv = cosv;
    M.logf = log_f;
    M.out = out;
    const uint32_t tiles = (n + kTileRows - 1) / kTileRows;
    static const uint32_t cap = resident_blocks((const void *)k_mlp_forward, 256);
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((tiles + 4 * kFwdTiles - 1) / (4 * kFwdTiles), cap));
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, (hipStream_t)stream, M);
    return hipGetLastError() == hipSuccess ? PCRT_OK : PCRT_EDEVICE;
}

pcrt_status pcrt_mlp_backward(const pcrt_mlp *net, uint32_t n, const uint16_t *label, const float *cosv, float log_f,
                              const float *g_out, void *ws, size_t ws_bytes, float *grad_w, float *grad_b,
                              float *grad_emb, void *stream) {
    if (!net || !net->w || !net->b || !net->emb || !label || !cosv || !g_out || !ws || !grad_w || !grad_b || !grad_emb)
        return PCRT_EINVAL;
    if (n == 0) return PCRT_EINVAL;
    if (net->n_labels == 0 || net->n_labels > 64) return PCRT_EUNSUPPORTED;
    MlpLayout L = mlp_layout(net->n_labels);
    if (ws_bytes < L.total) return PCRT_ENOMEM;
    char *w = (char *)ws;
    hipStream_t s = (hipStream_t)stream;
    MlpArgs M;
    memset(&M, 0, sizeof M);
    M.w = net->w;
    M.b = net->b;
    M.emb = net->emb;
    M.n_labels = net->n_labels;
    M.n = n;
    M.label = label;
    M.cosv = cosv;
    M.logf = log_f;
    M.gout = g_out;
    M.part = (float *)(w + L.part);
    M.part_stride = L.stride;
    float *part2 = (float *)(w + L.part2);
    hipLaunchKernelGGL(k_mlp_backward, dim3(kBwdWaves / 4), dim3(256), 0, s, M);
    sum_parts(M.part, kBwdWaves, kWAll, L.stride, part2, grad_w, s);
    sum_parts(M.part + kWAll, kBwdWaves, kBAll, L.stride, part2, grad_b, s);
    sum_parts(M.part + kPartW, kBwdWaves, net->n_labels * kEmb, L.stride, part2, grad_emb, s);
    return hipGetLastError() == hipSuccess ? PCRT_OK : PCRT_EDEVICE;
}

}  // extern "C"
