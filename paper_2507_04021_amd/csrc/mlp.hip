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
// The forward pass runs all four layers per 16-row tile in one kernel with the
// weights in LDS; activations change layout (C -> A) through a per-wave LDS
// tile. The backward pass recomputes the forward per tile, back-propagates to
// the pre-activation gradients (also MFMA), and a GEMM over fixed row blocks
// forms the weight gradients, reduced in a fixed order.
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
constexpr int kHPad = kHid + 8;                    // LDS row pitch (bf16) of activation tiles
constexpr int kGradRows = 1024;                    // rows per weight-gradient block

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
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

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
    uint16_t *x0, *h1, *h2, *h3;       // saved bf16 activations [n][32], [n][64] x3
    uint16_t *dz1, *dz2, *dz3, *dz4;   // bf16 pre-activation gradients [n][64] x3, [n][16]
    float *dx0;                        // [n][16] input (embedding) gradients
    float *part;                       // weight-gradient partials
    uint32_t n_blocks;
};

// LDS copy of the weights, forward (row = output) and, for the backward
// chain, transposed (row = input).
struct WLds {
    uint16_t w1[kHid][kIn], w2[kHid][kHid], w3[kHid][kHid], w4[kOut][kHid];
    float b[kBAll];
};
struct WtLds {
    uint16_t w1t[kIn][kHid], w2t[kHid][kHid], w3t[kHid][kHid], w4t[kHid][kOut + 16];  // w4t padded to K = 32
};

__device__ void load_weights(const MlpArgs &M, WLds &W) {
    const uint16_t *src = M.w;
    uint16_t *dst = &W.w1[0][0];
    for (int i = threadIdx.x; i < kWAll; i += blockDim.x) dst[i] = src[i];  // the four arrays are contiguous
    for (int i = threadIdx.x; i < kBAll; i += blockDim.x) W.b[i] = M.b[i];
}

__device__ void load_weights_t(const WLds &W, WtLds &T) {
    for (int i = threadIdx.x; i < kIn * kHid; i += blockDim.x) T.w1t[i % kIn][i / kIn] = W.w1[i / kIn][i % kIn];
    for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x) {
        T.w2t[i % kHid][i / kHid] = W.w2[i / kHid][i % kHid];
        T.w3t[i % kHid][i / kHid] = W.w3[i / kHid][i % kHid];
    }
    for (int i = threadIdx.x; i < kHid * (kOut + 16); i += blockDim.x) {
        int in = i / (kOut + 16), o = i % (kOut + 16);
        T.w4t[in][o] = o < kOut ? W.w4[o][in] : (uint16_t)0;
    }
}

__device__ __forceinline__ bf16x8 frag16(const uint16_t *p) {  // 8 consecutive bf16 from LDS
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = as_b(p[j]);
    return v;
}

// Input features of this lane's A fragment (row = tile row l % 16, columns
// 8 kb .. 8 kb + 7) as bf16 bits.
__device__ __forceinline__ void input_bits(const MlpArgs &M, uint32_t row, int kb, uint16_t *xb) {
    uint16_t lab = row < M.n ? M.label[row] : (uint16_t)0xffff;
    const bool live = lab != 0xffff && lab < M.n_labels;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        int k = 8 * kb + j;
        float x = 0.f;
        if (live) {
            if (k < kEmb) x = M.emb[(size_t)lab * kEmb + k];
            else if (k == kEmb) x = M.cosv[row];
            else if (k == kEmb + 1) x = M.logf;
        }
        xb[j] = to_bf(x);
    }
}

__device__ __forceinline__ bf16x8 bits_frag(const uint16_t *xb) {
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = as_b(xb[j]);
    return v;
}

// One hidden layer: acc[n] (C layout, 64 outputs) from an activation tile in
// LDS (row pitch kHPad) or, for layer 1, from the input fragment.
template <int KSTEPS>
__device__ __forceinline__ void layer_mfma(const uint16_t *Hrow /* this lane's A row in LDS */, const bf16x8 *a_in,
                                          const uint16_t (*Wrows)[KSTEPS * 32], int lane, f32x4 *acc) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
        bf16x8 a = a_in ? a_in[ks] : frag16(Hrow + ks * 32 + 8 * (lane >> 4));
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            bf16x8 bv = frag16(&Wrows[nt * 16 + (lane & 15)][ks * 32 + 8 * (lane >> 4)]);
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[nt], 0, 0, 0);
        }
    }
}

// acc (C layout) + bias -> GELU -> bf16 tile in LDS (and optionally the
// pre-activation values kept in LDS for the backward pass).
__device__ __forceinline__ void store_act(const f32x4 *acc, const float *bias, uint16_t (*H)[kHPad], float (*Z)[kHid],
                                          int lane) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int row = 4 * (lane >> 4) + r, col = nt * 16 + (lane & 15);
            float z = acc[nt][r] + bias[col];
            if (Z) Z[row][col] = z;
            H[row][col] = to_bf(gelu(z));
        }
}

// Output layer: z4 (16 wide) for the tile into LDS.
__device__ __forceinline__ void out_layer(const WLds &W, uint16_t (*H)[kHPad], float (*Z4)[kOut], int lane) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        bf16x8 a = frag16(&H[lane & 15][ks * 32 + 8 * (lane >> 4)]);
        bf16x8 bv = frag16(&W.w4[lane & 15][ks * 32 + 8 * (lane >> 4)]);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        int row = 4 * (lane >> 4) + r, col = lane & 15;
        Z4[row][col] = acc[r] + W.b[3 * kHid + col];
    }
}

struct WaveTile {
    uint16_t H[kTileRows][kHPad];
    float Z4[kTileRows][kOut];
};

__global__ __launch_bounds__(256) void k_mlp_forward(MlpArgs M) {
    __shared__ WLds W;
    __shared__ WaveTile wt[4];
    load_weights(M, W);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveTile &T = wt[wave];
    const uint32_t n_tiles = (M.n + kTileRows - 1) / kTileRows;
    for (uint32_t t = blockIdx.x * 4 + wave; t < n_tiles; t += gridDim.x * 4) {
        const uint32_t r0 = t * kTileRows;
        uint16_t xb[8];
        input_bits(M, r0 + (lane & 15), lane >> 4, xb);
        bf16x8 a_in = bits_frag(xb);
        f32x4 acc[4];
        layer_mfma<1>(nullptr, &a_in, W.w1, lane, acc);
        wave_sync();  // previous tile's reads of H are done
        store_act(acc, W.b, T.H, nullptr, lane);
        wave_sync();
        layer_mfma<2>(&T.H[lane & 15][0], nullptr, W.w2, lane, acc);
        wave_sync();
        store_act(acc, W.b + kHid, T.H, nullptr, lane);
        wave_sync();
        layer_mfma<2>(&T.H[lane & 15][0], nullptr, W.w3, lane, acc);
        wave_sync();
        store_act(acc, W.b + 2 * kHid, T.H, nullptr, lane);
        wave_sync();
        out_layer(W, T.H, T.Z4, lane);
        wave_sync();
        if (lane < kTileRows) {
            const uint32_t row = r0 + lane;
            if (row < M.n) {
                uint16_t lab = M.label[row];
                float4 o0 = make_float4(0.f, 0.f, 0.f, 0.f), o1 = o0;
                if (lab != 0xffff && lab < M.n_labels) {
                    const float *z = T.Z4[lane];
                    float a, b, d;
                    radial(z[0], z[1], o0.x, o0.y, a, b, d);
                    radial(z[2], z[3], o0.z, o0.w, a, b, d);
                    o1.x = 1.f / (1.f + expf(-z[4]));
                }
                float4 *o = (float4 *)(M.out + 8 * (size_t)row);
                o[0] = o0;
                o[1] = o1;
            }
        }
    }
}

// Backward chain per 16-row tile: forward recompute (saving inputs and
// activations for the weight GEMM), output-activation Jacobian, then
// dz_l = (dz_{l+1} W_{l+1}) * GELU'(z_l), all bf16-operand MFMAs.
struct BwdTile {
    uint16_t H[kTileRows][kHPad];      // activation / gradient tile (A operand)
    float Z[3][kTileRows][kHid];       // pre-activations of the hidden layers
    float Z4[kTileRows][kOut];
};

__device__ __forceinline__ void save_tile(uint16_t *dst, uint32_t r0, uint32_t n, int width, uint16_t (*H)[kHPad],
                                          int lane) {
    for (int i = lane; i < kTileRows * width; i += 64) {
        int row = i / width, col = i % width;
        if (r0 + row < n) dst[(size_t)(r0 + row) * width + col] = H[row][col];
    }
}

// dH = dZ (tile in LDS, K = KSTEPS*32) x W^T-rows (B from the transposed copy),
// N = 64 outputs in 4 tiles.
template <int KSTEPS, int LDW>
__device__ __forceinline__ void back_mfma(uint16_t (*G)[kHPad], const uint16_t (*Wt)[LDW], int lane, f32x4 *acc) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
        bf16x8 a = frag16(&G[lane & 15][ks * 32 + 8 * (lane >> 4)]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            bf16x8 bv = frag16(&Wt[nt * 16 + (lane & 15)][ks * 32 + 8 * (lane >> 4)]);
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[nt], 0, 0, 0);
        }
    }
}

__global__ __launch_bounds__(256) void k_mlp_backward_chain(MlpArgs M) {
    __shared__ WLds W;
    __shared__ WtLds WT;
    __shared__ BwdTile bt[4];
    load_weights(M, W);
    __syncthreads();
    load_weights_t(W, WT);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    BwdTile &T = bt[wave];
    const uint32_t n_tiles = (M.n + kTileRows - 1) / kTileRows;
    for (uint32_t t = blockIdx.x * 4 + wave; t < n_tiles; t += gridDim.x * 4) {
        const uint32_t r0 = t * kTileRows;
        uint16_t xb[8];
        input_bits(M, r0 + (lane & 15), lane >> 4, xb);
        bf16x8 a_in = bits_frag(xb);
        // save x0 (bf16) for the first layer's weight gradient
        {
            const uint32_t row = r0 + (lane & 15);
            if (row < M.n) {
                for (int j = 0; j < 8; ++j) M.x0[(size_t)row * kIn + 8 * (lane >> 4) + j] = xb[j];
            }
        }
        f32x4 acc[4];
        layer_mfma<1>(nullptr, &a_in, W.w1, lane, acc);
        wave_sync();  // previous tile's reads of H are done
        store_act(acc, W.b, T.H, T.Z[0], lane);
        wave_sync();
        save_tile(M.h1, r0, M.n, kHid, T.H, lane);
        layer_mfma<2>(&T.H[lane & 15][0], nullptr, W.w2, lane, acc);
        wave_sync();
        store_act(acc, W.b + kHid, T.H, T.Z[1], lane);
        wave_sync();
        save_tile(M.h2, r0, M.n, kHid, T.H, lane);
        layer_mfma<2>(&T.H[lane & 15][0], nullptr, W.w3, lane, acc);
        wave_sync();
        store_act(acc, W.b + 2 * kHid, T.H, T.Z[2], lane);
        wave_sync();
        save_tile(M.h3, r0, M.n, kHid, T.H, lane);
        out_layer(W, T.H, T.Z4, lane);
        wave_sync();
        // output-activation Jacobian: dz4 (16 wide, 5 used), bf16, into the H tile
        if (lane < kTileRows) {
            const uint32_t row = r0 + lane;
            float dz[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            if (row < M.n) {
                uint16_t lab = M.label[row];
                if (lab != 0xffff && lab < M.n_labels) {
                    const float *z = T.Z4[lane];
                    const float *g = M.gout + 8 * (size_t)row;
                    float re, im, a, b, d;
                    radial(z[0], z[1], re, im, a, b, d);
                    dz[0] = g[0] * a + g[1] * b;
                    dz[1] = g[0] * b + g[1] * d;
                    radial(z[2], z[3], re, im, a, b, d);
                    dz[2] = g[2] * a + g[3] * b;
                    dz[3] = g[2] * b + g[3] * d;
                    float S = 1.f / (1.f + expf(-z[4]));
                    dz[4] = g[4] * S * (1.f - S);
                }
            }
            for (int c = 0; c < 32; ++c) T.H[lane][c] = c < 5 ? to_bf(dz[c]) : (uint16_t)0;
            if (row < M.n)
                for (int c = 0; c < kOut; ++c) M.dz4[(size_t)row * kOut + c] = c < 5 ? to_bf(dz[c]) : (uint16_t)0;
        }
        wave_sync();
        // dh3 = dz4 W4 (K = 16 padded to 32); dz3 = dh3 * GELU'(z3)
        back_mfma<1, kOut + 16>(T.H, WT.w4t, lane, acc);
        wave_sync();
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = 4 * (lane >> 4) + r, col = nt * 16 + (lane & 15);
                T.H[row][col] = to_bf(acc[nt][r] * gelu_grad(T.Z[2][row][col]));
            }
        wave_sync();
        save_tile(M.dz3, r0, M.n, kHid, T.H, lane);
        back_mfma<2, kHid>(T.H, WT.w3t, lane, acc);
        wave_sync();
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = 4 * (lane >> 4) + r, col = nt * 16 + (lane & 15);
                T.H[row][col] = to_bf(acc[nt][r] * gelu_grad(T.Z[1][row][col]));
            }
        wave_sync();
        save_tile(M.dz2, r0, M.n, kHid, T.H, lane);
        back_mfma<2, kHid>(T.H, WT.w2t, lane, acc);
        wave_sync();
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = 4 * (lane >> 4) + r, col = nt * 16 + (lane & 15);
                T.H[row][col] = to_bf(acc[nt][r] * gelu_grad(T.Z[0][row][col]));
            }
        wave_sync();
        save_tile(M.dz1, r0, M.n, kHid, T.H, lane);
        // dx0 = dz1 W1: only the embedding columns (N tile 0)
        {
            f32x4 a0 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                bf16x8 a = frag16(&T.H[lane & 15][ks * 32 + 8 * (lane >> 4)]);
                bf16x8 bv = frag16(&WT.w1t[lane & 15][ks * 32 + 8 * (lane >> 4)]);
                a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, a0, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                uint32_t row = r0 + 4 * (lane >> 4) + r;
                if (row < M.n) M.dx0[(size_t)row * kEmb + (lane & 15)] = a0[r];
            }
        }
    }
}

// Weight gradient of one layer over a fixed block of rows:
// dW[o][i] = sum_rows dZ[row][o] H[row][i] (A = dZ^T, B = H, K = 32 rows per
// MFMA), and the bias gradient sum_rows dZ[row][o]. Partials per block.
template <int OUT, int IN>
__global__ __launch_bounds__(256) void k_mlp_wgrad(const uint16_t *dz, const uint16_t *h, uint32_t n, float *part) {
    __shared__ uint16_t sdz[32][OUT + 2];
    __shared__ uint16_t sh[32][IN + 2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int TO = OUT / 16, TI = IN / 16, NT = TO * TI, PER = (NT + 3) / 4;
    f32x4 acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    const uint32_t b0 = blockIdx.x * kGradRows, b1 = min(b0 + kGradRows, n);
    for (uint32_t r0 = b0; r0 < b1; r0 += 32) {
        __syncthreads();
        for (int i = threadIdx.x; i < 32 * OUT; i += 256) {
            int rr = i / OUT, c = i % OUT;
            sdz[rr][c] = r0 + rr < b1 ? dz[(size_t)(r0 + rr) * OUT + c] : (uint16_t)0;
        }
        for (int i = threadIdx.x; i < 32 * IN; i += 256) {
            int rr = i / IN, c = i % IN;
            sh[rr][c] = r0 + rr < b1 ? h[(size_t)(r0 + rr) * IN + c] : (uint16_t)0;
        }
        __syncthreads();
        if (threadIdx.x < OUT)
            for (int rr = 0; rr < 32; ++rr) bsum += bf(sdz[rr][threadIdx.x]);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int tile = wave * PER + q;
            if (tile >= NT) continue;
            const int o0 = (tile / TI) * 16, i0 = (tile % TI) * 16;
            bf16x8 a, bv;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                a[j] = as_b(sdz[8 * (lane >> 4) + j][o0 + (lane & 15)]);
                bv[j] = as_b(sh[8 * (lane >> 4) + j][i0 + (lane & 15)]);
            }
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[q], 0, 0, 0);
        }
    }
    float *P = part + (size_t)blockIdx.x * (OUT * IN + OUT);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int tile = wave * PER + q;
        if (tile >= NT) continue;
        const int o0 = (tile / TI) * 16, i0 = (tile % TI) * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) P[(o0 + 4 * (lane >> 4) + r) * IN + i0 + (lane & 15)] = acc[q][r];
    }
    if (threadIdx.x < OUT) P[OUT * IN + threadIdx.x] = bsum;
}

// Embedding gradient partial of one block of rows. Thread (g, d) -- row group
// g = 0..15, embedding dimension d -- adds dx0[row][d] of rows b0 + g,
// b0 + g + 16, ... in order into its group's LDS table acc[g][label][d]; the
// 16 group tables are then added in group order. Fixed order, no atomics.
constexpr int kEmbGroups = 16;
constexpr int kMaxLabels = 64;
__global__ __launch_bounds__(256) void k_mlp_embgrad(const uint16_t *label, const float *dx0, uint32_t n,
                                                     uint32_t n_labels, float *part) {
    __shared__ float acc[kEmbGroups][kMaxLabels * kEmb];
    for (uint32_t e = threadIdx.x; e < kEmbGroups * kMaxLabels * kEmb; e += blockDim.x) (&acc[0][0])[e] = 0.f;
    __syncthreads();
    const uint32_t g = threadIdx.x / kEmb, d = threadIdx.x % kEmb;
    const uint32_t b0 = blockIdx.x * kGradRows, b1 = min(b0 + kGradRows, n);
    for (uint32_t r = b0 + g; r < b1; r += kEmbGroups) {
        const uint32_t lab = label[r];
        if (lab < n_labels) acc[g][lab * kEmb + d] += dx0[(size_t)r * kEmb + d];
    }
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < n_labels * kEmb; e += blockDim.x) {
        float s = 0.f;
        for (int k = 0; k < kEmbGroups; ++k) s += acc[k][e];
        part[(size_t)blockIdx.x * n_labels * kEmb + e] = s;
    }
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
    size_t x0, h1, h2, h3, dz1, dz2, dz3, dz4, dx0, part, part2, total;
    uint32_t n_blocks;
};
MlpLayout mlp_layout(uint32_t n, uint32_t n_labels) {
    Bump b;
    MlpLayout L;
    L.n_blocks = std::max<uint32_t>((n + kGradRows - 1) / kGradRows, 1);
    L.x0 = b.take(2ull * n * kIn);
    L.h1 = b.take(2ull * n * kHid);
    L.h2 = b.take(2ull * n * kHid);
    L.h3 = b.take(2ull * n * kHid);
    L.dz1 = b.take(2ull * n * kHid);
    L.dz2 = b.take(2ull * n * kHid);
    L.dz3 = b.take(2ull * n * kHid);
    L.dz4 = b.take(2ull * n * kOut);
    L.dx0 = b.take(4ull * n * kEmb);
    size_t per = std::max<size_t>(kHid * kHid + kHid, (size_t)n_labels * kEmb);
    L.part = b.take(4ull * L.n_blocks * per);
    L.part2 = b.take(4ull * kSumSplits * per);
    L.total = b.off;
    return L;
}
}  // namespace

extern "C" {

pcrt_status pcrt_mlp_workspace_size(uint32_t n, uint32_t n_labels, size_t *bytes) {
    if (!bytes) return PCRT_EINVAL;
    *bytes = mlp_layout(n, n_labels).total;
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
    const uint32_t grid = std::min<uint32_t>((tiles + 3) / 4, 2048);
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
    MlpLayout L = mlp_layout(n, net->n_labels);
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
    M.x0 = (uint16_t *)(w + L.x0);
    M.h1 = (uint16_t *)(w + L.h1);
    M.h2 = (uint16_t *)(w + L.h2);
    M.h3 = (uint16_t *)(w + L.h3);
    M.dz1 = (uint16_t *)(w + L.dz1);
    M.dz2 = (uint16_t *)(w + L.dz2);
    M.dz3 = (uint16_t *)(w + L.dz3);
    M.dz4 = (uint16_t *)(w + L.dz4);
    M.dx0 = (float *)(w + L.dx0);
    float *part = (float *)(w + L.part), *part2 = (float *)(w + L.part2);
    const uint32_t tiles = (n + kTileRows - 1) / kTileRows;
    hipLaunchKernelGGL(k_mlp_backward_chain, dim3(std::min<uint32_t>((tiles + 3) / 4, 2048)), dim3(256), 0, s, M);
    const uint32_t nb = L.n_blocks;
    // layer 4 .. 1: (dz, input activation) -> grad_w slice, grad_b slice
    struct Job {
        int out, in;
        const uint16_t *dz, *h;
        size_t w_off, b_off;
    } jobs[4] = {{kOut, kHid, M.dz4, M.h3, (size_t)(kW1 + kW2 + kW3), 3 * kHid},
                 {kHid, kHid, M.dz3, M.h2, (size_t)(kW1 + kW2), 2 * kHid},
                 {kHid, kHid, M.dz2, M.h1, (size_t)kW1, kHid},
                 {kHid, kIn, M.dz1, M.x0, 0, 0}};
    for (const Job &j : jobs) {
        if (j.out == kOut)
            hipLaunchKernelGGL((k_mlp_wgrad<kOut, kHid>), dim3(nb), dim3(256), 0, s, j.dz, j.h, n, part);
        else if (j.in == kHid)
            hipLaunchKernelGGL((k_mlp_wgrad<kHid, kHid>), dim3(nb), dim3(256), 0, s, j.dz, j.h, n, part);
        else
            hipLaunchKernelGGL((k_mlp_wgrad<kHid, kIn>), dim3(nb), dim3(256), 0, s, j.dz, j.h, n, part);
        const uint32_t wsz = j.out * j.in, stride = wsz + j.out;
        sum_parts(part, nb, wsz, stride, part2, grad_w + j.w_off, s);
        sum_parts(part + wsz, nb, (uint32_t)j.out, stride, part2, grad_b + j.b_off, s);
    }
    hipLaunchKernelGGL(k_mlp_embgrad, dim3(nb), dim3(256), 0, s, label, M.dx0, n, net->n_labels, part);
    const uint32_t ew = net->n_labels * kEmb;
    sum_parts(part, nb, ew, ew, part2, grad_emb, s);
    return hipGetLastError() == hipSuccess ? PCRT_OK : PCRT_EDEVICE;
}

}  // extern "C"
