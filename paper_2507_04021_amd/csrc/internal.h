// Host-side declarations shared by the translation units of libpcrt.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstddef>

#include "common.h"
#include "pcrt.h"

namespace pcrt {

// Persistent launches: grids of as many blocks as the device holds at once
// (blocks per compute unit from the occupancy API x compute units); their
// waves pull work from atomic counters until it runs out.
uint32_t resident_blocks(const void *kernel, int block_threads);
constexpr uint32_t kMaxPairs = 262144;  // (transmitter, receiver) pairs in one solve
// Work counters of the persistent launches: [0] trace units, [1] refine chunks,
// [8, 16) diffuse chunks, one counter per XCD range.
constexpr uint32_t kWorkWords = 32;
constexpr uint32_t kXcds = 8;  // MI355X: 8 accelerator complex dies, workgroups dealt round robin
constexpr uint32_t kDefaultWidth = 4;    // 4-wide nodes: fastest on the 1M-point office (binary and 8-wide slower)
constexpr uint32_t kDefaultBuilder = 2;  // clustering: 6 % fewer node visits than the radix tree on the office
#ifndef PCRT_SAH_COLLAPSE
#define PCRT_SAH_COLLAPSE 1
#endif
constexpr bool kSahCollapse = PCRT_SAH_COLLAPSE != 0;  // wide nodes by surface-area cost (else greedy by area)

struct Bump {  // 256-byte aligned offsets inside one workspace
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};

constexpr uint32_t kBuildLbvh = 1;  // Karras radix tree over Morton codes
constexpr uint32_t kBuildPloc = 2;  // locally-ordered clustering (surface-area merges)

struct SceneLayout {
    size_t pos_id, nrm_id, disk, node, stat, bounds, blk_bounds;
    size_t code0, code1, idx0, idx1, hist, scan_blk, child, range, parent_int, parent_leaf, dbox, ibox, flags;
    uint32_t width = 2;                             // node width of the traversed hierarchy
    uint32_t n_internal = 1;                        // binary internal nodes (buffer capacity)
    uint32_t builder = kBuildLbvh;
    size_t cbox[2] = {0, 0}, cid[2] = {0, 0}, csz[2] = {0, 0};  // clustering build (builder == kBuildPloc)
    size_t nn = 0, mflag = 0, kflag = 0, pblk = 0, nsize = 0, noff = 0, leaf_pos = 0, perm2 = 0, pleaf2 = 0;
    size_t wnode = 0, front0 = 0, front1 = 0, wcnt = 0, wblk = 0;  // wide collapse (width > 2)
    size_t qnode = 0, qref = 0;                                     // its compact any-hit copy
    size_t sah_pending = 0, sah_cost = 0, sah_choice = 0;           // its surface-area choices
    size_t dps_pt = 0, dps_off = 0, dps_of = 0, dps_flag = 0, dps_blk = 0, dps_stat = 0, dps_recv = 0;  // point sets
    size_t total;
};

SceneLayout scene_layout(uint32_t n, uint32_t width, uint32_t builder, bool dps);
// Single-bounce edge diffraction: per-pair amplitudes, then per-receiver sums.
uint32_t diffraction_blocks(uint32_t n_edges, uint32_t n_rx);
void launch_diffraction(const DevScene &S, const pcrt_edge *edges, uint32_t n_edges, const float *mats,
                        uint32_t n_labels, const float tx[3], const float *rx, uint32_t n_rx, double freq,
                        float eps_self, float4 *amp, double *out, hipStream_t s);
// Visibility of the point sets' reception points from receivers (one uint8 per pair).
uint32_t visibility_grid(uint32_t width);
void launch_visibility(const DevScene &S, const float *rx, uint32_t n_rx, const float4 *recv, uint32_t n_sets,
                       float eps_self, uint8_t *out, hipStream_t s);
void launch_recv_copy(const float4 *recv, uint32_t n, float *out, hipStream_t s);
// Point sets: voxel keys, sort, set boundaries (after build_scene, reusing its sort buffers).
hipError_t build_point_sets(const SceneLayout &L, char *ws, uint32_t n, float rho, hipStream_t s);
hipError_t build_wide(const SceneLayout &L, char *ws, hipStream_t s, int broot, uint32_t *levels, uint32_t *nodes);
hipError_t build_scene(const float *pos, const float *nrm, const uint16_t *mat, const uint32_t *surf, uint32_t n,
                       float r, uint32_t leaf, char *ws, const SceneLayout &L, hipStream_t s, uint32_t *wide_levels,
                       uint32_t *wide_nodes, int *root);
void fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
uint32_t scan_blk_words(uint32_t n);
uint32_t radix_hist_words(uint32_t n);
void exclusive_scan(uint32_t *a, uint32_t n, uint32_t *blk, hipStream_t s);
bool radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, uint32_t n, int bit_lo, int bit_hi,
                    uint32_t *hist, uint32_t *blk, hipStream_t s);
void fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s);

// Per-(ray, interaction) records, dense [T * K].
struct RecBufs {
    int *id;          // hit disk id, -1 = none
    float4 *xl;       // hit point, unfolded length from TX
    float *cs;        // incidence cosine, sign = orientation of the hit normal (n_k = sign * n)
    float4 *coef;     // diffuse coefficient (TE re, im, TM re, im), incl. lambda/4pi and the chain before
    uint32_t *slot;   // key-table slot of the prefix key
    float4 *nk;       // point-set average only: normal of the interaction, facing the incoming ray
    uint32_t *dslot;  // reception-point launch with diffuse: key-table slot of the voxel diffuse key
};

struct HashBufs {
    unsigned long long *key;  // 0 = empty
    uint32_t *rep;            // smallest ray id with this key
    uint32_t cap;             // slots per item (power of two)
};

struct SpecBufs {  // specular results per (key, RX) pair, RECORD mode only
    uint8_t *valid;
    float *len;
    float4 *amp;
    int *hit;     // [pairs * K]
    float *cs;    // [pairs * K]
};

struct SolveDims {
    uint32_t T;        // flattened ray slots (items padded to kRayChunk)
    uint32_t K;
    uint32_t n_rx;
    uint32_t n_items;
    uint32_t max_keys;
    uint32_t max_key_chunks;
    uint32_t n_ray_chunks;
    uint32_t rec_keys;     // keys whose (key, RX) results are kept in RECORD mode
    uint32_t n_slots;      // tape interaction slots: T*K traced + rec_keys*n_rx*K specular
    uint32_t n_slot_chunks;
    uint32_t spill_lanes;  // lanes of the widest traversal launch of this solve
    uint32_t spill_depth;  // traversal stack entries beyond the LDS part (stack bound - kStackLds)
    uint32_t width;        // node width of the scene's hierarchy (2, 4, 8)
};

constexpr uint32_t kSlotChunk = 512;    // slots per label-gradient reduction chunk (one 64-lane block each)
// Receivers per specular refinement unit (with one key chunk). Measured on the
// 1M-point office: 16 -> 8.70 ms, 8 -> 8.55 ms, 32 -> 10.05 ms.
constexpr uint32_t kRefineRxSlice = 8;
// Result slots per refinement block: two open units of kKeyChunk keys x kRefineRxSlice receivers.
constexpr uint32_t kRefineResPerBlock = 2 * kKeyChunk * kRefineRxSlice;
constexpr uint32_t kRefineQueue = 128;  // refinement ring of queued candidates (at most 127 are live)
constexpr uint32_t kMaxGradLabels = 64;   // label-gradient LDS: 64 lanes x 64 labels x 3 doubles

struct SolveLayout {
    size_t items, counters, work, rec_id, rec_xl, rec_cs, rec_coef, rec_slot, hkey, hrep, scan, scan_blk, keylist,
        key_off, chunk_off, spec_part, diff_part, los_part, sp_valid, sp_len, sp_amp, sp_hit, sp_cs, dvis, spill,
        slot_label, slot_cos, slot_coef, slot_adj, grad_part, dkey0, dkey1, dval0, dval1, dhist, dblk, spec_res, dpack, rec_nk, spec_ovr,
        rec_dslot, dhkey, dhrep, dkeylist, dkey_off, dchunk_off, dcnt;
    size_t total;
};

SolveLayout solve_layout(const SolveDims &D, uint32_t flags);
uint32_t trace_grid(const SolveDims &D, uint32_t wave_rays);
uint32_t refine_grid(const SolveDims &D);
uint32_t diffuse_grid(const SolveDims &D);

struct SortBufs {  // spatial ordering of the diffuse records
    uint64_t *key0, *key1;
    uint32_t *val0, *val1, *hist, *blk;
    const uint32_t *order;  // sorted record indices (set by the launcher)
    // The records in that order, two float4 each: (hit point, unfolded length),
    // (normal on the lit side, disk id as int bits; -1 = no interaction).
    float4 *pack;
};

struct LaunchArgs {
    DevScene S;
    const Item *items;
    const uint32_t *subset;
    const float *rx;
    const float *mats;  // [n_labels][3]
    uint32_t n_labels;
    uint32_t n_surf1;   // surface labels + 1 (key radix)
    uint32_t flags;
    Thr thr;
    FieldConst fc;
    SolveDims D;
    RecBufs rb;
    HashBufs hb;
    SpecBufs sb;
    uint32_t wave_rays; // rays a wavefront takes per work fetch (multiple of 64)
    f3 pol_tx, pol_rx;  // polarised field: transmit and receive polarisation vectors
    float dps_area;     // point sets: the area rho^2 a voxel diffuse path stands for
    const uint8_t *dps_vis;  // launch at the reception points: [n_rx][n_sets] receiver sees reception point
    HashBufs dhb;            // ... and its voxel diffuse keys (labels before the last interaction, last set)
    uint32_t *dkeylist, *dkey_off, *dchunk_off;
    uint64_t *dcnt;
    uint32_t *work;     // [8] atomic work counters
    uint64_t *counters; // [16]
    uint32_t *scan;
    uint32_t *scan_blk;
    uint32_t *keylist;
    uint32_t *key_off;   // [n_items + 1]
    uint32_t *chunk_off; // [n_items + 1]
    double *spec_part;
    float4 *spec_res;      // refinement: per block, path amplitudes of its current unit's pairs
    float4 *spec_ovr;      // refinement with point-set averaging: per block and ring position, replaced planes
    double *diff_part;
    double *los_part;
    uint8_t *dvis;
    uint16_t *slot_label;  // RECORD tape: material label per interaction slot (0xffff: empty)
    float *slot_cos;
    float *slot_coef;      // [n_slots][8]: Gamma_TE re, im, Gamma_TM re, im, S
    float *slot_adj;       // [n_slots][8]: dL/d of the same values
    double *grad_part;     // [n_slot_chunks][kMaxGradLabels][3]
    SortBufs dsort;
};

// Voxel diffuse keys of the reception-point launch: block c of n_blocks (the
// ray chunks) takes an equal share of the n_keys keys, in key order, and each
// of its kDpsWaves wavefronts an equal share of that (receivers across the
// lanes); the wavefronts' sums are added in wavefront order, the blocks' in
// block order. Every wavefront has work and enough of them run to hide the
// chain of dependent loads per key. (With the ray chunks' 1 280 key positions
// per single-wavefront block, the office's 53 k keys sat in 42 blocks.)
constexpr uint32_t kDpsWaves = 8;
__device__ __forceinline__ void dps_key_range(uint32_t n_keys, uint32_t c, uint32_t n_blocks, uint32_t w,
                                              uint32_t &q0, uint32_t &q1) {
    const uint32_t per = (n_keys + n_blocks - 1) / n_blocks;
    const uint32_t b0 = min(n_keys, c * per), b1 = min(n_keys, b0 + per);
    const uint32_t sub = (b1 - b0 + kDpsWaves - 1) / kDpsWaves;
    q0 = min(b1, b0 + w * sub);
    q1 = min(b1, q0 + sub);
}

// Wavefront w of a voxel diffuse block hands its lane's five sums over in
// LDS; wavefront 0 adds them in wavefront order into out (if out is set).
__device__ __forceinline__ void dps_block_sum(double (*red)[kWave][5], uint32_t w, uint32_t lane, const double *acc,
                                              double *out) {
    for (int a = 0; a < 5; ++a) red[w][lane][a] = acc[a];
    __syncthreads();
    if (w == 0 && out) {
        double t[5] = {0, 0, 0, 0, 0};
        for (uint32_t v = 0; v < kDpsWaves; ++v)
            for (int a = 0; a < 5; ++a) t[a] += red[v][lane][a];
        for (int a = 0; a < 5; ++a) out[a] = t[a];
    }
}

// Normal of interaction record ri, turned to face the ray that arrived there:
// the point-set average's normal when it ran, else the hit disk's normal.
__device__ __forceinline__ f3 record_normal(const LaunchArgs &A, uint32_t ri) {
    if (A.rb.nk) return xyz(A.rb.nk[ri]);
    const f3 n = xyz(A.S.nrm[A.rb.id[ri]]);
    return A.rb.cs[ri] < 0.f ? (-1.f) * n : n;
}

void launch_trace(const LaunchArgs &A, hipStream_t s);
void launch_keys(const LaunchArgs &A, hipStream_t s);
void launch_refine(const LaunchArgs &A, hipStream_t s);
void launch_refine_pol(const LaunchArgs &A, dim3 grid, hipStream_t s);  // PCRT_POLARIZED instances
// Morton order of the interaction records: sorts them, fills A.dsort.pack and
// returns the sorted record indices
const uint32_t *launch_diffuse_order(const LaunchArgs &A, hipStream_t s);
void launch_diffuse(const LaunchArgs &A, hipStream_t s);  // needs A.dsort.order
// Reception-point launch: compact the voxel diffuse keys, then their fields (area rho^2 each).
void launch_dps_diffuse(const LaunchArgs &A, float area, hipStream_t s);
uint32_t dps_key_cap(const SolveDims &D);
void launch_los_and_combine(const LaunchArgs &A, double *gain, double *h_te, double *h_tm, double *parts,
                            hipStream_t s);
void launch_combine(const LaunchArgs &A, double *gain, double *h_te, double *h_tm, double *parts, hipStream_t s);
void launch_tape_slots(const LaunchArgs &A, hipStream_t s);
void launch_tape_fresnel(const LaunchArgs &A, const float *mats, uint32_t n_labels, hipStream_t s);
void launch_tape_forward(const LaunchArgs &A, double *gain, double *h_te, double *h_tm, double *parts,
                         hipStream_t s);
void launch_tape_backward(const LaunchArgs &A, const double *dldg, hipStream_t s);
void launch_tape_cfr(const LaunchArgs &A, double bw, uint32_t N, double *cfr, hipStream_t s);
void launch_tape_cfr_backward(const LaunchArgs &A, double bw, uint32_t N, const double *dldh, hipStream_t s);
void launch_material_grad(const LaunchArgs &A, const float *mats, uint32_t n_labels, double *out, hipStream_t s);
void launch_raygen(uint32_t n_budget, const uint32_t *ids, uint32_t n, float *out, hipStream_t s);
void launch_paths_copy(const LaunchArgs &A, uint32_t cap, uint32_t *key_ray, uint8_t *key_len, int32_t *key_seq,
                       uint8_t *valid, float *length, float *amp, int32_t *hit, hipStream_t s);

}  // namespace pcrt
