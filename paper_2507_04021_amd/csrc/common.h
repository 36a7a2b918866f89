// Device-side types and routines shared by the HIP kernels of libpcrt.
//
// Geometry and field arithmetic are FP32; only per-receiver reductions are FP64.
// Written for gfx950 (CDNA4): 64-lane wavefronts, LDS traversal stacks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcrt {

constexpr int kMaxK = 8;          // max interactions per path
constexpr int kWave = 64;         // wavefront width
constexpr int kStackLds = 23;     // traversal stack entries kept in LDS per lane (5.75 KiB per wavefront)
constexpr int kStackMax = 96;     // max stack entries (LDS + global spill)
constexpr int kRayChunk = 256;    // rays per diffuse reduction chunk (item ray ranges are padded to this);
                                   // office connections: 128 -> 30.3 ms, 256 -> 29.8, 512 -> 30.7
constexpr int kKeyChunk = 64;     // specular keys per reduction chunk
constexpr float kParallelEps = 1e-6f;  // |d.n| below this: ray parallel to a disk

// Instrumented builds (-DPCRT_COUNT_VISITS=1) count node visits and disk tests
// per kernel for the algorithmic-byte model; the product build compiles the
// counting away.
#ifndef PCRT_COUNT_VISITS
#define PCRT_COUNT_VISITS 0
#endif
constexpr bool kCountVisits = PCRT_COUNT_VISITS != 0;
constexpr int kNodeBytes = 64;   // one binary node: two child boxes + refs
constexpr int kDiskBytes = 32;   // one leaf-ordered disk: centre, id, normal

constexpr double kC0 = 299792458.0;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- vectors
struct f3 {
    float x, y, z;
};
__device__ __forceinline__ f3 mk(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(float s, f3 a) { return {s * a.x, s * a.y, s * a.z}; }
// s * a + b with one rounding per component (fused multiply-add)
__device__ __forceinline__ f3 fma3(float s, f3 a, f3 b) { return {fmaf(s, a.x, b.x), fmaf(s, a.y, b.y), fmaf(s, a.z, b.z)}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float len(f3 a) { return sqrtf(dot(a, a)); }
__device__ __forceinline__ f3 normalize(f3 a) { return (1.0f / len(a)) * a; }
__device__ __forceinline__ f3 xyz(float4 v) { return {v.x, v.y, v.z}; }

// ------------------------------------------------------------- scene
// Child reference of a node: >= 0 internal node index; < 0 leaf,
// v = -1 - ref, first disk = v >> 3, count = (v & 7) + 1.
__host__ __device__ __forceinline__ int leaf_ref(int first, int count) { return -1 - ((first << 3) | (count - 1)); }

// float4 at a 32-bit byte offset from a wavefront-uniform array base. The
// address is then one scalar base plus one per-lane 32-bit offset, instead of
// a 64-bit add per lane; scenes are capped (2^26 points) so that the node and
// disk arrays stay below 4 GiB.
__device__ __forceinline__ float4 ld4(const float4 *base, uint32_t off) {
    return *(const float4 *)((const char *)base + off);
}

struct DevScene {
    const float4 *node;  // binary nodes (4 float4: child boxes + refs) or wide nodes (2W float4)
    const float4 *qnode; // wide nodes only: compact copies for the any-hit walks (16 + 12 W bytes each), 8 octants
    const int *qref;     // wide nodes only: the child references, W per node
    uint32_t qstride;    // bytes between the octant copies of the compact nodes
    const float4 *disk;  // 2 float4 per leaf-ordered disk: (p.xyz, id bits), (n.xyz, point set bits or 0)
    const float4 *pos;   // by id: (p.xyz, surface bits)
    const float4 *nrm;   // by id: (n.xyz, material bits)
    const float *bounds; // scene bounds of the disk centres: lo xyz, hi xyz
    int width;           // node width: 2 (binary nodes, 64 B) or 4 / 8 (wide nodes, 32 W bytes)
    int *spill;          // global spill of traversal stacks, [stack bound - kStackLds][spill_lanes]
    uint32_t spill_lanes;
    int root;
    float r2;
    uint32_t n;
    // Discretised point sets (voxels of the point centres), null without them.
    const float4 *dps_pt;     // 2 float4 per member, grouped by set: (p.xyz, id bits), (n.xyz, 0)
    const uint32_t *dps_off;  // [n_sets + 1] first member of each set
    const uint32_t *dps_of;   // by id: set of the point
    const float4 *dps_recv;   // [n_sets] reception points (set means)
    uint32_t n_sets;
};

// Node layout (64 B): n0 = (lo0.x, lo0.y, lo0.z, hi0.x), n1 = (hi0.y, hi0.z, lo1.x, lo1.y),
// n2 = (lo1.z, hi1.x, hi1.y, hi1.z), n3 = (ref0, ref1, -, -).

struct Thr {
    float eps_tie, eps_self, cos_ta, t_d;
    int kappa;
    float lambda_d;  // depth attenuation of the point-set average
};

struct Item {  // one transmitter of a (batched) solve, 32 B
    float tx[3];
    uint32_t n_rays;   // rays traced for this item
    uint32_t ray_off;  // first flattened ray slot (multiple of kRayChunk)
    uint32_t budget;   // ray budget N (Fibonacci directions, diffuse weight)
    uint32_t pad[2];
};

// ---------------------------------------------------- traversal stack
// Entries 0..kStackLds-1 live in LDS ([depth][lane] so lanes hit distinct
// banks); deeper entries spill to a per-lane global region.
struct Stack {
    int *lds;        // this lane's column base: lds[s * kWave]
    int *gl;         // this lane's spill column base: gl[(s - kStackLds) * lanes]
    uint32_t lanes;
    uint32_t nv = 0, nd = 0;  // node visits, disk tests (instrumented builds only)
    __device__ __forceinline__ void visit() {
        if (kCountVisits) ++nv;
    }
    __device__ __forceinline__ void test(int n) {
        if (kCountVisits) nd += n;
    }
    __device__ __forceinline__ void put(int s, int v) {
        if (s < kStackLds) lds[s * kWave] = v;
        else gl[(size_t)(s - kStackLds) * lanes] = v;
    }
    __device__ __forceinline__ int get(int s) const {
        // The LDS read is always in bounds; the global read only for spilled
        // entries (keeps the common pop an LDS access, not a generic one).
        int v = lds[min(s, kStackLds - 1) * kWave];
        __asm__ volatile("" : "+v"(v));  // opaque use: the LDS read stays a read of its own
        if (s >= kStackLds) v = gl[(size_t)(s - kStackLds) * lanes];
        return v;
    }
};

// Rank of this lane among the lanes set in a ballot mask (lanes below it).
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ f3 safe_inv(f3 d) {
    const float tiny = 1e-30f;
    float x = fabsf(d.x) < tiny ? copysignf(tiny, d.x) : d.x;
    float y = fabsf(d.y) < tiny ? copysignf(tiny, d.y) : d.y;
    float z = fabsf(d.z) < tiny ? copysignf(tiny, d.z) : d.z;
    return {1.0f / x, 1.0f / y, 1.0f / z};
}

// Slab test of one box against [t_lo, t_hi]; returns entry distance in tn.
// oi = o * inv (per ray), so each slab distance is one fused multiply-add
// lo * inv - o * inv. Its extra rounding, at most |o * inv| * 2^-24, stays far
// below the boxes' padding (>= 1e-5 * |inv| per axis), so no box that the
// exact slab test would enter is skipped.
__device__ __forceinline__ bool box_hit(float lx, float ly, float lz, float hx, float hy, float hz, f3 inv, f3 oi,
                                        float t_lo, float t_hi, float &tn) {
    const float ax = fmaf(lx, inv.x, -oi.x), bx = fmaf(hx, inv.x, -oi.x);
    const float ay = fmaf(ly, inv.y, -oi.y), by = fmaf(hy, inv.y, -oi.y);
    const float az = fmaf(lz, inv.z, -oi.z), bz = fmaf(hz, inv.z, -oi.z);
    const float t0 = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), t_lo));
    const float t1 = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), t_hi));
    tn = t0;
    return t0 <= t1;
}

__device__ __forceinline__ f3 times(f3 a, f3 b) { return {a.x * b.x, a.y * b.y, a.z * b.z}; }

// Two-sided ray-disk test (Sec. II-C): plane hit t, squared distance of the
// hit point from the centre. Evaluated without early exits (a ray parallel
// to the plane gives a non-finite t and d2 and fails on |d.n|), so the loads
// of a disk are issued together and every caller rounds identically.
__device__ __forceinline__ bool disk_hit(f3 o, f3 d, f3 p, f3 n, float r2, float &t, float &d2) {
    const float a = dot(d, n);
    t = dot(p - o, n) / a;
    const f3 q = fma3(t, d, o);
    const f3 e = q - p;
    d2 = dot(e, e);
    return (fabsf(a) >= kParallelEps) & (d2 <= r2);
}

// Weighted-average intersection over the point set of the hit disk h
// (Sec. II-C, Eq. 3-4). The members are the disks of h's voxel that the ray
// meets farther than eps_self from o (excl aside); member i weighs
//   exp(-|q_i - p_i|^2 / (2 r^2)) * exp(-lambda_d * (t_i - t_min)),
// t_min being the nearest member intersection (|q_i - q_min| = t_i - t_min:
// both points lie on the ray and d is unit). t becomes the weighted mean
// distance, n the weighted sum of the member normals turned to face the ray,
// normalised. Members are visited in increasing id, which fixes the sums.
__device__ __forceinline__ void dps_average(const DevScene &S, f3 o, f3 d, int excl, float eps_self,
                                            float lambda_d, int h, float &t, f3 &n) {
    const uint32_t g = S.dps_of[h];
    const uint32_t b = S.dps_off[g], e = S.dps_off[g + 1];
    float tmin = INFINITY;
    for (uint32_t j = b; j < e; ++j) {
        const float4 pp = S.dps_pt[2 * (size_t)j], pn = S.dps_pt[2 * (size_t)j + 1];
        float tj, d2;
        const bool hit = disk_hit(o, d, xyz(pp), xyz(pn), S.r2, tj, d2);
        if (hit && __float_as_int(pp.w) != excl && tj > eps_self) tmin = fminf(tmin, tj);
    }
    const float inv2r2 = 0.5f / S.r2;
    float sw = 0.f, st = 0.f;
    f3 sn = mk(0.f, 0.f, 0.f);
    for (uint32_t j = b; j < e; ++j) {
        const float4 pp = S.dps_pt[2 * (size_t)j], pn = S.dps_pt[2 * (size_t)j + 1];
        float tj, d2;
        const bool hit = disk_hit(o, d, xyz(pp), xyz(pn), S.r2, tj, d2);
        if (!(hit && __float_as_int(pp.w) != excl && tj > eps_self)) continue;
        const float w = expf(-d2 * inv2r2) * expf(-lambda_d * (tj - tmin));
        const f3 m = xyz(pn);
        const float side = dot(d, m) > 0.f ? -w : w;
        sw += w;
        st += w * tj;
        sn = sn + side * m;
    }
    t = st / sw;
    n = normalize(sn);
}

// Nearest hit among disks != excl with t in (t_lo, inf), with the tie rule:
// t* = min t; among hits with t <= t* + eps_tie the smallest (d2, id) wins.
// Hits within the current window are kept in a short list that is pruned
// whenever t* shrinks; if the list overflows, a second, exact pass over the
// final window decides. Returns the disk id or -1; t of the winner.
struct Cand {
    float t, d2;
    int id;
};
// Three entries: no bounce of the office overflows them (as with four) and
// the walks hold fewer registers; one entry sends 1 % of its bounces to the
// second pass and slows the refinement by 7 %.
constexpr int kTieList = 3;  // entries of the tie-window candidate list

template <bool kSecond>
__device__ __forceinline__ void visit_disk(const DevScene &S, int i, f3 o, f3 d, int excl, float t_lo, float eps_tie,
                                           float &tmin, Cand *c, bool &spill, float t_win, float &best_d2,
                                           int &best_id, float &best_t) {
    const float4 dp = ld4(S.disk, (uint32_t)i * 32u);
    const float4 dn = ld4(S.disk, (uint32_t)i * 32u + 16u);
    const int id = __float_as_int(dp.w);
    if (id == excl) return;
    float t, d2;
    if (!disk_hit(o, d, xyz(dp), xyz(dn), S.r2, t, d2)) return;
    if (!(t > t_lo)) return;
    if (kSecond) {
        if (t <= t_win && (d2 < best_d2 || (d2 == best_d2 && id < best_id))) {
            best_d2 = d2;
            best_id = id;
            best_t = t;
        }
        return;
    }
    if (t > tmin + eps_tie) return;
    if (t < tmin) {
        tmin = t;
        const float lim = tmin + eps_tie;
#pragma unroll
        for (int k = 0; k < kTieList; ++k)
            if (c[k].id >= 0 && c[k].t > lim) c[k].id = -1;
    }
    bool placed = false;
#pragma unroll
    for (int k = 0; k < kTieList; ++k)
        if (!placed && c[k].id < 0) {
            c[k].t = t;
            c[k].d2 = d2;
            c[k].id = id;
            placed = true;
        }
    if (!placed) spill = true;
}

// Children of a wide node (8W floats: lo x[W], lo y[W], lo z[W], hi x[W],
// hi y[W], hi z[W], refs[W], pad): entry distance per child (INFINITY for a
// child the segment misses) and its reference.
// Same children test without the octant registers (the closest-hit walks are
// register-bound: per-box min / max instead of per-lane row offsets).
template <int W>
__device__ __forceinline__ void wide_hits_minmax(const float4 *node, int ref, f3 inv, f3 oi, float t_lo, float t_hi,
                                                 float (&tn)[W], int (&cr)[W]) {
    const uint32_t nb = (uint32_t)ref * (32u * W);
    float v[7 * W];
#pragma unroll
    for (int k = 0; k < 7 * W / 4; ++k) {
        const float4 q = ld4(node, nb + 16u * k);
        v[4 * k] = q.x;
        v[4 * k + 1] = q.y;
        v[4 * k + 2] = q.z;
        v[4 * k + 3] = q.w;
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
        float t;
        const bool h = box_hit(v[j], v[W + j], v[2 * W + j], v[3 * W + j], v[4 * W + j], v[5 * W + j], inv, oi, t_lo,
                               t_hi, t);
        tn[j] = h ? t : INFINITY;
        cr[j] = __float_as_int(v[6 * W + j]);
    }
}

// Compact wide nodes for the any-hit walks (16 + 12 W bytes: 64 for W = 4).
// A header holds the origin of a grid (xyz) and its per-axis steps 2^e (the
// three e as signed bytes in the fourth word); six rows of W FP16 values
// follow (near x, near y, near z, far x, far y, far z: lo or hi by the copy's
// octant, below), each a grid coordinate (an
// integer 0..2047, exact in FP16) rounded outward with at least one step of
// margin, so every compact child box contains its float child box. The child
// references are a separate array of W ints per node.
//
// Slab distance of a plane at grid coordinate g: g * (2^e inv) + (origin -
// o) * inv. 2^e inv is exact (ldexp); (origin - o) inv is one FMA per axis
// and node (origin * inv - o * inv, o * inv precomputed); each plane is then
// one mixed-precision FMA whose FP16 operand is widened exactly. The
// roundings, a few units of 2^-24 of the coordinates and distances, stay far
// below the float boxes' padding (1e-5 + 2e-6 (|c| + r)), so no box that the
// exact slab test of the float box would enter is skipped.
template <int W>
constexpr uint32_t qnode_bytes() {
    return 16u + 12u * W;
}

// Octant form of the slab test: the sign of each inverse direction
// component fixes which of lo / hi is the near plane on that axis for every
// box. The compact nodes are stored in eight copies, one per octant, with the
// near plane rows first, so a lane reads its octant's copy and needs neither
// a per-box min / max nor a row select (twelve selects per 4-wide node: diffuse
// 20.92 -> 20.47 ms on the office, for 7 x 15 MB more nodes). Rounding is
// monotonic, so each near / far value is exactly the one min / max would pick.
struct Octant {
    uint32_t oct;  // bit a set: the inverse direction component a is negative
};

template <int W>
__device__ __forceinline__ Octant octant(f3 inv) {
    return {(inv.x < 0.f ? 1u : 0u) | (inv.y < 0.f ? 2u : 0u) | (inv.z < 0.f ? 4u : 0u)};
}

// The whole compact node is loaded (four 16-byte loads for W = 4, then one
// for the references): the any-hit walks are bound by the number of vector
// load instructions (the texture address and data units stay busy about 17
// and 21 cycles per wavefront load, whatever its width). On the office's
// diffuse connections: float nodes (six 16-byte row loads chosen by octant +
// references) 27.0 ms; compact rows as six 8-byte loads chosen by octant
// 28.1 ms; whole compact node 21.75 ms, with the same visibility.
template <int W>
__device__ __forceinline__ void wide_hits(const DevScene &S, int ref, const Octant &q, f3 inv, f3 oi, float t_lo,
                                          float t_hi, float (&tn)[W], int (&cr)[W]) {
    constexpr int NQ = (int)qnode_bytes<W>() / 16;  // 16-byte loads per node
    constexpr int RW = W / 2;                       // dwords per row of W FP16 values
    const uint32_t nb = q.oct * S.qstride + (uint32_t)ref * qnode_bytes<W>();
    uint32_t w[4 * NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const uint4 v = *(const uint4 *)((const char *)S.qnode + nb + 16u * k);
        w[4 * k] = v.x;
        w[4 * k + 1] = v.y;
        w[4 * k + 2] = v.z;
        w[4 * k + 3] = v.w;
    }
#pragma unroll
    for (int k = 0; k < W / 4; ++k) {
        const int4 v = *(const int4 *)((const char *)S.qref + (uint32_t)ref * (4u * W) + 16u * k);
        cr[4 * k] = v.x;
        cr[4 * k + 1] = v.y;
        cr[4 * k + 2] = v.z;
        cr[4 * k + 3] = v.w;
    }
    _Float16 nx[W], ny[W], nz[W], fx[W], fy[W], fz[W];  // near rows, then far rows
    __builtin_memcpy(nx, w + 4, sizeof nx);
    __builtin_memcpy(ny, w + 4 + RW, sizeof ny);
    __builtin_memcpy(nz, w + 4 + 2 * RW, sizeof nz);
    __builtin_memcpy(fx, w + 4 + 3 * RW, sizeof fx);
    __builtin_memcpy(fy, w + 4 + 4 * RW, sizeof fy);
    __builtin_memcpy(fz, w + 4 + 5 * RW, sizeof fz);
    const int eb = (int)w[3];
    const f3 a = {ldexpf(inv.x, (eb << 24) >> 24), ldexpf(inv.y, (eb << 16) >> 24), ldexpf(inv.z, (eb << 8) >> 24)};
    const f3 b = {fmaf(__uint_as_float(w[0]), inv.x, -oi.x), fmaf(__uint_as_float(w[1]), inv.y, -oi.y),
                  fmaf(__uint_as_float(w[2]), inv.z, -oi.z)};
    // Entry and exit distances as integer max / min of the float bit patterns.
    // The bounds are positive (t_lo = eps_self, t_hi > t_lo), so the entry
    // distance is positive and, among non-negative floats, the integer order is
    // the float order; a negative exit distance stays negative (only its value
    // differs), so the test t0 <= t1 and the entry distance are those of the
    // float forms. The slab distances are never NaN (inv, the grid steps and
    // coordinates are finite). Unlike fmaxf / fminf, the integer forms need no
    // canonicalisation of their loop-invariant bound.
    const int lo_i = __float_as_int(t_lo), hi_i = __float_as_int(t_hi);
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int t0 = max(max(__float_as_int(fmaf((float)nx[j], a.x, b.x)), __float_as_int(fmaf((float)ny[j], a.y, b.y))),
                           max(__float_as_int(fmaf((float)nz[j], a.z, b.z)), lo_i));
        const int t1 = min(min(__float_as_int(fmaf((float)fx[j], a.x, b.x)), __float_as_int(fmaf((float)fy[j], a.y, b.y))),
                           min(__float_as_int(fmaf((float)fz[j], a.z, b.z)), hi_i));
        tn[j] = __int_as_float(t0) <= __int_as_float(t1) ? __int_as_float(t0) : INFINITY;
    }
}

__device__ __forceinline__ void cmp_swap(float *t, int *r, int i, int j) {
    const bool sw = t[j] < t[i];
    const float ti = sw ? t[j] : t[i], tj = sw ? t[i] : t[j];
    const int ri = sw ? r[j] : r[i], rj = sw ? r[i] : r[j];
    t[i] = ti;
    t[j] = tj;
    r[i] = ri;
    r[j] = rj;
}

// Children by increasing entry distance: optimal sorting networks for 4
// (5 comparators) and 8 (19 comparators) keys.
template <int W>
__device__ __forceinline__ void sort_hits(float (&t)[W], int (&r)[W]) {
    if constexpr (W == 4) {
        cmp_swap(t, r, 0, 1); cmp_swap(t, r, 2, 3);
        cmp_swap(t, r, 0, 2); cmp_swap(t, r, 1, 3);
        cmp_swap(t, r, 1, 2);
    } else {
        static_assert(W == 8, "wide nodes have 4 or 8 children");
        cmp_swap(t, r, 0, 2); cmp_swap(t, r, 1, 3); cmp_swap(t, r, 4, 6); cmp_swap(t, r, 5, 7);
        cmp_swap(t, r, 0, 4); cmp_swap(t, r, 1, 5); cmp_swap(t, r, 2, 6); cmp_swap(t, r, 3, 7);
        cmp_swap(t, r, 0, 1); cmp_swap(t, r, 2, 3); cmp_swap(t, r, 4, 5); cmp_swap(t, r, 6, 7);
        cmp_swap(t, r, 2, 4); cmp_swap(t, r, 3, 5);
        cmp_swap(t, r, 1, 4); cmp_swap(t, r, 3, 6);
        cmp_swap(t, r, 1, 2); cmp_swap(t, r, 3, 4); cmp_swap(t, r, 5, 6);
    }
}

// One step at a wide node: the nearest entered child becomes ref, the other
// entered children are pushed farthest first (so they come back nearest
// first). Returns false if no child is entered.
template <int W>
__device__ __forceinline__ bool wide_step(const DevScene &S, int &ref, int &sp, f3 inv, f3 oi, float t_lo,
                                          float t_hi, Stack &stk) {
    float tn[W];
    int cr[W];
    wide_hits_minmax<W>(S.node, ref, inv, oi, t_lo, t_hi, tn, cr);
    sort_hits<W>(tn, cr);
    if (!(tn[0] < INFINITY)) return false;
#pragma unroll
    for (int j = W - 1; j >= 1; --j)
        if (tn[j] < INFINITY) stk.put(sp++, cr[j]);
    ref = cr[0];
    return true;
}

// Any-hit step at a wide node: only the nearest entered child is singled out
// (walked next); the other entered children are pushed in slot order. The
// order cannot change an any-hit answer, only how soon it is found.
template <int W>
__device__ __forceinline__ bool wide_step_any(const DevScene &S, int &ref, int &sp, const Octant &q, f3 inv, f3 oi,
                                              float t_lo, float t_hi, Stack &stk) {
    float tn[W];
    int cr[W];
    wide_hits<W>(S, ref, q, inv, oi, t_lo, t_hi, tn, cr);
    float tb = tn[0];
    int jb = 0;
#pragma unroll
    for (int j = 1; j < W; ++j) {
        const bool lt = tn[j] < tb;
        tb = lt ? tn[j] : tb;
        jb = lt ? j : jb;
    }
    if (!(tb < INFINITY)) return false;
    int nref = cr[0];
#pragma unroll
    for (int j = 1; j < W; ++j) nref = jb == j ? cr[j] : nref;
    if (sp + (W - 1) <= kStackLds) {  // every push lands in LDS: no spill test per push
#pragma unroll
        for (int j = 0; j < W; ++j)
            if (tn[j] < INFINITY && j != jb) stk.lds[(sp++) * kWave] = cr[j];
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j)
            if (tn[j] < INFINITY && j != jb) stk.put(sp++, cr[j]);
    }
    ref = nref;
    return true;
}

template <int W, bool kSecond>
__device__ __forceinline__ void traverse_closest(const DevScene &S, f3 o, f3 d, f3 inv, int excl, float t_lo,
                                                 float eps_tie, Stack &stk, float &tmin, Cand *c, bool &spill,
                                                 float t_win, float &best_d2, int &best_id, float &best_t) {
    const f3 oi = times(o, inv);
    int ref = S.root;
    int sp = 0;
    for (;;) {
        if (ref >= 0) {
            stk.visit();
            const float tc = kSecond ? t_win : tmin + eps_tie;
            if constexpr (W > 2) {
                if (wide_step<W>(S, ref, sp, inv, oi, t_lo, tc, stk)) continue;
            } else {
                const uint32_t nb = (uint32_t)ref * 64u;
                const float4 a = ld4(S.node, nb), b = ld4(S.node, nb + 16u), e = ld4(S.node, nb + 32u),
                             r = ld4(S.node, nb + 48u);
                float n0, n1;
                const bool h0 = box_hit(a.x, a.y, a.z, a.w, b.x, b.y, inv, oi, t_lo, tc, n0);
                const bool h1 = box_hit(b.z, b.w, e.x, e.y, e.z, e.w, inv, oi, t_lo, tc, n1);
                const int r0 = __float_as_int(r.x), r1 = __float_as_int(r.y);
                if (h0 && h1) {
                    const bool f0 = n0 <= n1;
                    stk.put(sp++, f0 ? r1 : r0);
                    ref = f0 ? r0 : r1;
                    continue;
                }
                if (h0) { ref = r0; continue; }
                if (h1) { ref = r1; continue; }
            }
        } else {
            const int v = -1 - ref;
            const int first = v >> 3, cnt = (v & 7) + 1;
            stk.test(cnt);
            for (int i = 0; i < cnt; ++i)
                visit_disk<kSecond>(S, first + i, o, d, excl, t_lo, eps_tie, tmin, c, spill, t_win, best_d2, best_id,
                                    best_t);
        }
        if (sp == 0) break;
        ref = stk.get(--sp);
    }
}

template <int W>
__device__ __forceinline__ int closest_hit(const DevScene &S, f3 o, f3 d, int excl, float t_lo, float eps_tie,
                                           Stack &stk, float &t_out, bool &spilled) {
    f3 inv = safe_inv(d);
    float tmin = INFINITY;
    Cand c[kTieList];
#pragma unroll
    for (int k = 0; k < kTieList; ++k) c[k] = {INFINITY, INFINITY, -1};
    bool spill = false;
    float bd2 = INFINITY, bt = INFINITY;
    int bid = 0x7fffffff;
    traverse_closest<W, false>(S, o, d, inv, excl, t_lo, eps_tie, stk, tmin, c, spill, 0.f, bd2, bid, bt);
    spilled = spill;
    if (!(tmin < INFINITY)) return -1;
    if (spill) {
        float dummy = tmin;
        traverse_closest<W, true>(S, o, d, inv, excl, t_lo, eps_tie, stk, dummy, c, spill, tmin + eps_tie, bd2,
                                  bid, bt);
        t_out = bt;
        return bid;
    }
#pragma unroll
    for (int k = 0; k < kTieList; ++k)
        if (c[k].id >= 0 && (c[k].d2 < bd2 || (c[k].d2 == bd2 && c[k].id < bid))) {
            bd2 = c[k].d2;
            bid = c[k].id;
            bt = c[k].t;
        }
    t_out = bt;
    return bid;
}

// Any-hit step at a node of either layout: true if a child was entered (ref
// is then that child, the other entered children are on the stack), false
// if the segment enters none.
template <int W>
__device__ __forceinline__ bool step_any(const DevScene &S, int &ref, int &sp, const Octant &oq, f3 inv, f3 oi,
                                         float t_lo, float t_hi, Stack &stk) {
    if constexpr (W > 2) {
        return wide_step_any<W>(S, ref, sp, oq, inv, oi, t_lo, t_hi, stk);
    } else {
        const uint32_t o = (uint32_t)ref * 64u;
        const float4 na = ld4(S.node, o), nb = ld4(S.node, o + 16u), ne = ld4(S.node, o + 32u),
                     nr = ld4(S.node, o + 48u);
        float n0, n1;
        const bool h0 = box_hit(na.x, na.y, na.z, na.w, nb.x, nb.y, inv, oi, t_lo, t_hi, n0);
        const bool h1 = box_hit(nb.z, nb.w, ne.x, ne.y, ne.z, ne.w, inv, oi, t_lo, t_hi, n1);
        const int r0 = __float_as_int(nr.x), r1 = __float_as_int(nr.y);
        if (h0 && h1) {
            const bool f0 = n0 <= n1;
            stk.put(sp++, f0 ? r1 : r0);
            ref = f0 ? r0 : r1;
            return true;
        }
        if (h0) { ref = r0; return true; }
        if (h1) { ref = r1; return true; }
        return false;
    }
}

// "Nothing left to walk": never a node (>= 0) or leaf (>= -2^29 - 8) reference.
constexpr int kNoRef = -0x7fffffff - 1;

// True iff a disk != excl is hit with eps_self < t < |b - a| - eps_self on the
// segment from a towards b. eps_self > 0 (every entry point maps other values
// to its default), which the integer clamps of wide_hits rely on.
//
// Leaves are parked: a lane that reaches a leaf keeps it (one at a time) and
// walks on through nodes; the wavefront tests the parked leaves together once
// at least half of its live lanes hold one, or when no lane can take a node
// step. Node steps and disk tests then each run with more lanes busy than
// when every lane tests a leaf as soon as it reaches it. Parking only delays
// disk tests: the walk order, and so the stack bound, are those of the plain
// depth-first walk, and the answer is the same.
// excl: a disk id, or with BY_SET a point set whose disks are all ignored.
template <int W, bool BY_SET = false>
__device__ __forceinline__ bool occluded(const DevScene &S, f3 a, f3 b, int excl, float eps_self, Stack &stk) {
    const f3 dv = b - a;
    const float L = len(dv);
    const f3 d = (1.0f / L) * dv;
    const f3 inv = safe_inv(d);
    const float t_hi = L - eps_self;
    if (!(t_hi > eps_self)) return false;
    const f3 oi = times(a, inv);
    const Octant oq = octant<W>(inv);
    int ref = S.root, sp = 0, park = kNoRef;
    for (;;) {
        for (;;) {
            if (ref < 0 && ref != kNoRef && park == kNoRef) {
                park = ref;
                ref = sp > 0 ? stk.get(--sp) : kNoRef;
            }
            const uint32_t n_live = (uint32_t)__popcll(__ballot(1));
            const uint32_t n_park = (uint32_t)__popcll(__ballot(park != kNoRef));
            if (!__ballot(ref >= 0) || 2 * n_park >= n_live) break;
            if (ref >= 0) {
                stk.visit();
                if (!step_any<W>(S, ref, sp, oq, inv, oi, eps_self, t_hi, stk))
                    ref = sp > 0 ? stk.get(--sp) : kNoRef;
            }
        }
        if (park != kNoRef) {
            const int v = -1 - park;
            const int first = v >> 3, cnt = (v & 7) + 1;
            stk.test(cnt);
            for (int i = 0; i < cnt; ++i) {
                const float4 dp = ld4(S.disk, (uint32_t)(first + i) * 32u);
                const float4 dn = ld4(S.disk, (uint32_t)(first + i) * 32u + 16u);
                float t, d2;
                const bool h = disk_hit(a, d, xyz(dp), xyz(dn), S.r2, t, d2);
                const int who = BY_SET ? __float_as_int(dn.w) : __float_as_int(dp.w);
                if (h & (who != excl) & (t > eps_self) & (t < t_hi)) return true;
            }
            park = kNoRef;
        }
        if (ref == kNoRef) return false;
    }
}

// ------------------------------------------------------------- field
struct c32 {
    float re, im;
};
__device__ __forceinline__ c32 cmul(c32 a, c32 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ c32 cdiv(c32 a, c32 b) {
    // scale by the larger component to keep |b|^2 in range (metals give |eta| ~ 1e8)
    float s = fmaxf(fabsf(b.re), fabsf(b.im));
    float inv_s = 1.0f / s;
    c32 bs = {b.re * inv_s, b.im * inv_s};
    c32 as = {a.re * inv_s, a.im * inv_s};
    float den = bs.re * bs.re + bs.im * bs.im;
    return {(as.re * bs.re + as.im * bs.im) / den, (as.im * bs.re - as.re * bs.im) / den};
}
__device__ __forceinline__ c32 csqrt_p(c32 z) {  // principal branch
    float r = hypotf(z.re, z.im);
    if (r == 0.f) return {0.f, 0.f};
    if (z.re >= 0.f) {
        float re = sqrtf(0.5f * (r + z.re));
        return {re, z.im / (2.f * re)};
    }
    float im = copysignf(sqrtf(0.5f * (r - z.re)), z.im);
    return {z.im / (2.f * im), im};
}

// Fresnel coefficients for eta = eps_r - j sigma/(omega eps0) at incidence
// cosine c: w = sqrt(eta - (1 - c^2)), TE = (c - w)/(c + w),
// TM = (eta c - w)/(eta c + w).
__device__ __forceinline__ void fresnel(float eps_r, float sig_w /* sigma/(omega eps0) */, float c, c32 &te,
                                        c32 &tm) {
    c32 eta = {eps_r, -sig_w};
    float s2 = 1.0f - c * c;
    c32 w = csqrt_p({eta.re - s2, eta.im});
    te = cdiv({c - w.re, -w.im}, {c + w.re, w.im});
    c32 ec = {eta.re * c, eta.im * c};
    tm = cdiv({ec.re - w.re, ec.im - w.im}, {ec.re + w.re, ec.im + w.im});
}

// Derivatives of the coefficients with respect to eta:
// dTE/deta = -c / (w (c + w)^2), dTM/deta = c (eta - 2 s^2) / (w (eta c + w)^2).
__device__ __forceinline__ void fresnel_deta(float eps_r, float sig_w, float c, c32 &dte, c32 &dtm) {
    c32 eta = {eps_r, -sig_w};
    float s2 = 1.0f - c * c;
    c32 w = csqrt_p({eta.re - s2, eta.im});
    c32 cw = {c + w.re, w.im};
    c32 den = cmul(w, cmul(cw, cw));
    dte = cdiv({-c, 0.f}, den);
    c32 ecw = {eta.re * c + w.re, eta.im * c + w.im};
    c32 den2 = cmul(w, cmul(ecw, ecw));
    dtm = cdiv({c * (eta.re - 2.f * s2), c * eta.im}, den2);
}

// e^{-j 2 pi L / lambda} with the cycle count L/lambda reduced exactly:
// (hi + lo) = 1/lambda split in two floats, Dekker product, then the
// fractional part, so the phase error is that of L alone.
__device__ __forceinline__ c32 propagate(float L, float inv_lam_hi, float inv_lam_lo) {
    float p = L * inv_lam_hi;
    float e = fmaf(L, inv_lam_hi, -p) + L * inv_lam_lo;
    float f = (p - rintf(p)) + e;
    float s, c;
    sincospif(2.0f * f, &s, &c);
    return {c, -s};
}

// Polarised field (Jones vectors): a complex 3-vector carried along a path.
// The transmitter radiates its polarisation vector projected on the plane
// normal to the departure direction; a reflection (incoming di, outgoing
// dout, plane normal n) splits the field along s = di x n / |di x n| (TE) and
// p_in = s x di (TM) and sends R (Gamma_TE (E.s) s + Gamma_TM (E.p_in) p_out),
// p_out = s x dout; the receiver projects on its polarisation vector
// projected on the plane normal to the arrival direction. At normal
// incidence s is any unit vector normal to di: Gamma_TM = -Gamma_TE there, so
// the result does not depend on the choice.
struct cv3 {
    c32 x, y, z;
};
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ f3 transverse(f3 p, f3 d) { return p - dot(p, d) * d; }
__device__ __forceinline__ cv3 pol_launch(f3 p, f3 d) {
    const f3 t = transverse(p, d);
    return {{t.x, 0.f}, {t.y, 0.f}, {t.z, 0.f}};
}
__device__ __forceinline__ c32 cdot(const cv3 &e, f3 v) {
    return {e.x.re * v.x + e.y.re * v.y + e.z.re * v.z, e.x.im * v.x + e.y.im * v.y + e.z.im * v.z};
}
__device__ __forceinline__ void pol_reflect(cv3 &e, f3 di, f3 dout, f3 n, c32 gte, c32 gtm, float R) {
    f3 s = cross(di, n);
    const float ns = len(s);
    if (ns > 1e-6f) {
        s = (1.0f / ns) * s;
    } else {  // normal incidence: the axis least aligned with di, crossed with it
        const f3 ax = fabsf(di.x) <= fabsf(di.y) && fabsf(di.x) <= fabsf(di.z) ? mk(1.f, 0.f, 0.f)
                      : fabsf(di.y) <= fabsf(di.z)                         ? mk(0.f, 1.f, 0.f)
                                                                           : mk(0.f, 0.f, 1.f);
        s = normalize(cross(di, ax));
    }
    const f3 pin = cross(s, di), pout = cross(s, dout);
    const c32 a = cmul({R * gte.re, R * gte.im}, cdot(e, s));
    const c32 b = cmul({R * gtm.re, R * gtm.im}, cdot(e, pin));
    e.x = {a.re * s.x + b.re * pout.x, a.im * s.x + b.im * pout.x};
    e.y = {a.re * s.y + b.re * pout.y, a.im * s.y + b.im * pout.y};
    e.z = {a.re * s.z + b.re * pout.z, a.im * s.z + b.im * pout.z};
}
__device__ __forceinline__ c32 pol_receive(const cv3 &e, f3 p, f3 d) { return cdot(e, transverse(p, d)); }

struct FieldConst {
    float amp_iso;      // lambda / (4 pi)
    float inv_lam_hi;   // 1/lambda, high part
    float inv_lam_lo;   // 1/lambda, low part
    float inv_we0;      // 1 / (omega eps0)
};

// LDS written by some lanes of a wavefront is visible to the others after this.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum_d(double v) {  // fixed xor-butterfly order
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ float warp_sum_f(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ uint32_t warp_sum_u(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Instrumented builds: add this lane's visit counts to counters[slot], [slot+1].
__device__ __forceinline__ void flush_visits(const Stack &stk, uint64_t *counters, int slot) {
    if (!kCountVisits) return;
    uint64_t v = stk.nv, d = stk.nd;
    for (int o = 32; o > 0; o >>= 1) {
        v += __shfl_xor(v, o, kWave);
        d += __shfl_xor(d, o, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicAdd((unsigned long long *)&counters[slot], (unsigned long long)v);
        atomicAdd((unsigned long long *)&counters[slot + 1], (unsigned long long)d);
    }
}

// Item of a flattened ray slot (items sorted by ray_off).
__device__ __forceinline__ int find_item(const Item *items, int n_items, uint32_t g) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (items[mid].ray_off <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Fibonacci-sphere launch direction of ray j out of N, FP64 then rounded to FP32.
__device__ __forceinline__ f3 fib_dir(uint32_t j, uint32_t N) {
#pragma clang fp contract(off)
    const double g = (3.0 - 2.2360679774997896964) * 0.5;  // (3 - sqrt 5)/2
    double z = 1.0 - (2.0 * (double)j + 1.0) / (double)N;
    double rho = sqrt(fmax(0.0, 1.0 - z * z));
    double f = (double)j * g;
    f -= floor(f);
    double phi = 2.0 * kPi * f;
    double sp, cp;
    sincos(phi, &sp, &cp);
    return {(float)(rho * cp), (float)(rho * sp), (float)z};
}

// Unit direction from o towards c, FP64 then rounded to FP32 (no contraction,
// so both implementations round the same products).
__device__ __forceinline__ f3 aim_dir(const float *o, float4 c) {
#pragma clang fp contract(off)
    const double dx = (double)c.x - (double)o[0], dy = (double)c.y - (double)o[1], dz = (double)c.z - (double)o[2];
    const double il = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    return {(float)(dx * il), (float)(dy * il), (float)(dz * il)};
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {  // splitmix64 finaliser
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

}  // namespace pcrt
