// Scene ingest and linear BVH build over disk bounding boxes.
//
// The paper hands point-set AABBs to a hardware ray-tracing API (Sec. II-A).
// gfx950 has no ray-tracing units, so the hierarchy is built here: Morton
// codes of disk centres, a hand-written LSD radix sort, the Karras (2012)
// binary radix tree over the sorted codes, and a bottom-up refit that also
// collapses small subtrees into leaves of up to `leaf_size` disks.
#include "common.h"
#include "internal.h"

#include <vector>

namespace pcrt {

// --------------------------------------------------------------- ingest
// Validates and normalises each point; writes the by-id tables and the
// per-block bounds of disk centres. status bits: 1 non-finite position,
// 2 zero or non-finite normal.
__global__ void k_ingest(const float *__restrict__ pos, const float *__restrict__ nrm,
                         const uint16_t *__restrict__ mat, const uint32_t *__restrict__ surf, uint32_t n,
                         float4 *__restrict__ pos_id, float4 *__restrict__ nrm_id, float *__restrict__ blk_bounds,
                         uint32_t *__restrict__ stat) {
    __shared__ float red[6][256];
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    uint32_t bad = 0, ms = 0, mm = 0;
    if (i < n) {
        float px = pos[3 * i], py = pos[3 * i + 1], pz = pos[3 * i + 2];
        float nx = nrm[3 * i], ny = nrm[3 * i + 1], nz = nrm[3 * i + 2];
        if (!(isfinite(px) && isfinite(py) && isfinite(pz))) bad |= 1;
        float l2 = nx * nx + ny * ny + nz * nz;
        if (!(l2 > 0.f) || !isfinite(l2)) bad |= 2;
        float il = bad & 2 ? 0.f : 1.0f / sqrtf(l2);
        uint32_t s = surf[i], m = mat[i];
        ms = s;
        mm = m;
        pos_id[i] = make_float4(px, py, pz, __uint_as_float(s));
        nrm_id[i] = make_float4(nx * il, ny * il, nz * il, __uint_as_float(m));
        if (!bad) {
            lo[0] = hi[0] = px;
            lo[1] = hi[1] = py;
            lo[2] = hi[2] = pz;
        }
    }
    for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = lo[a];
        red[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) blk_bounds[6 * blockIdx.x + a] = red[a][0];
    if (bad) atomicOr(&stat[0], bad);
    if (i < n) {
        atomicMax(&stat[1], ms);
        atomicMax(&stat[2], mm);
    }
}

// Final bounds over the per-block bounds (one block).
__global__ void k_bounds(const float *__restrict__ blk, uint32_t nblk, float *__restrict__ out) {
    __shared__ float red[6][256];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (uint32_t b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int a = 0; a < 3; ++a) {
            v[a] = fminf(v[a], blk[6 * b + a]);
            v[3 + a] = fmaxf(v[3 + a], blk[6 * b + 3 + a]);
        }
    for (int a = 0; a < 6; ++a) red[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) out[a] = red[a][0];
}

__device__ __forceinline__ uint64_t spread21(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

// 63-bit Morton code of each disk centre in the scene bounds.
__global__ void k_morton(const float4 *__restrict__ pos_id, uint32_t n, const float *__restrict__ bounds,
                         uint64_t *__restrict__ code, uint32_t *__restrict__ idx) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 p = pos_id[i];
    float c[3] = {p.x, p.y, p.z};
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) {
        float ext = bounds[3 + a] - bounds[a];
        float u = ext > 0.f ? (c[a] - bounds[a]) / ext : 0.5f;
        u = fminf(fmaxf(u, 0.f), 1.f);
        q[a] = (uint64_t)(u * 2097151.0f);
    }
    code[i] = spread21(q[0]) << 2 | spread21(q[1]) << 1 | spread21(q[2]);
    idx[i] = i;
}

// -------------------------------------------------- Karras radix tree
__device__ __forceinline__ int delta(const uint64_t *k, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    uint64_t a = k[i], b = k[j];
    if (a == b) return 64 + __clz((uint32_t)i ^ (uint32_t)j);
    return __clzll(a ^ b);
}

// Internal node i of n-1: children (int index or leaf encoded as ~pos) and
// covered range [first, last] of sorted positions.
__global__ void k_karras(const uint64_t *__restrict__ k, int n, int2 *__restrict__ child, int2 *__restrict__ range,
                         int *__restrict__ parent_int, int *__restrict__ parent_leaf) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (delta(k, n, i, i + 1) - delta(k, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = delta(k, n, i, i - d);
    int lmax = 2;
    while (delta(k, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(k, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = delta(k, n, i, j);
    int s = 0;
    int div = 2;
    for (;;) {
        int t = (l + div - 1) / div;
        if (delta(k, n, i, i + (s + t) * d) > dnode) s += t;
        if (t == 1) break;
        div <<= 1;
    }
    int gamma = i + s * d + min(d, 0);
    int first = min(i, j), last = max(i, j);
    int left = (first == gamma) ? ~gamma : gamma;
    int right = (last == gamma + 1) ? ~(gamma + 1) : gamma + 1;
    child[i] = make_int2(left, right);
    range[i] = make_int2(first, last);
    if (left < 0) parent_leaf[~left] = i;
    else parent_int[left] = i;
    if (right < 0) parent_leaf[~right] = i;
    else parent_int[right] = i;
    if (i == 0) parent_int[0] = -1;
}

// Leaf-ordered disks and their padded bounding boxes.
__global__ void k_gather(const float4 *__restrict__ pos_id, const float4 *__restrict__ nrm_id,
                         const uint32_t *__restrict__ perm, uint32_t n, float r, float4 *__restrict__ disk,
                         float *__restrict__ dbox) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t id = perm[i];
    float4 p = pos_id[id], nn = nrm_id[id];
    disk[2 * i] = make_float4(p.x, p.y, p.z, __int_as_float((int)id));
    disk[2 * i + 1] = make_float4(nn.x, nn.y, nn.z, 0.f);
    float c[3] = {p.x, p.y, p.z}, nv[3] = {nn.x, nn.y, nn.z};
    for (int a = 0; a < 3; ++a) {
        // tight half-extent of a disk along axis a, padded so that FP32
        // slab tests stay conservative
        float h = r * sqrtf(fmaxf(0.f, 1.f - nv[a] * nv[a]));
        float pad = 1e-5f + 2e-6f * (fabsf(c[a]) + r);
        dbox[6 * i + a] = c[a] - h - pad;
        dbox[6 * i + 3 + a] = c[a] + h + pad;
    }
}

// Bottom-up refit: the second thread to reach a node computes its box and
// writes its traversal record; children covering <= L disks become leaves.
__global__ void k_refit(int n, int L, const int2 *__restrict__ child, const int2 *__restrict__ range,
                        const int *__restrict__ parent_int, const int *__restrict__ parent_leaf,
                        const float *__restrict__ dbox, float *ibox, uint32_t *flags, float4 *__restrict__ node) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cur = parent_leaf[i];
    while (cur >= 0) {
        __threadfence();
        if (atomicAdd(&flags[cur], 1u) == 0) return;
        __threadfence();
        int2 ch = child[cur];
        float b[2][6];
        int ref[2];
        int cc[2] = {ch.x, ch.y};
        for (int s = 0; s < 2; ++s) {
            int c = cc[s];
            if (c < 0) {
                int p = ~c;
                for (int a = 0; a < 6; ++a) b[s][a] = dbox[6 * p + a];
                ref[s] = leaf_ref(p, 1);
            } else {
                const volatile float *vb = ibox + 6 * c;
                for (int a = 0; a < 6; ++a) b[s][a] = vb[a];
                int2 rg = range[c];
                int cnt = rg.y - rg.x + 1;
                ref[s] = cnt <= L ? leaf_ref(rg.x, cnt) : c;
            }
        }
        volatile float *ob = ibox + 6 * cur;
        for (int a = 0; a < 3; ++a) {
            ob[a] = fminf(b[0][a], b[1][a]);
            ob[3 + a] = fmaxf(b[0][3 + a], b[1][3 + a]);
        }
        float4 *nd = node + 4 * (size_t)cur;
        nd[0] = make_float4(b[0][0], b[0][1], b[0][2], b[0][3]);
        nd[1] = make_float4(b[0][4], b[0][5], b[1][0], b[1][1]);
        nd[2] = make_float4(b[1][2], b[1][3], b[1][4], b[1][5]);
        nd[3] = make_float4(__int_as_float(ref[0]), __int_as_float(ref[1]), 0.f, 0.f);
        cur = parent_int[cur];
    }
}

// Depth (number of internal ancestors) of each sorted leaf; max into *depth.
// Node records when every internal node's box is already known (the
// clustering builder records them at merge time): one thread per node, no
// bottom-up climb. Same records as k_refit.
__global__ void k_node_records(int n_int, int L, const int2 *__restrict__ child, const int2 *__restrict__ range,
                               const float *__restrict__ dbox, const float *__restrict__ ibox,
                               float4 *__restrict__ node) {
    const int cur = blockIdx.x * blockDim.x + threadIdx.x;
    if (cur >= n_int) return;
    const int2 ch = child[cur];
    float b[2][6];
    int ref[2];
    const int cc[2] = {ch.x, ch.y};
    for (int s = 0; s < 2; ++s) {
        const int c = cc[s];
        if (c < 0) {
            const int p = ~c;
            for (int a = 0; a < 6; ++a) b[s][a] = dbox[6 * (size_t)p + a];
            ref[s] = leaf_ref(p, 1);
        } else {
            for (int a = 0; a < 6; ++a) b[s][a] = ibox[6 * (size_t)c + a];
            const int2 rg = range[c];
            const int cnt = rg.y - rg.x + 1;
            ref[s] = cnt <= L ? leaf_ref(rg.x, cnt) : c;
        }
    }
    float4 *nd = node + 4 * (size_t)cur;
    nd[0] = make_float4(b[0][0], b[0][1], b[0][2], b[0][3]);
    nd[1] = make_float4(b[0][4], b[0][5], b[1][0], b[1][1]);
    nd[2] = make_float4(b[1][2], b[1][3], b[1][4], b[1][5]);
    nd[3] = make_float4(__int_as_float(ref[0]), __int_as_float(ref[1]), 0.f, 0.f);
}

__global__ void k_depth(int n, const int *__restrict__ parent_int, const int *__restrict__ parent_leaf,
                        uint32_t *__restrict__ depth) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t dd = 0;
    for (int cur = parent_leaf[i]; cur >= 0; cur = parent_int[cur]) ++dd;
    atomicMax(depth, dd);
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// ------------------------------------------------------------ host side
static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

void fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
    if (!n) return;
    uint32_t g = (uint32_t)std::min<size_t>(cdiv(n, 256), 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, s, p, v, n);
}
void fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s) {
    if (!n) return;
    uint32_t g = (uint32_t)std::min<size_t>(cdiv(n, 256), 4096);
    hipLaunchKernelGGL(k_fill_u64, dim3(g), dim3(256), 0, s, p, v, n);
}

// --------------------------------------------------- clustering builder
// Parallel locally-ordered clustering (Meister & Bittner, 2018) over the
// Morton-ordered disks. Each pass: every cluster finds, within +-kPlocRadius
// positions, the cluster whose merged box has the smallest surface area
// (ties: smaller index); mutual nearest pairs merge into a new internal node
// (lower index keeps the slot) and the list is compacted by an exclusive
// scan. The order on pairs (area, lower index, higher index) is total, so
// the globally cheapest pair is always mutual and every pass merges at least
// one pair. Internal nodes are numbered in creation order; the root is the
// last. The disks are then renumbered in depth-first order so that every
// subtree owns a contiguous disk range, which is what the refit and the leaf
// references expect.
// Search radius, measured on the 1M-point office (diffuse / refine / trace
// ms): 4 -> 34.4 / 4.8 / 3.1, 6 -> 33.9 / 4.5 / 3.1, 8 -> 34.6 / 4.4 / 3.1,
// 16 -> 35.1 / 4.8 / 3.3, 32 -> 35.8 / 4.6 / 3.4, 64 -> 36.3 / 4.5 / 3.4.
constexpr int kPlocRadius = 6;

__device__ __forceinline__ float merged_half_area(const float *a, const float *b) {
    const float dx = fmaxf(a[3], b[3]) - fminf(a[0], b[0]);
    const float dy = fmaxf(a[4], b[4]) - fminf(a[1], b[1]);
    const float dz = fmaxf(a[5], b[5]) - fminf(a[2], b[2]);
    return dx * dy + dy * dz + dz * dx;
}

__global__ void k_ploc_nn(const float *__restrict__ cbox, uint32_t n, int *__restrict__ nn) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float bi[6];
    for (int a = 0; a < 6; ++a) bi[a] = cbox[6 * (size_t)i + a];
    const uint32_t lo = i > (uint32_t)kPlocRadius ? i - kPlocRadius : 0u;
    const uint32_t hi = min(n - 1, i + kPlocRadius);
    float best = INFINITY;
    int bj = -1;
    for (uint32_t j = lo; j <= hi; ++j) {  // increasing j: a strict < keeps the smaller index on ties
        if (j == i) continue;
        const float c = merged_half_area(bi, cbox + 6 * (size_t)j);
        if (c < best) {
            best = c;
            bj = (int)j;
        }
    }
    nn[i] = bj;
}

__global__ void k_ploc_flags(const int *__restrict__ nn, uint32_t n, uint32_t *__restrict__ merge,
                             uint32_t *__restrict__ keep) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j = nn[i];
    const bool mutual = nn[j] == (int)i;
    merge[i] = mutual && (int)i < j;
    keep[i] = !(mutual && (int)i > j);
}

__global__ void k_ploc_apply(const float *__restrict__ cbox, const int *__restrict__ cid,
                             const uint32_t *__restrict__ csize, const int *__restrict__ nn, uint32_t n,
                             const uint32_t *__restrict__ mpos, const uint32_t *__restrict__ kpos, uint32_t node_base,
                             float *__restrict__ obox, int *__restrict__ oid, uint32_t *__restrict__ osize,
                             int2 *__restrict__ child, uint32_t *__restrict__ nsize, int *__restrict__ parent_int,
                             int *__restrict__ parent_leaf, float *__restrict__ ibox) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j = nn[i];
    const bool mutual = nn[j] == (int)i;
    if (mutual && (int)i > j) return;  // merged into the lower slot
    const uint32_t p = kpos[i];
    if (!mutual) {
        for (int a = 0; a < 6; ++a) obox[6 * (size_t)p + a] = cbox[6 * (size_t)i + a];
        oid[p] = cid[i];
        osize[p] = csize[i];
        return;
    }
    const int node = (int)(node_base + mpos[i]);
    const int a = cid[i], b = cid[j];
    child[node] = make_int2(a, b);
    const uint32_t sz = csize[i] + csize[j];
    nsize[node] = sz;
    if (a < 0) parent_leaf[~a] = node;
    else parent_int[a] = node;
    if (b < 0) parent_leaf[~b] = node;
    else parent_int[b] = node;
    const float *x = cbox + 6 * (size_t)i, *y = cbox + 6 * (size_t)j;
    for (int k = 0; k < 3; ++k) {
        const float lo = fminf(x[k], y[k]), hi = fmaxf(x[3 + k], y[3 + k]);
        obox[6 * (size_t)p + k] = lo;
        obox[6 * (size_t)p + 3 + k] = hi;
        ibox[6 * (size_t)node + k] = lo;  // the node's box: min / max are exact, so the same
        ibox[6 * (size_t)node + 3 + k] = hi;  // values a refit over its disks would give
    }
    oid[p] = node;
    osize[p] = sz;
}

// Depth-first offsets, one creation pass at a time from the root's down
// (a node's parent is always created in a later pass).
__global__ void k_dfs_pass(const int2 *__restrict__ child, const uint32_t *__restrict__ nsize, uint32_t lo,
                           uint32_t hi, uint32_t *__restrict__ noff, uint32_t *__restrict__ leaf_pos) {
    const uint32_t node = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= hi) return;
    const uint32_t o = noff[node];
    const int2 c = child[node];
    const uint32_t sa = c.x < 0 ? 1u : nsize[c.x];
    if (c.x < 0) leaf_pos[~c.x] = o;
    else noff[c.x] = o;
    if (c.y < 0) leaf_pos[~c.y] = o + sa;
    else noff[c.y] = o + sa;
}

__global__ void k_dfs_leaves(uint32_t n, const uint32_t *__restrict__ leaf_pos, const uint32_t *__restrict__ sorted_id,
                             const int *__restrict__ parent_leaf_old, uint32_t *__restrict__ perm,
                             int *__restrict__ parent_leaf) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = leaf_pos[i];
    perm[p] = sorted_id[i];
    parent_leaf[p] = parent_leaf_old[i];
}

__global__ void k_dfs_nodes(uint32_t n_int, const uint32_t *__restrict__ leaf_pos, const uint32_t *__restrict__ noff,
                            const uint32_t *__restrict__ nsize, int2 *__restrict__ child, int2 *__restrict__ range) {
    const uint32_t node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= n_int) return;
    int2 c = child[node];
    if (c.x < 0) c.x = ~(int)leaf_pos[~c.x];
    if (c.y < 0) c.y = ~(int)leaf_pos[~c.y];
    child[node] = c;
    range[node] = make_int2((int)noff[node], (int)(noff[node] + nsize[node] - 1));
}

__global__ void k_ploc_init(const float *__restrict__ dbox, uint32_t n, float *__restrict__ cbox, int *__restrict__ cid,
                            uint32_t *__restrict__ csize) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int a = 0; a < 6; ++a) cbox[6 * (size_t)i + a] = dbox[6 * (size_t)i + a];
    cid[i] = ~(int)i;
    csize[i] = 1;
}

// --------------------------------------------------------- wide nodes
// Collapse of the binary hierarchy into nodes of up to W children, level by
// level from the root. Which binary nodes become wide nodes is chosen by the
// surface-area cost below (a pass over the binary tree before the collapse);
// the greedy rule it replaced (open the internal child with the largest box
// surface area until the node holds W children) is kept for comparison
// builds. On the 1M-point office: 285 369 -> 232 866 wide nodes, solve
// 37.2 -> 36.6 ms, results bitwise the same. Children get wide indices in
// level order through an
// exclusive scan of the per-node internal-child counts, so the layout is
// deterministic. Wide node: 7W floats -- lo x[W], lo y[W], lo z[W], hi x[W],
// hi y[W], hi z[W], child refs[W] -- padded to 8W floats (128 B for W = 4,
// 256 B for W = 8). An empty slot holds a point box at 1e30, which no slab
// test over a finite segment accepts, and a one-disk leaf reference.
struct WSlot {
    float b[6];
    int ref;
};

__device__ __forceinline__ float half_area(const float *b) {
    const float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return dx * dy + dy * dz + dz * dx;
}

__device__ __forceinline__ void binary_children(const float4 *__restrict__ bnode, int b, WSlot &c0, WSlot &c1) {
    const float4 *nd = bnode + 4 * (size_t)b;
    const float4 x0 = nd[0], x1 = nd[1], x2 = nd[2], x3 = nd[3];
    c0 = {{x0.x, x0.y, x0.z, x0.w, x1.x, x1.y}, __float_as_int(x3.x)};
    c1 = {{x1.z, x1.w, x2.x, x2.y, x2.z, x2.w}, __float_as_int(x3.y)};
}

// Surface-area cost of the collapse into W-wide nodes, chosen per node
// (the cost-based collapse of Ylitie, Karras and Laine 2017). For a binary
// node n and i = 1..W, C(n, i) is the least expected traversal cost of n's
// subtree when it may take up to i child slots of its wide parent, with A
// the half surface area (a ray's chance of entering a box is proportional to
// it), c_node the cost of one wide node visit (W box tests) and c_disk that of
// one disk test:
//   C1(n) = A(n) c_node + D(n, W)                      n becomes a wide node
//   D(n, j) = min over j_l + j_r = j of C(l, j_l) + C(r, j_r)   n dissolved
//   C(n, 1) = C1(n),  C(n, i) = min(C1(n), D(n, i))     (i >= 2)
//   C(leaf, i) = A(leaf) c_disk |leaf|
// choice[n * W + i - 1] keeps, for i >= 2, the split j_l of D(n, i) in its low
// four bits and whether C(n, i) takes n as one slot in bit 4. The rows are
// filled bottom-up by one thread per node whose children are both leaves; a
// thread climbs while it is the last child to arrive at the parent (atomic
// countdown), and stops where the parent does not reference the node (the
// node lies inside a leaf the build collapsed).
constexpr float kSahNode = 1.0f, kSahDisk = 0.4f;  // a node step costs about 2.5 disk tests (4-wide any-hit walk)

__global__ void k_sah_pending(const float4 *__restrict__ bnode, uint32_t ni, uint32_t *pending) {
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= ni) return;
    const float4 r = bnode[4 * (size_t)n + 3];
    pending[n] = (__float_as_int(r.x) >= 0) + (__float_as_int(r.y) >= 0);
}

template <int W>
__global__ void k_sah_rows(const float4 *__restrict__ bnode, const int *__restrict__ parent, uint32_t ni,
                           uint32_t *pending, float *cost, uint8_t *choice) {
    const uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 >= ni) return;
    int n = (int)i0;
    {
        const float4 r = bnode[4 * (size_t)n + 3];
        if (__float_as_int(r.x) >= 0 || __float_as_int(r.y) >= 0) return;
    }
    for (;;) {
        WSlot c[2];
        binary_children(bnode, n, c[0], c[1]);
        float row[2][W];
        for (int s = 0; s < 2; ++s) {
            if (c[s].ref < 0) {
                const int v = -1 - c[s].ref;
                const float leaf = half_area(c[s].b) * kSahDisk * (float)((v & 7) + 1);
                for (int i = 0; i < W; ++i) row[s][i] = leaf;
            } else {
                const volatile float *cr = cost + (size_t)c[s].ref * W;
                for (int i = 0; i < W; ++i) row[s][i] = cr[i];
            }
        }
        float d[W + 1];
        uint8_t split[W + 1];
        for (int j = 2; j <= W; ++j) {
            d[j] = INFINITY;
            split[j] = 1;
            for (int jl = 1; jl < j; ++jl) {
                const float v = row[0][jl - 1] + row[1][j - jl - 1];
                if (v < d[j]) {
                    d[j] = v;
                    split[j] = (uint8_t)jl;
                }
            }
        }
        float lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(c[0].b[a], c[1].b[a]);
            hi[a] = fmaxf(c[0].b[3 + a], c[1].b[3 + a]);
        }
        const float box[6] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]};
        const float c1 = half_area(box) * kSahNode + d[W];
        volatile float *out = cost + (size_t)n * W;
        volatile uint8_t *ch = choice + (size_t)n * W;
        out[0] = c1;
        ch[0] = 0;
        for (int i = 2; i <= W; ++i) {
            const bool single = c1 <= d[i];
            out[i - 1] = single ? c1 : d[i];
            ch[i - 1] = (uint8_t)(split[i] | (single ? 16 : 0));
        }
        __threadfence();
        const int p = parent[n];
        if (p < 0) return;
        const float4 pr = bnode[4 * (size_t)p + 3];
        if (__float_as_int(pr.x) != n && __float_as_int(pr.y) != n) return;  // inside a collapsed leaf
        if (atomicSub(&pending[p], 1u) != 1u) return;  // the other child is not done yet
        __threadfence();
        n = p;
    }
}

// The children of the wide node standing for binary node b, by the choices
// above: b is dissolved into W slots; a child given j slots takes one if it
// is a leaf, if j = 1 or if its row says so, else it is dissolved in turn.
template <int W>
__device__ int wide_children_sah(const float4 *__restrict__ bnode, const uint8_t *__restrict__ choice, int b,
                                 WSlot *sl) {
    int st_n[W], st_j[W];
    int sp = 0, cnt = 0;
    st_n[sp] = b;
    st_j[sp++] = W;
    while (sp > 0) {
        --sp;
        const int n = st_n[sp], j = st_j[sp];
        WSlot c[2];
        binary_children(bnode, n, c[0], c[1]);
        const int jl = choice[(size_t)n * W + j - 1] & 15;
        const int js[2] = {jl, j - jl};
        for (int s = 0; s < 2; ++s) {
            if (c[s].ref < 0 || js[s] == 1 || (choice[(size_t)c[s].ref * W + js[s] - 1] & 16)) {
                sl[cnt++] = c[s];
            } else {
                st_n[sp] = c[s].ref;
                st_j[sp++] = js[s];
            }
        }
    }
    return cnt;
}

template <int W>
__device__ int wide_children(const float4 *__restrict__ bnode, int b, WSlot *sl) {
    binary_children(bnode, b, sl[0], sl[1]);
    int cnt = 2;
    while (cnt < W) {
        int best = -1;
        float ba = -1.f;
        for (int j = 0; j < cnt; ++j)
            if (sl[j].ref >= 0) {
                const float ar = half_area(sl[j].b);
                if (ar > ba) {
                    ba = ar;
                    best = j;
                }
            }
        if (best < 0) break;
        WSlot c0, c1;
        binary_children(bnode, sl[best].ref, c0, c1);
        sl[best] = c0;
        sl[cnt++] = c1;
    }
    return cnt;
}

template <int W>
__global__ void k_wide_count(const float4 *__restrict__ bnode, const uint8_t *__restrict__ choice,
                             const int *__restrict__ frontier, uint32_t nf, uint32_t *__restrict__ cnt) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    WSlot sl[W];
    const int c = choice ? wide_children_sah<W>(bnode, choice, frontier[i], sl) : wide_children<W>(bnode, frontier[i], sl);
    uint32_t k = 0;
    for (int j = 0; j < c; ++j) k += sl[j].ref >= 0;
    cnt[i] = k;
}

template <int W>
__global__ void k_wide_emit(const float4 *__restrict__ bnode, const uint8_t *__restrict__ choice,
                            const int *__restrict__ frontier, uint32_t nf, const uint32_t *__restrict__ pos,
                            uint32_t base_cur, uint32_t base_next, int *__restrict__ next, float *__restrict__ wnode) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    WSlot sl[W];
    const int c = choice ? wide_children_sah<W>(bnode, choice, frontier[i], sl) : wide_children<W>(bnode, frontier[i], sl);
    float *o = wnode + (size_t)(base_cur + i) * 8 * W;
    uint32_t k = pos[i];
    for (int j = 0; j < W; ++j) {
        int ref = leaf_ref(0, 1);
        float bx[6] = {1e30f, 1e30f, 1e30f, 1e30f, 1e30f, 1e30f};
        if (j < c) {
            for (int a = 0; a < 6; ++a) bx[a] = sl[j].b[a];
            ref = sl[j].ref;
            if (ref >= 0) {
                next[k] = ref;
                ref = (int)(base_next + k);
                ++k;
            }
        }
        for (int a = 0; a < 6; ++a) o[a * W + j] = bx[a];
        o[6 * W + j] = __int_as_float(ref);
        o[7 * W + j] = 0.f;
    }
}

// Compact copy of the wide nodes for the any-hit walks (layout and error
// bound at wide_hits): per axis, the grid step is the power of two 2^e with
// 2^e >= the node's extent / 2040 and >= 2^-19 times its largest coordinate
// (so the origin's rounding stays below 1/16 step); the origin is the largest
// float at or below lo - 2^e; lower planes round down, upper planes up (in
// FP64, where these differences and quotients are exact). Coordinates then
// lie in 1..2042. Empty slots get lo = 2047, hi = 0 on every axis, a box no
// segment enters. The node is written in eight copies, one per direction
// octant (copy o: bit a set for a negative direction component on axis a),
// the near plane rows first: lo rows on positive axes, hi rows on negative
// ones.
template <int W>
__global__ void k_wide_quant(const float *__restrict__ wnode, uint32_t n_nodes, float4 *__restrict__ qnode,
                             int *__restrict__ qref) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    const float *o = wnode + (size_t)i * 8 * W;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int j = 0; j < W; ++j) {
        if (!(o[j] < 1e30f)) continue;  // empty slot
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], o[a * W + j]);
            hi[a] = fmaxf(hi[a], o[(3 + a) * W + j]);
        }
    }
    float org[3];
    double step[3];
    uint32_t eb = 0;
    for (int a = 0; a < 3; ++a) {
        if (!(lo[a] <= hi[a])) lo[a] = hi[a] = 0.f;  // no child (never for a built node)
        const double ext = (double)hi[a] - (double)lo[a];
        const double m = fmax(fmax(fabs((double)lo[a]), fabs((double)hi[a])), 1.0);
        const double need = fmax(ext / 2040.0, m * 0x1p-19);
        int e;
        frexp(need, &e);  // need < 2^e
        e = max(e, -100);
        step[a] = ldexp(1.0, e);
        const double od = (double)lo[a] - step[a];
        float of = (float)od;
        if ((double)of > od) of = nextafterf(of, -INFINITY);
        org[a] = of;
        eb |= ((uint32_t)e & 0xffu) << (8 * a);
    }
    for (uint32_t oc = 0; oc < 8u; ++oc) {
        char *q = (char *)qnode + ((size_t)oc * n_nodes + i) * (16 + 12 * W);
        *(float4 *)q = make_float4(org[0], org[1], org[2], __uint_as_float(eb));
        _Float16 *rows = (_Float16 *)(q + 16);
        for (int j = 0; j < W; ++j) {
            const bool empty = !(o[j] < 1e30f);
            for (int a = 0; a < 3; ++a) {
                double gl = 2047.0, gh = 0.0;
                if (!empty) {
                    gl = floor(((double)o[a * W + j] - (double)org[a]) / step[a]);
                    gh = ceil(((double)o[(3 + a) * W + j] - (double)org[a]) / step[a]);
                    gl = fmin(fmax(gl, 0.0), 2047.0);
                    gh = fmin(fmax(gh, 0.0), 2047.0);
                }
                const bool neg = (oc >> a) & 1u;  // copy for a negative direction component
                rows[a * W + j] = (_Float16)(neg ? gh : gl);      // near plane first
                rows[(3 + a) * W + j] = (_Float16)(neg ? gl : gh);
            }
            qref[(size_t)i * W + j] = __float_as_int(o[6 * W + j]);
        }
    }
}

SceneLayout scene_layout(uint32_t n, uint32_t width, uint32_t builder, bool dps) {
    Bump b;
    SceneLayout L;
    uint32_t ni = n > 1 ? n - 1 : 1;
    uint32_t blk = cdiv(n, 256);
    L.pos_id = b.take(sizeof(float4) * n);
    L.nrm_id = b.take(sizeof(float4) * n);
    L.disk = b.take(sizeof(float4) * 2 * n);
    L.node = b.take(sizeof(float4) * 4 * (size_t)ni);
    L.stat = b.take(sizeof(uint32_t) * 8);
    L.bounds = b.take(sizeof(float) * 8);
    L.blk_bounds = b.take(sizeof(float) * 6 * blk);
    L.code0 = b.take(sizeof(uint64_t) * n);
    L.code1 = b.take(sizeof(uint64_t) * n);
    L.idx0 = b.take(sizeof(uint32_t) * n);
    L.idx1 = b.take(sizeof(uint32_t) * n);
    L.hist = b.take(sizeof(uint32_t) * radix_hist_words(n));
    L.scan_blk = b.take(sizeof(uint32_t) * scan_blk_words(radix_hist_words(n)));
    L.child = b.take(sizeof(int2) * ni);
    L.range = b.take(sizeof(int2) * ni);
    L.parent_int = b.take(sizeof(int) * ni);
    L.parent_leaf = b.take(sizeof(int) * n);
    L.dbox = b.take(sizeof(float) * 6 * n);
    L.ibox = b.take(sizeof(float) * 6 * ni);
    L.flags = b.take(sizeof(uint32_t) * ni);
    L.width = width;
    L.n_internal = ni;
    L.builder = builder;
    if (builder == kBuildPloc) {
        for (int k = 0; k < 2; ++k) {
            L.cbox[k] = b.take(sizeof(float) * 6 * (size_t)n);
            L.cid[k] = b.take(sizeof(int) * n);
            L.csz[k] = b.take(sizeof(uint32_t) * n);
        }
        L.nn = b.take(sizeof(int) * n);
        L.mflag = b.take(sizeof(uint32_t) * n);
        L.kflag = b.take(sizeof(uint32_t) * n);
        L.pblk = b.take(sizeof(uint32_t) * scan_blk_words(n));
        L.nsize = b.take(sizeof(uint32_t) * ni);
        L.noff = b.take(sizeof(uint32_t) * ni);
        L.leaf_pos = b.take(sizeof(uint32_t) * n);
        L.perm2 = b.take(sizeof(uint32_t) * n);
        L.pleaf2 = b.take(sizeof(int) * n);
    }
    if (width > 2) {  // every wide node stands for a distinct binary internal node
        L.wnode = b.take(sizeof(float) * 8 * width * (size_t)ni);
        L.qnode = b.take((16 + 12 * (size_t)width) * ni * 8);  // one copy per octant
        L.qref = b.take(sizeof(int) * width * (size_t)ni);
        L.front0 = b.take(sizeof(int) * ni);
        L.front1 = b.take(sizeof(int) * ni);
        L.wcnt = b.take(sizeof(uint32_t) * ni);
        L.wblk = b.take(sizeof(uint32_t) * scan_blk_words(ni));
        L.sah_pending = b.take(sizeof(uint32_t) * ni);
        L.sah_cost = b.take(sizeof(float) * width * (size_t)ni);
        L.sah_choice = b.take((size_t)width * ni);
    }
    if (dps) {  // point sets; their sort reuses the build's code / idx / hist buffers
        L.dps_pt = b.take(sizeof(float4) * 2 * (size_t)n);
        L.dps_off = b.take(sizeof(uint32_t) * ((size_t)n + 1));
        L.dps_of = b.take(sizeof(uint32_t) * n);
        L.dps_flag = b.take(sizeof(uint32_t) * n);
        L.dps_blk = b.take(sizeof(uint32_t) * scan_blk_words(n));
        L.dps_stat = b.take(sizeof(uint32_t) * 2);
        L.dps_recv = b.take(sizeof(float4) * n);
    }
    L.total = b.off;
    return L;
}

// Clustering build over the Morton-ordered disk boxes in dbox (n >= 2):
// fills child / parent arrays, renumbers the disks depth-first (perm2,
// pleaf2, range) and returns the root.
hipError_t build_ploc(const SceneLayout &L, char *ws, uint32_t n, const uint32_t *sorted_id, hipStream_t s,
                      int *root) {
    auto P = [&](size_t off) { return ws + off; };
    float *cbox[2] = {(float *)P(L.cbox[0]), (float *)P(L.cbox[1])};
    int *cid[2] = {(int *)P(L.cid[0]), (int *)P(L.cid[1])};
    uint32_t *csz[2] = {(uint32_t *)P(L.csz[0]), (uint32_t *)P(L.csz[1])};
    int *nn = (int *)P(L.nn);
    uint32_t *mflag = (uint32_t *)P(L.mflag), *kflag = (uint32_t *)P(L.kflag), *pblk = (uint32_t *)P(L.pblk);
    uint32_t *nsize = (uint32_t *)P(L.nsize), *noff = (uint32_t *)P(L.noff), *leaf_pos = (uint32_t *)P(L.leaf_pos);
    int2 *child = (int2 *)P(L.child), *range = (int2 *)P(L.range);
    int *pint = (int *)P(L.parent_int), *pleaf = (int *)P(L.parent_leaf);
    hipLaunchKernelGGL(k_ploc_init, dim3(cdiv(n, 256)), dim3(256), 0, s, (const float *)P(L.dbox), n, cbox[0], cid[0],
                       csz[0]);
    std::vector<uint32_t> bases;
    uint32_t m = n, node_base = 0;
    int cur = 0;
    while (m > 1) {
        if (bases.size() >= n) return hipErrorUnknown;  // every pass merges at least one pair
        const uint32_t g = cdiv(m, 256);
        hipLaunchKernelGGL(k_ploc_nn, dim3(g), dim3(256), 0, s, cbox[cur], m, nn);
        hipLaunchKernelGGL(k_ploc_flags, dim3(g), dim3(256), 0, s, nn, m, mflag, kflag);
        exclusive_scan(kflag, m, pblk, s);
        exclusive_scan(mflag, m, pblk, s);  // merge count lands in pblk[cdiv(m, 1024)]
        hipLaunchKernelGGL(k_ploc_apply, dim3(g), dim3(256), 0, s, cbox[cur], cid[cur], csz[cur], nn, m, mflag, kflag,
                           node_base, cbox[cur ^ 1], cid[cur ^ 1], csz[cur ^ 1], child, nsize, pint, pleaf,
                           (float *)P(L.ibox));
        uint32_t merges = 0;
        hipError_t e = hipMemcpyAsync(&merges, pblk + cdiv(m, 1024), sizeof merges, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (merges == 0 || merges > m / 2) return hipErrorUnknown;
        bases.push_back(node_base);
        node_base += merges;
        m -= merges;
        cur ^= 1;
    }
    if (node_base != n - 1) return hipErrorUnknown;
    const int r = (int)(n - 2);
    fill_u32((uint32_t *)pint + r, 0xffffffffu, 1, s);
    fill_u32(noff + r, 0, 1, s);
    for (size_t t = bases.size(); t-- > 0;) {
        const uint32_t lo = bases[t], hi = t + 1 < bases.size() ? bases[t + 1] : node_base;
        hipLaunchKernelGGL(k_dfs_pass, dim3(cdiv(hi - lo, 256)), dim3(256), 0, s, child, nsize, lo, hi, noff, leaf_pos);
    }
    hipLaunchKernelGGL(k_dfs_leaves, dim3(cdiv(n, 256)), dim3(256), 0, s, n, leaf_pos, sorted_id, pleaf,
                       (uint32_t *)P(L.perm2), (int *)P(L.pleaf2));
    hipLaunchKernelGGL(k_dfs_nodes, dim3(cdiv(n - 1, 256)), dim3(256), 0, s, n - 1, leaf_pos, noff, nsize, child,
                       range);
    *root = r;
    return hipGetLastError();
}

// Level-by-level collapse (one scan per level); the host reads each level's
// size, so this synchronises the stream once per level. Host outputs: the
// number of wide levels and of wide nodes.
template <int W>
hipError_t build_wide_w(const SceneLayout &L, char *ws, hipStream_t s, int broot, uint32_t *levels, uint32_t *nodes) {
    const float4 *bnode = (const float4 *)(ws + L.node);
    int *fr[2] = {(int *)(ws + L.front0), (int *)(ws + L.front1)};
    uint32_t *cnt = (uint32_t *)(ws + L.wcnt), *blk = (uint32_t *)(ws + L.wblk);
    float *wnode = (float *)(ws + L.wnode);
    const uint32_t ni = L.n_internal;
    const uint8_t *choice = nullptr;
    if (kSahCollapse) {
        uint32_t *pending = (uint32_t *)(ws + L.sah_pending);
        float *cost = (float *)(ws + L.sah_cost);
        uint8_t *ch = (uint8_t *)(ws + L.sah_choice);
        hipLaunchKernelGGL(k_sah_pending, dim3(cdiv(ni, 256)), dim3(256), 0, s, bnode, ni, pending);
        hipLaunchKernelGGL(k_sah_rows<W>, dim3(cdiv(ni, 256)), dim3(256), 0, s, bnode, (const int *)(ws + L.parent_int),
                           ni, pending, cost, ch);
        choice = ch;
    }
    fill_u32((uint32_t *)fr[0], (uint32_t)broot, 1, s);  // binary root
    uint32_t nf = 1, base = 0, lv = 0;
    while (nf > 0) {
        // every wide node stands for a distinct binary internal node
        if (base + nf > ni || lv >= 128) return hipErrorUnknown;
        const uint32_t g = cdiv(nf, 256);
        hipLaunchKernelGGL(k_wide_count<W>, dim3(g), dim3(256), 0, s, bnode, choice, fr[lv & 1], nf, cnt);
        exclusive_scan(cnt, nf, blk, s);
        hipLaunchKernelGGL(k_wide_emit<W>, dim3(g), dim3(256), 0, s, bnode, choice, fr[lv & 1], nf, cnt, base,
                           base + nf, fr[(lv + 1) & 1], wnode);
        uint32_t total = 0;
        hipError_t e = hipMemcpyAsync(&total, blk + cdiv(nf, 1024), sizeof total, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        base += nf;
        nf = total;
        ++lv;
    }
    *levels = lv;
    *nodes = base;
    hipLaunchKernelGGL(k_wide_quant<W>, dim3(cdiv(base, 256)), dim3(256), 0, s, wnode, base, (float4 *)(ws + L.qnode),
                       (int *)(ws + L.qref));
    return hipGetLastError();
}

hipError_t build_wide(const SceneLayout &L, char *ws, hipStream_t s, int broot, uint32_t *levels, uint32_t *nodes) {
    return L.width == 4 ? build_wide_w<4>(L, ws, s, broot, levels, nodes)
                        : build_wide_w<8>(L, ws, s, broot, levels, nodes);
}

hipError_t build_scene(const float *pos, const float *nrm, const uint16_t *mat, const uint32_t *surf, uint32_t n,
                       float r, uint32_t leaf, char *ws, const SceneLayout &L, hipStream_t s, uint32_t *wide_levels,
                       uint32_t *wide_nodes, int *root) {
    auto P = [&](size_t off) { return ws + off; };
    float4 *pos_id = (float4 *)P(L.pos_id), *nrm_id = (float4 *)P(L.nrm_id);
    uint32_t *stat = (uint32_t *)P(L.stat);
    float *bounds = (float *)P(L.bounds), *blkb = (float *)P(L.blk_bounds);
    uint64_t *c0 = (uint64_t *)P(L.code0), *c1 = (uint64_t *)P(L.code1);
    uint32_t *i0 = (uint32_t *)P(L.idx0), *i1 = (uint32_t *)P(L.idx1);
    uint32_t *hist = (uint32_t *)P(L.hist);
    uint32_t blk = cdiv(n, 256);
    fill_u32(stat, 0, 8, s);
    hipLaunchKernelGGL(k_ingest, dim3(blk), dim3(256), 0, s, pos, nrm, mat, surf, n, pos_id, nrm_id, blkb, stat);
    hipLaunchKernelGGL(k_bounds, dim3(1), dim3(256), 0, s, blkb, blk, bounds);
    hipLaunchKernelGGL(k_morton, dim3(blk), dim3(256), 0, s, pos_id, n, bounds, c0, i0);
    const bool in_tmp = radix_sort_u64(c0, i0, c1, i1, n, 0, 64, hist, (uint32_t *)P(L.scan_blk), s);
    if (in_tmp) {
        std::swap(c0, c1);
        std::swap(i0, i1);
    }
    float *dbox = (float *)P(L.dbox);
    hipLaunchKernelGGL(k_gather, dim3(blk), dim3(256), 0, s, pos_id, nrm_id, i0, n, r, (float4 *)P(L.disk), dbox);
    int broot = 0;
    if (n > 1) {
        int2 *child = (int2 *)P(L.child), *range = (int2 *)P(L.range);
        int *pint = (int *)P(L.parent_int), *pleaf = (int *)P(L.parent_leaf);
        if (L.builder == kBuildPloc) {
            hipError_t e = build_ploc(L, ws, n, i0, s, &broot);
            if (e != hipSuccess) return e;
            // disks and their boxes again, now in depth-first order
            hipLaunchKernelGGL(k_gather, dim3(blk), dim3(256), 0, s, pos_id, nrm_id, (const uint32_t *)P(L.perm2), n, r,
                               (float4 *)P(L.disk), dbox);
            pleaf = (int *)P(L.pleaf2);
        } else {
            hipLaunchKernelGGL(k_karras, dim3(cdiv(n - 1, 256)), dim3(256), 0, s, c0, (int)n, child, range, pint,
                               pleaf);
        }
        if (L.builder == kBuildPloc) {
            hipLaunchKernelGGL(k_node_records, dim3(cdiv(n - 1, 256)), dim3(256), 0, s, (int)(n - 1), (int)leaf,
                               child, range, dbox, (const float *)P(L.ibox), (float4 *)P(L.node));
        } else {
            fill_u32((uint32_t *)P(L.flags), 0, n - 1, s);
            hipLaunchKernelGGL(k_refit, dim3(blk), dim3(256), 0, s, (int)n, (int)leaf, child, range, pint, pleaf,
                               dbox, (float *)P(L.ibox), (uint32_t *)P(L.flags), (float4 *)P(L.node));
        }
        hipLaunchKernelGGL(k_depth, dim3(blk), dim3(256), 0, s, (int)n, pint, pleaf, stat + 3);
    }
    *root = broot;
    *wide_levels = *wide_nodes = 0;
    if (L.width > 2 && n > leaf) {
        hipError_t e = build_wide(L, ws, s, broot, wide_levels, wide_nodes);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace pcrt
