// C ABI of libpcrt: argument checks, workspace planning, launch sequence.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "pcrt.h"

using namespace pcrt;

struct pcrt_scene {
    DevScene dev;
    pcrt_scene_info info;
    char *ws;
    size_t ws_bytes;
    SceneLayout L;
};

namespace {

thread_local std::string g_err;

// Per-stage device timing of the last PCRT_TIMING solve on this thread:
// events around init, trace, keys, refine, diffuse, LOS + combine.
constexpr int kStages = 7;
thread_local hipEvent_t g_ev[kStages + 1];
thread_local bool g_ev_ok = false;
thread_local bool g_ev_used[kStages];

void stage_mark(bool on, int i, hipStream_t s) {
    if (!on) return;
    if (!g_ev_ok) {
        for (auto &e : g_ev) hipEventCreate(&e);
        g_ev_ok = true;
    }
    hipEventRecord(g_ev[i], s);
}

pcrt_status fail(pcrt_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

pcrt_status ok() {
    g_err.clear();
    return PCRT_OK;
}

#define HIP_TRY(x)                                                                            \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) return fail(PCRT_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

uint32_t next_pow2(uint64_t v) {
    uint64_t p = 64;
    while (p < v && p < (1ull << 31)) p <<= 1;
    return (uint32_t)p;
}

uint32_t round_up(uint32_t a, uint32_t b) { return (a + b - 1) / b * b; }

struct Plan {
    SolveDims D;
    SolveLayout L;
    uint32_t cap;
    uint32_t n_trace;
    Thr thr;
    FieldConst fc;
    uint64_t slots_wanted;  // tape slots before the 32-bit check (RECORD only)
};

Thr make_thr(const pcrt_thresholds &t) {
    Thr r;
    r.eps_tie = t.eps_tie > 0 ? t.eps_tie : 1e-4f;
    r.eps_self = t.eps_self > 0 ? t.eps_self : 1e-3f;
    float ta = t.t_a_deg > 0 ? t.t_a_deg : 1.0f;
    r.cos_ta = (float)std::cos((double)ta * kPi / 180.0);
    r.t_d = t.t_d > 0 ? t.t_d : 0.01f;
    r.kappa = t.kappa == PCRT_KAPPA_NONE ? 0 : (t.kappa == 0 ? 10 : (int)t.kappa);
    return r;
}

FieldConst make_fc(double f) {
    FieldConst fc;
    double lam = kC0 / f;
    fc.amp_iso = (float)(lam / (4.0 * kPi));
    double inv = 1.0 / lam;
    fc.inv_lam_hi = (float)inv;
    fc.inv_lam_lo = (float)(inv - (double)fc.inv_lam_hi);
    fc.inv_we0 = (float)(1.0 / (2.0 * kPi * f * kEps0));
    return fc;
}

// Per-item key-table capacity: twice the number of distinct keys possible.
uint32_t key_capacity(uint64_t max_rays, uint32_t K, uint32_t n_surf) {
    double combos = 0, p = 1;
    for (uint32_t k = 1; k <= K; ++k) {
        p *= (double)n_surf;
        combos += p;
    }
    double lim = std::min<double>(combos, (double)max_rays * K);
    return next_pow2((uint64_t)std::min<double>(2.0 * lim + 1, 2147483648.0));
}

pcrt_status check_params(const pcrt_scene *sc, const pcrt_solve_params *p) {
    if (!sc || !p) return fail(PCRT_EINVAL, "scene and params are required");
    if (p->max_interactions < 1 || p->max_interactions > (uint32_t)kMaxK)
        return fail(PCRT_EUNSUPPORTED, "max_interactions must be in 1..%d (got %u)", kMaxK, p->max_interactions);
    if (!(p->freq_hz > 0) || !std::isfinite(p->freq_hz)) return fail(PCRT_EINVAL, "freq_hz must be > 0");
    if (p->n_rx == 0 || !p->rx) return fail(PCRT_EINVAL, "n_rx must be > 0 and rx non-NULL");
    if ((p->flags & (PCRT_SPECULAR | PCRT_DIFFUSE)) && p->n_rays == 0)
        return fail(PCRT_EINVAL, "n_rays must be > 0 with SPECULAR or DIFFUSE");
    if (p->ray_subset && p->n_subset == 0) return fail(PCRT_EINVAL, "n_subset must be > 0 with ray_subset");
    if (!std::isfinite(p->tx[0]) || !std::isfinite(p->tx[1]) || !std::isfinite(p->tx[2]))
        return fail(PCRT_EINVAL, "tx must be finite");
    if (p->flags & PCRT_SPECULAR) {
        double bits = p->max_interactions * std::log2((double)sc->info.n_surfaces + 1.0);
        if (bits >= 63.9)
            return fail(PCRT_EUNSUPPORTED, "(n_surfaces + 1)^K = 2^%.1f: keys do not fit 64 bits", bits);
    }
    uint64_t nt = p->ray_subset ? p->n_subset : p->n_rays;
    if (nt * p->max_interactions > 0x7fffffffull) return fail(PCRT_EUNSUPPORTED, "too many rays x interactions");
    if ((uint64_t)p->n_rx > kMaxPairs) return fail(PCRT_EUNSUPPORTED, "too many receivers");
    if (p->flags & PCRT_POLARIZED) {
        if (p->flags & PCRT_DIFFUSE)
            return fail(PCRT_EUNSUPPORTED, "PCRT_POLARIZED covers line-of-sight and specular paths");
        for (int c = 0; c < 3; ++c)
            if (!std::isfinite(p->pol_tx[c]) || !std::isfinite(p->pol_rx[c]))
                return fail(PCRT_EINVAL, "pol_tx and pol_rx must be finite");
    }
    if ((p->flags & PCRT_AVERAGE) && !sc->dev.dps_pt)
        return fail(PCRT_EINVAL, "PCRT_AVERAGE needs a scene built with dps_voxel > 0");
    if (!(p->lambda_d >= 0.f) || !std::isfinite(p->lambda_d)) return fail(PCRT_EINVAL, "lambda_d must be >= 0");
    if (p->flags & PCRT_DPS_LAUNCH) {
        if (!sc->dev.dps_pt) return fail(PCRT_EINVAL, "PCRT_DPS_LAUNCH needs a scene built with dps_voxel > 0");
        if (p->n_rays != sc->info.n_point_sets) return fail(PCRT_EINVAL, "PCRT_DPS_LAUNCH: n_rays must be n_point_sets");
        if ((p->flags & (PCRT_SPECULAR | PCRT_DIFFUSE)) && !p->dps_vis)
            return fail(PCRT_EINVAL, "PCRT_DPS_LAUNCH needs dps_vis");
        if (p->flags & PCRT_DIFFUSE) {
            double bits = (p->max_interactions - 1) * std::log2((double)sc->info.n_surfaces + 1.0) +
                          std::log2((double)sc->info.n_point_sets + 1.0);
            if (bits >= 63.0) return fail(PCRT_EUNSUPPORTED, "voxel diffuse keys do not fit 64 bits");
        }
    }
    return PCRT_OK;
}

// Transmitters of a solve: one for pcrt_solve, many for pcrt_solve_batch.
// Ray slots of item i start at ray_off (a multiple of kRayChunk) so that
// reduction chunks never straddle two transmitters.
std::vector<Item> single_items(const pcrt_solve_params *p) {
    Item it;
    memset(&it, 0, sizeof it);
    for (int a = 0; a < 3; ++a) it.tx[a] = p->tx[a];
    it.n_rays = (p->flags & (PCRT_SPECULAR | PCRT_DIFFUSE)) ? (p->ray_subset ? p->n_subset : p->n_rays) : 0;
    it.budget = p->n_rays ? p->n_rays : 1;
    return {it};
}

std::vector<Item> batch_items(const pcrt_solve_params *p, const pcrt_batch_item *b, uint32_t n) {
    std::vector<Item> v(n);
    for (uint32_t i = 0; i < n; ++i) {
        memset(&v[i], 0, sizeof(Item));
        for (int a = 0; a < 3; ++a) v[i].tx[a] = b[i].tx[a];
        v[i].n_rays = (p->flags & (PCRT_SPECULAR | PCRT_DIFFUSE)) ? b[i].n_rays : 0;
        v[i].budget = b[i].n_rays ? b[i].n_rays : 1;
    }
    return v;
}

Plan make_plan(const pcrt_scene *sc, const pcrt_solve_params *p, std::vector<Item> &items) {
    Plan P{};  // every field zero until set
    const uint32_t K = p->max_interactions;
    SolveDims &D = P.D;
    D.K = K;
    D.n_rx = p->n_rx;
    D.n_items = (uint32_t)items.size();
    D.width = sc->info.width;
    uint64_t off = 0, total = 0, max_rays = 0;
    for (auto &it : items) {
        it.ray_off = (uint32_t)off;
        off += (uint64_t)round_up(it.n_rays, kRayChunk);
        total += it.n_rays;
        max_rays = std::max<uint64_t>(max_rays, it.n_rays);
    }
    P.n_trace = (uint32_t)total;
    D.T = (uint32_t)std::max<uint64_t>(off, kRayChunk);
    P.cap = key_capacity(max_rays, K, sc->info.n_surfaces);
    D.max_keys = (uint32_t)std::min<uint64_t>((uint64_t)D.T * K, (uint64_t)P.cap * D.n_items);
    D.max_key_chunks = (D.max_keys + kKeyChunk - 1) / kKeyChunk + D.n_items;
    D.n_ray_chunks = D.T / kRayChunk;
    if (p->flags & PCRT_RECORD) {
        uint32_t want = p->key_capacity ? p->key_capacity : 262144u;
        D.rec_keys = (p->flags & PCRT_SPECULAR) ? std::min(D.max_keys, want) : 0;
        // slot indices are 32-bit in the tape kernels: the count is formed in
        // 64 bits and a plan beyond 2^32 - 1 slots is refused (plan_check)
        P.slots_wanted = (uint64_t)D.T * K + (uint64_t)D.rec_keys * D.n_rx * K;
        D.n_slots = (uint32_t)std::min<uint64_t>(P.slots_wanted, 0xffffffffull);
        D.n_slot_chunks = (uint32_t)((P.slots_wanted + kSlotChunk - 1) / kSlotChunk);
    } else {
        D.rec_keys = D.n_slots = D.n_slot_chunks = 0;
    }
    // every traversal launch indexes the stack spill by its global lane
    const uint32_t wr = p->wave_rays ? p->wave_rays : kWave;
    // the first kStackLds stack entries live in LDS, the rest in the spill area
    // (set first: the diffuse grid depends on whether there is one)
    D.spill_depth = sc->info.stack_entries > (uint32_t)kStackLds ? sc->info.stack_entries - kStackLds : 0;
    D.spill_lanes = std::max({trace_grid(D, wr) * kWave, diffuse_grid(D) * kWave, refine_grid(D) * kWave,
                              round_up(D.n_items * D.n_rx, kWave)});
    P.L = solve_layout(D, p->flags);
    P.thr = make_thr(p->thr);
    P.thr.lambda_d = p->lambda_d > 0.f ? p->lambda_d : 100.f;
    P.fc = make_fc(p->freq_hz);
    return P;
}

Plan make_plan(const pcrt_scene *sc, const pcrt_solve_params *p) {
    std::vector<Item> items = single_items(p);
    return make_plan(sc, p, items);
}

// Limits that depend on the whole plan (checked wherever a plan is used).
pcrt_status plan_check(const Plan &P) {
    if (P.slots_wanted > 0xffffffffull)
        return fail(PCRT_EUNSUPPORTED,
                    "the tape would need %llu interaction slots (at most 2^32 - 1): lower key_capacity, "
                    "receivers or max_interactions",
                    (unsigned long long)P.slots_wanted);
    return PCRT_OK;
}

struct ItemBatch {
    Item it[96];
    uint32_t n, base;
};

__global__ void k_put_items(ItemBatch b, Item *dst) {
    uint32_t i = threadIdx.x;
    if (i < b.n) dst[b.base + i] = b.it[i];
}

__global__ void k_copy_seq(const int *id, uint32_t n, int32_t *out) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = id[i];
}

LaunchArgs make_args(const pcrt_scene *sc, const pcrt_material *mats, uint32_t n_labels, const pcrt_solve_params *p,
                     const Plan &P, char *ws, uint64_t *counters) {
    LaunchArgs A;
    memset(&A, 0, sizeof A);
    const SolveLayout &L = P.L;
    auto at = [&](size_t off) { return (void *)(ws + off); };
    A.S = sc->dev;
    A.S.spill = (int *)at(L.spill);
    A.S.spill_lanes = P.D.spill_lanes;
    A.items = (const Item *)at(L.items);
    A.subset = p->ray_subset;
    A.rx = p->rx;
    A.mats = (const float *)mats;
    A.n_labels = n_labels;
    A.n_surf1 = sc->info.n_surfaces + 1;
    A.flags = p->flags;
    if (p->flags & PCRT_POLARIZED) {
        A.pol_tx = {p->pol_tx[0], p->pol_tx[1], p->pol_tx[2]};
        A.pol_rx = {p->pol_rx[0], p->pol_rx[1], p->pol_rx[2]};
    }
    A.dps_vis = (p->flags & PCRT_DPS_LAUNCH) ? p->dps_vis : nullptr;
    if ((p->flags & PCRT_DPS_LAUNCH) && (p->flags & PCRT_DIFFUSE)) {
        A.rb.dslot = (uint32_t *)at(L.rec_dslot);
        A.dhb.key = (unsigned long long *)at(L.dhkey);
        A.dhb.rep = (uint32_t *)at(L.dhrep);
        A.dhb.cap = dps_key_cap(P.D);
        A.dkeylist = (uint32_t *)at(L.dkeylist);
        A.dkey_off = (uint32_t *)at(L.dkey_off);
        A.dchunk_off = (uint32_t *)at(L.dchunk_off);
        A.dcnt = (uint64_t *)at(L.dcnt);
    }
    A.thr = P.thr;
    A.fc = P.fc;
    A.D = P.D;
    A.wave_rays = p->wave_rays ? p->wave_rays : kWave;
    A.rb.id = (int *)at(L.rec_id);
    A.rb.xl = (float4 *)at(L.rec_xl);
    A.rb.cs = (float *)at(L.rec_cs);
    A.rb.coef = (p->flags & PCRT_DIFFUSE) ? (float4 *)at(L.rec_coef) : nullptr;
    A.rb.slot = (p->flags & PCRT_SPECULAR) ? (uint32_t *)at(L.rec_slot) : nullptr;
    A.rb.nk = (p->flags & PCRT_AVERAGE) ? (float4 *)at(L.rec_nk) : nullptr;
    A.hb.key = (unsigned long long *)at(L.hkey);
    A.hb.rep = (uint32_t *)at(L.hrep);
    A.hb.cap = P.cap;
    if ((p->flags & PCRT_RECORD) && (p->flags & PCRT_SPECULAR)) {
        A.sb.valid = (uint8_t *)at(L.sp_valid);
        A.sb.len = (float *)at(L.sp_len);
        A.sb.amp = (float4 *)at(L.sp_amp);
        A.sb.hit = (int *)at(L.sp_hit);
        A.sb.cs = (float *)at(L.sp_cs);
    }
    A.work = (uint32_t *)at(L.work);
    A.counters = counters ? counters : (uint64_t *)at(L.counters);
    A.scan = (uint32_t *)at(L.scan);
    A.scan_blk = (uint32_t *)at(L.scan_blk);
    A.keylist = (uint32_t *)at(L.keylist);
    A.key_off = (uint32_t *)at(L.key_off);
    A.chunk_off = (uint32_t *)at(L.chunk_off);
    A.spec_part = (double *)at(L.spec_part);
    A.spec_res = (p->flags & PCRT_SPECULAR) ? (float4 *)at(L.spec_res) : nullptr;
    A.spec_ovr = ((p->flags & PCRT_SPECULAR) && (p->flags & PCRT_AVERAGE)) ? (float4 *)at(L.spec_ovr) : nullptr;
    A.diff_part = (double *)at(L.diff_part);
    A.los_part = (double *)at(L.los_part);
    A.dvis = ((p->flags & PCRT_RECORD) && (p->flags & PCRT_DIFFUSE) && !(p->flags & PCRT_DPS_LAUNCH))
                 ? (uint8_t *)at(L.dvis)
                 : nullptr;
    A.dps_area = sc->info.dps_voxel * sc->info.dps_voxel;
    if (p->flags & PCRT_DIFFUSE) {
        A.dsort.key0 = (uint64_t *)at(L.dkey0);
        A.dsort.key1 = (uint64_t *)at(L.dkey1);
        A.dsort.val0 = (uint32_t *)at(L.dval0);
        A.dsort.val1 = (uint32_t *)at(L.dval1);
        A.dsort.hist = (uint32_t *)at(L.dhist);
        A.dsort.blk = (uint32_t *)at(L.dblk);
        A.dsort.pack = (float4 *)at(L.dpack);
    }
    if (p->flags & PCRT_RECORD) {
        A.slot_label = (uint16_t *)at(L.slot_label);
        A.slot_cos = (float *)at(L.slot_cos);
        A.slot_coef = (float *)at(L.slot_coef);
        A.slot_adj = (float *)at(L.slot_adj);
        A.grad_part = (double *)at(L.grad_part);
    }
    return A;
}

}  // namespace

namespace pcrt {
SolveLayout solve_layout(const SolveDims &D, uint32_t flags) {
    Bump b;
    SolveLayout L;
    memset(&L, 0, sizeof L);
    const size_t nrec = (size_t)D.T * D.K;
    const bool spec = flags & PCRT_SPECULAR, diff = flags & PCRT_DIFFUSE, rec = flags & PCRT_RECORD;
    L.items = b.take(sizeof(Item) * D.n_items);
    L.counters = b.take(sizeof(uint64_t) * PCRT_CNT_COUNT);
    L.work = b.take(sizeof(uint32_t) * kWorkWords);
    L.rec_id = b.take(sizeof(int) * nrec);
    L.rec_xl = b.take(sizeof(float4) * nrec);
    L.rec_cs = b.take(sizeof(float) * nrec);
    if (flags & PCRT_AVERAGE) L.rec_nk = b.take(sizeof(float4) * nrec);
    L.key_off = b.take(sizeof(uint32_t) * (D.n_items + 1));
    L.chunk_off = b.take(sizeof(uint32_t) * (D.n_items + 1));
    L.los_part = b.take(sizeof(double) * 5 * (size_t)D.n_items * D.n_rx);
    if (diff) {
        L.dkey0 = b.take(sizeof(uint64_t) * nrec);
        L.dkey1 = b.take(sizeof(uint64_t) * nrec);
        L.dval0 = b.take(sizeof(uint32_t) * nrec);
        L.dval1 = b.take(sizeof(uint32_t) * nrec);
        L.dhist = b.take(sizeof(uint32_t) * radix_hist_words((uint32_t)nrec));
        L.dblk = b.take(sizeof(uint32_t) * scan_blk_words(radix_hist_words((uint32_t)nrec)));
        L.rec_coef = b.take(sizeof(float4) * nrec);
        L.dpack = b.take(2 * sizeof(float4) * nrec);
        L.diff_part = b.take(sizeof(double) * 5 * (size_t)D.n_ray_chunks * D.n_rx);
        if (rec && !(flags & PCRT_DPS_LAUNCH)) L.dvis = b.take(nrec * D.n_rx);  // ray-tube connections only
        if (flags & PCRT_DPS_LAUNCH) {  // voxel diffuse keys of the reception-point launch
            const size_t cap = dps_key_cap(D);
            L.rec_dslot = b.take(sizeof(uint32_t) * nrec);
            L.dhkey = b.take(sizeof(uint64_t) * cap);
            L.dhrep = b.take(sizeof(uint32_t) * cap);
            L.dkeylist = b.take(sizeof(uint32_t) * nrec);
            L.dkey_off = b.take(sizeof(uint32_t) * (D.n_items + 1));
            L.dchunk_off = b.take(sizeof(uint32_t) * (D.n_items + 1));
            L.dcnt = b.take(sizeof(uint64_t) * PCRT_CNT_COUNT);
            if (!spec) {  // the compaction's scan buffers
                L.scan = b.take(sizeof(uint32_t) * nrec);
                L.scan_blk = b.take(sizeof(uint32_t) * ((nrec + 1023) / 1024 + 1));
            }
        }
    }
    if (spec) {
        L.rec_slot = b.take(sizeof(uint32_t) * nrec);
        L.scan = b.take(sizeof(uint32_t) * nrec);
        L.scan_blk = b.take(sizeof(uint32_t) * ((nrec + 1023) / 1024 + 1));
        L.keylist = b.take(sizeof(uint32_t) * D.max_keys);
        L.spec_part = b.take(sizeof(double) * 5 * (size_t)D.max_key_chunks * D.n_rx);
        L.spec_res = b.take(sizeof(float4) * (size_t)refine_grid(D) * kRefineResPerBlock);
        if (flags & PCRT_AVERAGE) L.spec_ovr = b.take(sizeof(float4) * 2 * (size_t)refine_grid(D) * kRefineQueue * D.K);
        if (rec) {
            const size_t pairs = (size_t)D.rec_keys * D.n_rx;
            L.sp_valid = b.take(pairs);
            L.sp_len = b.take(sizeof(float) * pairs);
            L.sp_amp = b.take(sizeof(float4) * pairs);
            L.sp_hit = b.take(sizeof(int) * pairs * D.K);
            L.sp_cs = b.take(sizeof(float) * pairs * D.K);
        }
    }
    if (rec) {
        L.slot_label = b.take(sizeof(uint16_t) * (size_t)D.n_slots);
        L.slot_cos = b.take(sizeof(float) * (size_t)D.n_slots);
        L.slot_coef = b.take(sizeof(float) * 8 * (size_t)D.n_slots);
        L.slot_adj = b.take(sizeof(float) * 8 * (size_t)D.n_slots);
        L.grad_part = b.take(sizeof(double) * 3 * kMaxGradLabels * (size_t)std::max<uint32_t>(D.n_slot_chunks, 1));
    }
    L.spill = b.take(sizeof(int) * (size_t)D.spill_depth * D.spill_lanes);
    L.total = b.off;
    return L;
}
}  // namespace pcrt

// Hash-table sizes depend on the key capacity, which the layout does not
// know; they are appended after the common layout.
static size_t hash_bytes(const Plan &P, uint32_t flags) {
    if (!(flags & PCRT_SPECULAR)) return 0;
    size_t slots = (size_t)P.cap * P.D.n_items;
    return ((sizeof(uint64_t) * slots + 255) & ~size_t(255)) + ((sizeof(uint32_t) * slots + 255) & ~size_t(255));
}

static void place_hash(Plan &P, uint32_t flags) {
    if (!(flags & PCRT_SPECULAR)) {
        P.L.hkey = P.L.hrep = 0;
        return;
    }
    size_t slots = (size_t)P.cap * P.D.n_items;
    P.L.hkey = P.L.total;
    P.L.hrep = P.L.total + ((sizeof(uint64_t) * slots + 255) & ~size_t(255));
    P.L.total += hash_bytes(P, flags);
}

extern "C" {

const char *pcrt_last_error(void) { return g_err.c_str(); }
const char *pcrt_version(void) { return "pcrt 0.1 (gfx950)"; }

pcrt_status pcrt_scene_workspace_size(uint32_t n_points, const pcrt_bvh_opts *opts, size_t *bytes) {
    if (!bytes) return fail(PCRT_EINVAL, "bytes is NULL");
    if (n_points == 0) return fail(PCRT_EINVAL, "n_points must be > 0");
    if (n_points > (1u << 26)) return fail(PCRT_EUNSUPPORTED, "at most 2^26 points");
    const uint32_t width = opts && opts->width ? opts->width : kDefaultWidth;
    if (width != 2 && width != 4 && width != 8) return fail(PCRT_EUNSUPPORTED, "width must be 2, 4 or 8");
    if (opts && opts->leaf_size > 8) return fail(PCRT_EUNSUPPORTED, "leaf_size must be in 1..8");
    const uint32_t builder = opts && opts->builder ? opts->builder : kDefaultBuilder;
    if (builder != kBuildLbvh && builder != kBuildPloc) return fail(PCRT_EUNSUPPORTED, "builder must be 1 or 2");
    const bool dps = opts && opts->dps_voxel > 0.f;
    *bytes = scene_layout(n_points, width, builder, dps).total;
    return ok();
}

pcrt_status pcrt_scene_create(const pcrt_points *pts, const pcrt_bvh_opts *opts, void *ws, size_t ws_bytes,
                              void *stream, pcrt_scene **out) {
    if (!pts || !out || !ws) return fail(PCRT_EINVAL, "pts, ws and out are required");
    if (!pts->pos || !pts->normal || !pts->material || !pts->surface)
        return fail(PCRT_EINVAL, "point arrays must be non-NULL");
    if (pts->n_points == 0) return fail(PCRT_EINVAL, "n_points must be > 0");
    if (pts->n_points > (1u << 26)) return fail(PCRT_EUNSUPPORTED, "at most 2^26 points");
    if (!(pts->disk_radius > 0.f) || !std::isfinite(pts->disk_radius))
        return fail(PCRT_EINVAL, "disk_radius must be > 0");
    uint32_t leaf = opts && opts->leaf_size ? opts->leaf_size : 4;
    if (leaf < 1 || leaf > 8) return fail(PCRT_EUNSUPPORTED, "leaf_size must be in 1..8");
    const uint32_t width = opts && opts->width ? opts->width : kDefaultWidth;
    if (width != 2 && width != 4 && width != 8) return fail(PCRT_EUNSUPPORTED, "width must be 2, 4 or 8");
    const uint32_t builder = opts && opts->builder ? opts->builder : kDefaultBuilder;
    if (builder != kBuildLbvh && builder != kBuildPloc) return fail(PCRT_EUNSUPPORTED, "builder must be 1 or 2");
    const float rho = opts ? opts->dps_voxel : 0.f;
    if (!(rho >= 0.f) || !std::isfinite(rho)) return fail(PCRT_EINVAL, "dps_voxel must be finite and >= 0");
    SceneLayout L = scene_layout(pts->n_points, width, builder, rho > 0.f);
    if (ws_bytes < L.total) return fail(PCRT_ENOMEM, "scene workspace too small: need %zu bytes", L.total);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s));
    uint32_t wide_levels = 0, wide_nodes = 0;
    int broot = 0;
    HIP_TRY(build_scene(pts->pos, pts->normal, pts->material, pts->surface, pts->n_points, pts->disk_radius, leaf,
                        (char *)ws, L, s, &wide_levels, &wide_nodes, &broot));
    if (rho > 0.f) HIP_TRY(build_point_sets(L, (char *)ws, pts->n_points, rho, s));
    HIP_TRY(hipEventRecord(e1, s));
    uint32_t stat[8], dstat[2] = {0, 0};
    float bounds[6];
    HIP_TRY(hipMemcpyAsync(stat, (char *)ws + L.stat, sizeof stat, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(bounds, (char *)ws + L.bounds, sizeof bounds, hipMemcpyDeviceToHost, s));
    if (rho > 0.f) HIP_TRY(hipMemcpyAsync(dstat, (char *)ws + L.dps_stat, sizeof dstat, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (stat[0] & 1) return fail(PCRT_EINVAL, "non-finite point position");
    if (stat[0] & 2) return fail(PCRT_EINVAL, "zero or non-finite normal");
    if (dstat[0] & 1) return fail(PCRT_EUNSUPPORTED, "voxel index beyond +-2^20 (dps_voxel too small for the scene)");
    // a depth-first walk holds at most (width - 1) entries per level of its path
    const uint32_t n_pts = pts->n_points;
    const uint32_t stack_entries = n_pts <= leaf ? 0 : width == 2 ? stat[3] : (width - 1) * wide_levels;
    if (stack_entries > (uint32_t)kStackMax)
        return fail(PCRT_EUNSUPPORTED, "hierarchy needs %u traversal stack entries (at most %d)", stack_entries,
                    kStackMax);
    pcrt_scene *sc = new pcrt_scene;
    memset(sc, 0, sizeof *sc);
    sc->ws = (char *)ws;
    sc->ws_bytes = ws_bytes;
    sc->L = L;
    const uint32_t n = pts->n_points;
    sc->dev.node = (const float4 *)(sc->ws + (width > 2 ? L.wnode : L.node));
    sc->dev.width = (int)width;
    if (width > 2) {
        sc->dev.qnode = (const float4 *)(sc->ws + L.qnode);
        sc->dev.qref = (const int *)(sc->ws + L.qref);
        sc->dev.qstride = (uint32_t)((16 + 12 * width) * wide_nodes);
    }
    sc->dev.disk = (const float4 *)(sc->ws + L.disk);
    sc->dev.pos = (const float4 *)(sc->ws + L.pos_id);
    sc->dev.nrm = (const float4 *)(sc->ws + L.nrm_id);
    sc->dev.bounds = (const float *)(sc->ws + L.bounds);
    sc->dev.r2 = pts->disk_radius * pts->disk_radius;
    sc->dev.n = n;
    if (rho > 0.f) {
        sc->dev.dps_pt = (const float4 *)(sc->ws + L.dps_pt);
        sc->dev.dps_off = (const uint32_t *)(sc->ws + L.dps_off);
        sc->dev.dps_of = (const uint32_t *)(sc->ws + L.dps_of);
        sc->dev.dps_recv = (const float4 *)(sc->ws + L.dps_recv);
        sc->dev.n_sets = dstat[1];
    }
    // the wide hierarchy's root is node 0; the binary root is the builder's
    sc->dev.root = n == 1 ? leaf_ref(0, 1) : (n <= leaf ? leaf_ref(0, (int)n) : (width > 2 ? 0 : broot));
    pcrt_scene_info &I = sc->info;
    I.n_points = n;
    I.n_surfaces = stat[1] + 1;
    I.n_materials = stat[2] + 1;
    I.depth = stat[3];
    I.n_nodes = n <= leaf ? 0 : width == 2 ? n - 1 : wide_nodes;
    I.leaf_size = leaf;
    I.width = width;
    I.stack_entries = stack_entries;
    I.builder = builder;
    memcpy(I.bbox, bounds, sizeof bounds);
    I.build_ms = ms;
    I.n_point_sets = dstat[1];
    I.dps_voxel = rho;
    *out = sc;
    return ok();
}

static size_t visibility_spill_bytes(const pcrt_scene *sc) {
    const uint32_t depth = sc->info.stack_entries > (uint32_t)kStackLds ? sc->info.stack_entries - kStackLds : 0;
    return sizeof(int) * (size_t)depth * visibility_grid(sc->info.width) * kWave;
}

pcrt_status pcrt_visibility_workspace_size(const pcrt_scene *scene, size_t *bytes) {
    if (!scene || !bytes) return fail(PCRT_EINVAL, "scene and bytes are required");
    *bytes = std::max<size_t>(256, visibility_spill_bytes(scene));
    return ok();
}

pcrt_status pcrt_visibility(const pcrt_scene *scene, const float *rx, uint32_t n_rx, float eps_self, void *ws,
                            size_t ws_bytes, uint8_t *vis, void *stream) {
    if (!scene || !rx || !vis || !ws) return fail(PCRT_EINVAL, "scene, rx, ws and vis are required");
    if (!scene->dev.dps_pt) return fail(PCRT_EINVAL, "the scene has no point sets (dps_voxel = 0)");
    if (n_rx == 0) return fail(PCRT_EINVAL, "n_rx must be > 0");
    if (!(eps_self >= 0.f) || !std::isfinite(eps_self)) return fail(PCRT_EINVAL, "eps_self must be >= 0");
    const size_t need = std::max<size_t>(256, visibility_spill_bytes(scene));
    if (ws_bytes < need) return fail(PCRT_ENOMEM, "visibility workspace too small: need %zu bytes", need);
    if ((uint64_t)n_rx * scene->info.n_point_sets > 0xffffffffull)
        return fail(PCRT_EUNSUPPORTED, "n_rx x point sets must stay below 2^32");
    DevScene S = scene->dev;
    S.spill = (int *)ws;
    S.spill_lanes = visibility_grid(scene->info.width) * kWave;
    launch_visibility(S, rx, n_rx, (const float4 *)(scene->ws + scene->L.dps_recv), scene->info.n_point_sets,
                      eps_self > 0.f ? eps_self : 1e-3f, vis, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return ok();
}

static size_t diffraction_ws(const pcrt_scene *sc, uint32_t n_edges, uint32_t n_rx, size_t *spill) {
    const uint32_t depth = sc->info.stack_entries > (uint32_t)kStackLds ? sc->info.stack_entries - kStackLds : 0;
    *spill = ((sizeof(int) * (size_t)depth * diffraction_blocks(n_edges, n_rx) * kWave) + 255) & ~size_t(255);
    return *spill + sizeof(float4) * (size_t)n_edges * n_rx;
}

pcrt_status pcrt_diffraction_workspace_size(const pcrt_scene *scene, uint32_t n_edges, uint32_t n_rx, size_t *bytes) {
    if (!scene || !bytes) return fail(PCRT_EINVAL, "scene and bytes are required");
    if (n_edges == 0 || n_rx == 0) return fail(PCRT_EINVAL, "n_edges and n_rx must be > 0");
    if ((uint64_t)n_edges * n_rx > (1ull << 30)) return fail(PCRT_EUNSUPPORTED, "at most 2^30 (edge, receiver) pairs");
    size_t spill;
    *bytes = diffraction_ws(scene, n_edges, n_rx, &spill);
    return ok();
}

}  // extern "C"

static pcrt_status check_diffraction(const pcrt_scene *scene, const pcrt_edge *edges, uint32_t n_edges,
                                     const pcrt_material *mats, uint32_t n_labels, const float tx[3], const float *rx,
                                     uint32_t n_rx, double freq_hz, float eps_self, const double *out) {
    if (!scene || !edges || !mats || !tx || !rx || !out)
        return fail(PCRT_EINVAL, "scene, edges, mats, tx, rx, ws and out are required");
    if (n_edges == 0 || n_rx == 0 || n_labels == 0) return fail(PCRT_EINVAL, "n_edges, n_rx and n_labels must be > 0");
    if ((uint64_t)n_edges * n_rx > (1ull << 30)) return fail(PCRT_EUNSUPPORTED, "at most 2^30 (edge, receiver) pairs");
    if (!(freq_hz > 0) || !std::isfinite(freq_hz)) return fail(PCRT_EINVAL, "freq_hz must be > 0");
    if (!(eps_self >= 0.f) || !std::isfinite(eps_self)) return fail(PCRT_EINVAL, "eps_self must be >= 0");
    if (!std::isfinite(tx[0]) || !std::isfinite(tx[1]) || !std::isfinite(tx[2])) return fail(PCRT_EINVAL, "tx must be finite");
    return PCRT_OK;
}

// ws holds the traversal stack spill, then (unless the caller takes the
// per-pair amplitudes in pair_amp) the amplitudes; spill bytes come first.
static pcrt_status diffraction_impl(const pcrt_scene *scene, const pcrt_edge *edges, uint32_t n_edges,
                                    const pcrt_material *mats, uint32_t n_labels, const float tx[3], const float *rx,
                                    uint32_t n_rx, double freq_hz, float eps_self, char *ws, size_t spill,
                                    double *out, float *pair_amp, hipStream_t stream) {
    DevScene S = scene->dev;
    S.spill = (int *)ws;
    S.spill_lanes = diffraction_blocks(n_edges, n_rx) * kWave;
    float4 *amp = pair_amp ? (float4 *)pair_amp : (float4 *)(ws + spill);
    launch_diffraction(S, edges, n_edges, (const float *)mats, n_labels, tx, rx, n_rx, freq_hz,
                       eps_self > 0.f ? eps_self : 1e-3f, amp, out, stream);
    HIP_TRY(hipGetLastError());
    return ok();
}

// Scratch of pcrt_diffraction_noalloc: one array per device, in the code
// object, so that call allocates nothing. Host code never uses the array's
// name as an address: the device address is looked up once per device.
static constexpr size_t kNoallocScratch = 16u << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratch];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static pcrt_status scratch_ptr(char **p) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PCRT_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(PCRT_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *p = (char *)g_scratch_ptr[dev];
    return PCRT_OK;
}

extern "C" {

pcrt_status pcrt_diffraction(const pcrt_scene *scene, const pcrt_edge *edges, uint32_t n_edges,
                             const pcrt_material *mats, uint32_t n_labels, const float tx[3], const float *rx,
                             uint32_t n_rx, double freq_hz, float eps_self, void *ws, size_t ws_bytes, double *out,
                             float *pair_amp, void *stream) {
    pcrt_status st = check_diffraction(scene, edges, n_edges, mats, n_labels, tx, rx, n_rx, freq_hz, eps_self, out);
    if (st) return st;
    if (!ws) return fail(PCRT_EINVAL, "scene, edges, mats, tx, rx, ws and out are required");
    size_t spill;
    const size_t need = diffraction_ws(scene, n_edges, n_rx, &spill);
    if (ws_bytes < need) return fail(PCRT_ENOMEM, "diffraction workspace too small: need %zu bytes", need);
    return diffraction_impl(scene, edges, n_edges, mats, n_labels, tx, rx, n_rx, freq_hz, eps_self, (char *)ws, spill,
                            out, pair_amp, (hipStream_t)stream);
}

pcrt_status pcrt_diffraction_noalloc(const pcrt_scene *scene, const pcrt_edge *edges, uint32_t n_edges,
                                     const pcrt_material *mats, uint32_t n_labels, const float tx[3], const float *rx,
                                     uint32_t n_rx, double freq_hz, float eps_self, double *out, float *pair_amp,
                                     void *stream) {
    pcrt_status st = check_diffraction(scene, edges, n_edges, mats, n_labels, tx, rx, n_rx, freq_hz, eps_self, out);
    if (st) return st;
    size_t spill;
    const size_t full = diffraction_ws(scene, n_edges, n_rx, &spill);
    const size_t need = pair_amp ? spill : full;
    if (need > kNoallocScratch)
        return fail(PCRT_EUNSUPPORTED,
                    "pcrt_diffraction_noalloc: %zu scratch bytes needed, its fixed scratch holds %zu; "
                    "use pcrt_diffraction with a workspace",
                    need, kNoallocScratch);
    char *ptr = nullptr;
    st = scratch_ptr(&ptr);
    if (st) return st;
    return diffraction_impl(scene, edges, n_edges, mats, n_labels, tx, rx, n_rx, freq_hz, eps_self, ptr, spill, out,
                            pair_amp, (hipStream_t)stream);
}

pcrt_status pcrt_reception_points(const pcrt_scene *scene, float *out, void *stream) {
    if (!scene || !out) return fail(PCRT_EINVAL, "scene and out are required");
    if (!scene->dev.dps_pt) return fail(PCRT_EINVAL, "the scene has no point sets (dps_voxel = 0)");
    launch_recv_copy((const float4 *)(scene->ws + scene->L.dps_recv), scene->info.n_point_sets, out,
                     (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return ok();
}

pcrt_status pcrt_scene_get_info(const pcrt_scene *scene, pcrt_scene_info *info) {
    if (!scene || !info) return fail(PCRT_EINVAL, "scene and info are required");
    *info = scene->info;
    return ok();
}

pcrt_status pcrt_scene_destroy(pcrt_scene *scene) {
    delete scene;
    return ok();
}

pcrt_status pcrt_solve_workspace_size(const pcrt_scene *scene, const pcrt_solve_params *p, size_t *bytes) {
    pcrt_status st = check_params(scene, p);
    if (st) return st;
    if (!bytes) return fail(PCRT_EINVAL, "bytes is NULL");
    Plan P = make_plan(scene, p);
    st = plan_check(P);
    if (st) return st;
    place_hash(P, p->flags);
    *bytes = P.L.total;
    return ok();
}

}  // extern "C"

static pcrt_status check_common(const pcrt_scene *scene, const pcrt_material *mats, uint32_t n_labels,
                                const pcrt_solve_params *p, void *ws, const pcrt_outputs *out) {
    pcrt_status st = check_params(scene, p);
    if (st) return st;
    if (!out || !out->gain) return fail(PCRT_EINVAL, "out->gain is required");
    if (!ws) return fail(PCRT_EINVAL, "ws is required");
    if ((p->flags & (PCRT_SPECULAR | PCRT_DIFFUSE)) && (!mats || n_labels == 0))
        return fail(PCRT_EINVAL, "materials are required");
    if (p->wave_rays && (p->wave_rays % kWave || p->wave_rays > 16 * kWave))
        return fail(PCRT_EUNSUPPORTED, "wave_rays must be a multiple of 64 up to 1024");
    return PCRT_OK;
}

// The whole launch sequence of a (batched) solve. Only kernels are enqueued:
// no allocation, no memset node, no host synchronisation (except the event
// records of PCRT_TIMING), so it can be captured in a HIP graph.
static pcrt_status solve_impl(const pcrt_scene *scene, const pcrt_material *mats, uint32_t n_labels,
                              const pcrt_solve_params *p, std::vector<Item> &items, void *ws, size_t ws_bytes,
                              const pcrt_outputs *out, hipStream_t s) {
    Plan P = make_plan(scene, p, items);
    pcrt_status st = plan_check(P);
    if (st) return st;
    place_hash(P, p->flags);
    if (ws_bytes < P.L.total) return fail(PCRT_ENOMEM, "solve workspace too small: need %zu bytes", P.L.total);
    char *w = (char *)ws;
    LaunchArgs A = make_args(scene, mats, n_labels, p, P, w, out->counters);
    const bool tm = p->flags & PCRT_TIMING;
    for (int i = 0; i < kStages; ++i) g_ev_used[i] = tm;
    stage_mark(tm, 0, s);
    fill_u32(A.work, 0, kWorkWords, s);
    fill_u64(A.counters, 0, PCRT_CNT_COUNT, s);
    fill_u32(A.key_off, 0, P.D.n_items + 1, s);
    fill_u32(A.chunk_off, 0, P.D.n_items + 1, s);
    for (size_t b = 0; b < items.size(); b += 96) {
        ItemBatch ib;
        memset(&ib, 0, sizeof ib);
        ib.n = (uint32_t)std::min<size_t>(96, items.size() - b);
        ib.base = (uint32_t)b;
        memcpy(ib.it, items.data() + b, sizeof(Item) * ib.n);
        hipLaunchKernelGGL(k_put_items, dim3(1), dim3(96), 0, s, ib, (Item *)A.items);
    }
    if (p->flags & PCRT_SPECULAR) {
        fill_u64((uint64_t *)A.hb.key, 0, (size_t)P.cap * P.D.n_items, s);
        fill_u32(A.hb.rep, 0xffffffffu, (size_t)P.cap * P.D.n_items, s);
    }
    const bool dps_diff = (p->flags & PCRT_DPS_LAUNCH) && (p->flags & PCRT_DIFFUSE);
    if (dps_diff) {
        fill_u64((uint64_t *)A.dhb.key, 0, A.dhb.cap, s);
        fill_u32(A.dhb.rep, 0xffffffffu, A.dhb.cap, s);
    }
    stage_mark(tm, 1, s);
    if (p->flags & (PCRT_SPECULAR | PCRT_DIFFUSE)) {
        launch_trace(A, s);
        if (out->ray_seq && P.D.n_items == 1) {
            uint32_t n = P.n_trace * P.D.K;
            hipLaunchKernelGGL(k_copy_seq, dim3((n + 255) / 256), dim3(256), 0, s, A.rb.id, n, out->ray_seq);
        }
    }
    stage_mark(tm, 2, s);
    if (p->flags & PCRT_SPECULAR) launch_keys(A, s);
    stage_mark(tm, 3, s);
    if (p->flags & PCRT_SPECULAR) launch_refine(A, s);
    stage_mark(tm, 4, s);
    if ((p->flags & PCRT_DIFFUSE) && !dps_diff) A.dsort.order = launch_diffuse_order(A, s);
    stage_mark(tm, 5, s);
    if (dps_diff) launch_dps_diffuse(A, scene->info.dps_voxel * scene->info.dps_voxel, s);
    else if (p->flags & PCRT_DIFFUSE) launch_diffuse(A, s);
    stage_mark(tm, 6, s);
    launch_los_and_combine(A, out->gain, out->h_te, out->h_tm, out->gain_parts, s);
    if (p->flags & PCRT_RECORD) launch_tape_slots(A, s);
    stage_mark(tm, 7, s);
    HIP_TRY(hipGetLastError());
    return ok();
}

static pcrt_status check_batch(const pcrt_solve_params *p, const pcrt_batch_item *items, uint32_t n_items) {
    if (!items || n_items == 0) return fail(PCRT_EINVAL, "items are required");
    if (n_items > 65536) return fail(PCRT_EUNSUPPORTED, "at most 65536 items");
    if (p->ray_subset) return fail(PCRT_EINVAL, "ray_subset is not supported in a batch");
    if (p->flags & PCRT_RECORD) return fail(PCRT_EUNSUPPORTED, "tapes are kept for single-transmitter solves only");
    if (p->flags & PCRT_DPS_LAUNCH) return fail(PCRT_EUNSUPPORTED, "the reception-point launch is for single solves");
    uint64_t total = 0;
    for (uint32_t i = 0; i < n_items; ++i) {
        if (!std::isfinite(items[i].tx[0]) || !std::isfinite(items[i].tx[1]) || !std::isfinite(items[i].tx[2]))
            return fail(PCRT_EINVAL, "item %u: tx must be finite", i);
        if ((p->flags & (PCRT_SPECULAR | PCRT_DIFFUSE)) && items[i].n_rays == 0)
            return fail(PCRT_EINVAL, "item %u: n_rays must be > 0", i);
        total += round_up(items[i].n_rays, kRayChunk);
    }
    if (total * p->max_interactions > 0x7fffffffull) return fail(PCRT_EUNSUPPORTED, "too many rays x interactions");
    if ((uint64_t)n_items * p->n_rx > kMaxPairs) return fail(PCRT_EUNSUPPORTED, "too many items x receivers");
    return PCRT_OK;
}

struct pcrt_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {

pcrt_status pcrt_solve(const pcrt_scene *scene, const pcrt_material *mats, uint32_t n_labels,
                       const pcrt_solve_params *p, void *ws, size_t ws_bytes, const pcrt_outputs *out,
                       void *stream) {
    pcrt_status st = check_common(scene, mats, n_labels, p, ws, out);
    if (st) return st;
    std::vector<Item> items = single_items(p);
    return solve_impl(scene, mats, n_labels, p, items, ws, ws_bytes, out, (hipStream_t)stream);
}

pcrt_status pcrt_batch_workspace_size(const pcrt_scene *scene, const pcrt_solve_params *p,
                                      const pcrt_batch_item *items, uint32_t n_items, size_t *bytes) {
    pcrt_status st = check_params(scene, p);
    if (st) return st;
    st = check_batch(p, items, n_items);
    if (st) return st;
    if (!bytes) return fail(PCRT_EINVAL, "bytes is NULL");
    std::vector<Item> v = batch_items(p, items, n_items);
    Plan P = make_plan(scene, p, v);
    place_hash(P, p->flags);
    *bytes = P.L.total;
    return ok();
}

pcrt_status pcrt_solve_batch(const pcrt_scene *scene, const pcrt_material *mats, uint32_t n_labels,
                             const pcrt_solve_params *p, const pcrt_batch_item *items, uint32_t n_items, void *ws,
                             size_t ws_bytes, const pcrt_outputs *out, void *stream) {
    pcrt_status st = check_common(scene, mats, n_labels, p, ws, out);
    if (st) return st;
    st = check_batch(p, items, n_items);
    if (st) return st;
    std::vector<Item> v = batch_items(p, items, n_items);
    return solve_impl(scene, mats, n_labels, p, v, ws, ws_bytes, out, (hipStream_t)stream);
}

pcrt_status pcrt_graph_capture_batch(const pcrt_scene *scene, const pcrt_material *mats, uint32_t n_labels,
                                     const pcrt_solve_params *p, const pcrt_batch_item *items, uint32_t n_items,
                                     void *ws, size_t ws_bytes, const pcrt_outputs *out, void *stream,
                                     pcrt_graph **graph) {
    if (!graph) return fail(PCRT_EINVAL, "graph is NULL");
    if (!stream) return fail(PCRT_EINVAL, "capture needs a non-default stream");
    if (p && (p->flags & PCRT_TIMING)) return fail(PCRT_EINVAL, "PCRT_TIMING cannot be captured");
    pcrt_status st = check_common(scene, mats, n_labels, p, ws, out);
    if (st) return st;
    st = check_batch(p, items, n_items);
    if (st) return st;
    std::vector<Item> v = batch_items(p, items, n_items);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    pcrt_status rs = solve_impl(scene, mats, n_labels, p, v, ws, ws_bytes, out, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rs != PCRT_OK) {
        if (g) hipGraphDestroy(g);
        return rs;
    }
    if (e != hipSuccess) return fail(PCRT_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        return fail(PCRT_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    *graph = new pcrt_graph{g, x};
    return ok();
}

pcrt_status pcrt_graph_launch(pcrt_graph *graph, void *stream) {
    if (!graph) return fail(PCRT_EINVAL, "graph is NULL");
    HIP_TRY(hipGraphLaunch(graph->exec, (hipStream_t)stream));
    return ok();
}

pcrt_status pcrt_graph_destroy(pcrt_graph *graph) {
    if (!graph) return ok();
    hipGraphExecDestroy(graph->exec);
    hipGraphDestroy(graph->graph);
    delete graph;
    return ok();
}

pcrt_status pcrt_autotune(const pcrt_scene *const *scenes, uint32_t n_scenes, const pcrt_solve_params *p,
                          const pcrt_material *mats, uint32_t n_labels, const uint32_t *wave_rays, uint32_t n_wave,
                          uint32_t reps, void *solve_ws, size_t solve_ws_bytes, const pcrt_outputs *out, void *stream,
                          pcrt_tuning *table, pcrt_tuning *best) {
    if (!scenes || !n_scenes || !p || !wave_rays || !n_wave || !best || !out)
        return fail(PCRT_EINVAL, "scenes, p, wave_rays, out and best are required");
    for (uint32_t a = 0; a < n_scenes; ++a) {
        if (!scenes[a]) return fail(PCRT_EINVAL, "scene %u is NULL", a);
        for (uint32_t b = 0; b < n_wave; ++b) {
            pcrt_solve_params q = *p;
            q.wave_rays = wave_rays[b];
            size_t need = 0;
            pcrt_status st = pcrt_solve_workspace_size(scenes[a], &q, &need);
            if (st) return st;
            if (need > solve_ws_bytes)
                return fail(PCRT_ENOMEM, "solve workspace too small for scene %u: need %zu bytes", a, need);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    best->ms = INFINITY;
    uint32_t idx = 0;
    for (uint32_t a = 0; a < n_scenes; ++a) {
        const pcrt_scene *sc = scenes[a];
        for (uint32_t b = 0; b < n_wave; ++b, ++idx) {
            pcrt_solve_params q = *p;
            q.wave_rays = wave_rays[b];
            q.flags &= ~(uint32_t)PCRT_TIMING;
            pcrt_status st = pcrt_solve(sc, mats, n_labels, &q, solve_ws, solve_ws_bytes, out, stream);  // warm-up
            if (st) return st;
            HIP_TRY(hipEventRecord(e0, s));
            for (uint32_t r = 0; r < std::max<uint32_t>(reps, 1); ++r)
                pcrt_solve(sc, mats, n_labels, &q, solve_ws, solve_ws_bytes, out, stream);
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            pcrt_tuning t = {a, sc->info.leaf_size, sc->info.width, wave_rays[b], ms / std::max<uint32_t>(reps, 1)};
            if (table) table[idx] = t;
            if (t.ms < best->ms) *best = t;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return ok();
}

pcrt_status pcrt_paths_copy(const pcrt_scene *scene, const pcrt_solve_params *p, const void *ws, uint32_t cap,
                            uint32_t *key_ray, uint8_t *key_len, int32_t *key_seq, uint8_t *valid, float *length,
                            float *amp, int32_t *hit, uint32_t *n_keys, void *stream) {
    pcrt_status st = check_params(scene, p);
    if (st) return st;
    if (!(p->flags & PCRT_RECORD) || !(p->flags & PCRT_SPECULAR))
        return fail(PCRT_EINVAL, "paths need a solve with RECORD and SPECULAR");
    if (!ws) return fail(PCRT_EINVAL, "ws is required");
    Plan P = make_plan(scene, p);
    st = plan_check(P);
    if (st) return st;
    place_hash(P, p->flags);
    hipStream_t s = (hipStream_t)stream;
    LaunchArgs A = make_args(scene, nullptr, 0, p, P, (char *)ws, nullptr);
    launch_paths_copy(A, cap, key_ray, key_len, key_seq, valid, length, amp, hit, s);
    if (n_keys) {
        HIP_TRY(hipMemcpyAsync(n_keys, A.key_off + P.D.n_items, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return ok();
}

pcrt_status pcrt_diffuse_vis_copy(const pcrt_scene *scene, const pcrt_solve_params *p, const void *ws, uint8_t *vis,
                                  void *stream) {
    pcrt_status st = check_params(scene, p);
    if (st) return st;
    if (!(p->flags & PCRT_RECORD) || !(p->flags & PCRT_DIFFUSE))
        return fail(PCRT_EINVAL, "visibility needs a solve with RECORD and DIFFUSE");
    if (p->flags & PCRT_DPS_LAUNCH)
        return fail(PCRT_EUNSUPPORTED, "the reception-point launch gates its diffuse paths by the visibility matrix");
    if (!ws || !vis) return fail(PCRT_EINVAL, "ws and vis are required");
    Plan P = make_plan(scene, p);
    st = plan_check(P);
    if (st) return st;
    place_hash(P, p->flags);
    size_t bytes = (size_t)P.n_trace * P.D.K * P.D.n_rx;
    HIP_TRY(hipMemcpyAsync(vis, (const char *)ws + P.L.dvis, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return ok();
}

static pcrt_status tape_args(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws, LaunchArgs *A,
                             Plan *P) {
    pcrt_status st = check_params(scene, p);
    if (st) return st;
    if (!(p->flags & PCRT_RECORD)) return fail(PCRT_EINVAL, "the tape needs a solve with PCRT_RECORD");
    if (p->flags & PCRT_POLARIZED)
        return fail(PCRT_EUNSUPPORTED, "the tape evaluates the scalar TE/TM field, not PCRT_POLARIZED");
    if (!ws) return fail(PCRT_EINVAL, "ws is required");
    *P = make_plan(scene, p);
    st = plan_check(*P);
    if (st) return st;
    place_hash(*P, p->flags);
    *A = make_args(scene, nullptr, 0, p, *P, (char *)ws, nullptr);
    return PCRT_OK;
}

pcrt_status pcrt_tape_get(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws, pcrt_tape *out) {
    LaunchArgs A;
    Plan P{};  // every field zero until set
    pcrt_status st = tape_args(scene, p, ws, &A, &P);
    if (st) return st;
    if (!out) return fail(PCRT_EINVAL, "out is NULL");
    out->n_slots = P.D.n_slots;
    out->n_trace_slots = P.D.T * P.D.K;
    out->key_capacity = P.D.rec_keys;
    out->label = A.slot_label;
    out->cos = A.slot_cos;
    out->coef = A.slot_coef;
    out->adj = A.slot_adj;
    return ok();
}

pcrt_status pcrt_tape_fresnel(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws,
                              const pcrt_material *mats, uint32_t n_labels, void *stream) {
    LaunchArgs A;
    Plan P{};  // every field zero until set
    pcrt_status st = tape_args(scene, p, ws, &A, &P);
    if (st) return st;
    if (!mats || n_labels == 0) return fail(PCRT_EINVAL, "materials are required");
    launch_tape_fresnel(A, (const float *)mats, n_labels, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return ok();
}

pcrt_status pcrt_tape_forward(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws,
                              const pcrt_outputs *out, void *stream) {
    LaunchArgs A;
    Plan P{};  // every field zero until set
    pcrt_status st = tape_args(scene, p, ws, &A, &P);
    if (st) return st;
    if (!out || !out->gain) return fail(PCRT_EINVAL, "out->gain is required");
    launch_tape_forward(A, out->gain, out->h_te, out->h_tm, out->gain_parts, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return ok();
}

pcrt_status pcrt_tape_backward(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws,
                               const double *dL_dgain, void *stream) {
    LaunchArgs A;
    Plan P{};  // every field zero until set
    pcrt_status st = tape_args(scene, p, ws, &A, &P);
    if (st) return st;
    if (!dL_dgain) return fail(PCRT_EINVAL, "dL_dgain is required");
    launch_tape_backward(A, dL_dgain, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return ok();
}

pcrt_status pcrt_tape_cfr(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws, double bandwidth_hz,
                          uint32_t n_freq, double *cfr, void *stream) {
    LaunchArgs A;
    Plan P{};  // every field zero until set
    pcrt_status st = tape_args(scene, p, ws, &A, &P);
    if (st) return st;
    if ((p->flags & PCRT_DPS_LAUNCH) && (p->flags & PCRT_DIFFUSE))
        return fail(PCRT_EUNSUPPORTED, "frequency responses of the voxel diffuse paths are not kept");
    if (!cfr) return fail(PCRT_EINVAL, "cfr is required");
    if (n_freq == 0 || n_freq > 65535) return fail(PCRT_EINVAL, "n_freq must be in 1..65535");
    if (!(bandwidth_hz >= 0.0) || !std::isfinite(bandwidth_hz)) return fail(PCRT_EINVAL, "bandwidth_hz must be >= 0");
    launch_tape_cfr(A, bandwidth_hz, n_freq, cfr, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return ok();
}

pcrt_status pcrt_tape_cfr_backward(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws,
                                   double bandwidth_hz, uint32_t n_freq, const double *dL_dcfr, void *stream) {
    LaunchArgs A;
    Plan P{};  // every field zero until set
    pcrt_status st = tape_args(scene, p, ws, &A, &P);
    if (st) return st;
    if ((p->flags & PCRT_DPS_LAUNCH) && (p->flags & PCRT_DIFFUSE))
        return fail(PCRT_EUNSUPPORTED, "frequency responses of the voxel diffuse paths are not kept");
    if (!dL_dcfr) return fail(PCRT_EINVAL, "dL_dcfr is required");
    if (n_freq == 0 || n_freq > 65535) return fail(PCRT_EINVAL, "n_freq must be in 1..65535");
    if (!(bandwidth_hz >= 0.0) || !std::isfinite(bandwidth_hz)) return fail(PCRT_EINVAL, "bandwidth_hz must be >= 0");
    launch_tape_cfr_backward(A, bandwidth_hz, n_freq, dL_dcfr, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return ok();
}

pcrt_status pcrt_material_grad(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws,
                               const pcrt_material *mats, uint32_t n_labels, double *dL_dmat, void *stream) {
    LaunchArgs A;
    Plan P{};  // every field zero until set
    pcrt_status st = tape_args(scene, p, ws, &A, &P);
    if (st) return st;
    if (!mats || !dL_dmat || n_labels == 0) return fail(PCRT_EINVAL, "mats and dL_dmat are required");
    if (n_labels > kMaxGradLabels) return fail(PCRT_EUNSUPPORTED, "at most %u labels", kMaxGradLabels);
    launch_material_grad(A, (const float *)mats, n_labels, dL_dmat, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return ok();
}

pcrt_status pcrt_status_poll(const uint64_t *counters_host_copy) {
    if (!counters_host_copy) return fail(PCRT_EINVAL, "counters_host_copy is NULL");
    const uint64_t w = counters_host_copy[PCRT_CNT_STATUS];
    if (!w) return ok();
    std::string why;
    if (w & 2) why += "a material label >= n_labels was met (label 0 used); ";
    if (w & 1) why += "the key table overflowed (keys dropped from the paths); ";
    if (w & 4) why += "more keys than key_capacity (paths left off the tape and the gradients); ";
    if (w & ~7ull) why += "unknown status bits; ";
    why.resize(why.size() - 2);
    return fail((w & 2) ? PCRT_EINVAL : PCRT_EOVERFLOW, "device status 0x%llx: %s", (unsigned long long)w, why.c_str());
}

pcrt_status pcrt_stage_times(double *ms, uint32_t n) {
    if (!ms) return fail(PCRT_EINVAL, "ms is NULL");
    if (!g_ev_ok || !g_ev_used[0]) return fail(PCRT_EINVAL, "no PCRT_TIMING solve on this thread");
    HIP_TRY(hipEventSynchronize(g_ev[kStages]));
    for (uint32_t i = 0; i < n && i < (uint32_t)kStages; ++i) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, g_ev[i], g_ev[i + 1]));
        ms[i] = t;
    }
    return ok();
}

pcrt_status pcrt_raygen(uint32_t n_budget, const uint32_t *ids, uint32_t n, float *out, void *stream) {
    if (n_budget == 0 || !out) return fail(PCRT_EINVAL, "n_budget > 0 and out are required");
    if (n == 0) return ok();
    launch_raygen(n_budget, ids, n, out, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return ok();
}

}  // extern "C"
