// Single-bounce edge diffraction (Sec. II-B.3): per (receiver, edge) the edge
// point that minimises the path length, a check that the transmitter and the
// receiver both see it, and the wedge field of the uniform theory of
// diffraction (Kouyoumjian and Pathak 1974) with face reflection coefficients
// in the reflection terms (Luebbers 1984); the paper leaves the field to its
// EM back end.
//
// The geometry, the coefficient and the amplitude are evaluated in FP64 (a
// few thousand pairs; the shadow and reflection boundary terms cancel poles
// against zeros, which FP32 would resolve poorly); the visibility walks are
// the FP32 any-hit walks of the diffuse connections, one lane per pair, the
// lanes of a wavefront sharing the receiver.
#include "common.h"
#include "internal.h"

namespace pcrt {

namespace {

struct z64 {
    double re, im;
};
__device__ __forceinline__ z64 zadd(z64 a, z64 b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ z64 zmul(z64 a, z64 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ z64 zscale(z64 a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ z64 zexpj(double t) {  // e^{jt}
    double s, c;
    sincos(t, &s, &c);
    return {c, s};
}
__device__ __forceinline__ z64 zdiv(z64 a, z64 b) {
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ z64 zsqrt(z64 z) {  // principal branch
    const double r = hypot(z.re, z.im);
    if (r == 0.0) return {0.0, 0.0};
    if (z.re >= 0.0) {
        const double t = sqrt(0.5 * (r + z.re));
        return {t, z.im / (2.0 * t)};
    }
    const double t = sqrt(0.5 * (r - z.re));
    return {fabs(z.im) / (2.0 * t), z.im >= 0.0 ? t : -t};
}

struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 dsub(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ d3 dadd(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ d3 dmul(double s, d3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double ddot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 dcross(d3 a, d3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double dlen(d3 a) { return sqrt(ddot(a, a)); }
__device__ __forceinline__ d3 dunit(d3 a) { return dmul(1.0 / dlen(a), a); }
__device__ __forceinline__ d3 dload(const float *p) { return {p[0], p[1], p[2]}; }

// F(x) = 2j sqrt(x) e^{jx} int_{sqrt x}^inf e^{-j t^2} dt, x >= 0. Below x = 20
// the tail is the whole integral, sqrt(pi)/2 e^{-j pi/4}, minus the power
// series int_0^u e^{-j t^2} dt = sum_m (-j)^m u^{2m+1} / (m! (2m+1)) (largest
// term ~ e^x, so FP64 keeps ~9 digits at x = 20); above, the asymptotic
// series F = sum_m (-1)^m (2m-1)!! / (2 j x)^m, cut at its smallest term.
__device__ z64 transition_fn(double x) {
    if (x < 20.0) {
        const double u = sqrt(x);
        z64 a = {u, 0.0}, sum = {u, 0.0};
        for (int m = 1; m < 200; ++m) {
            a = zscale(zmul(a, {0.0, -1.0}), x / m);  // a_m = a_{m-1} (-j) x / m
            sum = zadd(sum, zscale(a, 1.0 / (2 * m + 1)));
            if (m > x && hypot(a.re, a.im) < 1e-18 * hypot(sum.re, sum.im)) break;
        }
        const double h = 0.5 * sqrt(kPi) * 0.70710678118654752440;  // sqrt(pi)/2 * cos(pi/4)
        const z64 tail = {h - sum.re, -h - sum.im};
        return zmul(zmul({0.0, 2.0 * u}, zexpj(x)), tail);
    }
    z64 t = {1.0, 0.0}, sum = {1.0, 0.0};
    double prev = 1.0;
    for (int m = 1; m < 60; ++m) {
        const z64 nt = zmul(t, {0.0, (2.0 * m - 1.0) / (2.0 * x)});  // t_m = t_{m-1} (2m-1) j / (2x)
        const double mag = hypot(nt.re, nt.im);
        if (mag >= prev || mag < 1e-18) break;
        t = nt;
        prev = mag;
        sum = zadd(sum, t);
    }
    return sum;
}

// cot((pi + sign beta) / (2n)) F(kL a^sign(beta)) with a^{+-}(beta) =
// 2 cos^2((2 n pi N - beta) / 2), N the integer nearest to 2 pi n N - beta =
// +-pi, and the term's finite limit where the cotangent's pole meets F's zero.
__device__ z64 utd_term(double beta, double n, double kL, double sign) {
    const double N = rint((beta + sign * kPi) / (2.0 * kPi * n));
    const double c = cos((2.0 * n * kPi * N - beta) / 2.0);
    const double eps = kPi + sign * beta - 2.0 * kPi * n * N;
    if (fabs(eps) < 1e-9) {
        const z64 e4 = zexpj(kPi / 4.0);
        const double sg = eps > 0.0 ? 1.0 : (eps < 0.0 ? -1.0 : 0.0);
        const z64 in = {n * (sqrt(2.0 * kPi * kL) * sg - 2.0 * kL * eps * e4.re), -n * 2.0 * kL * eps * e4.im};
        return zmul(in, e4);
    }
    return zscale(transition_fn(kL * 2.0 * c * c), 1.0 / tan((kPi + sign * beta) / (2.0 * n)));
}

// Reflection coefficients of a face (eta = eps_r - j sigma / (omega eps0)) at
// incidence cosine cs: TE (perpendicular) and TM (parallel).
__device__ void face_gamma(double eps_r, double sig_w, double cs, z64 &te, z64 &tm) {
    const z64 eta = {eps_r, -sig_w};
    const double s2 = 1.0 - cs * cs;
    const z64 root = zsqrt({eta.re - s2, eta.im});
    te = zdiv({cs - root.re, -root.im}, {cs + root.re, root.im});
    const z64 ec = zscale(eta, cs);
    tm = zdiv({ec.re - root.re, ec.im - root.im}, {ec.re + root.re, ec.im + root.im});
}

// angle of direction v about the edge e from face 0 (in-face t0, outward n0), in [0, 2 pi)
__device__ __forceinline__ double wedge_angle(d3 v, d3 e, d3 t0, d3 n0) {
    const d3 w = dsub(v, dmul(ddot(v, e), e));
    const double ph = atan2(ddot(w, n0), ddot(w, t0));
    return ph < 0.0 ? ph + 2.0 * kPi : ph;
}

}  // namespace

struct DiffArgs {
    DevScene S;
    const pcrt_edge *edges;
    uint32_t n_edges;
    const float *mats;  // [n_labels][3]
    uint32_t n_labels;
    float tx[3];
    const float *rx;
    uint32_t n_rx;
    double k, lam, inv_we0;
    float eps_self, trim;
    float4 *amp;  // [n_rx][n_edges]: TE re, im, TM re, im (0 where no path)
};

template <int W>
__global__ __launch_bounds__(kWave) void k_diffraction(DiffArgs A) {
    __shared__ int lds_stack[kStackLds * kWave];
    const int lane = threadIdx.x;
    const uint32_t glane = blockIdx.x * kWave + lane;
    Stack stk{lds_stack + lane, A.S.spill + glane, A.S.spill_lanes};
    const uint32_t p = glane;
    if (p >= A.n_rx * A.n_edges) return;
    const uint32_t r = p / A.n_edges, i = p % A.n_edges;
    const pcrt_edge E = A.edges[i];
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    const d3 a = dload(E.a), b = dload(E.b), tx = dload(A.tx), rx = dload(A.rx + 3 * r);
    const d3 n0 = dunit(dload(E.n0)), n1 = dunit(dload(E.n1));
    const d3 ev = dsub(b, a);
    const d3 e = dunit(ev);
    // edge point: the straight line of the two ends unfolded about the edge
    const double l2 = ddot(ev, ev);
    const double tp = ddot(dsub(tx, a), ev) / l2, tq = ddot(dsub(rx, a), ev) / l2;
    const double dp = dlen(dsub(tx, dadd(a, dmul(tp, ev)))), dq = dlen(dsub(rx, dadd(a, dmul(tq, ev))));
    bool ok = dp + dq > 0.0;
    const double t = ok ? tp + (tq - tp) * dp / (dp + dq) : 0.0;
    ok = ok && t > 0.0 && t < 1.0;
    d3 t0 = dunit(dcross(n0, e));
    if (ddot(t0, n1) > 0.0) t0 = dmul(-1.0, t0);
    d3 t1 = dunit(dcross(n1, e));
    if (ddot(t1, n0) > 0.0) t1 = dmul(-1.0, t1);
    const double n = (2.0 * kPi - acos(fmin(1.0, fmax(-1.0, ddot(t0, t1))))) / kPi;
    const d3 D = dadd(a, dmul(t, ev));
    const d3 vi = dsub(tx, D), vo = dsub(rx, D);
    const double sp = dlen(vi), s = dlen(vo);
    const double phip = wedge_angle(vi, e, t0, n0), phi = wedge_angle(vo, e, t0, n0);
    ok = ok && sp > 0.0 && s > 0.0 && phip > 0.0 && phip < n * kPi && phi > 0.0 && phi < n * kPi;
    if (ok) {  // both ends see the edge point (segments cut short by trim at the edge)
        const d3 ui = dmul(1.0 / sp, vi), uo = dmul(1.0 / s, vo);
        const d3 ci = dadd(D, dmul(A.trim, ui)), co = dadd(D, dmul(A.trim, uo));
        ok = !occluded<W>(A.S, mk((float)tx.x, (float)tx.y, (float)tx.z), mk((float)ci.x, (float)ci.y, (float)ci.z),
                          -1, A.eps_self, stk);
        ok = ok && !occluded<W>(A.S, mk((float)rx.x, (float)rx.y, (float)rx.z),
                                mk((float)co.x, (float)co.y, (float)co.z), -1, A.eps_self, stk);
        if (ok) {
            const double sin_b0 = dlen(dcross(ui, e));
            const double kL = A.k * s * sp * sin_b0 * sin_b0 / (s + sp);
            const double bm = phi - phip, bp = phi + phip;
            const z64 f1 = utd_term(bm, n, kL, +1.0), f2 = utd_term(bm, n, kL, -1.0);
            const z64 f3 = utd_term(bp, n, kL, -1.0), f4 = utd_term(bp, n, kL, +1.0);
            const uint32_t l0 = min((uint32_t)E.label0, A.n_labels - 1), ln = min((uint32_t)E.label1, A.n_labels - 1);
            z64 r0te, r0tm, rnte, rntm;
            face_gamma(A.mats[3 * l0], A.mats[3 * l0 + 1] * A.inv_we0, sin(phip), r0te, r0tm);
            face_gamma(A.mats[3 * ln], A.mats[3 * ln + 1] * A.inv_we0, sin(n * kPi - phi), rnte, rntm);
            const z64 pre = zscale(zexpj(-kPi / 4.0), -1.0 / (2.0 * n * sqrt(2.0 * kPi * A.k) * sin_b0));
            const z64 common = zadd(f1, f2);
            const z64 dte = zmul(pre, zadd(common, zadd(zmul(r0te, f3), zmul(rnte, f4))));
            const z64 dtm = zmul(pre, zadd(common, zadd(zmul(r0tm, f3), zmul(rntm, f4))));
            const z64 base = zscale(zexpj(-A.k * (sp + s)), A.lam / (4.0 * kPi) / sp * sqrt(sp / (s * (s + sp))));
            const z64 ate = zmul(base, dte), atm = zmul(base, dtm);
            out = make_float4((float)ate.re, (float)ate.im, (float)atm.re, (float)atm.im);
        }
    }
    A.amp[(size_t)r * A.n_edges + i] = out;
}

// Per receiver, the paths in edge order (FP64): G, h_TE re, im, h_TM re, im.
__global__ void k_diffraction_sum(const float4 *amp, uint32_t n_edges, uint32_t n_rx, double *out) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n_rx; r += gridDim.x * blockDim.x) {
        double acc[5] = {0, 0, 0, 0, 0};
        for (uint32_t i = 0; i < n_edges; ++i) {
            const float4 v = amp[(size_t)r * n_edges + i];
            const double tr = v.x, ti = v.y, mr = v.z, mi = v.w;
            acc[0] += 0.5 * (tr * tr + ti * ti + mr * mr + mi * mi);
            acc[1] += tr;
            acc[2] += ti;
            acc[3] += mr;
            acc[4] += mi;
        }
        for (int a = 0; a < 5; ++a) out[(size_t)r * 5 + a] = acc[a];
    }
}

uint32_t diffraction_blocks(uint32_t n_edges, uint32_t n_rx) { return (n_edges * n_rx + kWave - 1) / kWave; }

void launch_diffraction(const DevScene &S, const pcrt_edge *edges, uint32_t n_edges, const float *mats,
                        uint32_t n_labels, const float tx[3], const float *rx, uint32_t n_rx, double freq,
                        float eps_self, float4 *amp, double *out, hipStream_t s) {
    DiffArgs A;
    A.S = S;
    A.edges = edges;
    A.n_edges = n_edges;
    A.mats = mats;
    A.n_labels = n_labels;
    for (int c = 0; c < 3; ++c) A.tx[c] = tx[c];
    A.rx = rx;
    A.n_rx = n_rx;
    A.k = 2.0 * kPi * freq / kC0;
    A.lam = kC0 / freq;
    A.inv_we0 = 1.0 / (2.0 * kPi * freq * kEps0);
    A.eps_self = eps_self;
    A.trim = 2.0f * sqrtf(S.r2);
    A.amp = amp;
    const dim3 g(diffraction_blocks(n_edges, n_rx));
    switch (S.width) {
        case 8: hipLaunchKernelGGL(k_diffraction<8>, g, dim3(kWave), 0, s, A); break;
        case 4: hipLaunchKernelGGL(k_diffraction<4>, g, dim3(kWave), 0, s, A); break;
        default: hipLaunchKernelGGL(k_diffraction<2>, g, dim3(kWave), 0, s, A); break;
    }
    hipLaunchKernelGGL(k_diffraction_sum, dim3((n_rx + 255) / 256), dim3(256), 0, s, amp, n_edges, n_rx, out);
}

}  // namespace pcrt
