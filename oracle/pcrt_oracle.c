/*
 * pcrt_oracle.c -- plain, slow, FP64 CPU oracle for point-cloud radio ray tracing.
 *
 * TEST INFRASTRUCTURE. This is the checker that the GPU library is compared
 * against. Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may build, load or call it; the product path never does. It shares
 * no code, header, table or helper with the GPU library.
 *
 * Method: Vaara et al., "Differentiable High-Performance Ray Tracing-Based
 * Simulation of Radio Propagation with Point Clouds" (arXiv 2507.04021).
 *   - Input: augmented point cloud (position, normal, surface label, material
 *     label per point), TX and RX positions (Sec. II, opening paragraph).
 *   - Each point is a planar disk of radius r_p (Sec. II-C).
 *   - Optionally, the points are grouped into voxels of edge rho (Sec. II-A)
 *     and an interaction is the weighted average over the intersected disks
 *     of the hit disk's voxel (Sec. II-C, Eq. 3-4). Each set's reception
 *     point and its visibility from every receiver form the visibility
 *     matrix (Sec. II-A, II-B).
 *   - Rays keep a constant count; every interaction continues as a specular
 *     reflection (Sec. II-B).
 *   - Diffuse scattering is the last interaction, validated by a ray from the
 *     scatter point to the RX (Sec. II-B.1).
 *   - Specular paths minimise the path length of Eq. (1) on infinite planes,
 *     then every interaction is validated with thresholds t_a, t_d and up to
 *     kappa retries (Sec. II-B.2, Table I).
 *   - Duplicates are removed with a key of surface labels (Sec. II-B.4).
 *   - Field: Fresnel reflection from complex permittivity, scattering
 *     coefficient, free-space spreading (the paper delegates this to its EM
 *     back end; the readings used here are spelled out next to each function).
 *     Two field models: the scalar TE and TM chains, or (ORC_POLARIZED) the
 *     field vector carried through every reflection (Jones vectors).
 *
 * Everything is brute force: every query tests every disk. All arithmetic is
 * double precision; FP32 input arrays are promoted on entry. Parallelism is
 * OpenMP over independent rays / (key, receiver) pairs only; every reduction
 * is serial in a fixed order.
 *
 * Pins: tests/test_oracle_pins.py checks these functions against closed forms,
 * brute force on tiny inputs, textbook special cases and invariants. Parity
 * unpinned (conventions the paper leaves open, with no independent value to
 * check them against; the GPU library is only compared with them): the tie
 * window eps_tie and the self-hit distance eps_self of the nearest-hit rule,
 * the pick between coplanar disks at the tiny room's holes and door edge, and,
 * under ORC_AVERAGE, that the refinement takes its planes from the key's
 * representative's averaged records.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_C0 299792458.0
#define ORC_EPS0 8.8541878128e-12
#define ORC_PI 3.14159265358979323846
#define ORC_KMAX 8

enum { ORC_LOS = 1, ORC_SPECULAR = 2, ORC_DIFFUSE = 4, ORC_TRACE = 8 /* trace even without paths */,
       ORC_AVERAGE = 16 /* weighted-average intersection over point sets */,
       ORC_DPS_LAUNCH = 32 /* rays towards the reception points, visibility-gated specular candidates */,
       ORC_POLARIZED = 64 /* Jones-vector field of line-of-sight and specular paths */ };

typedef struct {
    int64_t n;
    double *p;  /* [n][3] centres */
    double *nr; /* [n][3] unit normals */
    const uint16_t *mat;
    const uint32_t *surf;
    double r;
} scene_t;

typedef struct {
    double eps_tie;  /* nearest-hit tie window (m) */
    double eps_self; /* minimum hit distance from a ray origin (m) */
    double cos_ta;   /* cos of the angle threshold t_a */
    double t_d;      /* plane-distance threshold (m) */
    int kappa;       /* refinement retries */
} thr_t;

typedef struct {
    int n_labels;
    const double *eps_r, *sigma, *scat;
    double freq, omega, lambda, k0;
} em_t;

/* ------------------------------------------------------------------ vectors */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(double *r, const double *a, const double *b) { r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2]; }
static double norm3(const double *a) { return sqrt(dot3(a, a)); }
static void scale3(double *a, double s) { a[0] *= s; a[1] *= s; a[2] *= s; }
static void copy3(double *d, const double *s) { d[0] = s[0]; d[1] = s[1]; d[2] = s[2]; }
static void from_f32(double *d, const float *s) { d[0] = s[0]; d[1] = s[1]; d[2] = s[2]; }
static void cross3(double *r, const double *a, const double *b)
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

static int scene_init(scene_t *s, int64_t n, const float *pos, const float *nrm, const uint16_t *mat,
                      const uint32_t *surf, double r)
{
    s->n = n;
    s->mat = mat;
    s->surf = surf;
    s->r = r;
    s->p = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    s->nr = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!s->p || !s->nr) return -2;
    for (int64_t i = 0; i < n; ++i) {
        from_f32(s->p + 3 * i, pos + 3 * i);
        from_f32(s->nr + 3 * i, nrm + 3 * i);
        double l = norm3(s->nr + 3 * i);
        if (!(l > 0.0) || !isfinite(l)) return -1;
        scale3(s->nr + 3 * i, 1.0 / l);
    }
    return 0;
}

static void scene_free(scene_t *s)
{
    free(s->p);
    free(s->nr);
}

/* ------------------------------------------------- launch directions (a3) */
/* Fibonacci sphere: z = 1 - (2j+1)/N, phi = 2 pi frac(j g), g = (3 - sqrt 5)/2.
 * Computed in FP64 and rounded to FP32; both implementations trace these FP32
 * vectors. (The paper launches one ray per discretised point set; a uniform
 * sphere is the launch used here.) */
void orc_fib_dirs(int64_t n_budget, const int64_t *ids, int64_t n_ids, float *out)
{
    const double g = (3.0 - sqrt(5.0)) / 2.0;
    for (int64_t q = 0; q < n_ids; ++q) {
        int64_t j = ids[q];
        double z = 1.0 - (2.0 * (double)j + 1.0) / (double)n_budget;
        double rho = sqrt(fmax(0.0, 1.0 - z * z));
        double f = (double)j * g;
        f -= floor(f);
        double phi = 2.0 * ORC_PI * f;
        out[3 * q + 0] = (float)(rho * cos(phi));
        out[3 * q + 1] = (float)(rho * sin(phi));
        out[3 * q + 2] = (float)z;
    }
}

/* ------------------------------------------------- ray-disk test (Sec. II-C) */
/* Two-sided disk of centre p, unit normal n, radius r. Returns 1 on a hit with
 * ray parameter t, hit point q and squared distance |q - p|^2. */
static int ray_disk(const scene_t *s, int64_t i, const double *o, const double *d, double *t, double *q,
                    double *d2)
{
    const double *p = s->p + 3 * i, *n = s->nr + 3 * i;
    double a = dot3(d, n);
    if (fabs(a) < 1e-6) return 0;
    double w[3];
    sub3(w, p, o);
    double tt = dot3(w, n) / a;
    double qq[3] = {o[0] + tt * d[0], o[1] + tt * d[1], o[2] + tt * d[2]};
    double e[3];
    sub3(e, qq, p);
    double dd = dot3(e, e);
    if (dd > s->r * s->r) return 0;
    *t = tt;
    copy3(q, qq);
    *d2 = dd;
    return 1;
}

/* Nearest hit with an order-independent two-pass rule:
 *   t* = smallest t over hits in (t_lo, t_hi) not excluded;
 *   candidates = hits with t <= t* + eps_tie;
 *   winner = smallest (|q - p|^2, index), compared lexicographically.
 * The paper picks the closest points at an intersection (Sec. II-B.4); the
 * window makes coplanar overlapping disks resolve by disk centre distance. */
static int64_t nearest(const scene_t *s, const double *o, const double *d, int64_t excl, double t_lo,
                       double t_hi, double eps_tie, double *t_out, double *q_out)
{
    double tstar = INFINITY, t, q[3], d2;
    for (int64_t i = 0; i < s->n; ++i) {
        if (i == excl) continue;
        if (ray_disk(s, i, o, d, &t, q, &d2) && t > t_lo && t < t_hi && t < tstar) tstar = t;
    }
    if (!(tstar < INFINITY)) return -1;
    int64_t best = -1;
    double bd2 = INFINITY;
    for (int64_t i = 0; i < s->n; ++i) {
        if (i == excl) continue;
        if (ray_disk(s, i, o, d, &t, q, &d2) && t > t_lo && t < t_hi && t <= tstar + eps_tie) {
            if (d2 < bd2) { /* ascending i: ties on d2 keep the smaller index */
                bd2 = d2;
                best = i;
                *t_out = t;
                copy3(q_out, q);
            }
        }
    }
    return best;
}

/* True iff some disk other than excl is hit strictly between a and b, more
 * than eps_self away from both ends. */
static int occluded(const scene_t *s, const double *a, const double *b, int64_t excl, double eps_self)
{
    double d[3];
    sub3(d, b, a);
    double len = norm3(d);
    scale3(d, 1.0 / len);
    double t, q[3], d2;
    for (int64_t i = 0; i < s->n; ++i) {
        if (i == excl) continue;
        if (ray_disk(s, i, a, d, &t, q, &d2) && t > eps_self && t < len - eps_self) return 1;
    }
    return 0;
}

/* ------------------------------------ discretised point sets (Sec. II-A) */
/* The points are grouped by the voxel of edge rho that holds their centre:
 * voxel = floor(p / rho) per axis, both in FP64 from the FP32 inputs. Each
 * non-empty voxel is one point set. */
typedef struct {
    int64_t *of;  /* [n] set of each point */
    int64_t *off; /* [n_sets + 1] first member of each set in mem */
    int64_t *mem; /* [n] point indices grouped by set, ascending inside a set */
    int64_t n_sets;
} dps_t;

typedef struct {
    int64_t v[3], i;
} vox_t;

static int vox_cmp(const void *pa, const void *pb)
{
    const vox_t *a = (const vox_t *)pa, *b = (const vox_t *)pb;
    for (int c = 0; c < 3; ++c)
        if (a->v[c] != b->v[c]) return a->v[c] < b->v[c] ? -1 : 1;
    return a->i < b->i ? -1 : (a->i > b->i);
}

static int dps_build(dps_t *g, const scene_t *s, double rho)
{
    int64_t n = s->n;
    vox_t *v = (vox_t *)malloc(sizeof(vox_t) * (size_t)(n > 0 ? n : 1));
    g->of = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    g->off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    g->mem = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!v || !g->of || !g->off || !g->mem) { free(v); return -2; }
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < 3; ++c) v[i].v[c] = (int64_t)floor(s->p[3 * i + c] / rho);
        v[i].i = i;
    }
    qsort(v, (size_t)n, sizeof(vox_t), vox_cmp);
    g->n_sets = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == 0 || memcmp(v[j].v, v[j - 1].v, sizeof v[j].v)) g->off[g->n_sets++] = j;
        g->mem[j] = v[j].i;
        g->of[v[j].i] = g->n_sets - 1;
    }
    g->off[g->n_sets] = n;
    free(v);
    return 0;
}

static void dps_free(dps_t *g)
{
    free(g->of);
    free(g->off);
    free(g->mem);
}

/* Weighted-average intersection (Sec. II-C, Eq. 3-4). The averaging set is
 * every disk of the hit disk's point set that the ray meets farther than
 * eps_self from its origin (the excluded disk aside). Each member i has the
 * weight
 *   w_i = exp(-|q_i - p_i|^2 / (2 r^2)) * exp(-lambda_d |q_i - q_min|),
 * q_min being the member intersection nearest to the origin; the point is the
 * w-weighted mean of the q_i. All q_i lie on the ray, so the point is
 * o + t d with t the weighted mean of the t_i. The normal used to reflect is
 * the w-weighted sum of the member normals, each turned to face the incoming
 * ray, normalised. */
static void dps_average(const scene_t *s, const dps_t *g, const double *o, const double *d, int64_t excl,
                        double eps_self, int64_t h, double lambda_d, double *t_out, double *n_out)
{
    const int64_t set = g->of[h], b = g->off[set], e = g->off[set + 1];
    double t, q[3], d2, tmin = INFINITY, qmin[3] = {0, 0, 0};
    for (int64_t j = b; j < e; ++j) {
        int64_t i = g->mem[j];
        if (i == excl) continue;
        if (ray_disk(s, i, o, d, &t, q, &d2) && t > eps_self && t < tmin) {
            tmin = t;
            copy3(qmin, q);
        }
    }
    double sw = 0.0, st = 0.0, sn[3] = {0, 0, 0};
    for (int64_t j = b; j < e; ++j) {
        int64_t i = g->mem[j];
        if (i == excl) continue;
        if (!(ray_disk(s, i, o, d, &t, q, &d2) && t > eps_self)) continue;
        double dq[3];
        sub3(dq, q, qmin);
        double w = exp(-d2 / (2.0 * s->r * s->r)) * exp(-lambda_d * norm3(dq));
        const double *n = s->nr + 3 * i;
        double side = dot3(d, n) > 0.0 ? -1.0 : 1.0;
        sw += w;
        st += w * t;
        for (int c = 0; c < 3; ++c) sn[c] += w * side * n[c];
    }
    *t_out = st / sw;
    scale3(sn, 1.0 / norm3(sn));
    copy3(n_out, sn);
}

/* --------------------------------------------------------- Fresnel (field) */
/* eta = eps_r - j sigma/(omega eps0) (time convention e^{+j omega t});
 * w = sqrt(eta - sin^2) (principal branch);
 * Gamma_TE = (c - w)/(c + w), Gamma_TM = (eta c - w)/(eta c + w), c = cos(theta_i).
 * Derivatives with respect to eta are returned when requested. */
static void fresnel(const em_t *em, int label, double c, double complex *gte, double complex *gtm,
                    double complex *dte, double complex *dtm)
{
    double complex eta = em->eps_r[label] - I * (em->sigma[label] / (em->omega * ORC_EPS0));
    double s2 = 1.0 - c * c;
    double complex w = csqrt(eta - s2);
    *gte = (c - w) / (c + w);
    *gtm = (eta * c - w) / (eta * c + w);
    if (dte) *dte = -c / (w * (c + w) * (c + w));
    if (dtm) *dtm = c * (eta - 2.0 * s2) / (w * (eta * c + w) * (eta * c + w));
}

void orc_fresnel(double eps_r, double sigma, double freq, int64_t n, const double *cosv, double *out)
{
    em_t em = {1, &eps_r, &sigma, NULL, freq, 2.0 * ORC_PI * freq, ORC_C0 / freq, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        double complex a, b, da, db;
        fresnel(&em, 0, cosv[i], &a, &b, &da, &db);
        out[8 * i + 0] = creal(a);
        out[8 * i + 1] = cimag(a);
        out[8 * i + 2] = creal(b);
        out[8 * i + 3] = cimag(b);
        out[8 * i + 4] = creal(da);
        out[8 * i + 5] = cimag(da);
        out[8 * i + 6] = creal(db);
        out[8 * i + 7] = cimag(db);
    }
}

/* A path as a chain of interactions: each has a material label, an incidence
 * cosine and a factor kind (0: specular, amplitude R = sqrt(1 - S^2);
 * 1: diffuse, amplitude S). amp0 is the geometric amplitude (lambda/4pi times
 * spreading), len the phase length. Returns the two complex amplitudes and
 * accumulates 1/2(|a_TE|^2 + |a_TM|^2) and its gradient with respect to
 * (eps_r, sigma) of each label. */
static void path_field(const em_t *em, int k, const int *label, const double *cosv, const int *kind,
                       double amp0, double len, double complex *a_te, double complex *a_tm, double *g_acc,
                       double *jac /* [n_labels][3] or NULL */)
{
    double complex gte[ORC_KMAX], gtm[ORC_KMAX], dte[ORC_KMAX], dtm[ORC_KMAX];
    double fac[ORC_KMAX];
    double complex pte = 1.0, ptm = 1.0;
    for (int m = 0; m < k; ++m) {
        fresnel(em, label[m], cosv[m], &gte[m], &gtm[m], &dte[m], &dtm[m]);
        double S = em->scat[label[m]];
        fac[m] = kind[m] ? S : sqrt(fmax(0.0, 1.0 - S * S));
        pte *= fac[m] * gte[m];
        ptm *= fac[m] * gtm[m];
    }
    double complex ph = cexp(-I * em->k0 * len);
    *a_te = amp0 * pte * ph;
    *a_tm = amp0 * ptm * ph;
    *g_acc += 0.5 * (creal(*a_te * conj(*a_te)) + creal(*a_tm * conj(*a_tm)));
    if (!jac) return;
    /* d/d(eps_r, sigma) through Gamma, and d/dS through the factor:
     * d(R^2)/dS = -2S for a specular interaction, d(S^2)/dS = 2S for a diffuse one */
    const double complex deta[2] = {1.0, -I / (em->omega * ORC_EPS0)};
    for (int m = 0; m < k; ++m) {
        /* product of |f Gamma|^2 over every other interaction, per channel */
        double rest_te = amp0 * amp0, rest_tm = amp0 * amp0;
        for (int q = 0; q < k; ++q) {
            if (q == m) continue;
            rest_te *= fac[q] * fac[q] * creal(gte[q] * conj(gte[q]));
            rest_tm *= fac[q] * fac[q] * creal(gtm[q] * conj(gtm[q]));
        }
        for (int p = 0; p < 2; ++p) {
            double d_te = 2.0 * creal(conj(gte[m]) * dte[m] * deta[p]);
            double d_tm = 2.0 * creal(conj(gtm[m]) * dtm[m] * deta[p]);
            jac[3 * label[m] + p] += 0.5 * fac[m] * fac[m] * (rest_te * d_te + rest_tm * d_tm);
        }
        double S = em->scat[label[m]];
        double dfac2 = kind[m] ? 2.0 * S : -2.0 * S;
        jac[3 * label[m] + 2] += 0.5 * dfac2 *
                                 (rest_te * creal(gte[m] * conj(gte[m])) + rest_tm * creal(gtm[m] * conj(gtm[m])));
    }
}

/* Channel frequency response: every path adds its two complex amplitudes
 * (taken at the centre frequency f_c) times exp(-j 2 pi (f_n - f_c) tau),
 * tau = len / c0, at n_freq equally spaced frequencies
 * f_n = f_c + (n - (n_freq - 1) / 2) bw / (n_freq - 1) spanning bw. */
typedef struct {
    int n;
    double bw;
    double complex *h; /* [n_rx][n][2]: TE, TM */
} cfr_t;

static void cfr_add(cfr_t *c, int r, double complex a_te, double complex a_tm, double len)
{
    if (!c || c->n <= 0) return;
    const double tau = len / ORC_C0;
    for (int i = 0; i < c->n; ++i) {
        const double df = c->n > 1 ? (i - 0.5 * (c->n - 1)) * c->bw / (c->n - 1) : 0.0;
        const double complex w = cexp(-I * 2.0 * ORC_PI * df * tau);
        c->h[((size_t)r * c->n + i) * 2 + 0] += a_te * w;
        c->h[((size_t)r * c->n + i) * 2 + 1] += a_tm * w;
    }
}

/* Polarised field (Jones vectors; the paper takes its field from its EM back
 * end, which carries the field vector). The transmitter radiates pol_tx
 * projected on the plane normal to the departure direction (a short dipole);
 * at each specular interaction, with incoming direction d_in, outgoing d_out
 * and plane normal n, the field splits into its component along
 * s = (d_in x n)/|d_in x n| (perpendicular to the plane of incidence: TE) and
 * along p_in = s x d_in (in that plane: TM); the reflected field is
 *   R (Gamma_TE (E.s) s + Gamma_TM (E.p_in) p_out),  p_out = s x d_out,
 * which is the plane-wave relation E = Z H x k applied to the TM case, whose
 * coefficient (fresnel() above) is that of the magnetic field along s. At
 * normal incidence s is any unit vector normal to d_in (the result does not
 * depend on it there, since Gamma_TM = -Gamma_TE). The receiver takes the
 * projection of the arriving field on pol_rx projected on the plane normal
 * to the arrival direction. x: k + 2 points (TX, interactions, RX), n: the k
 * planes' normals. Returns the path's complex amplitude. */
static void unit_normal_to(const double *d, double *s)
{
    const double ax[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    int best = 0;
    for (int c = 1; c < 3; ++c)
        if (fabs(d[c]) < fabs(d[best])) best = c;
    cross3(s, d, ax[best]);
    scale3(s, 1.0 / norm3(s));
}

static double complex path_polarized(const em_t *em, int k, const double x[][3], const double n[][3],
                                     const int *label, double amp0, double len, const double *ptx,
                                     const double *prx)
{
    double din[3], dout[3];
    sub3(din, x[1], x[0]);
    scale3(din, 1.0 / norm3(din));
    double complex E[3];
    const double pd = dot3(ptx, din);
    for (int c = 0; c < 3; ++c) E[c] = ptx[c] - pd * din[c];
    for (int m = 1; m <= k; ++m) {
        sub3(dout, x[m + 1], x[m]);
        scale3(dout, 1.0 / norm3(dout));
        const double *nn = n[m - 1];
        double complex gte, gtm;
        fresnel(em, label[m - 1], fabs(dot3(din, nn)) / norm3(nn), &gte, &gtm, NULL, NULL);
        const double S = em->scat[label[m - 1]], R = sqrt(fmax(0.0, 1.0 - S * S));
        double s[3], pin[3], pout[3];
        cross3(s, din, nn);
        const double ns = norm3(s);
        if (ns < 1e-12 * norm3(nn)) unit_normal_to(din, s);
        else scale3(s, 1.0 / ns);
        cross3(pin, s, din);
        cross3(pout, s, dout);
        double complex es = 0.0, ep = 0.0;
        for (int c = 0; c < 3; ++c) {
            es += E[c] * s[c];
            ep += E[c] * pin[c];
        }
        for (int c = 0; c < 3; ++c) E[c] = R * (gte * es * s[c] + gtm * ep * pout[c]);
        copy3(din, dout);
    }
    const double pr = dot3(prx, din);
    double complex a = 0.0;
    for (int c = 0; c < 3; ++c) a += E[c] * (prx[c] - pr * din[c]);
    return amp0 * a * cexp(-I * em->k0 * len);
}

/* ------------------------------------------------------ bounce loop (a4-a5) */
typedef struct {
    int n;                 /* interactions recorded */
    int64_t id[ORC_KMAX];  /* hit disk */
    double x[ORC_KMAX][3]; /* hit point */
    double nk[ORC_KMAX][3];/* hit normal flipped against the incoming ray */
    double cs[ORC_KMAX];   /* incidence cosine */
    double L[ORC_KMAX];    /* unfolded length from TX to the hit */
} trace_t;

/* Every interaction is treated as a specular reflection and the ray count stays
 * constant (Sec. II-B). A miss ends the ray. */
static void trace_ray(const scene_t *s, const double *tx, const float *dir32, int K, const thr_t *th,
                      const dps_t *g, double lambda_d, trace_t *tr)
{
    double o[3], d[3];
    copy3(o, tx);
    from_f32(d, dir32);
    scale3(d, 1.0 / norm3(d));
    double L = 0.0;
    int64_t excl = -1;
    tr->n = 0;
    for (int k = 0; k < K; ++k) {
        double t, q[3];
        int64_t h = nearest(s, o, d, excl, th->eps_self, INFINITY, th->eps_tie, &t, q);
        if (h < 0) break;
        double n[3];
        copy3(n, s->nr + 3 * h);
        if (dot3(d, n) > 0.0) scale3(n, -1.0);
        if (g) { /* the point set's weighted average replaces the nearest disk's point and normal */
            dps_average(s, g, o, d, excl, th->eps_self, h, lambda_d, &t, n);
            for (int c = 0; c < 3; ++c) q[c] = o[c] + t * d[c];
        }
        L += t;
        tr->id[k] = h;
        copy3(tr->x[k], q);
        copy3(tr->nk[k], n);
        tr->cs[k] = -dot3(d, n);
        tr->L[k] = L;
        tr->n = k + 1;
        double dn = dot3(d, n);
        for (int c = 0; c < 3; ++c) d[c] -= 2.0 * dn * n[c];
        scale3(d, 1.0 / norm3(d));
        copy3(o, q);
        excl = h;
    }
}

/* -------------------------------------------- specular refine + validate (a8) */
/* Exact minimiser of Eq. (1) on infinite planes (image method), the convex
 * limit of the paper's iterative phase 1; phase 2 validates every interaction
 * with a ray from the previous point, thresholds t_a (angle) and t_d (plane
 * distance), and up to kappa retries that replace the failing plane with the
 * plane of the disk the validation ray hit. With point sets (Sec. II-C), the
 * planes are the representative's averaged interactions (point and normal),
 * every validation hit is averaged over its point set in the same way, and a
 * retry takes the averaged hit as the new plane. */
typedef struct {
    int valid, retries;
    int64_t hid[ORC_KMAX];
    double x[ORC_KMAX + 2][3];
    double len;
    double cs[ORC_KMAX];
    double n[ORC_KMAX][3]; /* the planes' normals the path was refined on */
} spec_t;

static int refine_on_planes(int k, const double *tx, const double *rx, double pp[][3], double pn[][3],
                            double eps_self, double x[][3])
{
    double img[ORC_KMAX + 1][3];
    copy3(img[0], tx);
    for (int m = 1; m <= k; ++m) {
        double w[3];
        sub3(w, img[m - 1], pp[m - 1]);
        double dd = dot3(w, pn[m - 1]);
        for (int c = 0; c < 3; ++c) img[m][c] = img[m - 1][c] - 2.0 * dd * pn[m - 1][c];
    }
    copy3(x[0], tx);
    copy3(x[k + 1], rx);
    double cur[3];
    copy3(cur, rx);
    for (int m = k; m >= 1; --m) {
        double seg[3], w[3];
        sub3(seg, img[m], cur);
        double den = dot3(seg, pn[m - 1]);
        if (den == 0.0) return 0;
        sub3(w, pp[m - 1], cur);
        double sp = dot3(w, pn[m - 1]) / den;
        if (!(sp > 0.0 && sp < 1.0)) return 0;
        for (int c = 0; c < 3; ++c) x[m][c] = cur[c] + sp * seg[c];
        copy3(cur, x[m]);
    }
    for (int m = 1; m <= k; ++m) {
        double a[3], b[3];
        sub3(a, x[m - 1], pp[m - 1]);
        sub3(b, x[m + 1], pp[m - 1]);
        double da = dot3(a, pn[m - 1]), db = dot3(b, pn[m - 1]);
        if (!(da * db > 0.0 && fabs(da) > eps_self && fabs(db) > eps_self)) return 0;
    }
    return 1;
}

static void specular_one(const scene_t *s, const double *tx, const double *rx, int k, const uint32_t *key,
                         const trace_t *rep, const dps_t *g, double lambda_d, const thr_t *th, spec_t *out)
{
    double pp[ORC_KMAX][3], pn[ORC_KMAX][3];
    for (int m = 0; m < k; ++m) {
        copy3(pp[m], g ? rep->x[m] : s->p + 3 * rep->id[m]);
        copy3(pn[m], g ? rep->nk[m] : s->nr + 3 * rep->id[m]);
    }
    out->valid = 0;
    out->retries = 0;
    for (;;) {
        if (!refine_on_planes(k, tx, rx, pp, pn, th->eps_self, out->x)) return;
        int64_t prev = -1;
        int retry = 0;
        for (int m = 1; m <= k; ++m) {
            double u[3], t, q[3];
            sub3(u, out->x[m], out->x[m - 1]);
            scale3(u, 1.0 / norm3(u));
            int64_t h = nearest(s, out->x[m - 1], u, prev, th->eps_self, INFINITY, th->eps_tie, &t, q);
            if (h < 0 || s->surf[h] != key[m - 1]) return;
            double hp[3], hn[3];
            copy3(hp, s->p + 3 * h);
            copy3(hn, s->nr + 3 * h);
            if (g) { /* the validation hit, averaged over its point set */
                dps_average(s, g, out->x[m - 1], u, prev, th->eps_self, h, lambda_d, &t, hn);
                for (int c = 0; c < 3; ++c) q[c] = out->x[m - 1][c] + t * u[c];
                copy3(hp, q);
            }
            double w[3];
            sub3(w, q, pp[m - 1]);
            int ang_ok = fabs(dot3(hn, pn[m - 1])) >= th->cos_ta;
            int dist_ok = fabs(dot3(w, pn[m - 1])) <= th->t_d;
            if (!(ang_ok && dist_ok)) {
                if (out->retries >= th->kappa) return;
                out->retries++;
                copy3(pp[m - 1], hp);
                copy3(pn[m - 1], hn);
                retry = 1;
                break;
            }
            out->hid[m - 1] = h;
            prev = h;
        }
        if (retry) continue;
        if (occluded(s, out->x[k], rx, out->hid[k - 1], th->eps_self)) return;
        double len = 0.0;
        for (int m = 0; m <= k; ++m) {
            double w[3];
            sub3(w, out->x[m + 1], out->x[m]);
            len += norm3(w);
        }
        out->len = len;
        for (int m = 1; m <= k; ++m) {
            double u[3];
            sub3(u, out->x[m], out->x[m - 1]);
            scale3(u, 1.0 / norm3(u));
            out->cs[m - 1] = fabs(dot3(u, pn[m - 1]));
            copy3(out->n[m - 1], pn[m - 1]);
        }
        out->valid = 1;
        return;
    }
}

/* ------------------------------------------------------- exported helpers */
/* Nearest hit for a batch of queries (unit tests). excl < 0 means none. */
int orc_nearest_batch(int64_t n_pts, const float *pos, const float *nrm, double r, int64_t n_q,
                      const double *o, const double *d, const int64_t *excl, double t_lo, double t_hi,
                      double eps_tie, int64_t *out_id, double *out_t, double *out_q)
{
    scene_t s;
    int rc = scene_init(&s, n_pts, pos, nrm, NULL, NULL, r);
    if (rc) { scene_free(&s); return rc; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_q; ++q) {
        double dd[3];
        copy3(dd, d + 3 * q);
        scale3(dd, 1.0 / norm3(dd));
        double t = NAN, qq[3] = {NAN, NAN, NAN};
        out_id[q] = nearest(&s, o + 3 * q, dd, excl[q], t_lo, t_hi, eps_tie, &t, qq);
        out_t[q] = t;
        copy3(out_q + 3 * q, qq);
    }
    scene_free(&s);
    return 0;
}

int orc_occluded_batch(int64_t n_pts, const float *pos, const float *nrm, double r, int64_t n_q,
                       const double *a, const double *b, const int64_t *excl, double eps_self,
                       uint8_t *out)
{
    scene_t s;
    int rc = scene_init(&s, n_pts, pos, nrm, NULL, NULL, r);
    if (rc) { scene_free(&s); return rc; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_q; ++q) out[q] = (uint8_t)occluded(&s, a + 3 * q, b + 3 * q, excl[q], eps_self);
    scene_free(&s);
    return 0;
}

/* Nearest hit followed by the point-set average (Eq. 3-4) for a batch of
 * queries: out_id = nearest disk (-1: miss), out_t = averaged distance,
 * out_n = averaged normal facing the incoming ray. */
int orc_average_batch(int64_t n_pts, const float *pos, const float *nrm, double r, double rho, double lambda_d,
                      int64_t n_q, const double *o, const double *d, const int64_t *excl, double eps_self,
                      double eps_tie, int64_t *out_id, double *out_t, double *out_n)
{
    scene_t s;
    int rc = scene_init(&s, n_pts, pos, nrm, NULL, NULL, r);
    if (rc) { scene_free(&s); return rc; }
    dps_t g;
    if (dps_build(&g, &s, rho)) { scene_free(&s); return -2; }
    for (int64_t k = 0; k < n_q; ++k) {
        double dd[3], t, q[3];
        copy3(dd, d + 3 * k);
        scale3(dd, 1.0 / norm3(dd));
        int64_t h = nearest(&s, o + 3 * k, dd, excl[k], eps_self, INFINITY, eps_tie, &t, q);
        out_id[k] = h;
        if (h < 0) {
            out_t[k] = NAN;
            for (int c = 0; c < 3; ++c) out_n[3 * k + c] = NAN;
            continue;
        }
        dps_average(&s, &g, o + 3 * k, dd, excl[k], eps_self, h, lambda_d, &out_t[k], out_n + 3 * k);
    }
    dps_free(&g);
    scene_free(&s);
    return 0;
}

/* ------------------------------------------ visibility matrix (Sec. II-B) */
/* Reception point of a point set: the mean of its members' centres (summed in
 * FP64 in ascending index, then rounded to FP32 like every scene coordinate).
 * Visibility of reception point j from receiver r: the open segment between
 * them meets no disk outside set j farther than eps_self from both ends (the
 * set's own disks surround its reception point and are not tested). */
static void reception_point(const scene_t *s, const dps_t *g, int64_t j, double *c)
{
    double acc[3] = {0, 0, 0};
    for (int64_t m = g->off[j]; m < g->off[j + 1]; ++m)
        for (int k = 0; k < 3; ++k) acc[k] += s->p[3 * g->mem[m] + k];
    const double n = (double)(g->off[j + 1] - g->off[j]);
    for (int k = 0; k < 3; ++k) c[k] = (double)(float)(acc[k] / n);
}

static int occluded_but_set(const scene_t *s, const dps_t *g, const double *a, const double *b, int64_t set,
                            double eps_self)
{
    double d[3];
    sub3(d, b, a);
    double len = norm3(d);
    scale3(d, 1.0 / len);
    double t, q[3], d2;
    for (int64_t i = 0; i < s->n; ++i) {
        if (g->of[i] == set) continue;
        if (ray_disk(s, i, a, d, &t, q, &d2) && t > eps_self && t < len - eps_self) return 1;
    }
    return 0;
}

/* Point sets of voxel edge rho: *n_sets; with out_recv (float[n_sets][3]) the
 * reception points; with out_vis (uint8[n_rx][n_sets]) the visibility matrix
 * from the receivers rx32 (float[n_rx][3]). */
int orc_visibility(int64_t n_pts, const float *pos, const float *nrm, double r, double rho, int32_t n_rx,
                   const float *rx32, double eps_self, int64_t *n_sets, float *out_recv, uint8_t *out_vis)
{
    scene_t s;
    int rc = scene_init(&s, n_pts, pos, nrm, NULL, NULL, r);
    if (rc) { scene_free(&s); return rc; }
    dps_t g;
    if (dps_build(&g, &s, rho)) { scene_free(&s); return -2; }
    *n_sets = g.n_sets;
    if (out_recv || out_vis) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t j = 0; j < g.n_sets; ++j) {
            double c[3];
            reception_point(&s, &g, j, c);
            if (out_recv)
                for (int k = 0; k < 3; ++k) out_recv[3 * j + k] = (float)c[k];
            if (out_vis)
                for (int32_t q = 0; q < n_rx; ++q) {
                    double a[3];
                    from_f32(a, rx32 + 3 * q);
                    out_vis[(int64_t)q * g.n_sets + j] = (uint8_t)!occluded_but_set(&s, &g, a, c, j, eps_self);
                }
        }
    }
    dps_free(&g);
    scene_free(&s);
    return 0;
}

/* ------------------------------------------------------------- full solve */
typedef struct {
    int len;
    uint32_t s[ORC_KMAX];
    int64_t ray_id;
    int64_t slot; /* index into the traced list */
} keyrec_t;

static int key_cmp(const void *pa, const void *pb)
{
    const keyrec_t *a = (const keyrec_t *)pa, *b = (const keyrec_t *)pb;
    if (a->len != b->len) return a->len < b->len ? -1 : 1;
    for (int m = 0; m < a->len; ++m)
        if (a->s[m] != b->s[m]) return a->s[m] < b->s[m] ? -1 : 1;
    if (a->ray_id != b->ray_id) return a->ray_id < b->ray_id ? -1 : 1;
    return 0;
}

/*
 * One TX, all RX. Traces the rays with the given ids out of a budget of
 * n_budget Fibonacci directions (the diffuse ray-tube weight always uses the
 * full budget).
 *
 * thr[13] = {eps_tie, eps_self, t_a (degrees), t_d, kappa, rho, lambda_d,
 * pol_tx (3), pol_rx (3)}; rho (voxel edge of the point sets) and lambda_d
 * (depth attenuation) are read with ORC_AVERAGE / ORC_DPS_LAUNCH only, the
 * polarisations with ORC_POLARIZED only. With ORC_POLARIZED every line-of-
 * sight and specular path has one complex amplitude a (path_polarized),
 * reported in both channels (a_TE = a_TM = a, so its power
 * 1/2(|a_TE|^2 + |a_TM|^2) is |a|^2); diffuse paths, the Jacobian and the
 * frequency response are refused (-1).
 *
 * Outputs (NULL = not wanted):
 *   seq      int64[n_trace*K]   hit disk per (ray, k), -1 after the ray ends
 *   rec      double[n_trace*K*5] x, y, z, L, cos per (ray, k)
 *   dvis     uint8[n_trace*K*n_rx] diffuse connection valid (lit side and unoccluded)
 *   dpow     double[n_trace*K*n_rx] power 1/2(|a_TE|^2 + |a_TM|^2) of every connection on
 *            the lit side, occluded or not (0 elsewhere): lets a comparison price the
 *            connections on which two runs disagree about occlusion
 *   keys     uint32[key_cap*K], key_len int32[key_cap], key_rep int64[key_cap]
 *   spec_valid uint8[key_cap*n_rx], spec_len double[key_cap*n_rx],
 *   spec_amp double[key_cap*n_rx*4] (TE re, im, TM re, im), spec_hid int64[key_cap*n_rx*K]
 *   out_rx   double[n_rx*8]: G_los, G_spec, G_diff, G, h_TE re, im, h_TM re, im
 *   jac      double[n_rx*n_labels*3]: dG/d(eps_r, sigma, S) per label
 *   out_cfr  double[n_rx*n_freq*4]: channel frequency response (TE re, im,
 *            TM re, im) at n_freq frequencies spanning bandwidth around freq
 * *n_keys receives the number of unique keys; returns -3 if key_cap is too small.
 */
int orc_solve(int64_t n_pts, const float *pos, const float *nrm, const uint16_t *mat, const uint32_t *surf,
              double r_p, int32_t n_labels, const double *eps_r, const double *sigma, const double *scat,
              const float *tx32, int32_t n_rx, const float *rx32, double freq, int64_t n_budget,
              int64_t n_trace, const int64_t *ray_ids, int32_t K, int32_t flags, const double *thr,
              int64_t *seq, double *rec, uint8_t *dvis, double *dpow, int64_t key_cap, uint32_t *keys,
              int32_t *key_len,
              int64_t *key_rep, int64_t *n_keys, uint8_t *spec_valid, double *spec_len, double *spec_amp,
              int64_t *spec_hid, double *out_rx, double *jac, int32_t n_freq, double bandwidth, double *out_cfr)
{
    if (K < 1 || K > ORC_KMAX) return -1;
    scene_t s;
    int rc = scene_init(&s, n_pts, pos, nrm, mat, surf, r_p);
    if (rc) { scene_free(&s); return rc; }
    for (int64_t i = 0; i < n_pts; ++i)
        if (mat[i] >= (uint32_t)n_labels) { scene_free(&s); return -1; }
    thr_t th = {thr[0], thr[1], cos(thr[2] * ORC_PI / 180.0), thr[3], (int)thr[4]};
    const int polarized = (flags & ORC_POLARIZED) != 0;
    if (polarized && ((flags & ORC_DIFFUSE) || jac || out_cfr)) { scene_free(&s); return -1; }
    const double *ptx = thr + 7, *prx = thr + 10;
    dps_t dps, *sets = NULL, *g = NULL; /* g: the sets when interactions are averaged */
    if (flags & (ORC_AVERAGE | ORC_DPS_LAUNCH)) {
        if (!(thr[5] > 0.0) || ((flags & ORC_AVERAGE) && !(thr[6] > 0.0))) { scene_free(&s); return -1; }
        if (dps_build(&dps, &s, thr[5])) { scene_free(&s); return -2; }
        sets = &dps;
        if (flags & ORC_AVERAGE) g = &dps;
        if (flags & ORC_DPS_LAUNCH)
            for (int64_t q = 0; q < n_trace; ++q)
                if (ray_ids[q] < 0 || ray_ids[q] >= dps.n_sets) { dps_free(&dps); scene_free(&s); return -1; }
    }
    em_t em = {n_labels, eps_r, sigma, scat, freq, 2.0 * ORC_PI * freq, ORC_C0 / freq, 0.0};
    em.k0 = 2.0 * ORC_PI / em.lambda;
    const double a_iso = em.lambda / (4.0 * ORC_PI);
    double tx[3];
    from_f32(tx, tx32);
    double *rx = (double *)malloc(sizeof(double) * 3 * (size_t)n_rx);
    for (int r = 0; r < n_rx; ++r) from_f32(rx + 3 * r, rx32 + 3 * r);

    double *G_los = calloc((size_t)n_rx, sizeof(double)), *G_spec = calloc((size_t)n_rx, sizeof(double));
    double *G_diff = calloc((size_t)n_rx, sizeof(double));
    double complex *h_te = calloc((size_t)n_rx, sizeof(double complex));
    double complex *h_tm = calloc((size_t)n_rx, sizeof(double complex));
    if (jac) memset(jac, 0, sizeof(double) * (size_t)n_rx * (size_t)n_labels * 3);
    cfr_t cfr = {out_cfr ? n_freq : 0, bandwidth, NULL};
    if (cfr.n > 0) cfr.h = calloc((size_t)n_rx * (size_t)cfr.n * 2, sizeof(double complex));

    /* line of sight */
    if (flags & ORC_LOS) {
        for (int r = 0; r < n_rx; ++r) {
            if (occluded(&s, tx, rx + 3 * r, -1, th.eps_self)) continue;
            double w[3];
            sub3(w, rx + 3 * r, tx);
            double d = norm3(w);
            double complex a = a_iso / d * cexp(-I * em.k0 * d);
            if (polarized) {
                double x2[2][3];
                copy3(x2[0], tx);
                copy3(x2[1], rx + 3 * r);
                a = path_polarized(&em, 0, (const double(*)[3])x2, NULL, NULL, a_iso / d, d, ptx, prx);
            }
            G_los[r] += 0.5 * (creal(a * conj(a)) * 2.0);
            h_te[r] += a;
            h_tm[r] += a;
            cfr_add(&cfr, r, a, a, d);
        }
    }

    /* trace every requested ray */
    trace_t *tr = (trace_t *)malloc(sizeof(trace_t) * (size_t)(n_trace > 0 ? n_trace : 1));
    float *dirs = (float *)malloc(sizeof(float) * 3 * (size_t)(n_trace > 0 ? n_trace : 1));
    if (flags & ORC_DPS_LAUNCH) {
        /* one ray towards each requested set's reception point (Sec. II-B):
         * the direction in FP64, rounded to FP32 like the sphere directions */
        for (int64_t q = 0; q < n_trace; ++q) {
            double c[3], d[3];
            reception_point(&s, sets, ray_ids[q], c);
            sub3(d, c, tx);
            scale3(d, 1.0 / norm3(d));
            for (int k = 0; k < 3; ++k) dirs[3 * q + k] = (float)d[k];
        }
    } else {
        orc_fib_dirs(n_budget, ray_ids, n_trace, dirs);
    }
    if (flags & (ORC_SPECULAR | ORC_DIFFUSE | ORC_TRACE)) {
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t q = 0; q < n_trace; ++q) trace_ray(&s, tx, dirs + 3 * q, K, &th, g, g ? thr[6] : 0.0, &tr[q]);
    } else {
        for (int64_t q = 0; q < n_trace; ++q) tr[q].n = 0;
    }
    if (seq || rec) {
        for (int64_t q = 0; q < n_trace; ++q)
            for (int k = 0; k < K; ++k) {
                int has = k < tr[q].n;
                if (seq) seq[q * K + k] = has ? tr[q].id[k] : -1;
                if (rec) {
                    double *o = rec + (q * K + k) * 5;
                    for (int c = 0; c < 3; ++c) o[c] = has ? tr[q].x[k][c] : NAN;
                    o[3] = has ? tr[q].L[k] : NAN;
                    o[4] = has ? tr[q].cs[k] : NAN;
                }
            }
    }

    if ((flags & ORC_DIFFUSE) && (flags & ORC_DPS_LAUNCH)) {
        /* Diffuse paths of the reception-point launch (Sec. II-B.1, II-B.4): one path
         * per unique (surface labels of the interactions before the last, point set of
         * the last); its representative (smallest ray id) gives the geometry. A path
         * reaches receiver r when r sees the set's reception point (the visibility
         * matrix) and lies on the lit side of the representative's interaction. It
         * stands for the field scattered by an area rho^2 there: a Lambertian patch lit
         * from the (image) transmitter at the unfolded length L,
         *   amp0 = lambda/(4 pi) sqrt(rho^2 cos_i cos_s / pi) / (L r_s),
         * which for the footprint of one ray tube, 4 pi L^2 / (N cos_i), is the ray-tube
         * amplitude of the per-interaction connections. */
        const double area = thr[5] * thr[5];
        int64_t total = 0;
        for (int64_t q = 0; q < n_trace; ++q) total += tr[q].n;
        keyrec_t *kr = (keyrec_t *)malloc(sizeof(keyrec_t) * (size_t)(total > 0 ? total : 1));
        int64_t e = 0;
        for (int64_t q = 0; q < n_trace; ++q)
            for (int k = 1; k <= tr[q].n; ++k) {
                memset(&kr[e], 0, sizeof(keyrec_t));
                kr[e].len = k;
                for (int m = 0; m < k - 1; ++m) kr[e].s[m] = s.surf[tr[q].id[m]];
                kr[e].s[k - 1] = (uint32_t)sets->of[tr[q].id[k - 1]];
                kr[e].ray_id = ray_ids[q];
                kr[e].slot = q;
                ++e;
            }
        qsort(kr, (size_t)total, sizeof(keyrec_t), key_cmp);
        for (int64_t i = 0; i < total; ++i) {
            if (i > 0 && kr[i].len == kr[i - 1].len && !memcmp(kr[i].s, kr[i - 1].s, sizeof(uint32_t) * (size_t)kr[i].len))
                continue;
            const trace_t *t = &tr[kr[i].slot];
            const int k = kr[i].len;
            const int64_t set = kr[i].s[k - 1];
            double c[3];
            reception_point(&s, sets, set, c);
            int label[ORC_KMAX], kind[ORC_KMAX];
            double cs[ORC_KMAX];
            for (int m = 0; m < k; ++m) {
                label[m] = s.mat[t->id[m]];
                cs[m] = t->cs[m];
                kind[m] = (m == k - 1);
            }
            for (int r = 0; r < n_rx; ++r) {
                if (occluded_but_set(&s, sets, rx + 3 * r, c, set, th.eps_self)) continue;
                double v[3];
                sub3(v, rx + 3 * r, t->x[k - 1]);
                double vn = dot3(v, t->nk[k - 1]);
                if (!(vn > 0.0)) continue;
                double rs = norm3(v);
                double amp0 = a_iso * sqrt(area * cs[k - 1] * (vn / rs) / ORC_PI) / (t->L[k - 1] * rs);
                double complex ate = 0, atm = 0;
                path_field(&em, k, label, cs, kind, amp0, t->L[k - 1] + rs, &ate, &atm, &G_diff[r],
                           jac ? jac + (int64_t)r * n_labels * 3 : NULL);
                h_te[r] += ate;
                h_tm[r] += atm;
                cfr_add(&cfr, r, ate, atm, t->L[k - 1] + rs);
            }
        }
        free(kr);
        if (dvis) memset(dvis, 0, (size_t)(n_trace * K * n_rx));
    } else if (flags & ORC_DIFFUSE) {
        /* diffuse connections from every interaction to every RX (Sec. II-B.1) */
        int64_t nslot = n_trace * K * (int64_t)n_rx;
        if (dpow) memset(dpow, 0, sizeof(double) * (size_t)nslot);
        double complex *ate = calloc((size_t)nslot, sizeof(double complex));
        double complex *atm = calloc((size_t)nslot, sizeof(double complex));
        double *pw = calloc((size_t)nslot, sizeof(double));
        double *plen = calloc((size_t)nslot, sizeof(double));
        double *jl = jac ? calloc((size_t)nslot * (size_t)n_labels * 3, sizeof(double)) : NULL;
        uint8_t *vis = calloc((size_t)nslot, 1);
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t q = 0; q < n_trace; ++q) {
            for (int k = 0; k < tr[q].n; ++k) {
                int label[ORC_KMAX], kind[ORC_KMAX];
                double cs[ORC_KMAX];
                for (int m = 0; m <= k; ++m) {
                    label[m] = s.mat[tr[q].id[m]];
                    cs[m] = tr[q].cs[m];
                    kind[m] = (m == k);
                }
                for (int r = 0; r < n_rx; ++r) {
                    int64_t slot = (q * K + k) * n_rx + r;
                    double v[3];
                    sub3(v, rx + 3 * r, tr[q].x[k]);
                    double vn = dot3(v, tr[q].nk[k]);
                    if (!(vn > 0.0)) continue;
                    const int occ = occluded(&s, tr[q].x[k], rx + 3 * r, tr[q].id[k], th.eps_self);
                    double rs = norm3(v);
                    double cos_s = vn / rs;
                    double amp0 = a_iso * sqrt(4.0 * cos_s / (double)n_budget) / rs;
                    if (dpow) { /* the connection's power as if unoccluded */
                        double complex a1 = 0, a2 = 0;
                        double p1 = 0.0;
                        path_field(&em, k + 1, label, cs, kind, amp0, tr[q].L[k] + rs, &a1, &a2, &p1, NULL);
                        dpow[slot] = p1;
                    }
                    if (occ) continue;
                    vis[slot] = 1;
                    plen[slot] = tr[q].L[k] + rs;
                    path_field(&em, k + 1, label, cs, kind, amp0, tr[q].L[k] + rs, &ate[slot], &atm[slot],
                               &pw[slot], jl ? jl + slot * n_labels * 3 : NULL);
                }
            }
        }
        for (int64_t q = 0; q < n_trace; ++q)
            for (int k = 0; k < K; ++k)
                for (int r = 0; r < n_rx; ++r) {
                    int64_t slot = (q * K + k) * n_rx + r;
                    if (dvis) dvis[slot] = vis[slot];
                    if (!vis[slot]) continue;
                    G_diff[r] += pw[slot];
                    h_te[r] += ate[slot];
                    h_tm[r] += atm[slot];
                    cfr_add(&cfr, r, ate[slot], atm[slot], plen[slot]);
                    if (jac)
                        for (int l = 0; l < 3 * n_labels; ++l) jac[r * n_labels * 3 + l] += jl[slot * n_labels * 3 + l];
                }
        free(ate); free(atm); free(pw); free(plen); free(jl); free(vis);
    } else if (dvis) {
        memset(dvis, 0, (size_t)(n_trace * K * n_rx));
    }

    /* specular: keys of surface labels, representative = smallest ray id */
    int64_t nk = 0;
    int ret = 0;
    if (flags & ORC_SPECULAR) {
        int64_t total = 0;
        for (int64_t q = 0; q < n_trace; ++q) total += tr[q].n;
        keyrec_t *kr = (keyrec_t *)malloc(sizeof(keyrec_t) * (size_t)(total > 0 ? total : 1));
        int64_t e = 0;
        for (int64_t q = 0; q < n_trace; ++q)
            for (int k = 1; k <= tr[q].n; ++k) {
                memset(&kr[e], 0, sizeof(keyrec_t));
                kr[e].len = k;
                for (int m = 0; m < k; ++m) kr[e].s[m] = s.surf[tr[q].id[m]];
                kr[e].ray_id = ray_ids[q];
                kr[e].slot = q;
                ++e;
            }
        qsort(kr, (size_t)total, sizeof(keyrec_t), key_cmp);
        keyrec_t *uk = (keyrec_t *)malloc(sizeof(keyrec_t) * (size_t)(total > 0 ? total : 1));
        for (int64_t i = 0; i < total; ++i) {
            if (i > 0 && kr[i].len == kr[i - 1].len && !memcmp(kr[i].s, kr[i - 1].s, sizeof(uint32_t) * (size_t)kr[i].len))
                continue;
            uk[nk++] = kr[i];
        }
        free(kr);
        if (nk > key_cap) {
            ret = -3;
        } else {
            spec_t *sp = (spec_t *)malloc(sizeof(spec_t) * (size_t)(nk * n_rx > 0 ? nk * n_rx : 1));
            int64_t npair = nk * n_rx;
#pragma omp parallel for schedule(dynamic, 1)
            for (int64_t pi = 0; pi < npair; ++pi) {
                int64_t ki = pi / n_rx;
                int r = (int)(pi % n_rx);
                const keyrec_t *key = &uk[ki];
                if (flags & ORC_DPS_LAUNCH) {
                    /* candidate only where the receiver sees the reception point of the
                     * set the representative's path ends in (the visibility matrix) */
                    const int64_t j = sets->of[tr[key->slot].id[key->len - 1]];
                    double c[3];
                    reception_point(&s, sets, j, c);
                    if (occluded_but_set(&s, sets, rx + 3 * r, c, j, th.eps_self)) {
                        sp[pi].valid = 0;
                        continue;
                    }
                }
                specular_one(&s, tx, rx + 3 * r, key->len, key->s, &tr[key->slot], g, g ? thr[6] : 0.0, &th, &sp[pi]);
            }
            for (int64_t ki = 0; ki < nk; ++ki) {
                if (keys)
                    for (int m = 0; m < K; ++m) keys[ki * K + m] = m < uk[ki].len ? uk[ki].s[m] : 0xffffffffu;
                if (key_len) key_len[ki] = uk[ki].len;
                if (key_rep) key_rep[ki] = uk[ki].ray_id;
                for (int r = 0; r < n_rx; ++r) {
                    spec_t *p = &sp[ki * n_rx + r];
                    int64_t o = ki * n_rx + r;
                    if (spec_valid) spec_valid[o] = (uint8_t)p->valid;
                    if (spec_hid)
                        for (int m = 0; m < K; ++m) spec_hid[o * K + m] = (p->valid && m < uk[ki].len) ? p->hid[m] : -1;
                    double complex ate = 0, atm = 0;
                    if (p->valid) {
                        int label[ORC_KMAX], kind[ORC_KMAX];
                        for (int m = 0; m < uk[ki].len; ++m) {
                            label[m] = s.mat[p->hid[m]];
                            kind[m] = 0;
                        }
                        double g = 0.0;
                        if (polarized) {
                            ate = atm = path_polarized(&em, uk[ki].len, (const double(*)[3])p->x,
                                                       (const double(*)[3])p->n, label, a_iso / p->len, p->len,
                                                       ptx, prx);
                            g = creal(ate * conj(ate));
                        } else {
                            path_field(&em, uk[ki].len, label, p->cs, kind, a_iso / p->len, p->len, &ate, &atm, &g,
                                       jac ? jac + (int64_t)r * n_labels * 3 : NULL);
                        }
                        G_spec[r] += g;
                        h_te[r] += ate;
                        h_tm[r] += atm;
                        cfr_add(&cfr, r, ate, atm, p->len);
                    }
                    if (spec_len) spec_len[o] = p->valid ? p->len : NAN;
                    if (spec_amp) {
                        spec_amp[4 * o + 0] = creal(ate);
                        spec_amp[4 * o + 1] = cimag(ate);
                        spec_amp[4 * o + 2] = creal(atm);
                        spec_amp[4 * o + 3] = cimag(atm);
                    }
                }
            }
            free(sp);
        }
        free(uk);
    }
    if (n_keys) *n_keys = nk;
    if (out_rx)
        for (int r = 0; r < n_rx; ++r) {
            double *o = out_rx + 8 * r;
            o[0] = G_los[r];
            o[1] = G_spec[r];
            o[2] = G_diff[r];
            o[3] = G_los[r] + G_spec[r] + G_diff[r];
            o[4] = creal(h_te[r]);
            o[5] = cimag(h_te[r]);
            o[6] = creal(h_tm[r]);
            o[7] = cimag(h_tm[r]);
        }
    if (cfr.n > 0)
        for (size_t i = 0; i < (size_t)n_rx * (size_t)cfr.n * 2; ++i) {
            out_cfr[2 * i] = creal(cfr.h[i]);
            out_cfr[2 * i + 1] = cimag(cfr.h[i]);
        }
    free(cfr.h);
    free(tr); free(dirs); free(rx); free(G_los); free(G_spec); free(G_diff); free(h_te); free(h_tm);
    if (sets) dps_free(sets);
    scene_free(&s);
    return ret;
}
