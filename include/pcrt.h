/*
 * pcrt.h -- C ABI of the MI355X (gfx950) point-cloud radio ray tracer.
 *
 * Method: Vaara et al., "Differentiable High-Performance Ray Tracing-Based
 * Simulation of Radio Propagation with Point Clouds", arXiv 2507.04021.
 *
 * Problem statement (Sec. II, opening paragraph): the input is an augmented
 * point cloud -- per point a position p_i, a surface normal n, a surface label
 * l_s and a material label l_m -- together with TX and RX positions. The
 * output here is, per receiver, the channel power gain and the coherent
 * complex field of all paths found: line of sight, specular reflections
 * (Sec. II-B.2) and diffuse scattering as the last interaction (Sec. II-B.1).
 *
 * Conventions
 *   - Units: metres, hertz, siemens per metre. Gains are linear power.
 *   - Time convention e^{+j omega t}: propagation over length L multiplies the
 *     field by e^{-j k0 L}; eta = eps_r - j sigma / (omega eps0).
 *   - Every device pointer is memory on the current HIP device, owned by the
 *     caller. The library never frees caller memory.
 *   - Every call returns a pcrt_status; none throws or aborts. On failure the
 *     reason is available from pcrt_last_error() (thread-local).
 *   - Calls that take a stream only enqueue work on that stream (no host
 *     synchronisation) unless the comment says otherwise. The solve calls
 *     allocate nothing; every scratch byte comes from the caller's workspace,
 *     so they can be captured in a HIP graph.
 */
#ifndef PCRT_H
#define PCRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PCRT_OK = 0,
    PCRT_EINVAL = -1,       /* invalid argument or input data */
    PCRT_ENOMEM = -2,       /* workspace too small (required size in the error text) */
    PCRT_EDEVICE = -3,      /* HIP runtime error */
    PCRT_EUNSUPPORTED = -4, /* valid request outside the supported range */
    PCRT_EOVERFLOW = -5     /* a device-side capacity was exceeded */
} pcrt_status;

/* Text of the last error on this thread; valid until the next call. */
const char *pcrt_last_error(void);
/* Library version string. */
const char *pcrt_version(void);

/* ------------------------------------------------------------------ scene */
/* The point cloud as surface-aligned disks (Sec. II-C): disk i has centre
 * pos[i], unit normal normal[i] (normalised by the library), radius
 * disk_radius (one radius for all points). Disks are two-sided.
 * pos, normal: device float[n_points][3]; material: device uint16[n_points]
 * (material label, < n_labels of the solve); surface: device uint32[n_points]
 * (surface label; keys of specular paths are sequences of these). */
typedef struct {
    const float *pos;
    const float *normal;
    const uint16_t *material;
    const uint32_t *surface;
    uint32_t n_points;
    float disk_radius;
} pcrt_points;

/* Bounding-volume hierarchy options. leaf_size: disks per leaf, 1..8
 * (0 = default 4). width: children per node -- 2 (binary radix tree), 4 or 8
 * (wide nodes collapsed from it, largest-area child opened first); 0 = 4.
 * Results do not depend on either option, only speed does. */
typedef struct {
    uint32_t leaf_size;
    uint32_t width;
    uint32_t builder; /* PCRT_BUILD_*; 0 = default (PCRT_BUILD_PLOC) */
    /* Discretised point sets (Sec. II-A): voxel edge rho in metres; each
     * non-empty voxel floor(p / rho) (per axis, evaluated in FP64 from the
     * FP32 centres) is one set. 0 = no sets; PCRT_AVERAGE solves need them.
     * Voxel indices must stay within +-2^20 (else EUNSUPPORTED). */
    float dps_voxel;
} pcrt_bvh_opts;

enum {
    PCRT_BUILD_LBVH = 1, /* Karras radix tree over Morton codes of the disk centres */
    PCRT_BUILD_PLOC = 2  /* locally-ordered clustering: mutual nearest neighbours by merged surface area within
                            +-16 positions of the Morton order, disks renumbered depth-first */
};

/* Scene statistics filled by pcrt_scene_create. */
typedef struct {
    uint32_t n_points;
    uint32_t n_surfaces;   /* max surface label + 1 */
    uint32_t n_materials;  /* max material label + 1 */
    uint32_t depth;        /* internal ancestors of the deepest leaf of the binary tree */
    uint32_t n_nodes;      /* nodes of the traversed hierarchy (wide nodes if width > 2) */
    uint32_t leaf_size;
    uint32_t width;
    uint32_t stack_entries; /* bound on traversal stack entries: (width - 1) x levels */
    uint32_t builder;
    float bbox[6];         /* lo xyz, hi xyz of the disk bounds */
    double build_ms;       /* device time of the build (point sets included) */
    uint32_t n_point_sets; /* non-empty voxels (0 without dps_voxel) */
    float dps_voxel;
} pcrt_scene_info;

typedef struct pcrt_scene pcrt_scene; /* opaque host handle */

/* Bytes of device workspace a scene of n_points needs (BVH, disk copies and,
 * with dps_voxel > 0, the point sets). */
pcrt_status pcrt_scene_workspace_size(uint32_t n_points, const pcrt_bvh_opts *opts, size_t *bytes);

/* Validate the points, copy them, build the hierarchy (Morton codes, radix
 * sort, linear BVH) in ws. The input arrays may be freed afterwards; ws must
 * outlive the scene. This call synchronises the stream once at the end to
 * read back validation results and statistics. Errors: EINVAL for NULL
 * pointers, n_points == 0, disk_radius <= 0, non-finite positions or zero
 * normals, a negative or non-finite dps_voxel; ENOMEM for a small ws;
 * EUNSUPPORTED for voxel indices beyond +-2^20, more than 2^26 points
 * (the traversal kernels address the node and disk arrays with 32-bit byte
 * offsets), an unsupported leaf size, width or builder, or a hierarchy whose
 * traversal stack bound exceeds the supported maximum. stream: hipStream_t
 * or NULL. */
pcrt_status pcrt_scene_create(const pcrt_points *pts, const pcrt_bvh_opts *opts, void *ws, size_t ws_bytes,
                              void *stream, pcrt_scene **out);
pcrt_status pcrt_scene_get_info(const pcrt_scene *scene, pcrt_scene_info *info);
pcrt_status pcrt_scene_destroy(pcrt_scene *scene);

/* ------------------------------------------ visibility matrix (Sec. II-A, II-B) */
/* Reception point of each point set: the mean of its members' centres (summed
 * in FP64 in increasing point index, rounded to FP32). out: device
 * float[n_point_sets][3]. Errors: EINVAL without point sets or NULL pointers. */
pcrt_status pcrt_reception_points(const pcrt_scene *scene, float *out, void *stream);

/* Device workspace of pcrt_visibility (traversal stack spill; >= 256 bytes). */
pcrt_status pcrt_visibility_workspace_size(const pcrt_scene *scene, size_t *bytes);

/* Visibility matrix: vis[r][j] = 1 when receiver r sees reception point j,
 * i.e. the open segment between them meets no disk outside set j farther
 * than eps_self (0 = 1e-3 m) from both ends; else 0. rx: device
 * float[n_rx][3]; vis: device uint8[n_rx][n_point_sets], overwritten. The
 * result does not depend on the hierarchy options. Asynchronous on stream,
 * allocates nothing. Errors: EINVAL without point sets, for NULL pointers,
 * n_rx == 0 or a negative eps_self; ENOMEM for a small ws; EUNSUPPORTED for
 * n_rx x n_point_sets >= 2^32. */
pcrt_status pcrt_visibility(const pcrt_scene *scene, const float *rx, uint32_t n_rx, float eps_self, void *ws,
                            size_t ws_bytes, uint8_t *vis, void *stream);

/* ------------------------------------------------------------------ solve */
/* Material of one label: relative permittivity, conductivity (S/m) and
 * scattering coefficient S in [0, 1]. Specular reflections carry
 * sqrt(1 - S^2) times the Fresnel coefficient, diffuse ones S times it. */
typedef struct {
    float eps_r, sigma, scatter;
} pcrt_material;

/* Thresholds. eps_tie: nearest-hit tie window (m); eps_self: minimum distance
 * from a ray origin to a hit (m); t_a_deg, t_d: validation thresholds of
 * Table I (angle in degrees, plane distance in m); kappa: refinement retries.
 * Zero fields take the defaults 1e-4, 1e-3, 1.0, 0.01, 10 (kappa = 0 is
 * expressed as PCRT_KAPPA_NONE). */
typedef struct {
    float eps_tie, eps_self, t_a_deg, t_d;
    uint32_t kappa;
} pcrt_thresholds;
#define PCRT_KAPPA_NONE 0xffffffffu

enum {
    PCRT_LOS = 1,      /* line of sight */
    PCRT_SPECULAR = 2, /* specular paths (keys, refinement, validation) */
    PCRT_DIFFUSE = 4,  /* diffuse scattering as the last interaction */
    PCRT_RECORD = 8,   /* keep the per-path tape in the workspace (for the gradient and path output) */
    PCRT_TIMING = 16,  /* record HIP events between stages (read with pcrt_stage_times) */
    /* Weighted-average intersection (Sec. II-C, Eq. 3-4): every interaction
     * is the weighted mean, over the hit disk's point set, of the ray's
     * intersections farther than eps_self, with weights
     * exp(-|q_i - p_i|^2 / (2 r_p^2)) exp(-lambda_d |q_i - q_min|) (q_min: the
     * member intersection nearest to the origin); the ray reflects about the
     * weighted sum of the member normals turned to face it. The nearest disk
     * still names the interaction (material, surface label, sequence).
     * Needs a scene built with dps_voxel > 0 (else EINVAL). */
    PCRT_AVERAGE = 32,
    /* The paper's launch (Sec. II-B): ray j goes from the transmitter towards
     * the reception point of point set j (n_rays must equal the scene's
     * n_point_sets; a ray_subset lists set indices, others end at once), and
     * a (key, receiver) pair is a specular candidate only where dps_vis says
     * the receiver sees the reception point of the set the key's
     * representative ray ends in. Needs point sets and dps_vis (EINVAL).
     * With PCRT_DIFFUSE, diffuse paths are deduplicated per voxel, each an
     * area rho^2 (Sec. II-B.4); with PCRT_RECORD the tape covers them (gains
     * and material gradients; pcrt_diffuse_vis_copy and the frequency-response
     * calls refuse such a solve: EUNSUPPORTED). Batches are refused. */
    PCRT_DPS_LAUNCH = 64,
    /* Polarised field (Jones vectors) of line-of-sight and specular paths, for
     * the field the paper takes from its EM back end: the transmitter radiates
     * pol_tx projected on the plane normal to the departure direction (a short
     * dipole); at every reflection the field splits into its components
     * normal to the plane of incidence (s = d_in x n / |d_in x n|, TE) and in
     * it (p_in = s x d_in, TM) and leaves as
     *   R (Gamma_TE (E.s) s + Gamma_TM (E.p_in) p_out),  p_out = s x d_out
     * (R = sqrt(1 - S^2)); the receiver takes the arriving field's projection
     * on pol_rx projected on the plane normal to the arrival direction. Each
     * path then has one complex amplitude a, reported in both channels
     * (a_TE = a_TM = a, as line of sight is in the scalar model): G = sum |a|^2
     * and h_te = h_tm = sum a; a PCRT_RECORD solve's path list
     * (pcrt_paths_copy) carries a in both amplitude pairs. PCRT_DIFFUSE is
     * refused with it, and so are the tape calls on such a solve
     * (EUNSUPPORTED: the tape holds the scalar model); pol_tx and pol_rx must
     * be finite (EINVAL). */
    PCRT_POLARIZED = 128
};

/* One transmitter. rx: device float[n_rx][3]. n_rays: ray budget N (Fibonacci
 * sphere directions; the diffuse ray-tube weight uses N). ray_subset
 * (optional device uint32[n_subset]): trace only these ray ids of the budget.
 * max_interactions K: 1..8. key_capacity: keys whose per-receiver results a
 * PCRT_RECORD solve keeps on its tape (0 = min(rays * K, 262144)); more keys
 * set bit 2 of the status word and are left off the tape (not off the gain). */
typedef struct {
    float tx[3];
    const float *rx;
    uint32_t n_rx;
    double freq_hz;
    uint32_t n_rays;
    uint32_t max_interactions;
    uint32_t flags;
    const uint32_t *ray_subset;
    uint32_t n_subset;
    pcrt_thresholds thr;
    uint32_t key_capacity;
    uint32_t wave_rays; /* rays a wavefront takes per work fetch, multiple of 64 up to 1024 (0 = 64) */
    float lambda_d;     /* depth attenuation of PCRT_AVERAGE, 1/m (0 = 100) */
    const uint8_t *dps_vis; /* PCRT_DPS_LAUNCH: device uint8[n_rx][n_point_sets] from pcrt_visibility for rx */
    float pol_tx[3];        /* PCRT_POLARIZED: transmit and receive polarisation vectors (any length; */
    float pol_rx[3];        /* the amplitude scales with both) */
} pcrt_solve_params;

/* Outputs (device pointers; NULL = not wanted unless marked required).
 *   gain       double[n_rx]         required: total power gain G_r
 *   h_te, h_tm double[n_rx][2]      coherent complex field sums (re, im)
 *   gain_parts double[n_rx][3]      G of LOS, specular, diffuse paths
 *   ray_seq    int32[n_trace][K]    hit disk per interaction, -1 after the ray ends
 *   counters   uint64[16]           see PCRT_CNT_* */
typedef struct {
    double *gain;
    double *h_te;
    double *h_tm;
    double *gain_parts;
    int32_t *ray_seq;
    uint64_t *counters;
} pcrt_outputs;

enum {
    PCRT_CNT_INTERACTIONS = 0, /* closest-hit interactions traced (sum of K_j) */
    PCRT_CNT_RAYS = 1,         /* rays traced */
    PCRT_CNT_SEGMENTS = 2,     /* diffuse connection segments tested for occlusion */
    PCRT_CNT_KEYS = 3,         /* unique specular keys */
    PCRT_CNT_SPECULAR = 4,     /* valid specular paths (over all receivers) */
    PCRT_CNT_DIFFUSE = 5,      /* visible diffuse connections */
    PCRT_CNT_STATUS = 6,       /* bit 0: key table overflow; bit 1: invalid material label; bit 2: tape key capacity exceeded */
    PCRT_CNT_CANDIDATES = 7,   /* (key, RX) pairs that passed the geometric refinement */
    PCRT_CNT_TIE_SPILL = 8,    /* nearest-hit queries that needed the exact second pass */
    PCRT_CNT_COUNT = 16
};

/* Decode the status word of a solve (counters[PCRT_CNT_STATUS] of a host copy
 * of the 16 counters, read back once the solve has finished). Returns PCRT_OK
 * when no bit is set; otherwise the reason text (pcrt_last_error) names every
 * set condition and the status is that of the first of:
 *   bit 1  a material label >= n_labels was met (label 0 was used) -> EINVAL
 *   bit 0  the key table overflowed: some specular (or voxel diffuse) keys
 *          were dropped, so their paths are missing from every output -> EOVERFLOW
 *   bit 2  a PCRT_RECORD solve found more keys than key_capacity: those
 *          paths are in the gains but not on the tape (nor in gradients) -> EOVERFLOW
 * counters_host_copy: host uint64[16]; NULL -> EINVAL. No device work. */
pcrt_status pcrt_status_poll(const uint64_t *counters_host_copy);

/* Workspace bytes for one solve with these parameters (plus, with
 * PCRT_RECORD, the tape). */
pcrt_status pcrt_solve_workspace_size(const pcrt_scene *scene, const pcrt_solve_params *p, size_t *bytes);

/* Trace and evaluate one transmitter against all receivers. mats: device
 * pcrt_material[n_labels]. Asynchronous on stream; allocates nothing.
 * Errors: EINVAL (bad sizes, NULL required pointers, freq <= 0, n_rays == 0
 * with SPECULAR or DIFFUSE), EUNSUPPORTED (K > 8, or surface labels too many
 * for exact keys: (n_surfaces + 1)^K must be < 2^64), ENOMEM (small ws).
 * Device-side problems set bits in counters[PCRT_CNT_STATUS]. */
pcrt_status pcrt_solve(const pcrt_scene *scene, const pcrt_material *mats, uint32_t n_labels,
                       const pcrt_solve_params *p, void *ws, size_t ws_bytes, const pcrt_outputs *out,
                       void *stream);

/* Specular path list of a PCRT_RECORD solve, copied out of its workspace.
 * Keys are ordered by (representative ray id, length). For key q:
 *   key_ray uint32[cap]   representative ray id (smallest ray id with this key)
 *   key_len uint8[cap]    number of interactions k
 *   key_seq int32[cap][K] disk ids of the representative ray's first k hits
 * For (key q, receiver r), index q * n_rx + r:
 *   valid uint8, length float (path length, m), amp float[4] (a_TE re, im,
 *   a_TM re, im), hit int32[K] (validated disk per interaction).
 * Any output pointer may be NULL. *n_keys receives the key count (host
 * pointer; this call synchronises the stream). ws/params: those of the solve. */
pcrt_status pcrt_paths_copy(const pcrt_scene *scene, const pcrt_solve_params *p, const void *ws,
                            uint32_t cap, uint32_t *key_ray, uint8_t *key_len, int32_t *key_seq,
                            uint8_t *valid, float *length, float *amp, int32_t *hit, uint32_t *n_keys,
                            void *stream);

/* Diffuse visibility of a PCRT_RECORD solve: uint8[n_trace][K][n_rx], 1 when
 * the connection from interaction k of ray j to receiver r is lit and
 * unoccluded (Sec. II-B.1). Device pointer; asynchronous. */
pcrt_status pcrt_diffuse_vis_copy(const pcrt_scene *scene, const pcrt_solve_params *p, const void *ws,
                                  uint8_t *vis, void *stream);

/* ------------------------------------------------------------- batching */
/* Many transmitter poses (e.g. a moving robot, Sec. I) against the same
 * receivers, traced in one persistent launch: the rays of every item share
 * one work queue; keys, refinement and reductions stay per item. */
typedef struct {
    float tx[3];
    uint32_t n_rays; /* ray budget of this item (its Fibonacci directions) */
} pcrt_batch_item;

/* Workspace for a batch; p supplies everything but tx, n_rays and
 * ray_subset (must be NULL). items: host array. */
pcrt_status pcrt_batch_workspace_size(const pcrt_scene *scene, const pcrt_solve_params *p,
                                      const pcrt_batch_item *items, uint32_t n_items, size_t *bytes);

/* As pcrt_solve for every item; outputs are indexed [item][rx] (gain
 * double[n_items][n_rx], h_te/h_tm double[n_items][n_rx][2], gain_parts
 * double[n_items][n_rx][3]); ray_seq is ignored. Allocates nothing and never
 * synchronises, so it can be captured. */
pcrt_status pcrt_solve_batch(const pcrt_scene *scene, const pcrt_material *mats, uint32_t n_labels,
                             const pcrt_solve_params *p, const pcrt_batch_item *items, uint32_t n_items, void *ws,
                             size_t ws_bytes, const pcrt_outputs *out, void *stream);

/* HIP graph of a batch solve: captured on stream (not the null stream) and
 * instantiated. Every pointer and value is frozen at capture: a launch
 * recomputes the batch from the current contents of the captured device
 * buffers (e.g. new materials written in place). */
typedef struct pcrt_graph pcrt_graph;
pcrt_status pcrt_graph_capture_batch(const pcrt_scene *scene, const pcrt_material *mats, uint32_t n_labels,
                                     const pcrt_solve_params *p, const pcrt_batch_item *items, uint32_t n_items,
                                     void *ws, size_t ws_bytes, const pcrt_outputs *out, void *stream,
                                     pcrt_graph **graph);
pcrt_status pcrt_graph_launch(pcrt_graph *graph, void *stream);
pcrt_status pcrt_graph_destroy(pcrt_graph *graph);

/* Autotuner: times reps solves of p on every given scene (built by the
 * caller with the leaf sizes and widths to compare) for every wave_rays
 * value (HIP events on stream; synchronises), fills table[n_scenes * n_wave]
 * (optional, scene-major) and the fastest configuration. solve_ws must fit
 * the solve on every scene (else ENOMEM, with the size needed). */
typedef struct {
    uint32_t scene;      /* index into scenes */
    uint32_t leaf_size;
    uint32_t width;
    uint32_t wave_rays;
    double ms;
} pcrt_tuning;
pcrt_status pcrt_autotune(const pcrt_scene *const *scenes, uint32_t n_scenes, const pcrt_solve_params *p,
                          const pcrt_material *mats, uint32_t n_labels, const uint32_t *wave_rays, uint32_t n_wave,
                          uint32_t reps, void *solve_ws, size_t solve_ws_bytes, const pcrt_outputs *out, void *stream,
                          pcrt_tuning *table, pcrt_tuning *best);

/* ------------------------------------------- edge diffraction (Sec. II-B.3) */
/* One straight wedge edge from a to b; n0, n1: outward normals of its two faces
 * (face 0 and face n); label0, label1: their material labels. The wedge is the
 * region behind both faces (a convex edge, exterior angle n pi with 1 < n <= 2). */
typedef struct {
    float a[3], b[3], n0[3], n1[3];
    uint16_t label0, label1;
} pcrt_edge;

/* Device workspace of pcrt_diffraction (stack spill + per-pair amplitudes). */
pcrt_status pcrt_diffraction_workspace_size(const pcrt_scene *scene, uint32_t n_edges, uint32_t n_rx, size_t *bytes);

/* Single-bounce diffracted paths from tx (host float[3]) to every receiver
 * over every edge: the edge point minimising the path length (strictly inside
 * the edge; source and receiver in the wedge's exterior), visible from both
 * ends (the segments are cut 2 r_p short at the edge, where the faces' own
 * disks meet, and eps_self (0 = 1e-3 m) at the other end), with the field of
 * the uniform theory of diffraction for a wedge (Kouyoumjian-Pathak) whose
 * two reflection terms carry the faces' Fresnel coefficients (Luebbers);
 * TE takes the perpendicular and TM the parallel coefficients. The paper
 * leaves this field to its EM back end. Amplitudes are normalised like the
 * other path types (isotropic antennas, lambda/4pi). edges, mats (pcrt_material
 * [n_labels]; labels beyond it read label n_labels - 1), rx (float[n_rx][3]):
 * device. out: device double[n_rx][5] = G, h_TE re, im, h_TM re, im (sums over
 * edges in edge order). pair_amp: optional device float[n_rx][n_edges][4]
 * (TE re, im, TM re, im; 0 where no path). Asynchronous, allocates nothing.
 * Errors: EINVAL for NULL pointers, zero sizes, freq <= 0; ENOMEM for a small ws. */
pcrt_status pcrt_diffraction(const pcrt_scene *scene, const pcrt_edge *edges, uint32_t n_edges,
                             const pcrt_material *mats, uint32_t n_labels, const float tx[3], const float *rx,
                             uint32_t n_rx, double freq_hz, float eps_self, void *ws, size_t ws_bytes, double *out,
                             float *pair_amp, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as pcrt_diffraction, with its workspace taken from
 * a fixed 16 MiB scratch array that the library holds on every device it runs
 * on until the process ends (the stack spill and, when pair_amp is NULL, the
 * per-pair amplitudes). Allocates nothing, including on its first call on a
 * device, where it looks up that device's scratch address. The caller still
 * passes edges, materials, receivers, out and (optionally) pair_amp. All calls
 * on one device share its scratch, so calls that overlap on one device (on
 * different streams, or from different threads without ordering) race; calls
 * ordered on one stream do not. Nothing in the scratch needs to start at zero.
 * Errors: as pcrt_diffraction; EUNSUPPORTED when the scratch needed
 * (diffraction workspace size, minus the amplitudes when pair_amp is given)
 * exceeds 16 MiB; EDEVICE if the scratch address cannot be found. */
pcrt_status pcrt_diffraction_noalloc(const pcrt_scene *scene, const pcrt_edge *edges, uint32_t n_edges,
                                     const pcrt_material *mats, uint32_t n_labels, const float tx[3], const float *rx,
                                     uint32_t n_rx, double freq_hz, float eps_self, double *out, float *pair_amp,
                                     void *stream);

/* ------------------------------------------------------ differentiation */
/* The tape of a PCRT_RECORD solve lives in its workspace. It holds the path
 * geometry, which does not depend on the materials, as interaction slots:
 * slots [0, n_trace_slots) are the traced interactions (ray slot g, bounce m
 * at g*K + m), the rest are the interactions of the specular paths
 * ((key q * n_rx + receiver r) * K + m). Per slot the tape has the material
 * label (0xffff for an empty slot) and the incidence cosine, a coefficient
 * row coef[8] = (Gamma_TE re, im, Gamma_TM re, im, S, 0, 0, 0) and an
 * adjoint row adj[8] = dL/d of those five values.
 *
 * The calls below use the workspace and parameters of that solve, run
 * asynchronously on stream and allocate nothing. Materials enter only
 * through the coefficient rows, so a learned coefficient model may write them
 * instead of pcrt_tape_fresnel. */
typedef struct {
    uint32_t n_slots;
    uint32_t n_trace_slots;
    uint32_t key_capacity;
    const uint16_t *label; /* device [n_slots] */
    const float *cos;      /* device [n_slots] */
    float *coef;           /* device [n_slots][8] */
    float *adj;            /* device [n_slots][8] */
} pcrt_tape;

/* Pointers into the workspace (host call, no device work). */
pcrt_status pcrt_tape_get(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws, pcrt_tape *out);

/* coef rows from per-label materials (the Fresnel model of the solve).
 * mats: device pcrt_material[n_labels]. */
pcrt_status pcrt_tape_fresnel(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws,
                              const pcrt_material *mats, uint32_t n_labels, void *stream);

/* Per-receiver gain and fields from the coef rows: the solve's reduction on
 * the recorded geometry (line of sight is taken from the solve). out as for
 * pcrt_solve (gain required). */
pcrt_status pcrt_tape_forward(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws,
                              const pcrt_outputs *out, void *stream);

/* Adjoint rows for a loss L(G): dL_dgain device double[n_rx] (dL/dG_r).
 * Each path's power 1/2 (|a_TE|^2 + |a_TM|^2) is differentiated with
 * respect to every coefficient of its chain. */
pcrt_status pcrt_tape_backward(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws,
                               const double *dL_dgain, void *stream);

/* Channel frequency response of the recorded paths with the current coef
 * rows (the material-learning experiment of Sec. III-B): per receiver r and
 * sample n, H_r(f_n) = sum over paths of a_p exp(-j 2 pi (f_n - f_c) L_p / c0),
 * a_p the path's TE / TM amplitudes at the solve's frequency f_c, L_p its
 * unfolded length, f_n = f_c + (n - (n_freq - 1) / 2) bandwidth_hz /
 * (n_freq - 1) (the centre frequency alone when n_freq == 1). The channel
 * impulse response is the inverse DFT of these samples. Paths: line of sight,
 * valid specular paths, visible diffuse connections, in that order, cut into
 * 16 contiguous ranges, each range into rounds of 64 paths and each round into
 * 4 interleaved subsets; each subset is summed in path order and the subset
 * and range sums are added in order, in FP64. The order does not depend on
 * n_freq, so results are reproducible. cfr: device double[n_rx][n_freq][4] = (H_TE re, im, H_TM
 * re, im). n_freq in 1..65535, bandwidth_hz >= 0; EINVAL otherwise. */
pcrt_status pcrt_tape_cfr(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws, double bandwidth_hz,
                          uint32_t n_freq, double *cfr, void *stream);

/* Adjoint rows (as pcrt_tape_backward writes them) for a loss L(H) of that
 * response: dL_dcfr device double[n_rx][n_freq][4] = dL/d of the four reals
 * of each sample. pcrt_material_grad then gives dL/d(eps_r, sigma, S). */
pcrt_status pcrt_tape_cfr_backward(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws,
                                   double bandwidth_hz, uint32_t n_freq, const double *dL_dcfr, void *stream);

/* dL/d(eps_r, sigma, S) per label from the adjoint rows and the Fresnel
 * derivatives dGamma/deta (deta/deps_r = 1, deta/dsigma = -j/(omega eps0)).
 * Fixed-order FP64 reduction. mats: device pcrt_material[n_labels],
 * n_labels <= 64; dL_dmat: device double[n_labels][3]. */
pcrt_status pcrt_material_grad(const pcrt_scene *scene, const pcrt_solve_params *p, void *ws,
                               const pcrt_material *mats, uint32_t n_labels, double *dL_dmat, void *stream);

/* ------------------------------------------------ learned material model */
/* A small network in place of the per-label Fresnel model: per interaction
 * slot, x = [emb[label] (16), cos theta_i, log10(f / 1 GHz), 0 x 14] (32),
 * h1..h3 = GELU(W h + b) (64 wide, exact erf GELU), z = W4 h3 + b4 (16, five
 * used); Gamma_TE = (z0 + j z1) tanh|.|/|.|, Gamma_TM = (z2 + j z3) tanh|.|/|.|
 * (|Gamma| < 1, a passive surface), S = sigmoid(z4). BF16 operands with FP32
 * accumulation on the matrix cores; biases and the embedding table are FP32
 * (the embedding is rounded to BF16 as an input).
 * w: device bf16 bits, packed W1 [64][32], W2 [64][64], W3 [64][64], W4 [16][64]
 * (row = output; W1 columns 18..31 and W4 rows 5..15 should be zero);
 * b: device float b1 [64], b2 [64], b3 [64], b4 [16]; emb: device float
 * [n_labels][16], n_labels <= 64. */
typedef struct {
    const uint16_t *w;
    const float *b;
    const float *emb;
    uint32_t n_labels;
} pcrt_mlp;

/* Rows of 8 floats, in the tape's coefficient-row format: out[i] = (Gamma_TE
 * re, im, Gamma_TM re, im, S, 0, 0, 0) for slot i; label 0xffff (an empty
 * slot) gives zeros. label, cos: device [n]. Allocates nothing. */
pcrt_status pcrt_mlp_forward(const pcrt_mlp *net, uint32_t n, const uint16_t *label, const float *cos, float log_f,
                             float *out, void *stream);

/* Workspace for pcrt_mlp_backward over n rows. */
pcrt_status pcrt_mlp_workspace_size(uint32_t n, uint32_t n_labels, size_t *bytes);

/* Gradients of sum_i g_out[i] . out[i] (g_out: device [n][8], e.g. the tape's
 * adjoint rows) with respect to the parameters, written (not accumulated) to
 * grad_w (float, packed like w), grad_b (float [208]) and grad_emb (float
 * [n_labels][16]). The pass recomputes the forward; weight gradients are
 * MFMA GEMMs over fixed row blocks summed in a fixed order. */
pcrt_status pcrt_mlp_backward(const pcrt_mlp *net, uint32_t n, const uint16_t *label, const float *cos, float log_f,
                              const float *g_out, void *ws, size_t ws_bytes, float *grad_w, float *grad_b,
                              float *grad_emb, void *stream);

/* Device time (ms) of the stages of the last PCRT_TIMING solve issued on
 * this host thread: [0] initialisation, [1] ray launch + bounce loop,
 * [2] key marking/compaction, [3] specular refine + validate + field,
 * [4] Morton ordering of the interaction records, [5] diffuse connections,
 * [6] line of sight + per-receiver combine.
 * Synchronises with the end of that solve. ms: host double[n], n <= 7. */
pcrt_status pcrt_stage_times(double *ms, uint32_t n);

/* Launch directions on the Fibonacci sphere: z = 1 - (2j+1)/N, phi = 2 pi
 * frac(j (3 - sqrt5)/2), evaluated in FP64 and rounded to FP32.
 * ids: device uint32[n] (NULL = 0..n-1); out: device float[n][3]. */
pcrt_status pcrt_raygen(uint32_t n_budget, const uint32_t *ids, uint32_t n, float *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PCRT_H */
