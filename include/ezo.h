/*
 * ezo.h -- C ABI of the MI355X (gfx950) EI-ZO hot path.
 *
 * EI-ZO ("Edge Inflation Zero-Order", Alg. 1 of Werner et al., "Superfast
 * Configuration-Space Convex Set Computation on GPUs for Online Motion
 * Planning", arXiv 2504.10783) inflates a collision-free configuration-space
 * segment L = conv{v1, v2} into a polytope P = {x : A x <= b} with L inside P,
 * P inside the domain D, such that with probability >= 1 - delta at most an
 * eps fraction of P's volume is in collision (eq:prob_polytope_cfree).  Its
 * bulk is batched collision checking: forward kinematics of a serial arm
 * followed by sphere-sphere tests (Sec. IV-D).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers marked "dev" are device pointers on the context's device (for
 *   instance torch tensors' data_ptr()); "host" pointers are ordinary host
 *   memory.  The caller owns every buffer it passes; the library keeps no
 *   caller pointer after a call returns.
 * - Work is enqueued on `stream` (a hipStream_t; NULL = the legacy default
 *   stream).  Results in dev buffers are valid once that stream reaches them;
 *   results in host buffers (stats) are valid when the call returns.
 *   ezo_inflate_edges synchronises with `stream` internally (it polls one
 *   4-byte counter per iteration); the other calls do not block.
 * - Floating point on the device is FP32.  Robot descriptions are given in
 *   FP64 and rounded to FP32 once, at ezo_robot_create.
 * - Errors: every call returns EZO_OK (0) or a negative ezo_status; the text
 *   of the last error on a context is returned by ezo_last_error.  Errors
 *   never cross the ABI as exceptions.  Per-edge outcomes of an inflation are
 *   reported in edge_status, so one colliding edge does not fail a batch.
 * - Threading: one context per host thread.  Calls on one context must not
 *   overlap.
 * - Limits: dof <= EZO_MAX_DOF; spheres <= EZO_MAX_SPHERES.
 */
#ifndef EZO_H
#define EZO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EZO_MAX_DOF 8
#define EZO_MAX_SPHERES 1024
#define EZO_MAX_BOXES 64
#define EZO_MAX_OBSTACLE_BOXES 64

typedef struct ezo_ctx ezo_ctx;
typedef struct ezo_robot ezo_robot;
typedef struct ezo_surrogate ezo_surrogate;
typedef int32_t ezo_status;

enum {
    EZO_OK = 0,
    EZO_E_INVALID = -1,     /* an argument is out of range or inconsistent   */
    EZO_E_HIP = -2,         /* a HIP runtime call failed                      */
    EZO_E_CAPACITY = -3,    /* face_capacity < 2 dof + n_f * max_iters        */
    EZO_E_NOMEM = -4,       /* a device or host allocation failed             */
    EZO_E_UNSUPPORTED = -5  /* shape beyond EZO_MAX_DOF / EZO_MAX_SPHERES     */
};

/* Per-edge outcome of an inflation (Alg. 1 and Sec. IV-C). */
enum {
    EZO_EDGE_CERTIFIED = 0,    /* the unadaptive test accepted P                      */
    EZO_EDGE_MAX_ITERS = 1,    /* max_iters rounds without acceptance; P uncertified  */
    EZO_EDGE_IN_COLLISION = 2, /* a candidate within t_col of L, or a projection onto
                                  L in collision: L is likely in collision            */
    EZO_EDGE_INVALID = 3,      /* a vertex outside D or not finite; P = D             */
    EZO_EDGE_CONTAINED = 4     /* not inflated: L lies in the set of an earlier edge
                                  of its path (ezo_inflate_paths); no rows            */
};

/* Serial arm with standard Denavit-Hartenberg links,
 *   T_i = T_{i-1} Rz(q_i) Tz(d_i) Tx(a_i) Rx(alpha_i),  T_0 = identity,
 * (a prismatic joint: Rz(0) Tz(d_i + q_i)), and collision spheres and boxes
 * rigidly attached to links (Sec. IV-D: sphere and box geometries; Sec. II:
 * kinematics and collision geometry are given).  A point robot in a plane
 * (the Forest scene, Sec. VI-A) is two prismatic joints and one sphere of
 * radius 0.
 * All arrays are host memory and are copied at ezo_robot_create. */
typedef struct {
    int32_t dof;                 /* 1..EZO_MAX_DOF                                   */
    const double *dh_a;          /* [dof] link length a_i                            */
    const double *dh_alpha;      /* [dof] link twist alpha_i                         */
    const double *dh_d;          /* [dof] link offset d_i                            */
    const double *q_lo, *q_hi;   /* [dof] joint limits; D = {q_lo <= q <= q_hi}      */
    int32_t n_spheres;           /* 0..EZO_MAX_SPHERES                               */
    const int32_t *sphere_link;  /* [S] link index 0..dof-1 of each sphere           */
    const double *sphere_xyz;    /* [S][3] centre in the frame of its link           */
    const double *sphere_r;      /* [S] radius (>= 0)                                */
    int32_t n_self_pairs;        /* >= 0                                             */
    const int32_t *self_pairs;   /* [P][2] sphere indices tested against each other  */
    /* boxes rigidly attached to links (Sec. IV-D: box and sphere geometries) */
    int32_t n_boxes;             /* 0..EZO_MAX_BOXES                                 */
    const int32_t *box_link;     /* [B] link of each box, 0-based                    */
    const double *box_pose;      /* [B][12] centre (x, y, z), then the rotation
                                    (3x3, row-major, columns = the box axes), in
                                    the link frame                                  */
    const double *box_half;      /* [B][3] half extents along the box axes, >= 0     */
    int32_t n_box_pairs;         /* >= 0                                             */
    const int32_t *box_pairs;    /* [Q][2] box indices tested against each other     */
    const int32_t *joint_type;   /* [dof] 0 revolute (theta = q), 1 prismatic (theta
                                    = 0, offset d + q); NULL = all revolute          */
} ezo_robot_desc;

/* EI-ZO parameters: Alg. 1 Input (delta, eps, tau, Delta_max, N_p, N_f, N_b)
 * plus the sampler's mixing steps N_mix (Sec. IV-D), the iteration cap N_it
 * and the collision tolerance t_col (Sec. IV-C). */
typedef struct {
    double eps;              /* admissible fraction in collision, (0, 1)            */
    double delta;            /* admissible uncertainty, (0, 1)                      */
    double tau;              /* test decision threshold, (0, 1); typically 0.5      */
    double step_back_max;    /* Delta_max > 0                                       */
    double t_col;            /* candidates with dist <= t_col abort the edge        */
    int32_t n_p;             /* N_p >= 1: samples updated per iteration; 0: chosen
                                by the autotuner (ezo_inflate_edges)                 */
    int32_t n_f;             /* N_f >= 1: faces placed per iteration                */
    int32_t n_b;             /* N_b >= 0: bisection steps                           */
    int32_t n_mix;           /* hit-and-run steps per sample, >= 0                  */
    int32_t max_iters;       /* N_it >= 1                                           */
    int32_t face_capacity;   /* rows reserved per edge in A/b, >= 2 dof + n_f N_it  */
    uint64_t seed;           /* Philox key                                          */
    int64_t edge_id_base;    /* edge e of this call draws the random stream of
                                edge id (edge_id_base + e)                           */
    const ezo_surrogate *surrogate;  /* NULL = exact checks only.  Otherwise the
                                learned screen skips the exact self-collision
                                pairs of samples after the first M_k (never of
                                the test samples) whose predicted self distance
                                is >= the screen's calibrated margin           */
    float *row_points;       /* dev f32 [E][face_capacity][dof] or NULL (caller-
                                owned).  ezo_inflate_edges writes, for every
                                hyperplane row f >= 2 dof it
                                places, the collision point c* that row was
                                placed for (Sec. IV-C: the row is a^T x <=
                                a^T c* - Delta with Delta > 0, so it excludes
                                c*); box rows and rows past n_faces are left
                                untouched.  Ignored by ezo_inflate_paths */
} ezo_params;

typedef struct {
    int32_t iterations;      /* unadaptive tests performed                          */
    int32_t planes;          /* hyperplanes added to D                              */
    int64_t final_m;         /* M_k of the last test                                */
    int64_t test_collisions; /* collisions among the first M_k samples, last test   */
    int64_t samples;         /* samples drawn (sum of |S| over iterations)          */
    int64_t exact_checks;    /* configurations collision-checked                    */
    int64_t screened_checks; /* of those, checks whose self pairs the screen skipped */
} ezo_edge_stats;

/* ---- context and robot ------------------------------------------------- */

/* Creates a context bound to HIP device `device`.  Allocates a small amount
 * of device memory and one internal stream (default priority). */
ezo_status ezo_ctx_create(int32_t device, ezo_ctx **out);
void ezo_ctx_destroy(ezo_ctx *ctx);

/* Obstacle boxes of the context (e.g. a table), in addition to the obstacle
 * spheres each call passes: every check, inflation, bisection and path check
 * on the context tests them.  boxes host f32 [n][15]: centre (x, y, z),
 * rotation (3x3, row-major, columns = the box axes), half extents, world
 * frame; copied.  n = 0 removes them.  EZO_E_UNSUPPORTED above
 * EZO_MAX_OBSTACLE_BOXES. */
ezo_status ezo_set_obstacle_boxes(ezo_ctx *ctx, const float *boxes, int32_t n);

/* Text of the last error on ctx (or of the last failed ezo_ctx_create when
 * ctx is NULL).  Valid until the next call on that context. */
const char *ezo_last_error(const ezo_ctx *ctx);

/* Uploads a robot (copied and rounded to FP32).  EZO_E_UNSUPPORTED beyond
 * the limits; EZO_E_INVALID for out-of-range link or sphere indices. */
ezo_status ezo_robot_create(ezo_ctx *ctx, const ezo_robot_desc *desc, ezo_robot **out);
/* Frees the robot; it may run before or after ezo_ctx_destroy of its
 * context (it reads only the robot), but not while a call uses the robot. */
void ezo_robot_destroy(ezo_robot *robot);

/* ---- collision checking (Sec. IV-D: PointsInCollision of Alg. 1) -------- */

/* For each configuration q_i (i < n), element j at q[i*stride_n + j*stride_d]
 * (dev, FP32), computes the minimum signed distance over
 *   robot-obstacle pairs  |c_s - o| - r_s - r_o   (obstacles obs[n_obs][4] =
 *                                                 x, y, z, r; dev, FP32)
 *   listed self pairs     |c_s - c_t| - r_s - r_t
 * and, with boxes (robot boxes, the context's obstacle boxes),
 *   sphere-box pairs      the exact signed distance: outside the box the
 *                         distance from the centre to the box minus r, inside
 *                         minus (the distance to the nearest face + r)
 *   box-box pairs         the separating-axis value: the largest, over the 6
 *                         face normals and the 9 edge-edge cross products
 *                         (unit; those with |A_i x B_j|^2 < 1e-12 skipped), of
 *                         |t.L| - r_A(L) - r_B(L) (t = centre offset, r_X(L) =
 *                         sum_k h_k |X_k . L|); the penetration depth when the
 *                         boxes overlap, a lower bound of their distance when
 *                         apart
 * (robot boxes against obstacle spheres and boxes, robot spheres against
 * obstacle boxes, the listed box self pairs) and flags[i] = 1 iff that
 * minimum is < 0 (dev u8[n]).
 * If min_sd and min_sd_self are both NULL only flags are computed, and a
 * configuration stops being tested at its first colliding pair.  Otherwise
 * min_sd[i] (dev f32[n], may be NULL) receives the overall minimum and
 * min_sd_self[i] (dev f32[n], may be NULL) the self-pair minimum (+inf when
 * there are none).  n = 0 is a no-op. */
ezo_status ezo_check_collisions(ezo_ctx *ctx, const ezo_robot *robot, const float *obs, int32_t n_obs,
                                const float *q, int64_t n, int64_t stride_n, int64_t stride_d,
                                uint8_t *flags, float *min_sd, float *min_sd_self, void *stream);

/* The same check with no allocation: for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, layouts, outputs and errors as in
 * ezo_check_collisions; the results are bit-identical to it.  Instead of the
 * context's growable workspace it uses a fixed scratch array in device
 * memory (obstacle records, frame shift, broad-phase grid counts and lists:
 * about 8.6 MB), one per device, allocated with the library's code object
 * and held until the process ends; the call itself allocates nothing and
 * never runs a launch-shape timing search (it uses the tuning cache, else
 * the size heuristic).  Limit: n_obs <= EZO_NOALLOC_MAX_OBSTACLES, else
 * EZO_E_CAPACITY (any n).  Every call on one device shares that device's
 * scratch, so calls that overlap on one device (two streams, two contexts,
 * two threads) race; calls in one stream are ordered.  Each call rewrites
 * every scratch byte it reads. */
#define EZO_NOALLOC_MAX_OBSTACLES 4096
ezo_status ezo_check_collisions_noalloc(ezo_ctx *ctx, const ezo_robot *robot, const float *obs, int32_t n_obs,
                                        const float *q, int64_t n, int64_t stride_n, int64_t stride_d,
                                        uint8_t *flags, float *min_sd, float *min_sd_self, void *stream);

/* Forward kinematics only: world-frame sphere centres, centres[i][s][0..2]
 * (dev f32 [n][S][3]), for the same q layout as ezo_check_collisions. */
ezo_status ezo_sphere_centres(ezo_ctx *ctx, const ezo_robot *robot, const float *q, int64_t n,
                              int64_t stride_n, int64_t stride_d, float *centres, void *stream);

/* ---- statistical test constants (Sec. IV-B) ----------------------------- */

/* Host helper: delta_k = 6 delta / (pi^2 k^2), M_k = ceil(2 ln(1/delta_k) /
 * (eps tau^2)), T_k = floor(M_k (1 - tau) eps + 1e-9); the test accepts iff
 * the collisions among the first M_k samples are <= T_k. */
ezo_status ezo_test_constants(double eps, double delta, double tau, int32_t k, int64_t *M, int64_t *T);

/* ---- the steps of one EI-ZO iteration, on E edges at once --------------- */
/* Layouts: edges dev f32 [E][2][dof] (v1 then v2); polytopes A dev f32
 * [E][face_capacity][dof], b dev f32 [E][face_capacity], n_faces dev i32 [E];
 * samples dev f32 [E][dof][sample_stride] (coordinate-major per edge);
 * candidate arrays are [E][cand_capacity] (per coordinate: [E][dof][cand_capacity]). */

/* UniformSample(P, .) of Alg. 1: n_samples hit-and-run walks per edge inside
 * its current polytope (Sec. IV-B/IV-D).  Walk i of edge e starts at
 * v1 + w (v2 - v1), w ~ U(0,1), then takes n_mix steps: direction
 * u = g/|g|, g ~ N(0, I) by Box-Muller, chord [t_lo, t_hi] over all rows,
 * t ~ U[t_lo, t_hi] (t = 0 if rounding empties the chord).  Randomness:
 * Philox4x32-10, key = (seed low, seed high), counter = (i, edge_id_base + e,
 * iteration, 16 s + word/4) with s = 0 for the start and 1..n_mix for steps;
 * words map to (0,1) by ((x >> 9) + 1/2) 2^-23.  sample_stride >= n_samples. */
ezo_status ezo_sample_polytopes(ezo_ctx *ctx, int32_t dof, const float *A, const float *b,
                                const int32_t *n_faces, int32_t face_capacity, const float *edges,
                                int32_t n_edges, int32_t n_samples, int32_t n_mix, uint64_t seed,
                                int64_t edge_id_base, int32_t iteration, float *samples,
                                int64_t sample_stride, void *stream);

/* UnadaptiveTest of Alg. 1 plus candidate selection (Sec. IV-B): per edge,
 * count = collisions among flags[e][0..M-1] (flags dev u8 [E][sample_stride],
 * n_samples valid); accept[e] = count <= T (dev u8 [E]); test_count[e] =
 * count (dev i32 [E]).  If not accepted, cand_idx[e][0..] (dev i32
 * [E][cand_capacity]) receives the indices of the first min(n_p,
 * #colliding) colliding samples in increasing order and n_cands[e] their
 * number (dev i32 [E]); if accepted n_cands[e] = 0.  n_p <= cand_capacity. */
ezo_status ezo_test_and_select(ezo_ctx *ctx, const uint8_t *flags, int32_t n_edges, int64_t sample_stride,
                               int32_t n_samples, int64_t M, int64_t T, int32_t n_p, int32_t *cand_idx,
                               int32_t *n_cands, int32_t cand_capacity, uint8_t *accept,
                               int32_t *test_count, void *stream);

/* ProjectPoints and UpdatePointsViaBisection of Alg. 1 (Sec. IV-A, IV-B):
 * for candidate j < n_cands[e] with sample c = samples[e][:, cand_idx[e][j]]:
 * c_proj = projection onto L (eq:proj, eq:proj_alpha), a = (c - c_proj) /
 * |c - c_proj| (eq:dist_grad), proj_collides[e][j] = collision flag of
 * c_proj (fail-fast check, Sec. IV-C), then n_b bisection steps on
 * [c_proj, c] keeping the colliding end; c_star = that end,
 * t_star = |c_star - c_proj|.  Outputs dev: c_star, a_dir f32
 * [E][dof][cand_capacity], t_star f32 [E][cand_capacity], proj_collides
 * u8 [E][cand_capacity]. */
ezo_status ezo_project_bisect(ezo_ctx *ctx, const ezo_robot *robot, const float *obs, int32_t n_obs,
                              const float *edges, int32_t n_edges, const float *samples,
                              int64_t sample_stride, const int32_t *cand_idx, const int32_t *n_cands,
                              int32_t cand_capacity, int32_t n_b, float *c_star, float *a_dir,
                              float *t_star, uint8_t *proj_collides, void *stream);

/* OrderAndPlaceHyperplanes of Alg. 1 (Sec. IV-B, step back Sec. IV-C): per
 * edge whose edge_status is not yet final (< 0 means running; the call only
 * reads/writes edges with edge_status[e] < 0), order candidates by (t_star,
 * candidate index); repeatedly take the closest one not yet discarded: if
 * its t_star <= t_col set edge_status[e] = EZO_EDGE_IN_COLLISION and stop;
 * else append the row a^T x <= b - Delta with b = a^T c_star,
 * r = max(a^T v1, a^T v2) - b + step_back_max and Delta = step_back_max - r
 * if r > 0 else step_back_max; discard every candidate with
 * a^T c_star > b - Delta.  At most n_f rows.  n_faces[e] is advanced;
 * placed_idx (dev i32 [E][n_f], may be NULL) receives the candidate index of
 * each new row; n_placed (dev i32 [E], may be NULL) their number.  If
 * face_capacity would be exceeded the edge stops adding rows. */
ezo_status ezo_place_hyperplanes(ezo_ctx *ctx, int32_t dof, const float *edges, int32_t n_edges,
                                 const float *c_star, const float *a_dir, const float *t_star,
                                 const int32_t *n_cands, int32_t cand_capacity, int32_t n_f,
                                 double step_back_max, double t_col, float *A, float *b,
                                 int32_t *n_faces, int32_t face_capacity, int32_t *edge_status,
                                 int32_t *placed_idx, int32_t *n_placed, void *stream);

/* ---- the whole method (Alg. 1) on E edges in one call ------------------- */

/* Inflates every edge e (edges dev f32 [E][2][dof]) against the robot and
 * obstacles: P_e = D (the robot's joint-limit box, rows +e_j <= q_hi then
 * -e_j <= -q_lo), then for k = 1..max_iters: |S| = max(N_p, M_k) samples,
 * collision checks, test (accept => CERTIFIED), candidates, projection +
 * bisection, placement.  All edges advance together; finished edges are
 * skipped.  Outputs: A dev f32 [E][face_capacity][dof], b dev f32
 * [E][face_capacity], n_faces dev i32 [E], edge_status dev i32 [E] (EZO_EDGE_*),
 * stats host [E] (may be NULL).  Returns EZO_E_CAPACITY if face_capacity <
 * 2 dof + n_f max_iters.  Blocks until the stream has finished the call.
 * params->n_p = 0: N_p is chosen by the autotuner (tuning kind "samples",
 * key: architecture, robot size, obstacle count, floor(log2 E)): the first
 * call with a new key inflates its own edges with N_p = 10000, 5000, 2000 and
 * 1000 (each once, then all again three times) and keeps the largest N_p
 * whose time is within 5 % of the fastest; with tuning off and nothing
 * cached N_p = 10000.  Those timed inflations draw from an independent
 * random stream (Philox key seed ^ 0x9E3779B97F4A7C15, recorded as
 * "tune_seed" in the cache entry) and are discarded; the returned sets are
 * one inflation with the chosen N_p on the call's own seed, so the choice
 * never depends on their draws.  The certification does not depend on
 * N_p (the test uses the first M_k samples); the sets do. */
ezo_status ezo_inflate_edges(ezo_ctx *ctx, const ezo_robot *robot, const float *obs, int32_t n_obs,
                             const float *edges, int32_t n_edges, const ezo_params *params, float *A,
                             float *b, int32_t *n_faces, int32_t *edge_status, ezo_edge_stats *stats,
                             void *stream);

/* ---- piecewise-linear paths in sequence (Sec. V-A) ---------------------- */

/* Inflates n_paths paths, each in sequence with the containment skip: edge k
 * of a path is inflated only if its segment L_k is not contained in the set
 * of an earlier edge of the same path (both ends satisfy every row of that
 * set, FP32), where only sets of edges that were inflated and ended
 * CERTIFIED or MAX_ITERS count.  Paths are independent of one another.
 * Since an edge's set does not depend on any other edge, the call works in
 * rounds over windows of s consecutive edges of every path (s chosen so that
 * a round holds about 128 edges): window edges inside a set of an earlier
 * round are skipped, the others are inflated in one batched pass, and then
 * resolved in path order (an edge inside the set of an earlier edge of its
 * window is dropped).  The result is that of the sequential process.
 *
 * vertices dev f32 [sum_p path_vertices[p]][dof], the paths' vertices back
 * to back; path_vertices host i32 [n_paths], each >= 2.  Edges are numbered
 * path by path (path p's edge k has global index g = sum_{q<p}
 * (path_vertices[q] - 1) + k) and every output is indexed by g: A dev f32
 * [n_edges][face_capacity][dof], b [n_edges][face_capacity], n_faces and
 * edge_status dev i32 [n_edges], covered_by dev i32 [n_edges] (-1 for an
 * inflated edge, else the first earlier edge whose set contains it; that
 * edge's status is EZO_EDGE_CONTAINED and n_faces 0), stats host [n_edges]
 * (may be NULL; zero for a contained edge).  Edge g draws the random stream
 * of edge id params->edge_id_base + g, so an inflated edge's set equals the
 * one ezo_inflate_edges gives for it with the same parameters.  Errors as in
 * ezo_inflate_edges, EZO_E_INVALID for a path with fewer than 2 vertices.
 * Blocks until the stream has finished the call. */
ezo_status ezo_inflate_paths(ezo_ctx *ctx, const ezo_robot *robot, const float *obs, int32_t n_obs,
                             const float *vertices, const int32_t *path_vertices, int32_t n_paths,
                             const ezo_params *params, float *A, float *b, int32_t *n_faces,
                             int32_t *edge_status, int32_t *covered_by, ezo_edge_stats *stats, void *stream);

/* ---- learned self-collision screen ------------------------------------ */
/* A multilayer perceptron dof -> H -> H -> H -> 1 with SiLU activations
 * predicting a configuration's minimum self-collision signed distance from
 * x = q / pi (BF16 MFMA layers, FP32 accumulation and master weights).
 * Trained with this library's own forward/backward kernels and Adam on
 * labels produced by the exact checker; used by ezo_inflate_edges only to
 * skip exact self pairs of optimizer samples (never of the unadaptive test's
 * samples), so certification never depends on it.  Callers: anyone wanting
 * to trade exact self-pair work for a network evaluation.
 * Parameters are one flat FP32 vector W1[H][dof] b1[H] W2[H][H] b2[H]
 * W3[H][H] b3[H] W4[H] b4[1] (z = W a + b). */
typedef struct {
    int32_t epochs;          /* passes over the training rows                       */
    int32_t batch;           /* rows per Adam step, a multiple of 64                */
    double lr;               /* peak learning rate, cosine decay to 0               */
    double beta1, beta2, adam_eps;
    double huber_delta;      /* Huber loss threshold                                */
    double clip_lo, clip_hi; /* targets are clipped to [clip_lo, clip_hi]           */
    uint64_t seed;           /* batch order                                         */
} ezo_train_params;

int64_t ezo_surrogate_num_params(int32_t dof, int32_t hidden);
/* hidden: multiple of 64 in [64, 4096].  Weights ~ U(+-1/sqrt(fan_in)) from seed;
 * margin = +inf (screens nothing) until calibrated. */
ezo_status ezo_surrogate_create(ezo_ctx *ctx, int32_t dof, int32_t hidden, uint64_t seed, ezo_surrogate **out);
/* Frees the screen; like ezo_robot_destroy it may outlive its context. */
void ezo_surrogate_destroy(ezo_surrogate *s);
/* host [n] parameter copies (n = ezo_surrogate_num_params); set resets Adam. */
ezo_status ezo_surrogate_set_params(ezo_surrogate *s, const float *params, int64_t n);
ezo_status ezo_surrogate_get_params(const ezo_surrogate *s, float *params, int64_t n);
/* Adam training on rows q dev f32 [n][dof] with targets dev f32 [n];
 * epoch_loss host [epochs] (mean Huber loss per epoch) may be NULL.  Blocks. */
ezo_status ezo_surrogate_train(ezo_ctx *ctx, ezo_surrogate *s, const float *q, const float *target, int64_t n,
                               const ezo_train_params *tp, float *epoch_loss, void *stream);
/* Mean loss (host) and its gradient (host f32 [num_params]) over n rows
 * (n a multiple of 64, <= 2^20) without updating the weights.  Blocks. */
ezo_status ezo_surrogate_loss_grad(ezo_ctx *ctx, ezo_surrogate *s, const float *q, const float *target, int64_t n,
                                   const ezo_train_params *tp, float *grad, double *loss, void *stream);
/* Predictions pred dev f32 [n] for q dev f32 [n][dof]. */
ezo_status ezo_surrogate_predict(ezo_ctx *ctx, const ezo_surrogate *s, const float *q, int64_t n, float *pred,
                                 void *stream);
/* Margin m = smallest value with #{pred >= m and target < 0} <= alpha
 * #{target < 0} on the given rows (conformal-style calibration); stored in
 * the screen and returned.  Blocks. */
ezo_status ezo_surrogate_calibrate(ezo_ctx *ctx, ezo_surrogate *s, const float *q, const float *target, int64_t n,
                                   double alpha, double *margin_out, void *stream);
ezo_status ezo_surrogate_set_margin(ezo_surrogate *s, double margin);
/* What an inflation screens (R22: always one-sided, never the unadaptive
 * test's first M_k samples nor the projections onto L): EZO_SCREEN_SAMPLES,
 * the samples after M_k; EZO_SCREEN_MIDPOINTS, the bisection midpoints; both
 * by default.  EZO_E_INVALID for other bits. */
enum { EZO_SCREEN_SAMPLES = 1, EZO_SCREEN_MIDPOINTS = 2 };
ezo_status ezo_surrogate_set_scope(ezo_surrogate *s, int32_t scope);
/* On held-out rows: miss rate = #{pred >= m and target < 0} / #{target < 0};
 * screened fraction = #{pred >= m} / n.  Blocks. */
ezo_status ezo_surrogate_miss_rate(ezo_ctx *ctx, const ezo_surrogate *s, const float *q, const float *target,
                                   int64_t n, double *miss_rate, double *screened_fraction, void *stream);

/* ---- instrumentation ------------------------------------------------- */

/* Kernel phases of one inflation iteration, in launch order. */
enum {
    EZO_PHASE_SAMPLE = 0,        /* hit-and-run sampler                       */
    EZO_PHASE_CHECK = 1,         /* collision checks of the samples           */
    EZO_PHASE_TEST = 2,          /* unadaptive test + candidate selection     */
    EZO_PHASE_BISECT = 3,        /* projection, fail-fast check, bisection    */
    EZO_PHASE_PLACE = 4,         /* ordering and placing hyperplanes          */
    EZO_PHASE_ADVANCE = 5,       /* iteration bookkeeping (a call with one
                                    edge does it inside the placement kernel:
                                    0 ms)                                     */
    EZO_NUM_PHASES = 6
};

/* Enables (1) or disables (0) per-phase GPU timing of ezo_inflate_edges on
 * this context.  While enabled, the iteration's kernels are launched directly
 * (not through the replayed hipGraph), each with a pair of hipEvents that its
 * dispatch records at kernel start and end on the stream it runs on, and the
 * kernel durations accumulate per phase.  Results are identical either way.
 * Enabling resets the totals. */
ezo_status ezo_set_phase_timing(ezo_ctx *ctx, int32_t enable);

/* Cumulative per-phase kernel time (ms_out[EZO_NUM_PHASES], host), the
 * number of timed iterations (iterations_out, host, may be NULL) and the
 * number of sphere-sphere tests the collision-check phases performed
 * (tests_out[EZO_NUM_PHASES], host, may be NULL; bound tests of the broad
 * phase included, pairs it proved separated excluded) since timing was
 * enabled.  Synchronises the context's stream when tests_out is given. */
ezo_status ezo_get_phase_timing(ezo_ctx *ctx, double *ms_out, int64_t *iterations_out, int64_t *tests_out);

/* ---------------------------------------------------------------------------
 * Collision map of a dynamic roadmap (appendix, DRM construction)
 *
 * The task space is cut into voxels of side `side`: voxel (i, j, k) of a
 * dims[0] x dims[1] x dims[2] grid from corner lo (host f32 [3]) has index
 * v = (k dims[1] + j) dims[0] + i and is represented by its circumscribing
 * sphere, centre lo + side (i + 1/2, j + 1/2, k + 1/2), radius sqrt(3)/2 side.
 * Every voxel is checked against every roadmap node.
 * ------------------------------------------------------------------------- */

/* map (dev u32 [V][row_words], V = dims[0] dims[1] dims[2], row_words >=
 * ceil(n_nodes / 32)): bit n of row v (word n / 32, bit n % 32) is set iff the
 * robot at node q_n (dev f32 [n_nodes][dof], row-major) collides with voxel
 * v: some robot sphere or box at signed distance < 0 from the voxel's sphere
 * (FP32; self pairs, obstacles and obstacle boxes play no part).  The call
 * clears the map first.  A dense bitset instead of id lists: 35 000 nodes x
 * 12 000 voxels is 52 MB, the online lookup is an OR of rows, and the result
 * does not depend on thread timing.  Does not synchronise. */
ezo_status ezo_collision_map(ezo_ctx *ctx, const ezo_robot *robot, const float *q, int64_t n_nodes,
                             const float *lo, float side, const int32_t *dims, uint32_t *map, int64_t row_words,
                             void *stream);

/* The map as id lists: offsets (dev i64 [n_rows + 1]) = exclusive prefix of
 * the rows' bit counts, ids (dev i32 [capacity]) = the set bits of each row
 * as node ids in increasing order, row v at ids[offsets[v] .. offsets[v+1]).
 * *total (host, may be NULL) = offsets[n_rows]; EZO_E_CAPACITY (ids not
 * written) if it exceeds capacity.  Synchronises `stream`. */
ezo_status ezo_collision_map_lists(ezo_ctx *ctx, const uint32_t *map, int64_t n_rows, int64_t row_words,
                                   int64_t n_nodes, int64_t *offsets, int32_t *ids, int64_t capacity,
                                   int64_t *total, void *stream);

/* ---------------------------------------------------------------------------
 * Recovery from collisions found on a trajectory (Sec. V-B)
 *
 * A trajectory through the sets is checked by fine discretisation; the
 * collisions found inside a set are excluded by repeating the last three
 * steps of Alg. 1 on them; then every path segment must still lie in some
 * set (a segment lies in a convex polytope iff both its ends do), else it is
 * inflated again (ezo_inflate_edges).
 * ------------------------------------------------------------------------- */

/* Discretises the piecewise-linear path through waypoints (dev [K][dof],
 * row-major, K >= 1) so that consecutive points differ by at most max_step
 * in every coordinate -- segment i is cut into m_i = max(1, ceil(max_j
 * |w_{i+1,j} - w_{i,j}| / max_step)) equal pieces (computed in FP64), points
 * w_i + (j / m_i)(w_{i+1} - w_i) in FP32, each shared vertex once -- and
 * checks every point (flags mode).  points_out (dev [point_capacity][dof],
 * may be NULL when point_capacity = 0) receives the first point_capacity
 * colliding points in path order; *n_points (host, may be NULL) the number
 * of path points and *n_colliding (host, may be NULL) the number of
 * colliding ones.  Synchronises `stream` (the point count sizes the check).
 * At most 2^28 path points. */
ezo_status ezo_check_path(ezo_ctx *ctx, const ezo_robot *robot, const float *obs_xyzr, int32_t n_obs,
                          const float *waypoints, int32_t n_waypoints, double max_step, float *points_out,
                          int32_t point_capacity, int64_t *n_points, int64_t *n_colliding, void *stream);

/* Edits sets after collisions were found (Sec. V-B).  points (dev
 * [n_points][dof], row-major) are the found collisions; they are expected to
 * collide and are not checked again.  For every edge whose status is
 * CERTIFIED or MAX_ITERS, the points inside its polytope (A x <= b over its
 * n_faces rows, FP32) are, in point order, the candidates of the last three
 * steps of Alg. 1: projection onto L with the fail-fast check, n_b bisection
 * steps, then ordering and placing up to n_f hyperplanes appended to
 * (A, b, n_faces) (layouts as in ezo_inflate_edges, face_capacity rows per
 * edge).  An edge whose chosen candidate lies within t_col of L, or whose
 * candidate's projection collides, becomes EZO_EDGE_IN_COLLISION; every other
 * status is left as it is.  planes_added (dev [n_edges] or NULL) receives the
 * planes placed per edge.  n_points <= 64512 per call. */
ezo_status ezo_update_polytopes(ezo_ctx *ctx, const ezo_robot *robot, const float *obs_xyzr, int32_t n_obs,
                                const float *edges, int32_t n_edges, const float *points, int32_t n_points,
                                int32_t n_b, int32_t n_f, double step_back_max, double t_col, float *A, float *b,
                                int32_t *n_faces, int32_t face_capacity, int32_t *edge_status,
                                int32_t *planes_added, void *stream);

/* covered[k] (dev [n_segments]) = the smallest set index whose polytope
 * contains both ends of segment k (segments dev [n_segments][2][dof]):
 * A v <= b + tol over its n_faces rows (FP32), -1 if no set does.  A set
 * with n_faces = 0 (an edge that holds no set, EZO_EDGE_CONTAINED) contains
 * nothing. */
ezo_status ezo_segments_contained(ezo_ctx *ctx, int32_t dof, const float *A, const float *b, const int32_t *n_faces,
                                  int32_t face_capacity, int32_t n_sets, const float *segments, int32_t n_segments,
                                  double tol, int32_t *covered, void *stream);

/* ---------------------------------------------------------------------------
 * Launch-shape autotuning
 *
 * The tile kernels (collision check in flags and signed-distance mode;
 * projection + bisection) run with a launch shape: configurations per
 * workgroup, waves per workgroup, and whether obstacle records are staged in
 * LDS; the sampler runs with a number of lanes per walk.  The shape never
 * changes a result (every flag, distance and bisection is computed from the
 * same pair tests whatever the split, and the sampler's split of the faces
 * is reduced with exact min/max), only the time.
 * With autotuning on (the default), the first call whose tuning key is new
 * times every candidate shape once on the device, times the four fastest
 * again over three launches each, and caches for the process the first of
 * them (in a fixed order: fewer bisection levels per round, larger tiles
 * first) whose time is within 3 % of the fastest; the key is (device
 * architecture, kernel, dof, spheres, self pairs, obstacles,
 * floor(log2(work items))).  That first call synchronises with
 * `stream` (it reads timing events), so it must not run under stream
 * capture: disable tuning or import a cache first.  ezo_check_collisions and
 * ezo_project_bisect time on the call's own inputs (launches that only write
 * the call's outputs); ezo_inflate_edges times on configurations uniform in
 * the joint box, before its first iteration.  With autotuning off, a cached
 * shape is still used; otherwise a size heuristic picks one.
 * ------------------------------------------------------------------------- */

/* Turn timing of new tuning keys on (enable != 0, default) or off. */
ezo_status ezo_set_autotune(ezo_ctx *ctx, int32_t enable);

/* The process-wide cache as text, one JSON object per line with keys arch,
 * kernel ("check_flags" | "check_sd" | "bisect" | "sample"), dof, spheres,
 * self_pairs, obstacles, log2_items, T, W, stage, depth and us (measured
 * time per launch).  For "bisect", T counts candidates per workgroup and
 * depth (1..3, optional on import, default 1) the bisection levels checked
 * per round, so a tile check holds T (2^depth - 1) configurations.  For
 * "samples" (the sample count N_p of ezo_inflate_edges), T is N_p and
 * tune_seed (export only) the Philox key of the timed inflations.  For
 * "sample", T is
 * the number of lanes per walk, W the waves per workgroup, and spheres =
 * self_pairs = obstacles = 0.
 * buf (host, may be NULL) receives at most capacity - 1 bytes and a NUL;
 * *length (host, may be NULL) receives the full text length.  Returns
 * EZO_E_CAPACITY when the text was truncated. */
ezo_status ezo_tune_cache_export(char *buf, int64_t capacity, int64_t *length);

/* Adds (or replaces) cache entries from text in the export format.  Returns
 * EZO_E_INVALID, importing nothing, when a line with '{' lacks a key or has
 * an invalid shape; *n_imported (host, may be NULL) receives the number of
 * entries added.  Entries whose shape does not fit a device's LDS are
 * ignored when looked up. */
ezo_status ezo_tune_cache_import(const char *text, int32_t *n_imported);

/* Empties the process-wide cache. */
void ezo_tune_cache_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* EZO_H */
