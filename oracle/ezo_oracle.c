/*
 * ezo_oracle.c -- plain FP64 CPU reference ("oracle") for the EI-ZO hot path
 * of "Superfast Configuration-Space Convex Set Computation on GPUs for Online
 * Motion Planning" (Werner, Cheng, Stewart, Tedrake, Rus; arXiv 2504.10783).
 *
 * TEST INFRASTRUCTURE ONLY.  The product library (HIP, FP32) never links,
 * loads or calls anything in this file; only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark do.  It shares no source with the
 * GPU path: its own kinematics, its own distance code, its own Philox, its own
 * statistical-test constants.
 *
 * Everything is computed in double precision, written for readability, in the
 * order the paper states it:
 *   - collision checking  : the plain definition (all pairs, min signed
 *                           distance, flag = min < 0), Sec. IV-D;
 *   - projection / gradient / tangent plane: Sec. IV-A (eq:proj, eq:proj_alpha,
 *                           eq:dist_grad, eqn:sl_tangent);
 *   - EI-ZO loop           : Alg. 1 and Sec. IV-B; step back Sec. IV-C;
 *   - hit-and-run sampling : Sec. IV-B (Lovasz' hit-and-run inside P).
 * Readings of points the paper leaves open are noted where they are used.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Robot and scenes                                                          */
/* ------------------------------------------------------------------------ */

/* Serial arm with standard Denavit-Hartenberg parameters and spheres rigidly
 * attached to its links (the sphere geometry of Sec. VI-A / Sec. IV-D). */
typedef struct {
    int32_t dof;
    const double *a, *alpha, *d;   /* [dof] DH link length, twist, offset    */
    const double *q_lo, *q_hi;     /* [dof] joint limits (the domain D)       */
    int32_t n_spheres;
    const int32_t *sphere_link;    /* [S] 0-based link the sphere is fixed to */
    const double *sphere_xyz;      /* [S][3] centre in that link's frame      */
    const double *sphere_r;        /* [S] radius                              */
    int32_t n_self;
    const int32_t *self_pairs;     /* [P][2] sphere indices checked for self-collision */
    /* boxes rigidly attached to links (the box geometry of Sec. IV-D) */
    int32_t n_boxes;
    const int32_t *box_link;       /* [B] 0-based link                                  */
    const double *box_pose;        /* [B][12] centre (3), then rotation (3x3, row-major,
                                      columns = the box axes) in that link's frame      */
    const double *box_half;        /* [B][3] half extents along the box axes            */
    int32_t n_box_pairs;
    const int32_t *box_pairs;      /* [Q][2] box indices checked for self-collision     */
    const int32_t *joint_type;     /* [dof] 0 revolute (theta = q), 1 prismatic (theta = 0,
                                      offset d + q); NULL = all revolute              */
} orc_robot;

/* A signed-distance function over configurations; the configuration is in
 * collision iff it is negative. */
typedef double (*orc_sd_fn)(const void *scene, const double *q);

typedef struct {
    const orc_robot *robot;
    const double *obs;             /* [n_obs][4] x, y, z, r (world frame) */
    int32_t n_obs;
    const double *ebox;            /* [n_ebox][15] obstacle boxes: centre (3), rotation (9,
                                      row-major, columns = axes), half extents (3), world */
    int32_t n_ebox;
} orc_arm_scene;

typedef struct {
    int32_t dim;
    const double *centres;         /* [n][dim] */
    const double *radii;           /* [n] */
    int32_t n;
} orc_ball_scene;

/* ------------------------------------------------------------------------ */
/* Forward kinematics: T_i = T_{i-1} Rz(q_i) Tz(d_i) Tx(a_i) Rx(alpha_i)      */
/* ------------------------------------------------------------------------ */

static void mat4_identity(double M[16]) {
    memset(M, 0, 16 * sizeof(double));
    M[0] = M[5] = M[10] = M[15] = 1.0;
}

static void mat4_mul(const double A[16], const double B[16], double C[16]) {
    double R[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += A[4 * i + k] * B[4 * k + j];
            R[4 * i + j] = s;
        }
    memcpy(C, R, sizeof(R));
}

static void rot_z(double th, double M[16]) {
    mat4_identity(M);
    M[0] = cos(th); M[1] = -sin(th);
    M[4] = sin(th); M[5] = cos(th);
}

static void rot_x(double al, double M[16]) {
    mat4_identity(M);
    M[5] = cos(al); M[6] = -sin(al);
    M[9] = sin(al); M[10] = cos(al);
}

static void trans(double x, double y, double z, double M[16]) {
    mat4_identity(M);
    M[3] = x; M[7] = y; M[11] = z;
}

/* Link frames T_1..T_dof (world <- link i), each a row-major 4x4.  A
 * prismatic joint keeps theta = 0 and slides along its z axis: d_i + q_i. */
void orc_link_frames(const orc_robot *rb, const double *q, double *frames /* [dof][16] */) {
    double T[16], E[16];
    mat4_identity(T);
    for (int i = 0; i < rb->dof; ++i) {
        const int prismatic = rb->joint_type && rb->joint_type[i] == 1;
        rot_z(prismatic ? 0.0 : q[i], E);                       mat4_mul(T, E, T);
        trans(0, 0, rb->d[i] + (prismatic ? q[i] : 0.0), E);   mat4_mul(T, E, T);
        trans(rb->a[i], 0, 0, E);     mat4_mul(T, E, T);
        rot_x(rb->alpha[i], E);       mat4_mul(T, E, T);
        memcpy(frames + 16 * i, T, sizeof(T));
    }
}

/* World-frame sphere centres c_s = T_{link(s)} [p_s; 1]. */
void orc_sphere_centres(const orc_robot *rb, const double *q, double *centres /* [S][3] */) {
    double *frames = (double *)malloc(sizeof(double) * 16 * (size_t)rb->dof);
    orc_link_frames(rb, q, frames);
    for (int s = 0; s < rb->n_spheres; ++s) {
        const double *T = frames + 16 * rb->sphere_link[s];
        const double *p = rb->sphere_xyz + 3 * s;
        for (int r = 0; r < 3; ++r)
            centres[3 * s + r] = T[4 * r + 0] * p[0] + T[4 * r + 1] * p[1] + T[4 * r + 2] * p[2] + T[4 * r + 3];
    }
    free(frames);
}

/* ------------------------------------------------------------------------ */
/* Collision checking: plain definition over all pairs                       */
/* ------------------------------------------------------------------------ */

static double dist3(const double *x, const double *y) {
    double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* ---- boxes ---------------------------------------------------------------- */

/* World pose of a box fixed to a link: c = R_T p + t, R = R_T R_local. */
static void box_world(const double T[16], const double *pose, double c[3], double R[9]) {
    for (int r = 0; r < 3; ++r) {
        c[r] = T[4 * r + 0] * pose[0] + T[4 * r + 1] * pose[1] + T[4 * r + 2] * pose[2] + T[4 * r + 3];
        for (int k = 0; k < 3; ++k)
            R[3 * r + k] = T[4 * r + 0] * pose[3 + k] + T[4 * r + 1] * pose[6 + k] + T[4 * r + 2] * pose[9 + k];
    }
}

/* Signed distance between a sphere (centre x, radius r) and a box (centre c,
 * rotation R whose columns are the axes, half extents h): the point in box
 * coordinates p = R^T (x - c); outside the box the Euclidean distance from p
 * to the box minus r, inside minus (the distance to the nearest face + r). */
double orc_sd_sphere_box(const double x[3], double r, const double c[3], const double R[9], const double h[3]) {
    double p[3], out2 = 0.0, depth = INFINITY;
    int inside = 1;
    for (int k = 0; k < 3; ++k) {
        p[k] = R[0 + k] * (x[0] - c[0]) + R[3 + k] * (x[1] - c[1]) + R[6 + k] * (x[2] - c[2]);
        const double a = fabs(p[k]);
        if (a > h[k]) {
            inside = 0;
            out2 += (a - h[k]) * (a - h[k]);
        }
        if (h[k] - a < depth) depth = h[k] - a;
    }
    return inside ? -depth - r : sqrt(out2) - r;
}

/* Separating-axis value of two boxes: the largest, over the 3 + 3 face
 * normals and the 9 cross products of an edge of each box (unit, those with
 * |A_i x B_j| < 1e-6 skipped as parallel), of |t . L| - r_A(L) - r_B(L), with
 * t the centre offset and r_X(L) = sum_k h_k |X_k . L| the box's half width
 * along L.  Positive: the boxes are apart (a lower bound on their distance);
 * otherwise minus the smallest overlap over the axes, which for two boxes is
 * the penetration depth.  *fragile (may be NULL) flags where FP32 rounding
 * of the poses, amplified on a cross axis of nearly parallel edges
 * (|A_i x B_j| < weak, a "weak" axis; weak and the band are set by
 * orc_set_fragility, default 0.05 and 5e-5), can change the result: bit 0
 * (the value) when a weak axis comes within 1e-3 of the value or within 1e-4
 * of 0; bit 1 (the sign) when the value is set by a weak axis, is above
 * -band, and the other axes alone give less than band. */
static double g_weak_axis = 0.05, g_fragile_band = 5e-5;

/* Thresholds of the fragility bits of orc_sat_boxes (test infrastructure: the
 * conditioning of a cross axis is about 1/|A_i x B_j|, so a smaller weak norm
 * needs a wider band).  Not thread-safe: set before checking. */
void orc_set_fragility(double weak_axis_norm, double band) {
    g_weak_axis = weak_axis_norm;
    g_fragile_band = band;
}

double orc_sat_boxes(const double cA[3], const double RA[9], const double hA[3], const double cB[3],
                     const double RB[9], const double hB[3], int *fragile) {
    double Ax[3][3], Bx[3][3], t[3];
    for (int k = 0; k < 3; ++k) {
        for (int r = 0; r < 3; ++r) {
            Ax[k][r] = RA[3 * r + k];
            Bx[k][r] = RB[3 * r + k];
        }
        t[k] = cB[k] - cA[k];
    }
    double best = -INFINITY, best_good = -INFINITY;
    double weak[9];
    int n_weak = 0;
    for (int a = 0; a < 15; ++a) {
        double L[3];
        double norm = 1.0;
        if (a < 3) {
            memcpy(L, Ax[a], sizeof(L));
        } else if (a < 6) {
            memcpy(L, Bx[a - 3], sizeof(L));
        } else {
            const double *u = Ax[(a - 6) / 3], *v = Bx[(a - 6) % 3];
            L[0] = u[1] * v[2] - u[2] * v[1];
            L[1] = u[2] * v[0] - u[0] * v[2];
            L[2] = u[0] * v[1] - u[1] * v[0];
            norm = sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
            if (norm < 1e-6) continue;
            for (int k = 0; k < 3; ++k) L[k] /= norm;
        }
        double rA = 0.0, rB = 0.0;
        for (int k = 0; k < 3; ++k) {
            rA += hA[k] * fabs(Ax[k][0] * L[0] + Ax[k][1] * L[1] + Ax[k][2] * L[2]);
            rB += hB[k] * fabs(Bx[k][0] * L[0] + Bx[k][1] * L[1] + Bx[k][2] * L[2]);
        }
        const double sep = fabs(t[0] * L[0] + t[1] * L[1] + t[2] * L[2]) - rA - rB;
        if (sep > best) best = sep;
        if (a >= 6 && norm < g_weak_axis)
            weak[n_weak++] = sep;
        else if (sep > best_good)
            best_good = sep;
    }
    if (fragile) {
        *fragile = 0;
        for (int i = 0; i < n_weak; ++i)
            if (weak[i] > best - 1e-3 || fabs(weak[i]) < 1e-4) *fragile |= 1;
        if (best > best_good && best > -g_fragile_band && best_good < g_fragile_band) *fragile |= 2;
    }
    return best;
}

/* Minimum signed distance over robot-obstacle pairs (sd_env) and over the
 * listed self pairs (sd_self); +inf when a set of pairs is empty.  Obstacle
 * pairs: robot spheres and boxes against obstacle spheres and boxes
 * (sphere-sphere: centre distance minus radii; sphere-box: orc_sd_sphere_box;
 * box-box: orc_sat_boxes).  Self pairs: the sphere pairs and the box pairs.
 * *fragile (may be NULL): bit 0 when some box-box pair within 1e-3 of the
 * minimum of its own kind (sd_env for obstacle boxes, sd_self for box self
 * pairs) has a fragile value, bit 1 when some box-box pair has a fragile
 * sign (orc_sat_boxes). */
void orc_check_config(const orc_robot *rb, const double *obs, int32_t n_obs, const double *ebox, int32_t n_ebox,
                      const double *q, double *sd_env, double *sd_self, int *fragile) {
    double *c = (double *)malloc(sizeof(double) * 3 * (size_t)(rb->n_spheres > 0 ? rb->n_spheres : 1));
    const int B = rb->n_boxes;
    double *bc = (double *)malloc(sizeof(double) * 12 * (size_t)(B > 0 ? B : 1));
    orc_sphere_centres(rb, q, c);
    if (B > 0) {
        double *frames = (double *)malloc(sizeof(double) * 16 * (size_t)rb->dof);
        orc_link_frames(rb, q, frames);
        for (int k = 0; k < B; ++k)
            box_world(frames + 16 * rb->box_link[k], rb->box_pose + 12 * k, bc + 12 * k, bc + 12 * k + 3);
        free(frames);
    }
    double env = INFINITY, self = INFINITY;
    for (int s = 0; s < rb->n_spheres; ++s)
        for (int o = 0; o < n_obs; ++o) {
            double sd = dist3(c + 3 * s, obs + 4 * o) - rb->sphere_r[s] - obs[4 * o + 3];
            if (sd < env) env = sd;
        }
    for (int s = 0; s < rb->n_spheres; ++s)
        for (int e = 0; e < n_ebox; ++e) {
            const double *E = ebox + 15 * e;
            double sd = orc_sd_sphere_box(c + 3 * s, rb->sphere_r[s], E, E + 3, E + 12);
            if (sd < env) env = sd;
        }
    /* box-box values with their fragility, kept until the minima are known;
       the first n_eb are obstacle-box pairs */
    const int n_bb = B * n_ebox + rb->n_box_pairs;
    double *bbv = (double *)malloc(sizeof(double) * (size_t)(n_bb > 0 ? n_bb : 1));
    int *bbf = (int *)malloc(sizeof(int) * (size_t)(n_bb > 0 ? n_bb : 1));
    int nb = 0;
    const int n_eb = B * n_ebox;
    for (int k = 0; k < B; ++k) {
        const double *h = rb->box_half + 3 * k;
        for (int o = 0; o < n_obs; ++o) {
            double sd = orc_sd_sphere_box(obs + 4 * o, obs[4 * o + 3], bc + 12 * k, bc + 12 * k + 3, h);
            if (sd < env) env = sd;
        }
        for (int e = 0; e < n_ebox; ++e) {
            const double *E = ebox + 15 * e;
            double sd = orc_sat_boxes(bc + 12 * k, bc + 12 * k + 3, h, E, E + 3, E + 12, &bbf[nb]);
            bbv[nb++] = sd;
            if (sd < env) env = sd;
        }
    }
    for (int p = 0; p < rb->n_self; ++p) {
        int s = rb->self_pairs[2 * p], t = rb->self_pairs[2 * p + 1];
        double sd = dist3(c + 3 * s, c + 3 * t) - rb->sphere_r[s] - rb->sphere_r[t];
        if (sd < self) self = sd;
    }
    for (int p = 0; p < rb->n_box_pairs; ++p) {
        int i = rb->box_pairs[2 * p], j = rb->box_pairs[2 * p + 1];
        double sd = orc_sat_boxes(bc + 12 * i, bc + 12 * i + 3, rb->box_half + 3 * i, bc + 12 * j, bc + 12 * j + 3,
                                  rb->box_half + 3 * j, &bbf[nb]);
        bbv[nb++] = sd;
        if (sd < self) self = sd;
    }
    if (fragile) {
        *fragile = 0;
        for (int i = 0; i < nb; ++i) {
            if ((bbf[i] & 1) && bbv[i] < (i < n_eb ? env : self) + 1e-3) *fragile |= 1;
            *fragile |= bbf[i] & 2;
        }
    }
    free(bbv);
    free(bbf);
    free(bc);
    free(c);
    *sd_env = env;
    *sd_self = self;
}

/* Batch form: flag = [min(sd_env, sd_self) < 0].  Any output may be NULL. */
void orc_check_batch(const orc_robot *rb, const double *obs, int32_t n_obs, const double *ebox, int32_t n_ebox,
                     const double *q, int64_t n, uint8_t *flags, double *min_sd, double *sd_env, double *sd_self,
                     uint8_t *fragile) {
    const int dof = rb->dof;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double e, s;
        int fr = 0;
        orc_check_config(rb, obs, n_obs, ebox, n_ebox, q + (size_t)i * dof, &e, &s, fragile ? &fr : NULL);
        double m = e < s ? e : s;
        if (flags) flags[i] = (uint8_t)(m < 0.0);
        if (min_sd) min_sd[i] = m;
        if (sd_env) sd_env[i] = e;
        if (sd_self) sd_self[i] = s;
        if (fragile) fragile[i] = (uint8_t)fr;
    }
}

/* ---- collision map of a dynamic roadmap (appendix, DRM construction) ------- */

/* The task space is cut into voxels of side s: voxel (i, j, k) of a grid of
 * dims[0] x dims[1] x dims[2] cells from corner lo has index v = (k dims[1] +
 * j) dims[0] + i and is represented by its circumscribing sphere, centre
 * lo + s (i + 1/2, j + 1/2, k + 1/2), radius sqrt(3)/2 s.  For each listed
 * voxel vox[m] and each node q_n, sd[m][n] = the minimum signed distance
 * between that sphere and the robot's spheres and boxes (self pairs play no
 * part); the node collides with the voxel iff sd < 0. */
void orc_collision_map(const orc_robot *rb, const double *q, int64_t n_nodes, const double lo[3], double side,
                       const int32_t dims[3], const int64_t *vox, int64_t n_vox, double *sd) {
    const double rv = 0.5 * sqrt(3.0) * side;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t n = 0; n < n_nodes; ++n) {
        const double *qn = q + (size_t)n * rb->dof;
        double *c = (double *)malloc(sizeof(double) * 3 * (size_t)(rb->n_spheres > 0 ? rb->n_spheres : 1));
        double *bc = (double *)malloc(sizeof(double) * 12 * (size_t)(rb->n_boxes > 0 ? rb->n_boxes : 1));
        orc_sphere_centres(rb, qn, c);
        if (rb->n_boxes > 0) {
            double *frames = (double *)malloc(sizeof(double) * 16 * (size_t)rb->dof);
            orc_link_frames(rb, qn, frames);
            for (int k = 0; k < rb->n_boxes; ++k)
                box_world(frames + 16 * rb->box_link[k], rb->box_pose + 12 * k, bc + 12 * k, bc + 12 * k + 3);
            free(frames);
        }
        for (int64_t m = 0; m < n_vox; ++m) {
            const int64_t v = vox[m];
            const int64_t i = v % dims[0], j = (v / dims[0]) % dims[1], k = v / ((int64_t)dims[0] * dims[1]);
            const double x[3] = {lo[0] + side * ((double)i + 0.5), lo[1] + side * ((double)j + 0.5),
                                 lo[2] + side * ((double)k + 0.5)};
            double best = INFINITY;
            for (int s = 0; s < rb->n_spheres; ++s) {
                const double d = dist3(c + 3 * s, x) - rb->sphere_r[s] - rv;
                if (d < best) best = d;
            }
            for (int b = 0; b < rb->n_boxes; ++b) {
                const double d = orc_sd_sphere_box(x, rv, bc + 12 * b, bc + 12 * b + 3, rb->box_half + 3 * b);
                if (d < best) best = d;
            }
            sd[(size_t)m * n_nodes + n] = best;
        }
        free(bc);
        free(c);
    }
}

double orc_arm_sd(const void *scene, const double *q) {
    const orc_arm_scene *sc = (const orc_arm_scene *)scene;
    double e, s;
    orc_check_config(sc->robot, sc->obs, sc->n_obs, sc->ebox, sc->n_ebox, q, &e, &s, NULL);
    return e < s ? e : s;
}

/* Point robot among balls (a 2-D disc forest is the Forest scene of Sec. VI-A
 * with identity kinematics). */
double orc_ball_sd(const void *scene, const double *q) {
    const orc_ball_scene *sc = (const orc_ball_scene *)scene;
    double best = INFINITY;
    for (int o = 0; o < sc->n; ++o) {
        double s2 = 0.0;
        for (int j = 0; j < sc->dim; ++j) {
            double t = q[j] - sc->centres[(size_t)o * sc->dim + j];
            s2 += t * t;
        }
        double sd = sqrt(s2) - sc->radii[o];
        if (sd < best) best = sd;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC'11): 10 rounds of the 4x32 S-box with multipliers     */
/* 0xD2511F53 / 0xCD9E8D57 and Weyl key increments 0x9E3779B9 / 0xBB67AE85.  */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 32-bit word -> uniform in (0, 1): ((x >> 9) + 1/2) * 2^-23.  The result
 * (2m + 1) 2^-24 with m < 2^23 needs 24 significant bits, so it is exact in
 * FP32 as well as FP64. */
double orc_u01(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

/* Word w of the random stream of (sample i, edge e, iteration k, step s).
 * Counter = (i, e, k, 16*s + w/4), key = (seed low, seed high). */
static double stream_u01(uint64_t seed, uint32_t i, uint32_t e, uint32_t k, uint32_t s, int w) {
    uint32_t ctr[4] = {i, e, k, 16u * s + (uint32_t)(w / 4)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return orc_u01(out[w % 4]);
}

/* ------------------------------------------------------------------------ */
/* Unadaptive test constants (Sec. IV-B)                                     */
/* ------------------------------------------------------------------------ */

/* delta_k = 6 delta / (pi^2 k^2); M_k = ceil(2 ln(1/delta_k) / (eps tau^2))
 * (natural log: the Chernoff lower-tail bound exp(-tau^2 eps M / 2) <= delta_k);
 * accept iff (#collisions in the first M_k samples) <= M_k (1 - tau) eps, taken
 * as the integer T_k = floor(M_k (1 - tau) eps + 1e-9). */
void orc_test_constants(double eps, double delta, double tau, int32_t k, int64_t *M, int64_t *T) {
    double dk = 6.0 * delta / (ORC_PI * ORC_PI * (double)k * (double)k);
    double m = ceil(2.0 * log(1.0 / dk) / (eps * tau * tau));
    *M = (int64_t)m;
    *T = (int64_t)floor(m * (1.0 - tau) * eps + 1e-9);
}

/* ------------------------------------------------------------------------ */
/* Hit-and-run inside P = {x : A x <= b} (Sec. IV-B, Lovasz 1999)            */
/* ------------------------------------------------------------------------ */

/* Step s (>= 1) of walk i from the point x (updated in place): draws a
 * direction u = g/|g|, g ~ N(0, I) (Box-Muller on word pairs), intersects the
 * line x + t u with every row to get the chord [t_lo, t_hi], and moves to
 * t ~ U[t_lo, t_hi].  If rounding leaves t_hi < t_lo the walk stays put.
 * den_bind (may be NULL) receives a^T u of the rows that set t_lo and t_hi
 * (0 where no row bounds that end): how well conditioned the two chord ends
 * are. */
void orc_hit_and_run_step(int32_t d, const double *A, const double *b, int32_t F, uint64_t seed,
                          uint32_t i, uint32_t e, uint32_t k, uint32_t s, double *x, double *den_bind) {
    const int npair = (d + 1) / 2;
    double g[64], u[64];
    for (int m = 0; m < npair; ++m) {
        double ua = stream_u01(seed, i, e, k, s, 2 * m);
        double ub = stream_u01(seed, i, e, k, s, 2 * m + 1);
        double r = sqrt(-2.0 * log(ua));
        g[2 * m] = r * cos(2.0 * ORC_PI * ub);
        g[2 * m + 1] = r * sin(2.0 * ORC_PI * ub);
    }
    double nrm = 0.0;
    for (int j = 0; j < d; ++j) nrm += g[j] * g[j];
    nrm = sqrt(nrm);
    for (int j = 0; j < d; ++j) u[j] = g[j] / nrm;
    double t_lo = -INFINITY, t_hi = INFINITY, den_lo = 0.0, den_hi = 0.0;
    for (int f = 0; f < F; ++f) {
        double den = 0.0, ax = 0.0;
        for (int j = 0; j < d; ++j) {
            den += A[(size_t)f * d + j] * u[j];
            ax += A[(size_t)f * d + j] * x[j];
        }
        double num = b[f] - ax;
        if (den > 0.0) {
            double t = num / den;
            if (t < t_hi) { t_hi = t; den_hi = den; }
        } else if (den < 0.0) {
            double t = num / den;
            if (t > t_lo) { t_lo = t; den_lo = den; }
        }
    }
    double wt = stream_u01(seed, i, e, k, s, 2 * npair);
    double t = 0.0;
    if (t_hi >= t_lo && isfinite(t_lo) && isfinite(t_hi)) t = t_lo + wt * (t_hi - t_lo);
    for (int j = 0; j < d; ++j) x[j] += t * u[j];
    if (den_bind) {
        den_bind[0] = den_lo;
        den_bind[1] = den_hi;
    }
}

/* One walk: start uniform on L = conv{v1, v2}, then n_mix steps. */
void orc_hit_and_run_walk(int32_t d, const double *A, const double *b, int32_t F,
                          const double *v1, const double *v2, int32_t n_mix, uint64_t seed,
                          uint32_t i, uint32_t e, uint32_t k, double *x) {
    double w0 = stream_u01(seed, i, e, k, 0, 0);
    for (int j = 0; j < d; ++j) x[j] = v1[j] + w0 * (v2[j] - v1[j]);
    for (int s = 1; s <= n_mix; ++s) orc_hit_and_run_step(d, A, b, F, seed, i, e, k, (uint32_t)s, x, NULL);
}

/* Step s of walks first .. first + n - 1, each from its own point X[i] (in
 * place); den_bind [n][2] or NULL. */
void orc_hit_and_run_steps(int32_t d, const double *A, const double *b, int32_t F, uint64_t seed, uint32_t e,
                           uint32_t k, uint32_t s, int64_t first, int64_t n, double *X, double *den_bind) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        orc_hit_and_run_step(d, A, b, F, seed, (uint32_t)(first + i), e, k, s, X + (size_t)i * d,
                             den_bind ? den_bind + 2 * (size_t)i : NULL);
}

void orc_hit_and_run(int32_t d, const double *A, const double *b, int32_t F, const double *v1,
                     const double *v2, int32_t n_mix, uint64_t seed, uint32_t e, uint32_t k,
                     int64_t n, double *S /* [n][d] */) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        orc_hit_and_run_walk(d, A, b, F, v1, v2, n_mix, seed, (uint32_t)i, e, k, S + (size_t)i * d);
}

/* ------------------------------------------------------------------------ */
/* Projection, gradient, bisection (Sec. IV-A, IV-B)                         */
/* ------------------------------------------------------------------------ */

/* c_proj = v1 if v1 = v2, else (1 - alpha) v1 + alpha v2 with
 * alpha = min(max((c - v1)^T (v2 - v1) / |v2 - v1|^2, 0), 1). */
void orc_project(int32_t d, const double *v1, const double *v2, const double *c, double *c_proj, double *alpha_out) {
    double num = 0.0, den = 0.0;
    for (int j = 0; j < d; ++j) {
        num += (c[j] - v1[j]) * (v2[j] - v1[j]);
        den += (v2[j] - v1[j]) * (v2[j] - v1[j]);
    }
    double alpha = 0.0;
    if (den > 0.0) {
        alpha = num / den;
        if (alpha < 0.0) alpha = 0.0;
        if (alpha > 1.0) alpha = 1.0;
    }
    for (int j = 0; j < d; ++j) c_proj[j] = (1.0 - alpha) * v1[j] + alpha * v2[j];
    if (alpha_out) *alpha_out = alpha;
}

/* For one colliding sample c: project onto L, take the gradient direction
 * a = (c - c_proj)/|c - c_proj| (eq:dist_grad), optionally check c_proj for
 * collision (fail-fast), then n_b bisection steps on the segment
 * [c_proj, c] keeping the colliding end: mid = (lo + hi)/2, hi = mid if mid
 * collides else lo = mid.  c* = hi, t* = |c* - c_proj|.  Also reports the
 * smallest |sd| met at any evaluated point (projection and midpoints), and
 * optionally every evaluated signed distance (sd_trace[0] = projection,
 * sd_trace[1 + i] = midpoint of step i), so a caller can tell where a
 * lower-precision evaluation may legitimately decide differently.  Returns 1
 * if c_proj collides. */
int orc_bisect(const void *scene, orc_sd_fn sd, int32_t d, const double *v1, const double *v2,
               const double *c, int32_t n_b, double *c_star, double *t_star, double *a_dir,
               double *c_proj_out, double *min_abs_sd, double *sd_trace) {
    double cp[64], lo[64], hi[64], mid[64];
    orc_project(d, v1, v2, c, cp, NULL);
    double nrm = 0.0;
    for (int j = 0; j < d; ++j) nrm += (c[j] - cp[j]) * (c[j] - cp[j]);
    nrm = sqrt(nrm);
    for (int j = 0; j < d; ++j) a_dir[j] = nrm > 0.0 ? (c[j] - cp[j]) / nrm : 0.0;
    double sp = sd(scene, cp);
    double mabs = fabs(sp);
    if (sd_trace) sd_trace[0] = sp;
    int proj_col = sp < 0.0;
    for (int j = 0; j < d; ++j) { lo[j] = cp[j]; hi[j] = c[j]; }
    for (int it = 0; it < n_b; ++it) {
        for (int j = 0; j < d; ++j) mid[j] = 0.5 * (lo[j] + hi[j]);
        double sm = sd(scene, mid);
        if (sd_trace) sd_trace[1 + it] = sm;
        if (fabs(sm) < mabs) mabs = fabs(sm);
        if (sm < 0.0) memcpy(hi, mid, sizeof(double) * d);
        else memcpy(lo, mid, sizeof(double) * d);
    }
    double t = 0.0;
    for (int j = 0; j < d; ++j) {
        c_star[j] = hi[j];
        t += (hi[j] - cp[j]) * (hi[j] - cp[j]);
        if (c_proj_out) c_proj_out[j] = cp[j];
    }
    *t_star = sqrt(t);
    if (min_abs_sd) *min_abs_sd = mabs;
    return proj_col;
}

/* ------------------------------------------------------------------------ */
/* Ordering and placing hyperplanes with step back (Sec. IV-B, IV-C)         */
/* ------------------------------------------------------------------------ */

enum { ORC_CERTIFIED = 0, ORC_MAX_ITERS = 1, ORC_IN_COLLISION = 2, ORC_INVALID = 3 };

typedef struct { double t; int32_t j; } orc_key;

static int key_cmp(const void *pa, const void *pb) {
    const orc_key *a = (const orc_key *)pa, *b = (const orc_key *)pb;
    if (a->t < b->t) return -1;
    if (a->t > b->t) return 1;
    return (a->j > b->j) - (a->j < b->j);
}

/* Candidates j = 0..n-1 (in candidate order) with c*_j, a_j, t*_j.  Sort by
 * (t*, j); repeatedly take the closest candidate not yet discarded, fail with
 * IN_COLLISION if its t* <= t_col, place a_j^T x <= b_j - Delta with
 * b_j = a_j^T c*_j and the relaxed step back
 *   r = max(a^T v1, a^T v2) - b + Delta_max,  Delta = Delta_max - r if r > 0
 *   else Delta_max,
 * then discard every remaining candidate with a^T c* > b - Delta.  At most
 * n_f planes.  Rows are appended to A/b at index *n_faces (capacity cap).
 * placed_idx (optional) receives the candidate index behind each new row.
 * Returns ORC_CERTIFIED (0) on success or ORC_IN_COLLISION. */
int orc_place(int32_t d, const double *v1, const double *v2, int32_t n, const double *c_star,
              const double *a_dir, const double *t_star, int32_t n_f, double step_back_max,
              double t_col, double *A, double *b, int32_t *n_faces, int32_t cap, int32_t *placed_idx,
              int32_t *n_placed) {
    orc_key *keys = (orc_key *)malloc(sizeof(orc_key) * (size_t)(n > 0 ? n : 1));
    uint8_t *alive = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    for (int j = 0; j < n; ++j) { keys[j].t = t_star[j]; keys[j].j = j; alive[j] = 1; }
    qsort(keys, (size_t)n, sizeof(orc_key), key_cmp);
    int placed = 0, status = ORC_CERTIFIED;
    for (int q = 0; q < n && placed < n_f; ++q) {
        int j = keys[q].j;
        if (!alive[j]) continue;
        if (t_star[j] <= t_col) { status = ORC_IN_COLLISION; break; }
        if (*n_faces >= cap) break;
        const double *a = a_dir + (size_t)j * d;
        double bj = 0.0, av1 = 0.0, av2 = 0.0;
        for (int k = 0; k < d; ++k) {
            bj += a[k] * c_star[(size_t)j * d + k];
            av1 += a[k] * v1[k];
            av2 += a[k] * v2[k];
        }
        double r = (av1 > av2 ? av1 : av2) - bj + step_back_max;
        double delta = r > 0.0 ? step_back_max - r : step_back_max;
        double rhs = bj - delta;
        for (int k = 0; k < d; ++k) A[(size_t)(*n_faces) * d + k] = a[k];
        b[*n_faces] = rhs;
        if (placed_idx) placed_idx[placed] = j;
        ++(*n_faces);
        ++placed;
        for (int l = 0; l < n; ++l) {
            if (!alive[l]) continue;
            double ac = 0.0;
            for (int k = 0; k < d; ++k) ac += a[k] * c_star[(size_t)l * d + k];
            if (ac > rhs) alive[l] = 0;
        }
    }
    if (n_placed) *n_placed = placed;
    free(keys);
    free(alive);
    return status;
}

/* ------------------------------------------------------------------------ */
/* EI-ZO (Alg. 1)                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    double eps, delta, tau, step_back_max, t_col;
    int32_t n_p, n_f, n_b, n_mix, max_iters;
    uint64_t seed;
    int64_t edge_id;
} orc_params;

typedef struct {
    int32_t iterations, planes;
    int64_t final_m, test_collisions, samples, checks;
} orc_stats;

/* P <- D (rows A_D, b_D);  for k = 1..max_iters:
 *   |S| = max(N_p, M_k) hit-and-run samples in P; flags by collision checks;
 *   accept (CERTIFIED) iff the collisions among the first M_k are <= T_k;
 *   candidates = first min(N_p, |S_col|) colliding samples in index order;
 *   projection + fail-fast + bisection per candidate; order and place planes.
 * Returns the edge status; rows of P are written to A/b (capacity cap). */
int orc_eizo(const void *scene, orc_sd_fn sd, int32_t d, const double *A_D, const double *b_D,
             int32_t n_D, const double *v1, const double *v2, const orc_params *prm, double *A,
             double *b, int32_t cap, int32_t *n_faces, orc_stats *st) {
    memset(st, 0, sizeof(*st));
    *n_faces = 0;
    for (int f = 0; f < n_D && f < cap; ++f) {
        for (int j = 0; j < d; ++j) A[(size_t)f * d + j] = A_D[(size_t)f * d + j];
        b[f] = b_D[f];
        ++(*n_faces);
    }
    /* An edge is usable only if both vertices are finite and inside D. */
    for (int f = 0; f < n_D; ++f) {
        double a1 = 0.0, a2 = 0.0;
        for (int j = 0; j < d; ++j) {
            if (!isfinite(v1[j]) || !isfinite(v2[j])) return ORC_INVALID;
            a1 += A_D[(size_t)f * d + j] * v1[j];
            a2 += A_D[(size_t)f * d + j] * v2[j];
        }
        if (a1 > b_D[f] || a2 > b_D[f]) return ORC_INVALID;
    }
    int64_t M0, T0;
    orc_test_constants(prm->eps, prm->delta, prm->tau, prm->max_iters, &M0, &T0);
    int64_t cap_s = prm->n_p > M0 ? prm->n_p : M0;
    double *S = (double *)malloc(sizeof(double) * (size_t)cap_s * d);
    uint8_t *flg = (uint8_t *)malloc((size_t)cap_s);
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(prm->n_p > 0 ? prm->n_p : 1));
    double *cs = (double *)malloc(sizeof(double) * (size_t)(prm->n_p > 0 ? prm->n_p : 1) * d);
    double *ad = (double *)malloc(sizeof(double) * (size_t)(prm->n_p > 0 ? prm->n_p : 1) * d);
    double *ts = (double *)malloc(sizeof(double) * (size_t)(prm->n_p > 0 ? prm->n_p : 1));
    uint8_t *pc = (uint8_t *)malloc((size_t)(prm->n_p > 0 ? prm->n_p : 1));
    int status = ORC_MAX_ITERS;
    for (int k = 1; k <= prm->max_iters; ++k) {
        int64_t M, T;
        orc_test_constants(prm->eps, prm->delta, prm->tau, k, &M, &T);
        int64_t nS = prm->n_p > M ? prm->n_p : M;
        orc_hit_and_run(d, A, b, *n_faces, v1, v2, prm->n_mix, prm->seed, (uint32_t)prm->edge_id,
                        (uint32_t)k, nS, S);
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < nS; ++i) flg[i] = (uint8_t)(sd(scene, S + (size_t)i * d) < 0.0);
        int64_t cnt = 0;
        for (int64_t i = 0; i < M; ++i) cnt += flg[i];
        st->iterations = k;
        st->final_m = M;
        st->test_collisions = cnt;
        st->samples += nS;
        st->checks += nS;
        if (cnt <= T) { status = ORC_CERTIFIED; break; }
        int32_t nc = 0;
        for (int64_t i = 0; i < nS && nc < prm->n_p; ++i)
            if (flg[i]) cand[nc++] = (int32_t)i;
        int any_proj = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : any_proj)
        for (int j = 0; j < nc; ++j) {
            int p = orc_bisect(scene, sd, d, v1, v2, S + (size_t)cand[j] * d, prm->n_b, cs + (size_t)j * d,
                               ts + j, ad + (size_t)j * d, NULL, NULL, NULL);
            pc[j] = (uint8_t)p;
            any_proj |= p;
        }
        st->checks += (int64_t)nc * (1 + prm->n_b);
        if (any_proj) { status = ORC_IN_COLLISION; break; }
        int32_t np = 0;
        int ps = orc_place(d, v1, v2, nc, cs, ad, ts, prm->n_f, prm->step_back_max, prm->t_col, A, b,
                           n_faces, cap, NULL, &np);
        st->planes += np;
        if (ps == ORC_IN_COLLISION) { status = ORC_IN_COLLISION; break; }
    }
    free(S); free(flg); free(cand); free(cs); free(ad); free(ts); free(pc);
    return status;
}

/* Convenience entry points for the two scene kinds. */
int orc_eizo_arm(const orc_robot *rb, const double *obs, int32_t n_obs, const double *ebox, int32_t n_ebox,
                 const double *A_D, const double *b_D, int32_t n_D, const double *v1, const double *v2,
                 const orc_params *prm, double *A, double *b, int32_t cap, int32_t *n_faces,
                 orc_stats *st) {
    orc_arm_scene sc = {rb, obs, n_obs, ebox, n_ebox};
    return orc_eizo(&sc, orc_arm_sd, rb->dof, A_D, b_D, n_D, v1, v2, prm, A, b, cap, n_faces, st);
}

int orc_eizo_balls(int32_t dim, const double *centres, const double *radii, int32_t n,
                   const double *A_D, const double *b_D, int32_t n_D, const double *v1,
                   const double *v2, const orc_params *prm, double *A, double *b, int32_t cap,
                   int32_t *n_faces, orc_stats *st) {
    orc_ball_scene sc = {dim, centres, radii, n};
    return orc_eizo(&sc, orc_ball_sd, dim, A_D, b_D, n_D, v1, v2, prm, A, b, cap, n_faces, st);
}

int orc_bisect_arm(const orc_robot *rb, const double *obs, int32_t n_obs, const double *ebox, int32_t n_ebox,
                   const double *v1, const double *v2, const double *c, int32_t n_b, double *c_star,
                   double *t_star, double *a_dir, double *c_proj, double *min_abs_sd, double *sd_trace) {
    orc_arm_scene sc = {rb, obs, n_obs, ebox, n_ebox};
    return orc_bisect(&sc, orc_arm_sd, rb->dof, v1, v2, c, n_b, c_star, t_star, a_dir, c_proj, min_abs_sd,
                      sd_trace);
}

int orc_bisect_balls(int32_t dim, const double *centres, const double *radii, int32_t n,
                     const double *v1, const double *v2, const double *c, int32_t n_b,
                     double *c_star, double *t_star, double *a_dir, double *c_proj,
                     double *min_abs_sd, double *sd_trace) {
    orc_ball_scene sc = {dim, centres, radii, n};
    return orc_bisect(&sc, orc_ball_sd, dim, v1, v2, c, n_b, c_star, t_star, a_dir, c_proj, min_abs_sd,
                      sd_trace);
}

/* Threads used by the OpenMP loops above (0 = runtime default). */
void orc_set_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
