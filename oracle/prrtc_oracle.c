/*
 * prrtc_oracle.c -- plain serial reference for the pRRTC hot path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product library.  Written for
 * obviousness, not speed: 4x4 homogeneous matrices multiplied in the order
 * the kinematic convention states, closed-form clearances evaluated one test
 * at a time, exhaustive nearest neighbour, rounds replayed worker by worker.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fopenmp -shared -fPIC -lm.
 * -ffp-contract=off matters: the FP32 contract below forbids fused
 * multiply-adds except where fmaf() is written out.
 */
#include "prrtc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_CAPACITY (-3)
#define ORC_E_INVALID_ENDPOINT (-4)
#define ORC_E_NO_SOLUTION (-5)

int orc_dof(const orc_robot *R) {
    int d = 0;
    for (int c = 0; c < R->n_chains; c++) d += R->chain_dof[c];
    return d;
}

int orc_n_frames(const orc_robot *R) {
    int f = 0;
    for (int c = 0; c < R->n_chains; c++) f += R->chain_dof[c] + 1;
    return f;
}

/* ---------------------------------------------------------------------------
 * Forward kinematics (Sec. III-A: FK of the robot's collision spheres).
 * Modified DH: frame j+1 = frame j * Rx(alpha_j) * Tx(a_j) * Rz(q_j) * Tz(d_j);
 * frame 0 of a chain is its base pose.
 * ------------------------------------------------------------------------- */
typedef struct {
    double m[4][4];
} mat4;

static mat4 mat_identity(void) {
    mat4 r;
    memset(&r, 0, sizeof r);
    for (int i = 0; i < 4; i++) r.m[i][i] = 1.0;
    return r;
}

static mat4 mat_mul(const mat4 *A, const mat4 *B) {
    mat4 r;
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            double s = 0.0;
            for (int k = 0; k < 4; k++) s += A->m[i][k] * B->m[k][j];
            r.m[i][j] = s;
        }
    return r;
}

static mat4 mat_rot_x(double t) {
    mat4 r = mat_identity();
    r.m[1][1] = cos(t);
    r.m[1][2] = -sin(t);
    r.m[2][1] = sin(t);
    r.m[2][2] = cos(t);
    return r;
}

static mat4 mat_rot_z(double t) {
    mat4 r = mat_identity();
    r.m[0][0] = cos(t);
    r.m[0][1] = -sin(t);
    r.m[1][0] = sin(t);
    r.m[1][1] = cos(t);
    return r;
}

static mat4 mat_trans(double x, double y, double z) {
    mat4 r = mat_identity();
    r.m[0][3] = x;
    r.m[1][3] = y;
    r.m[2][3] = z;
    return r;
}

static void store_frame(const mat4 *T, double *out) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 4; j++) out[i * 4 + j] = T->m[i][j];
}

void orc_fk_frames(const orc_robot *R, const double *q, double *frames) {
    int qi = 0, f = 0;
    for (int c = 0; c < R->n_chains; c++) {
        mat4 T = mat_identity();
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 4; j++) T.m[i][j] = (double)R->base_pose[c][i * 4 + j];
        store_frame(&T, frames + 12 * f++);
        for (int j = 0; j < R->chain_dof[c]; j++, qi++) {
            const double alpha = R->dh[3 * qi + 0], a = R->dh[3 * qi + 1], d = R->dh[3 * qi + 2];
            mat4 A = mat_rot_x(alpha), B = mat_trans(a, 0.0, 0.0), C = mat_rot_z(q[qi]),
                 D = mat_trans(0.0, 0.0, d);
            mat4 t1 = mat_mul(&T, &A);
            mat4 t2 = mat_mul(&t1, &B);
            mat4 t3 = mat_mul(&t2, &C);
            T = mat_mul(&t3, &D);
            store_frame(&T, frames + 12 * f++);
        }
    }
}

static void spheres_world(const orc_robot *R, const double *q, double *xyz) {
    double frames[12 * (ORC_MAX_DOF + ORC_MAX_CHAINS)];
    orc_fk_frames(R, q, frames);
    for (int k = 0; k < R->n_spheres; k++) {
        const double *F = frames + 12 * R->sphere_frame[k];
        const float *p = R->sphere_xyzr + 4 * k;
        for (int i = 0; i < 3; i++)
            xyz[3 * k + i] = F[4 * i + 0] * p[0] + F[4 * i + 1] * p[1] + F[4 * i + 2] * p[2] + F[4 * i + 3];
    }
}

void orc_fk_spheres(const orc_robot *R, const float *q, double *xyz) {
    double qd[ORC_MAX_DOF];
    for (int j = 0; j < orc_dof(R); j++) qd[j] = (double)q[j];
    spheres_world(R, qd, xyz);
}

void orc_fk_spheres_batch(const orc_robot *R, const float *q, int64_t n, double *xyz, int32_t n_threads) {
    const int dof = orc_dof(R);
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(n_threads)
    for (int64_t i = 0; i < n; i++) orc_fk_spheres(R, q + i * dof, xyz + i * 3 * R->n_spheres);
}

/* ---------------------------------------------------------------------------
 * Signed clearance of a sphere to a primitive (Sec. III-A: sphere tests
 * against primitive obstacles).  Negative = penetration, i.e. collision.
 * ------------------------------------------------------------------------- */
static double norm3(double x, double y, double z) { return sqrt(x * x + y * y + z * z); }

double orc_clearance(const double c[3], double r, const orc_prim *p) {
    const double v[3] = {c[0] - (double)p->c[0], c[1] - (double)p->c[1], c[2] - (double)p->c[2]};
    if (p->type == 0) { /* sphere: centre distance minus both radii */
        return norm3(v[0], v[1], v[2]) - (r + (double)p->dims[0]);
    }
    if (p->type == 1) { /* oriented cuboid: local coordinates along the box axes */
        double l[3], h[3];
        int inside = 1;
        for (int i = 0; i < 3; i++) {
            l[i] = (double)p->rot[0 * 3 + i] * v[0] + (double)p->rot[1 * 3 + i] * v[1] +
                   (double)p->rot[2 * 3 + i] * v[2];
            h[i] = (double)p->dims[i];
            if (fabs(l[i]) > h[i]) inside = 0;
        }
        if (inside) {
            double depth = h[0] - fabs(l[0]);
            for (int i = 1; i < 3; i++)
                if (h[i] - fabs(l[i]) < depth) depth = h[i] - fabs(l[i]);
            return -depth - r;
        }
        double e[3];
        for (int i = 0; i < 3; i++) {
            double cl = l[i] < -h[i] ? -h[i] : (l[i] > h[i] ? h[i] : l[i]);
            e[i] = l[i] - cl;
        }
        return norm3(e[0], e[1], e[2]) - r;
    }
    /* solid cylinder with flat caps; axis = column 2 of rot */
    const double u[3] = {(double)p->rot[2], (double)p->rot[5], (double)p->rot[8]};
    const double R = (double)p->dims[0], H = (double)p->dims[1];
    const double z = v[0] * u[0] + v[1] * u[1] + v[2] * u[2];
    const double w[3] = {v[0] - z * u[0], v[1] - z * u[1], v[2] - z * u[2]};
    const double rho = norm3(w[0], w[1], w[2]);
    if (fabs(z) <= H && rho <= R) {
        double depth = H - fabs(z);
        if (R - rho < depth) depth = R - rho;
        return -depth - r;
    }
    const double dz = fabs(z) > H ? fabs(z) - H : 0.0;
    const double dr = rho > R ? rho - R : 0.0;
    return sqrt(dz * dz + dr * dr) - r;
}

/* ---------------------------------------------------------------------------
 * ESDF grid: trilinear interpolation of the node values (clamped coordinates).
 * ------------------------------------------------------------------------- */
static const orc_esdf *g_esdf = NULL;

void orc_esdf_attach(const orc_esdf *g) { g_esdf = g; }

double orc_esdf_value(const orc_esdf *g, const double p[3]) {
    int32_t i0[3];
    double t[3];
    for (int a = 0; a < 3; a++) {
        const int32_t n = g->dims[a];
        double x = (p[a] - (double)g->origin[a]) / (double)g->voxel;
        if (x < 0.0) x = 0.0;
        if (x > (double)(n - 1)) x = (double)(n - 1);
        int32_t i = (int32_t)floor(x);
        if (i > n - 2) i = n - 2;
        i0[a] = i;
        t[a] = x - (double)i;
    }
    double e = 0.0;
    for (int dz = 0; dz < 2; dz++)
        for (int dy = 0; dy < 2; dy++)
            for (int dx = 0; dx < 2; dx++) {
                const double w = (dx ? t[0] : 1.0 - t[0]) * (dy ? t[1] : 1.0 - t[1]) * (dz ? t[2] : 1.0 - t[2]);
                const size_t at = ((size_t)(i0[2] + dz) * g->dims[1] + (size_t)(i0[1] + dy)) * g->dims[0] +
                                  (size_t)(i0[0] + dx);
                e += w * (double)g->values[at];
            }
    return e;
}

void orc_esdf_from_prims(const orc_prim *prims, int32_t n, const float origin[3], float voxel,
                         const int32_t dims[3], float *values, int32_t n_threads) {
    const int64_t total = (int64_t)dims[0] * dims[1] * dims[2];
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(n_threads)
    for (int64_t at = 0; at < total; at++) {
        const int64_t i = at % dims[0], j = (at / dims[0]) % dims[1], k = at / ((int64_t)dims[0] * dims[1]);
        const double p[3] = {(double)origin[0] + (double)voxel * (double)i, (double)origin[1] + (double)voxel * (double)j,
                             (double)origin[2] + (double)voxel * (double)k};
        double m = INFINITY;
        for (int32_t o = 0; o < n; o++) {
            const double s = orc_clearance(p, 0.0, prims + o);
            if (s < m) m = s;
        }
        values[at] = (float)m;
    }
}

/* min clearance at one configuration; stops early once below stop_below. */
static double point_clearance(const orc_robot *R, const orc_prim *prims, int32_t n_prims,
                              const double *q, double stop_below) {
    double xyz[3 * 256];
    double *buf = R->n_spheres <= 256 ? xyz : (double *)malloc(sizeof(double) * 3 * R->n_spheres);
    spheres_world(R, q, buf);
    double m = INFINITY;
    for (int k = 0; k < R->n_spheres && m >= stop_below; k++) {
        const double r = R->sphere_xyzr[4 * k + 3];
        for (int o = 0; o < n_prims; o++) {
            const double s = orc_clearance(buf + 3 * k, r, prims + o);
            if (s < m) m = s;
            if (m < stop_below) break;
        }
        if (g_esdf) {
            const double s = orc_esdf_value(g_esdf, buf + 3 * k) - r;
            if (s < m) m = s;
        }
    }
    for (int pidx = 0; pidx < R->n_self_pairs && m >= stop_below; pidx++) {
        const int i = R->self_pairs[2 * pidx], j = R->self_pairs[2 * pidx + 1];
        const double *ci = buf + 3 * i, *cj = buf + 3 * j;
        const double s = norm3(ci[0] - cj[0], ci[1] - cj[1], ci[2] - cj[2]) -
                         ((double)R->sphere_xyzr[4 * i + 3] + (double)R->sphere_xyzr[4 * j + 3]);
        if (s < m) m = s;
    }
    if (buf != xyz) free(buf);
    return m;
}

double orc_config_clearance(const orc_robot *R, const orc_prim *prims, int32_t n_prims,
                            const double *q) {
    return point_clearance(R, prims, n_prims, q, -INFINITY);
}

/* ---------------------------------------------------------------------------
 * Edge discretisation (Alg. 2; Sec. III-A).  The point count is an integer
 * decided in floating point, so it follows the FP32 contract:
 *   S = sum_j (b_j - a_j)^2 in order, no FMA;  L = sqrtf(S);
 *   n = max(1, ceil(res * L)), capped at 2^24.
 * Point i is a + (i/n)(b - a), evaluated here in FP64.
 * ------------------------------------------------------------------------- */
static float f32_norm_diff(const float *a, const float *b, int32_t dof) {
    float s = 0.0f;
    for (int j = 0; j < dof; j++) {
        const float d = b[j] - a[j];
        const float sq = d * d;
        s = s + sq;
    }
    return sqrtf(s);
}

int32_t orc_edge_count(const float *a, const float *b, int32_t dof, float res) {
    const float L = f32_norm_diff(a, b, dof);
    const float prod = res * L;
    const float x = ceilf(prod);
    if (!(x >= 1.0f)) return 1;
    if (x > 16777216.0f) return 16777216;
    return (int32_t)x;
}

double orc_edge_clearance(const orc_robot *R, const orc_prim *prims, int32_t n_prims,
                          const float *a, const float *b, float res, int32_t i_first,
                          int32_t early_exit) {
    const int dof = orc_dof(R);
    const int32_t n = orc_edge_count(a, b, dof, res);
    const double stop = early_exit ? -ORC_FLAG_BAND : -INFINITY;
    double m = INFINITY;
    double q[ORC_MAX_DOF];
    for (int32_t i = i_first; i <= n; i++) {
        const double t = (double)i / (double)n;
        for (int j = 0; j < dof; j++) q[j] = (double)a[j] + t * ((double)b[j] - (double)a[j]);
        const double s = point_clearance(R, prims, n_prims, q, stop);
        if (s < m) m = s;
        if (m < stop) break;
    }
    return m;
}

void orc_check_edges(const orc_robot *R, const orc_prim *prims, int32_t n_prims,
                     const float *a, const float *b, int64_t n_edges, float res,
                     uint8_t *valid, uint8_t *flagged, double *m_out, int32_t early_exit,
                     int32_t n_threads) {
    const int dof = orc_dof(R);
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(n_threads)
#endif
    for (int64_t e = 0; e < n_edges; e++) {
        const double m = orc_edge_clearance(R, prims, n_prims, a + e * dof, b + e * dof, res, 0,
                                            early_exit);
        if (valid) valid[e] = m >= 0.0;
        if (flagged) flagged[e] = fabs(m) <= ORC_FLAG_BAND;
        if (m_out) m_out[e] = m;
    }
    (void)n_threads;
}

/* ---------------------------------------------------------------------------
 * Nearest neighbour (Sec. III-B): exact argmin of the FP32 squared distance
 * (summed in order, no FMA) over the non-blocked nodes; ties -> lowest index.
 * ------------------------------------------------------------------------- */
int32_t orc_nearest(const float *tree, int32_t cap, int32_t size, const uint8_t *blocked,
                    const float *x, int32_t dof) {
    int32_t best = -1;
    float bd = INFINITY;
    for (int32_t i = 0; i < size; i++) {
        if (blocked && blocked[i]) continue;
        float s = 0.0f;
        for (int j = 0; j < dof; j++) {
            const float d = x[j] - tree[(int64_t)j * cap + i];
            const float sq = d * d;
            s = s + sq;
        }
        if (best < 0 || s < bd) {
            bd = s;
            best = i;
        }
    }
    return best;
}

/* Steer (Alg. 2, INTERPOLATE toward c_rand by at most delta):
 * L = |to - from| (FP32 contract); L <= delta -> to; else
 * out_j = fmaf(delta / L, to_j - from_j, from_j). */
void orc_steer(const float *from, const float *to, int32_t dof, float delta, float *out) {
    const float L = f32_norm_diff(from, to, dof);
    if (L <= delta) {
        for (int j = 0; j < dof; j++) out[j] = to[j];
        return;
    }
    const float k = delta / L;
    for (int j = 0; j < dof; j++) out[j] = fmaf(k, to[j] - from[j], from[j]);
}

/* ---------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
 * 32x32->64 multiplies with the Weyl key schedule.  Used for RANDOM_CONFIG
 * (Alg. 1) in place of the paper's Halton sequence so runs are reproducible.
 * ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* RANDOM_CONFIG: key = seed (low word, high word); counter = (draw, worker,
 * round, query) with draw = attempt * ceil(dof / 4) + block; u = (word >> 8) *
 * 2^-24; q_j = fmaf(u, hi_j - lo_j, lo_j), joint j from word j % 4 of block
 * j / 4. */
void orc_sample_config_try(uint64_t seed, uint32_t query, uint32_t round, uint32_t worker,
                           uint32_t attempt, const float *lo, const float *hi, int32_t dof, float *out) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint32_t nblk = (uint32_t)(dof + 3) / 4;
    for (int32_t draw = 0; draw * 4 < dof; draw++) {
        const uint32_t ctr[4] = {attempt * nblk + (uint32_t)draw, worker, round, query};
        uint32_t w[4];
        orc_philox4x32_10(ctr, key, w);
        for (int m = 0; m < 4 && draw * 4 + m < dof; m++) {
            const int j = draw * 4 + m;
            const float u = (float)(w[m] >> 8) * 0x1p-24f;
            out[j] = fmaf(u, hi[j] - lo[j], lo[j]);
        }
    }
}

void orc_sample_config(uint64_t seed, uint32_t query, uint32_t round, uint32_t worker,
                       const float *lo, const float *hi, int32_t dof, float *out) {
    orc_sample_config_try(seed, query, round, worker, 0, lo, hi, dof, out);
}

/* Halton points (the sampler of the paper's experiments, Sec. IV-A). */
float orc_radical_inverse(uint32_t i, uint32_t b) {
    uint64_t v = 0, bm = 1; /* v / b^m with the digits reversed */
    for (uint32_t x = i; x > 0; x /= b) {
        v = v * b + x % b;
        bm *= b;
    }
    return (float)((double)v / (double)bm);
}

static const uint32_t kPrimes[ORC_MAX_DOF] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53};

void orc_halton_config(uint64_t seed, uint32_t query, uint32_t round, uint32_t worker, uint32_t workers,
                       uint32_t tries, uint32_t attempt, const float *lo, const float *hi, int32_t dof, float *out) {
    const uint32_t i = (uint32_t)seed + 65536u * query + (round * workers + worker) * tries + attempt + 1u;
    for (int j = 0; j < dof; j++) out[j] = fmaf(orc_radical_inverse(i, kPrimes[j]), hi[j] - lo[j], lo[j]);
}

/* ---------------------------------------------------------------------------
 * Planner (Alg. 1) in deterministic rounds.
 *
 * Readings of the paper adopted here (its blocks run asynchronously with
 * atomic tree insertion, which is not reproducible):
 *  - Each round, every worker sees the same snapshot of both trees; the
 *    smaller tree (tie -> start tree) is grown (balanced RRT-Connect).
 *  - Worker w samples, finds the nearest node, steers by at most delta and
 *    checks that edge at points i = 1..n (the tree node itself is known free).
 *  - Greedy connect: n_ext = max(1, ceil(L/delta)) equal steps toward the
 *    nearest node of the other tree, targets measured from the fixed origin;
 *    the last target is that node itself.  Valid intermediate targets join
 *    the grown tree; the trees connect iff all n_ext steps are valid.
 *  - Staged nodes are appended in worker order.  A worker whose nodes do not
 *    all fit in the tree loses its connection.
 *  - Dynamic-domain sampling (Yershova et al.; the paper uses it, Sec. III):
 *    every node carries a radius, infinite at first.  A sample farther from
 *    its nearest node than that node's radius is rejected and the worker
 *    draws again (up to dds_tries samples per round); a failed extension sets
 *    its start node's radius to dds_radius at the commit.  dds_radius = 0
 *    turns this off.
 *  - The lowest-numbered connected worker gives the path.  Its segments are
 *    re-checked at validate_factor x res (points i = 0..n); on a failure the
 *    failing segment's deeper node is blocked (excluded from nearest
 *    neighbour) and the rounds continue.
 * ------------------------------------------------------------------------- */
typedef struct {
    float *q; /* [dof][cap] */
    int32_t *parent;
    uint8_t *blocked;
    float *radius; /* dynamic-domain radius */
    int32_t size, cap;
} orc_tree;

static int tree_init(orc_tree *T, int dof, int cap, const float *root) {
    T->q = (float *)calloc((size_t)dof * cap, sizeof(float));
    T->parent = (int32_t *)calloc((size_t)cap, sizeof(int32_t));
    T->blocked = (uint8_t *)calloc((size_t)cap, 1);
    T->radius = (float *)malloc(sizeof(float) * (size_t)cap);
    if (!T->q || !T->parent || !T->blocked || !T->radius) return -1;
    for (int32_t i = 0; i < cap; i++) T->radius[i] = INFINITY;
    T->cap = cap;
    for (int j = 0; j < dof; j++) T->q[(int64_t)j * cap] = root[j];
    T->parent[0] = -1;
    T->size = 1;
    return 0;
}

static void tree_free(orc_tree *T) {
    free(T->q);
    free(T->parent);
    free(T->blocked);
    free(T->radius);
}

static void tree_get(const orc_tree *T, int dof, int32_t i, float *out) {
    for (int j = 0; j < dof; j++) out[j] = T->q[(int64_t)j * T->cap + i];
}

typedef struct {
    float *nodes; /* [stage_cap][dof] */
    int32_t count, nn, other, connected, edges, flagged;
    int32_t fail_nn; /* node whose extension failed this round, or -1 */
    int32_t last; /* tree index of the last committed node */
} orc_stage;

static int is_flag(double m) { return fabs(m) <= ORC_FLAG_BAND; }

static void worker_round(const orc_robot *R, const orc_prim *prims, int32_t n_prims,
                         const orc_plan_params *p, int dof, uint32_t round, uint32_t w,
                         const orc_tree *Ts, const orc_tree *To, int32_t ns, int32_t no,
                         orc_stage *st) {
    float c_rand[ORC_MAX_DOF], c_nn[ORC_MAX_DOF], c_new[ORC_MAX_DOF], c_nno[ORC_MAX_DOF];
    float prev[ORC_MAX_DOF], tgt[ORC_MAX_DOF], D[ORC_MAX_DOF];
    st->count = 0;
    st->connected = 0;
    st->edges = 0;
    st->flagged = 0;
    st->fail_nn = -1;
    st->nn = -1;
    const int tries = p->dds_tries > 0 ? p->dds_tries : 1;
    for (int t = 0; t < tries; t++) {
        if (p->sampler == 2)
            orc_halton_config(p->seed, p->query, round, w, (uint32_t)p->workers, (uint32_t)tries, (uint32_t)t,
                              R->q_lo, R->q_hi, dof, c_rand);
        else
            orc_sample_config_try(p->seed, p->query, round, w, (uint32_t)t, R->q_lo, R->q_hi, dof, c_rand);
        const int32_t nn = orc_nearest(Ts->q, Ts->cap, ns, Ts->blocked, c_rand, dof);
        if (nn < 0) return;
        tree_get(Ts, dof, nn, c_nn);
        /* dynamic domain: reject samples beyond the nearest node's radius */
        if (p->dds_radius > 0.0f && !(f32_norm_diff(c_nn, c_rand, dof) <= Ts->radius[nn])) continue;
        st->nn = nn;
        break;
    }
    if (st->nn < 0) return;
    orc_steer(c_nn, c_rand, dof, p->delta, c_new);
    double m = orc_edge_clearance(R, prims, n_prims, c_nn, c_new, p->res, 1, 1);
    st->edges++;
    st->flagged += is_flag(m);
    if (m < 0.0) {
        st->fail_nn = st->nn;
        return;
    }
    memcpy(st->nodes, c_new, sizeof(float) * dof);
    st->count = 1;
    st->other = orc_nearest(To->q, To->cap, no, To->blocked, c_new, dof);
    if (st->other < 0) return;
    tree_get(To, dof, st->other, c_nno);
    for (int j = 0; j < dof; j++) D[j] = c_nno[j] - c_new[j];
    const float L = f32_norm_diff(c_new, c_nno, dof);
    const float ratio = L / p->delta;
    const float xf = ceilf(ratio);
    const int32_t n_ext = xf >= 1.0f ? (int32_t)xf : 1;
    memcpy(prev, c_new, sizeof(float) * dof);
    for (int32_t k = 1; k <= n_ext; k++) {
        if (k == n_ext) {
            memcpy(tgt, c_nno, sizeof(float) * dof);
        } else {
            const float t = (float)k / (float)n_ext;
            for (int j = 0; j < dof; j++) tgt[j] = fmaf(t, D[j], c_new[j]);
        }
        m = orc_edge_clearance(R, prims, n_prims, prev, tgt, p->res, 1, 1);
        st->edges++;
        st->flagged += is_flag(m);
        if (m < 0.0) return;
        if (k < n_ext) {
            memcpy(st->nodes + (size_t)st->count * dof, tgt, sizeof(float) * dof);
            st->count++;
        }
        memcpy(prev, tgt, sizeof(float) * dof);
    }
    st->connected = 1;
}

/* root -> ... -> node for tree walk; returns length. */
static int32_t walk_to_root(const orc_tree *T, int32_t node, int32_t *out, int32_t cap) {
    int32_t n = 0;
    for (int32_t x = node; x >= 0; x = T->parent[x]) {
        if (n >= cap) return -1;
        out[n++] = x;
    }
    return n; /* node first, root last */
}

static void tree_dump(const orc_tree *T, int dof, float *nodes, int32_t *parent, uint8_t *blocked) {
    for (int32_t i = 0; i < T->size; i++) {
        if (nodes) tree_get(T, dof, i, nodes + (size_t)i * dof);
        if (parent) parent[i] = T->parent[i];
        if (blocked) blocked[i] = T->blocked[i];
    }
}

int32_t orc_plan(const orc_robot *R, const orc_prim *prims, int32_t n_prims, const float *start,
                 const float *goal, const orc_plan_params *p, float *path, int32_t path_cap,
                 int32_t *path_len, orc_plan_stats *st_out, int32_t n_threads) {
    return orc_plan_dump(R, prims, n_prims, start, goal, p, path, path_cap, path_len, st_out,
                         n_threads, NULL);
}

int32_t orc_plan_dump(const orc_robot *R, const orc_prim *prims, int32_t n_prims, const float *start,
                      const float *goal, const orc_plan_params *p, float *path, int32_t path_cap,
                      int32_t *path_len, orc_plan_stats *st_out, int32_t n_threads,
                      orc_tree_dump *dump) {
    const int dof = orc_dof(R);
    orc_plan_stats st;
    memset(&st, 0, sizeof st);
    st.connect_worker = -1;
    if (path_len) *path_len = 0;
    if (dof < 1 || dof > ORC_MAX_DOF || p->workers < 1 || !(p->delta > 0.0f) || !(p->res > 0.0f) ||
        p->tree_capacity < 2 || p->max_rounds < 0) {
        if (st_out) *st_out = st;
        return ORC_E_ARG;
    }
    /* endpoints: inside the limits and collision-free */
    const float *ends[2] = {start, goal};
    for (int e = 0; e < 2; e++) {
        double qd[ORC_MAX_DOF];
        for (int j = 0; j < dof; j++) {
            if (!(ends[e][j] >= R->q_lo[j] && ends[e][j] <= R->q_hi[j])) {
                if (st_out) *st_out = st;
                return ORC_E_INVALID_ENDPOINT;
            }
            qd[j] = ends[e][j];
        }
        const double m = orc_config_clearance(R, prims, n_prims, qd);
        st.flagged_edges += is_flag(m);
        if (m < 0.0) {
            if (st_out) *st_out = st;
            return ORC_E_INVALID_ENDPOINT;
        }
    }
    orc_tree A, B;
    if (tree_init(&A, dof, p->tree_capacity, start) || tree_init(&B, dof, p->tree_capacity, goal)) {
        tree_free(&A);
        tree_free(&B);
        return ORC_E_ARG;
    }
    /* longest possible connect: ceil(|hi - lo| / delta) steps */
    const float diag = f32_norm_diff(R->q_lo, R->q_hi, dof);
    const int32_t stage_cap = (int32_t)ceilf(diag / p->delta) + 2;
    const int W = p->workers;
    orc_stage *stages = (orc_stage *)calloc((size_t)W, sizeof(orc_stage));
    float *stage_mem = (float *)calloc((size_t)W * stage_cap * dof, sizeof(float));
    int32_t *walk_a = (int32_t *)malloc(sizeof(int32_t) * p->tree_capacity);
    int32_t *walk_b = (int32_t *)malloc(sizeof(int32_t) * p->tree_capacity);
    for (int w = 0; w < W; w++) stages[w].nodes = stage_mem + (size_t)w * stage_cap * dof;
    int32_t status = ORC_E_NO_SOLUTION;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#endif
    for (int32_t round = 0; round < p->max_rounds; round++) {
        st.rounds = round + 1;
        const int s_is_a = A.size <= B.size;
        orc_tree *Ts = s_is_a ? &A : &B, *To = s_is_a ? &B : &A;
        const int32_t ns = Ts->size, no = To->size;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
        for (int w = 0; w < W; w++)
            worker_round(R, prims, n_prims, p, dof, (uint32_t)round, (uint32_t)w, Ts, To, ns, no,
                         &stages[w]);
        /* commit in worker order */
        int first = -1;
        for (int w = 0; w < W; w++) {
            orc_stage *sw = &stages[w];
            st.edges_checked += sw->edges;
            st.flagged_edges += sw->flagged;
            if (p->dds_radius > 0.0f && sw->fail_nn >= 0) Ts->radius[sw->fail_nn] = p->dds_radius;
            if (sw->count == 0) continue;
            const int32_t room = Ts->cap - Ts->size;
            const int32_t c = sw->count < room ? sw->count : room;
            for (int32_t k = 0; k < c; k++) {
                const int32_t idx = Ts->size + k;
                for (int j = 0; j < dof; j++)
                    Ts->q[(int64_t)j * Ts->cap + idx] = sw->nodes[(size_t)k * dof + j];
                Ts->parent[idx] = k == 0 ? sw->nn : idx - 1;
                Ts->blocked[idx] = 0;
                Ts->radius[idx] = INFINITY;
            }
            Ts->size += c;
            if (c < sw->count) sw->connected = 0;
            sw->last = Ts->size - 1;
            if (sw->connected && first < 0) first = w;
        }
        if (first < 0) continue;
        /* path: root_a .. x_a, x_b .. root_b */
        const orc_stage *sw = &stages[first];
        const int32_t xa = s_is_a ? sw->last : sw->other;
        const int32_t xb = s_is_a ? sw->other : sw->last;
        const int32_t na = walk_to_root(&A, xa, walk_a, A.cap);
        const int32_t nb = walk_to_root(&B, xb, walk_b, B.cap);
        const int32_t len = na + nb;
        float *tmp = (float *)malloc(sizeof(float) * (size_t)len * dof);
        int32_t *tree_of = (int32_t *)malloc(sizeof(int32_t) * len);
        int32_t *idx_of = (int32_t *)malloc(sizeof(int32_t) * len);
        for (int32_t k = 0; k < na; k++) {
            tree_get(&A, dof, walk_a[na - 1 - k], tmp + (size_t)k * dof);
            tree_of[k] = 0;
            idx_of[k] = walk_a[na - 1 - k];
        }
        for (int32_t k = 0; k < nb; k++) {
            tree_get(&B, dof, walk_b[k], tmp + (size_t)(na + k) * dof);
            tree_of[na + k] = 1;
            idx_of[na + k] = walk_b[k];
        }
        int ok = 1;
        if (p->validate_factor > 0) {
            const float res_v = p->res * (float)p->validate_factor;
            int blocked_in_path = 0;
            for (int32_t k = 0; k < len; k++) {
                const orc_tree *T = tree_of[k] == 0 ? &A : &B;
                if (T->blocked[idx_of[k]]) blocked_in_path = 1;
            }
            uint8_t *bad = (uint8_t *)calloc((size_t)len, 1);
            for (int32_t k = 0; k + 1 < len; k++) {
                const double m = orc_edge_clearance(R, prims, n_prims, tmp + (size_t)k * dof,
                                                    tmp + (size_t)(k + 1) * dof, res_v, 0, 1);
                st.edges_checked++;
                st.flagged_edges += is_flag(m);
                if (m < 0.0) bad[k] = 1;
            }
            for (int32_t k = 0; k + 1 < len; k++) {
                if (!bad[k]) continue;
                ok = 0;
                if (k + 1 < na) { /* edge inside the start tree: block the deeper node */
                    A.blocked[idx_of[k + 1]] = 1;
                } else if (k + 1 == na) { /* the connection: block the grown tree's end */
                    if (s_is_a) A.blocked[xa] = 1; else B.blocked[xb] = 1;
                } else { /* inside the goal tree: the deeper node comes first */
                    B.blocked[idx_of[k]] = 1;
                }
            }
            if (blocked_in_path) {
                ok = 0;
                if (xa != 0) A.blocked[xa] = 1;
                if (xb != 0) B.blocked[xb] = 1;
            }
            free(bad);
        }
        if (ok) {
            st.connect_worker = first;
            if (path_len) *path_len = len;
            if (len > path_cap || !path) {
                status = ORC_E_CAPACITY;
            } else {
                memcpy(path, tmp, sizeof(float) * (size_t)len * dof);
                status = ORC_OK;
            }
        } else {
            st.validation_failures++;
        }
        free(tmp);
        free(tree_of);
        free(idx_of);
        if (ok) break;
    }
    st.nodes_a = A.size;
    st.nodes_b = B.size;
    if (st_out) *st_out = st;
    if (dump) {
        tree_dump(&A, dof, dump->nodes_a, dump->parent_a, dump->blocked_a);
        tree_dump(&B, dof, dump->nodes_b, dump->parent_b, dump->blocked_b);
    }
    free(stages);
    free(stage_mem);
    free(walk_a);
    free(walk_b);
    tree_free(&A);
    tree_free(&B);
    return status;
}

double orc_path_clearance(const orc_robot *R, const orc_prim *prims, int32_t n_prims,
                          const float *path, int32_t len, float res, int32_t *n_flag) {
    const int dof = orc_dof(R);
    double m = INFINITY;
    int32_t nf = 0;
    for (int32_t k = 0; k + 1 < len; k++) {
        const double s = orc_edge_clearance(R, prims, n_prims, path + (size_t)k * dof,
                                            path + (size_t)(k + 1) * dof, res, 0, 0);
        nf += is_flag(s);
        if (s < m) m = s;
    }
    if (n_flag) *n_flag = nf;
    return m;
}
