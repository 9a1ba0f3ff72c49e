/*
 * prrtc_oracle.h -- serial reference ("oracle") for the pRRTC hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes,
 * links or calls this code; only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header, table or
 * constant generator with the HIP implementation.
 *
 * What it follows (pRRTC, Huang et al., arXiv 2503.06757):
 *   - Alg. 1 (pRRTC main loop: balanced tree choice, sample, nearest
 *     neighbour, extend, add, greedy connect, path),
 *   - Alg. 2 (pEXTEND: steer by at most delta, check the discretised edge),
 *   - Sec. III-A (forward kinematics of collision spheres, sphere tests
 *     against primitive obstacles, discretised edge checking),
 *   - Sec. III-B (nearest neighbour = exact argmin over the tree).
 * Geometry (FK, clearances, interpolated points) is in FP64.  The steps
 * whose floating point decides an integer or a tree node (edge point count,
 * steer, nearest-neighbour argmin, connect targets, random configurations)
 * follow a fixed FP32 contract that the GPU side implements identically:
 * sequential sums with no fused multiply-add, correctly rounded sqrtf and
 * division, explicit fmaf where stated.
 *
 * Status codes match the product library's (0 ok, negative errors).
 */
#ifndef PRRTC_ORACLE_H
#define PRRTC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_DOF 16
#define ORC_MAX_CHAINS 2
#define ORC_FLAG_BAND 1e-5 /* metres: |clearance| within this is "near contact" */

typedef struct {
    int32_t n_chains;
    int32_t chain_dof[ORC_MAX_CHAINS];
    float base_pose[ORC_MAX_CHAINS][12]; /* row-major 3x4 */
    const float *dh;                     /* [dof][3] = (alpha, a, d), modified DH */
    const float *q_lo, *q_hi;            /* [dof] */
    int32_t n_spheres;
    const int32_t *sphere_frame; /* global frame id: chain c's frames follow chain c-1's */
    const float *sphere_xyzr;    /* [n][4], centre in its frame + radius */
    int32_t n_self_pairs;
    const int32_t *self_pairs; /* [m][2] sphere indices */
} orc_robot;

typedef struct {
    int32_t type; /* 0 sphere, 1 cuboid, 2 cylinder */
    float c[3];
    float rot[9]; /* row-major; columns are the primitive's axes */
    float dims[3];
} orc_prim;

typedef struct {
    uint64_t seed;
    uint32_t query;
    int32_t workers;
    float delta;
    float res;
    int32_t max_rounds;
    int32_t tree_capacity;
    int32_t validate_factor;
    float dds_radius;  /* dynamic-domain radius after a failed extension; 0 = off */
    int32_t dds_tries; /* samples drawn per worker and round before giving up */
    int32_t sampler;   /* 0: Philox uniform draws; 2: Halton points (orc_halton_config) */
} orc_plan_params;

typedef struct {
    int32_t rounds;
    int32_t nodes_a, nodes_b;
    int64_t edges_checked;
    int32_t flagged_edges;      /* edges whose verdict lay within the flag band */
    int32_t validation_failures;
    int32_t connect_worker;
} orc_plan_stats;

/* ESDF grid (Sec. III-A: with camera-built maps the planner checks spheres
 * against a Euclidean signed distance field instead of primitives).  Node
 * (i, j, k) sits at origin + voxel (i, j, k); values[(k dims[1] + j) dims[0] +
 * i] is the signed distance there.  A sphere (c, r) collides iff E(c) < r,
 * E the trilinear interpolation of the node values, with c's grid
 * coordinates clamped to the grid's box (outside, the field continues as its
 * value at the nearest point of the box). */
typedef struct {
    float origin[3];
    float voxel;
    int32_t dims[3]; /* each >= 2 */
    const float *values;
} orc_esdf;

/* The ESDF that every clearance below also takes into account (NULL: none).
 * Test infrastructure: one grid at a time, set while no check runs. */
void orc_esdf_attach(const orc_esdf *g);
/* E(p): trilinear interpolation in FP64 of the FP32 node values. */
double orc_esdf_value(const orc_esdf *g, const double p[3]);
/* Node values of the signed distance to the union of n primitives (the least
 * signed clearance at radius 0; +inf for none) at origin + voxel (i, j, k),
 * in FP64 rounded to FP32; OpenMP over nodes. */
void orc_esdf_from_prims(const orc_prim *prims, int32_t n, const float origin[3], float voxel,
                         const int32_t dims[3], float *values, int32_t n_threads);

int orc_dof(const orc_robot *R);
int orc_n_frames(const orc_robot *R);

/* FK: frames[f] as row-major 3x4 (FP64) for every global frame. */
void orc_fk_frames(const orc_robot *R, const double *q, double *frames);
/* Sphere centres in world coordinates for configuration q (float32 input). */
void orc_fk_spheres(const orc_robot *R, const float *q, double *xyz);
/* Radical inverse of index i in base b (van der Corput): with i's base-b
 * digits d_0 (least significant) .. d_{m-1}, the value sum_k d_k b^-(k+1) =
 * v / b^m as an exact rational, rounded to FP64 and then to FP32. */
float orc_radical_inverse(uint32_t i, uint32_t b);
/* Halton RANDOM_CONFIG (Sec. IV-A samples configurations from Halton
 * sequences): point i = (low word of seed) + 65536 query + (round W + worker)
 * tries + attempt + 1 (mod 2^32); joint j takes the radical inverse of i in
 * the j-th prime base (2, 3, 5, ..., 53) and q_j = fmaf(u_j, hi_j - lo_j, lo_j). */
void orc_halton_config(uint64_t seed, uint32_t query, uint32_t round, uint32_t worker, uint32_t workers,
                       uint32_t tries, uint32_t attempt, const float *lo, const float *hi, int32_t dof, float *out);
/* orc_fk_spheres for n configurations q[n][dof] -> xyz[n][n_spheres][3],
 * OpenMP over configurations (n_threads <= 0: all). */
void orc_fk_spheres_batch(const orc_robot *R, const float *q, int64_t n, double *xyz, int32_t n_threads);

/* Signed clearance of a sphere (centre c, radius r) to one primitive. */
double orc_clearance(const double c[3], double r, const orc_prim *p);
/* min over environment and self pairs at configuration q (FP64). */
double orc_config_clearance(const orc_robot *R, const orc_prim *prims, int32_t n_prims,
                            const double *q);

/* FP32-contract point count of an edge. */
int32_t orc_edge_count(const float *a, const float *b, int32_t dof, float res);

/* min clearance over points i = i_first..n of edge (a, b).  With early_exit
 * the scan stops once a clearance below -flag band is seen. */
double orc_edge_clearance(const orc_robot *R, const orc_prim *prims, int32_t n_prims,
                          const float *a, const float *b, float res, int32_t i_first,
                          int32_t early_exit);

/* Batch edge verdicts: valid = (m >= 0), flagged = (|m| <= flag band). */
void orc_check_edges(const orc_robot *R, const orc_prim *prims, int32_t n_prims,
                     const float *a, const float *b, int64_t n_edges, float res,
                     uint8_t *valid, uint8_t *flagged, double *m_out, int32_t early_exit,
                     int32_t n_threads);

/* Nearest neighbour over tree[dof][cap] (nodes 0..size-1), FP32 contract. */
int32_t orc_nearest(const float *tree, int32_t cap, int32_t size, const uint8_t *blocked,
                    const float *x, int32_t dof);
/* Steer: at most delta from `from` toward `to` (FP32 contract). */
void orc_steer(const float *from, const float *to, int32_t dof, float delta, float *out);

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_sample_config(uint64_t seed, uint32_t query, uint32_t round, uint32_t worker,
                       const float *lo, const float *hi, int32_t dof, float *out);
/* Sample number `attempt` of a worker in a round (attempt 0 = the above). */
void orc_sample_config_try(uint64_t seed, uint32_t query, uint32_t round, uint32_t worker,
                           uint32_t attempt, const float *lo, const float *hi, int32_t dof, float *out);

int32_t orc_plan(const orc_robot *R, const orc_prim *prims, int32_t n_prims, const float *start,
                 const float *goal, const orc_plan_params *p, float *path, int32_t path_cap,
                 int32_t *path_len, orc_plan_stats *st, int32_t n_threads);

/* Final state of both trees, for tests of the round structure: node k of a
 * tree is nodes[k * dof .. k * dof + dof - 1], its parent parent[k] (-1 for
 * the root); every array holds tree_capacity entries.  Sizes are the stats'
 * nodes_a / nodes_b.  Any pointer may be NULL. */
typedef struct {
    float *nodes_a, *nodes_b;
    int32_t *parent_a, *parent_b;
    uint8_t *blocked_a, *blocked_b;
} orc_tree_dump;

/* orc_plan, also writing the final trees into *dump (when not NULL). */
int32_t orc_plan_dump(const orc_robot *R, const orc_prim *prims, int32_t n_prims, const float *start,
                      const float *goal, const orc_plan_params *p, float *path, int32_t path_cap,
                      int32_t *path_len, orc_plan_stats *st, int32_t n_threads, orc_tree_dump *dump);

/* Re-check a path's segments (points i = 0..n at resolution res).  Returns
 * the minimum clearance over all segments; *n_flag counts segments within
 * the flag band. */
double orc_path_clearance(const orc_robot *R, const orc_prim *prims, int32_t n_prims,
                          const float *path, int32_t len, float res, int32_t *n_flag);

#ifdef __cplusplus
}
#endif
#endif
