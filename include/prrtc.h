/*
 * prrtc.h -- C ABI of the MI355X (gfx950) pRRTC hot-path library, libprrtc.so.
 *
 * pRRTC (Huang, Jadhav, Plancher, Kingston; arXiv 2503.06757) is RRT-Connect
 * with many sample-extend-connect iterations running at once on two shared
 * trees (Alg. 1), every candidate edge validated by checking all of its
 * discretised configurations at once (Alg. 2, Sec. III-A): forward kinematics
 * of the robot's collision spheres, then sphere tests against primitive
 * obstacles and between the robot's own spheres.
 *
 * Conventions shared by every call
 *   - Every call returns a prrtc_status; no C++ exception crosses the ABI.
 *     Argument errors are detected on the host before any GPU work; the
 *     reason is readable through prrtc_last_error() until the next call on
 *     the same context.
 *   - A context owns every device table it creates.  One context per host
 *     thread; calls on one context are not thread-safe.
 *   - Descriptor memory passed in is copied; the caller may free it when the
 *     call returns.
 *   - Pointers documented as "device" are HIP device pointers on the
 *     context's device; "host" pointers are ordinary host memory.
 *   - Angles in radians, lengths in metres, all floating point is IEEE FP32.
 */
#ifndef PRRTC_H
#define PRRTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PRRTC_OK = 0,
    PRRTC_E_ARG = -1,              /* invalid argument (detail in prrtc_last_error) */
    PRRTC_E_STATE = -2,            /* unknown robot/scene id, or context unusable */
    PRRTC_E_CAPACITY = -3,         /* output buffer too small; required size reported */
    PRRTC_E_INVALID_ENDPOINT = -4, /* start/goal outside the limits or in collision */
    PRRTC_E_NO_SOLUTION = -5,      /* round or time budget exhausted: a result, not a fault */
    PRRTC_E_BUSY = -6,             /* admission refused (resource budget full) */
    PRRTC_E_HIP = -7               /* a HIP runtime call failed */
} prrtc_status;

typedef struct prrtc_ctx prrtc_ctx;

#define PRRTC_MAX_DOF 16
#define PRRTC_MAX_CHAINS 2
#define PRRTC_MAX_SPHERES 256
#define PRRTC_MAX_PRIMS 1024
#define PRRTC_MAX_SELF_PAIRS 16384

/* Create a context on HIP device `device` (plan runs on the context's own
 * non-blocking stream; the asynchronous calls take the caller's stream, or
 * that stream when they are given NULL). */
prrtc_status prrtc_create(prrtc_ctx **out, int device);
/* Free every table and buffer of the context.  destroy(NULL) is a no-op. */
void prrtc_destroy(prrtc_ctx *ctx);
/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char *prrtc_last_error(const prrtc_ctx *ctx);

/*
 * Robot: one or two serial chains of revolute joints with collision spheres
 * (Sec. III-A represents the robot by bounding spheres attached to its links).
 *
 * Joint j of a chain applies, in modified DH form,
 *     frame_{j+1} = frame_j * Rx(alpha_j) * Tx(a_j) * Rz(q_j) * Tz(d_j),
 * with frame_0 = the chain's base pose.  Global frame ids number chain 0's
 * frames 0..dof_0, then chain 1's dof_0+1 .. dof_0+1+dof_1.  The
 * configuration vector is chain 0's joints followed by chain 1's.
 */
typedef struct {
    int32_t n_chains;                          /* 1 or 2 */
    int32_t chain_dof[PRRTC_MAX_CHAINS];       /* joints per chain; total <= 16 */
    float base_pose[PRRTC_MAX_CHAINS][12];     /* row-major 3x4 [R | t], R orthonormal */
    const float *dh;                           /* host [dof][3] = (alpha, a, d) */
    const float *q_lo;                         /* host [dof] lower joint limit */
    const float *q_hi;                         /* host [dof] upper joint limit (> q_lo) */
    int32_t n_spheres;                         /* 1..256 */
    const int32_t *sphere_frame;               /* host [n_spheres] global frame id */
    const float *sphere_xyzr;                  /* host [n_spheres][4] centre in frame, radius > 0 */
    int32_t n_self_pairs;                      /* 0..16384 */
    const int32_t *self_pairs;                 /* host [n_self_pairs][2] sphere indices, i != j */
    /* Two-stage checks (Sec. III-A: a low-resolution pass over coarse spheres
     * flags the links that may collide; only their fine spheres are checked).
     * n_coarse = 0 (all three NULL): one stage.  Else sphere k lies inside
     * coarse sphere sphere_coarse[k], on the same frame (|p_k - c| + r_k <=
     * R, checked: E_ARG).  Verdicts do not change, only the work: the
     * planner always runs the two-stage pass for such a robot; check_edges
     * times it against one stage per (robot, scene) pair (schedules). */
    int32_t n_coarse;                          /* 0..256 */
    const int32_t *coarse_frame;               /* host [n_coarse] global frame id */
    const float *coarse_xyzr;                  /* host [n_coarse][4] centre in frame, radius */
    const int32_t *sphere_coarse;              /* host [n_spheres] coarse sphere of each sphere */
} prrtc_robot_desc;

/* Validate and copy a robot to the device.  E_ARG on non-finite values,
 * lo >= hi, frame ids or pair indices out of range, non-positive radii. */
prrtc_status prrtc_load_robot(prrtc_ctx *ctx, const prrtc_robot_desc *desc, int32_t *robot_id);

/*
 * Scene primitive, 64 bytes (Sec. III-A: environments as primitive shapes).
 *   type 0 sphere:   c = centre, dims[0] = radius
 *   type 1 cuboid:   c = centre, columns of rot = box axes, dims = half-extents
 *   type 2 cylinder: c = centre, column 2 of rot = axis, dims[0] = radius,
 *                    dims[1] = half-height (solid, flat caps)
 * rot is row-major and must be orthonormal to 1e-5 (not re-orthonormalised).
 */
typedef struct {
    int32_t type;
    float c[3];
    float rot[9];
    float dims[3];
} prrtc_prim;

/* Validate and copy n primitives (0 allowed: empty scene). */
prrtc_status prrtc_load_scene(prrtc_ctx *ctx, const prrtc_prim *prims, int32_t n,
                              int32_t *scene_id);

/* Release a scene's device memory (waits for all work on the device first).
 * Its id stays retired: later calls naming it return E_STATE. */
prrtc_status prrtc_unload_scene(prrtc_ctx *ctx, int32_t scene_id);

/*
 * ESDF grid (Sec. III-A: with maps built from camera data, the planner checks
 * the robot's spheres against a Euclidean signed distance field instead of
 * primitives).  Node (i, j, k) sits at origin + voxel (i, j, k) and holds the
 * signed distance values[(k dims[1] + j) dims[0] + i] (metres, negative
 * inside obstacles).  A sphere (centre c, radius r) collides iff E(c) < r, E
 * the trilinear interpolation of the node values at c, with c's grid
 * coordinates clamped to the grid's box (outside the box the field continues
 * as its value at the box's nearest point).  FP32 throughout.
 */
typedef struct {
    float origin[3];
    float voxel;             /* node spacing, > 0 */
    int32_t dims[3];         /* nodes along x, y, z: each 2..1024, at most 2^27 in all */
    const float *values;     /* host [dims[2]][dims[1]][dims[0]], no NaN */
} prrtc_esdf_desc;

/* Attach a copy of an ESDF grid to a scene (replacing any it had; desc NULL
 * detaches it).  The scene's primitives, if any, still count: a sphere
 * collides if it meets either.  Waits for the device; the scene's timed
 * check_edges schedules are timed again.  E_ARG on bad geometry or NaN. */
prrtc_status prrtc_scene_set_esdf(prrtc_ctx *ctx, int32_t scene_id, const prrtc_esdf_desc *desc);

/* Build a grid from a scene's primitives (standing in for a map from camera
 * data): values (device float32 [dims[2]][dims[1]][dims[0]]) = the signed
 * distance of each node to the union of the primitives (the least of their
 * signed distances; +inf for a scene without primitives), FP32.  Async on
 * stream.  An attached grid is not part of the union. */
prrtc_status prrtc_esdf_from_scene(prrtc_ctx *ctx, int32_t scene_id, const float origin[3], float voxel,
                                   const int32_t dims[3], float *values, void *stream);

/*
 * check_edges (Alg. 2 / Sec. III-A).  For edge e with endpoints a_e, b_e:
 *     L = |b_e - a_e| (FP32, squares summed in joint order, no fused
 *         multiply-add, correctly rounded sqrt),
 *     n = max(1, ceil(res * L)) (capped at 2^24),
 *     q_i = a_e + (i/n)(b_e - a_e), i = 0..n,
 * and valid[e] = 1 iff no q_i puts a robot sphere strictly inside an
 * obstacle or another robot sphere of a self-collision pair; else 0.
 *
 * a, b:   device float32 [n_edges][dof], row-major, finite.
 * valid:  device uint8 [n_edges], written.
 * res:    points per radian (> 0).
 * stream: hipStream_t to enqueue on (NULL = the context's own stream, a
 *         non-blocking stream that prrtc_plan also uses; hipDeviceSynchronize
 *         waits for it; the null stream itself is named hipStreamLegacy).
 *         The call is asynchronous; buffers must stay alive
 *         until the stream is synchronised.  n_edges = 0 is a no-op.  Launches on one context
 *         draw from a ring of 256 work counters, so at most 256 launches of
 *         one context may be in flight at once.
 *
 * Kernel schedules give the same verdicts at different speeds: 0 and 1
 * differ in items per lane and the order of the obstacle types; for a robot
 * with coarse spheres, 2 and 3 are the same with the two-stage pass (coarse
 * spheres gating the fine ones), 0 and 1 then ignoring the coarse spheres.
 * The first batch of at least 8192 edges on a (robot, scene) pair times every
 * schedule the robot has on its first 2^20 edges (all of a smaller batch) and
 * keeps the fastest for that pair; that one call waits for the stream.  Until
 * then a pair runs schedule 0 (2 with coarse spheres).
 */
prrtc_status prrtc_check_edges(prrtc_ctx *ctx, int32_t robot_id, int32_t scene_id,
                               const float *a, const float *b, int64_t n_edges, float res,
                               uint8_t *valid, void *stream);

/* The check_edges schedule of a (robot, scene) pair: set = 0 or 1 (2 or 3
 * for a robot with coarse spheres) pins that schedule, -1 forgets the choice
 * and its tuning record (the next large batch times every schedule again),
 * -2 changes nothing (a stored tuning record for the pair's key is taken
 * up).  *schedule (may be NULL) = the schedule in force after the call, -1
 * while none is chosen.  E_ARG for another set value. */
prrtc_status prrtc_edge_schedule(prrtc_ctx *ctx, int32_t robot_id, int32_t scene_id, int32_t set,
                                 int32_t *schedule);

/*
 * FK (Sec. III-A): world-frame sphere centres of every configuration, from
 * the same four-lanes-per-configuration FK the collision checks use.
 * q: device float32 [n][dof]; xyz: device float32 [n][n_spheres][3], in the
 * robot descriptor's sphere order.  Asynchronous on `stream`.
 */
prrtc_status prrtc_fk_spheres(prrtc_ctx *ctx, int32_t robot_id, const float *q, int64_t n,
                              float *xyz, void *stream);

/*
 * plan (Alg. 1): parallel RRT-Connect from start to goal.
 *
 * Rounds r = 0..max_rounds-1 run on the GPU inside one persistent launch.
 * In each round every worker w sees the same snapshot of both trees, grows
 * the smaller one (tie: start tree): RANDOM_CONFIG from Philox4x32-10
 * (key = seed, counter = (draw, w, r, query)), nearest neighbour (exact
 * argmin, ties to the lowest node index), steer by at most delta, edge check
 * at points i = 1..n, then greedy connect toward the nearest node of the
 * other tree in ceil(L/delta) equal steps.  Staged nodes are appended in
 * worker order, so a given seed gives the same trees and path on every run.
 * The lowest-numbered connected worker yields the path, which is re-checked
 * at validate_factor * res (i = 0..n); on failure its offending node is
 * excluded and rounds continue.
 */
typedef struct {
    uint64_t seed;
    uint32_t query;          /* counter word; 0 for a single query */
    int32_t workers;         /* parallel workers W (default 256) */
    float delta;             /* extension range (default 0.5 rad) */
    float res;               /* edge resolution, points per radian (default 32) */
    int32_t max_rounds;      /* >= 0 */
    int32_t tree_capacity;   /* nodes per tree, >= 2 */
    float time_budget_ms;    /* <= 0: none.  Checked between rounds on the GPU clock */
    int32_t validate_factor; /* 0 disables the final re-check (default 4) */
    float dds_radius;        /* dynamic-domain sampling (Sec. III, after Yershova et
                                al.): a failed extension sets its start node's
                                sampling radius to this; 0 (default) turns it off */
    int32_t dds_tries;       /* samples a worker draws per round until one lies
                                within its nearest node's radius (1..64, default 1) */
    int32_t sampler;         /* 0: uniform Philox draws (default); 1: learned proposal,
                                see below; 2: Halton points (the sampler of the paper's
                                experiments, Sec. IV-A): point i = (low word of seed) +
                                65536 query + (round W + worker) dds_tries + try + 1
                                (mod 2^32), joint j the radical inverse of i in the j-th
                                prime base (2, 3, 5, ..., 53) as the exact rational
                                rounded to FP64 then FP32, q_j = fmaf(u, hi_j - lo_j, lo_j) */
    int32_t model_id;        /* proposal model for sampler 1; its dof must match */
    float mix;               /* sampler 1: probability that a draw comes from the
                                mixture (0..1, default 0.5); 0 gives the uniform plan */
    int32_t tile;            /* configurations per FK tile of the collision checks:
                                64 (0 = default; lowest latency per query) or 16
                                (a quarter of the LDS: more groups per batched
                                launch); a single plan of tile 64 runs workers
                                of eight waves when all of them can be resident,
                                else of four; results do not depend on it */
} prrtc_plan_params;

typedef struct {
    int32_t rounds;
    int32_t nodes_a, nodes_b;
    int64_t edges_checked;
    int32_t validation_failures;
    int32_t connect_worker;
    float gpu_ms;            /* device time of the launch(es), proposal inference included */
    int32_t fallback;        /* 1: the proposal's mixture was not finite; uniform draws only */
    int32_t pad;
    int64_t learned_samples; /* draws taken from the mixture */
} prrtc_plan_stats;

/* Fill *p with the defaults above (seed 1, 256 workers, 0.5 rad, 32/rad,
 * 1000 rounds, 65536 nodes, no time budget, factor 4, no dynamic domain,
 * uniform sampler, model -1, mix 0.5). */
void prrtc_plan_params_default(prrtc_plan_params *p);

/*
 * start, goal: host float32 [dof].  path: host float32 [path_cap][dof].
 * Synchronous.  Returns OK with *path_len nodes written (path[0] == start,
 * path[len-1] == goal bit for bit; every segment no longer than delta);
 * E_CAPACITY if path_cap is too small (then *path_len = nodes needed and
 * nothing is written: call again with a larger buffer), or, before any work,
 * if params->workers workgroups of the chosen tile cannot all be resident on
 * the device at once (*path_len = 0);
 * E_INVALID_ENDPOINT, E_NO_SOLUTION as documented above.  stats may be NULL.
 */
prrtc_status prrtc_plan(prrtc_ctx *ctx, int32_t robot_id, int32_t scene_id, const float *start,
                        const float *goal, const prrtc_plan_params *params, float *path,
                        int32_t path_cap, int32_t *path_len, prrtc_plan_stats *stats);

/*
 * Batched planning: many independent queries in one persistent launch (the
 * paper's high-level parallelism, one query per group of workers instead of
 * one query per launch).  The launch holds G groups of params->workers
 * workgroups; group g runs queries g, g + G, g + 2G, ... one after another,
 * each exactly as prrtc_plan would with the same parameters, seed and query
 * word (identical trees, path and statistics).  Queries may mix robots and
 * scenes; all share *params (its seed and query fields are ignored).  With
 * sampler 1 each query uses its own model_id (or params->model_id) and the
 * group that runs it computes its mixture from the scene's occupancy-grid
 * embedding, with the arithmetic of prrtc_plan's, so learned queries also
 * plan exactly as prrtc_plan would.
 *
 * groups: G, or 0 for as many as are resident at once (capped at n).  More
 *   than fit on the device at once is E_CAPACITY.
 * memory_budget: bytes of device memory the launch may use for trees and
 *   per-query buffers (0: no limit); G shrinks to fit (admission by tree
 *   memory), E_CAPACITY if not even one group fits.
 * paths: host float32 [n][path_cap][PRRTC_MAX_DOF]; query k's path is the
 *   row-major [path_len][dof] block at paths + k path_cap PRRTC_MAX_DOF.
 * results: host [n]; status per query (OK, E_CAPACITY with path_len = nodes
 *   needed, E_INVALID_ENDPOINT, E_NO_SOLUTION, E_STATE/E_ARG for a query
 *   rejected on the host (not launched), E_HIP if its group aborted);
 *   stats.gpu_ms is the whole launch.
 * groups_used: may be NULL.  Synchronous.  The return value is OK when the
 * launch ran, whatever the queries' outcomes.
 */
typedef struct {
    int32_t robot_id, scene_id;
    float start[PRRTC_MAX_DOF], goal[PRRTC_MAX_DOF];
    uint64_t seed;
    uint32_t query;
    int32_t model_id;        /* sampler 1: this query's proposal model (its dof must
                                match the robot's); -1 = params->model_id */
} prrtc_query;

typedef struct {
    int32_t status;
    int32_t path_len;
    prrtc_plan_stats stats;
} prrtc_query_result;

prrtc_status prrtc_plan_batch(prrtc_ctx *ctx, const prrtc_query *queries, int32_t n,
                              const prrtc_plan_params *params, int32_t groups, int64_t memory_budget,
                              float *paths, int32_t path_cap, prrtc_query_result *results,
                              int32_t *groups_used);

/*
 * Launch-shape tuning for batched planning: the queries are planned once per
 * (worker count, tile) pair (each pass a complete prrtc_plan_batch with the
 * largest resident group count and memory_budget), timed on the host clock.
 * rates (may be NULL): host float [n_workers][n_tiles], queries per second
 * of each pair (0 if it cannot launch).  *best_workers, *best_tile = the
 * fastest pair.  Synchronous; E_CAPACITY if no pair can launch.
 */
prrtc_status prrtc_tune_launch(prrtc_ctx *ctx, const prrtc_query *queries, int32_t n,
                               const prrtc_plan_params *params, const int32_t *workers, int32_t n_workers,
                               const int32_t *tiles, int32_t n_tiles, int64_t memory_budget, float *rates,
                               int32_t *best_workers, int32_t *best_tile);

/*
 * Tuning records (kept across processes).  The library records what it
 * timed: each check_edges schedule it chose, keyed by the device
 * architecture and the robot's and scene's shape (DoF, moving spheres,
 * coarse spheres or not, self pairs, and primitive counts by type, counts in
 * power-of-two buckets, ESDF or not), and each prrtc_tune_launch result,
 * keyed by the device, the queries' DoF set, the largest obstacle count's
 * bucket and the candidate lists.  A (robot, scene) pair whose key has a
 * record takes its schedule without timing.
 *
 * prrtc_tuned_launch: the stored result of prrtc_tune_launch for these
 *   queries and candidates (E_STATE if none).
 * prrtc_tuning_save: write every record to a text file (one "key | value"
 *   line each).  prrtc_tuning_load: add a file's records (later ones win).
 *   E_ARG if the file cannot be written / read or a line is malformed.
 */
prrtc_status prrtc_tuned_launch(prrtc_ctx *ctx, const prrtc_query *queries, int32_t n, const int32_t *workers,
                                int32_t n_workers, const int32_t *tiles, int32_t n_tiles, int32_t *best_workers,
                                int32_t *best_tile);
prrtc_status prrtc_tuning_save(prrtc_ctx *ctx, const char *path);
prrtc_status prrtc_tuning_load(prrtc_ctx *ctx, const char *path);

/*
 * Serving: a thread owned by the context plans submitted queries as they
 * arrive.  It keeps one persistent launch running: queries are published
 * into a ring of 64 x slots entries (32 to 16384, and within about 256 MiB
 * of pinned host memory for the entries' arguments and paths) that the
 * launch's worker groups take from while it runs (at most `slots` in
 * flight), and each result returns as soon as its query ends.  The launch
 * closes once no query has been claimed for 50 ms (every group leaves at its
 * next claim) and is started again by the next submission; a used-up ring
 * drains the launch and the next one starts on the reset ring.  Group
 * buffers are sized for the largest robot loaded when serving starts
 * (robots cannot be loaded while serving).  With the learned sampler
 * (params->sampler 1) each group computes its query's mixture inside the
 * launch from tables of every (scene, model) pair loaded when serving
 * starts.  Groups
 * are sized by memory_budget as in prrtc_plan_batch.  Results equal those
 * of prrtc_plan / prrtc_plan_batch for the same query, seed and parameters.
 * While serving, the context accepts only prrtc_submit, prrtc_poll,
 * prrtc_serve_stop and prrtc_last_error (everything else: E_STATE).  The
 * serving thread never writes the message prrtc_last_error returns: served
 * queries report their outcome through their result status only.
 *
 * prrtc_serve_start: params as for prrtc_plan_batch; slots >= 1;
 *   max_pending >= slots bounds the queries admitted and not yet polled;
 *   path_cap >= 1 nodes kept per query.  E_STATE if no robot is loaded; E_CAPACITY if one worker group does not fit;
 *   E_HIP if the ring buffers (pinned host and device memory) cannot be
 *   allocated.  A query rejected by the host checks (unknown ids, endpoints
 *   outside the limits) comes back through prrtc_poll with that status;
 *   one whose worker group aborted comes back as E_HIP.
 * prrtc_submit: copies *query and returns a ticket; E_BUSY (admission
 *   refused) when max_pending queries are queued, running or unpolled.
 * prrtc_poll: E_BUSY while the ticket is queued or running; OK with *result
 *   (its status is the query's outcome) and, for a solved query, the path in
 *   path (host float32 [path_cap][dof]) once done — the ticket is then
 *   released; E_CAPACITY if path_cap < result->path_len (ticket kept);
 *   E_STATE for an unknown or released ticket.
 * prrtc_serve_stop: plans everything still queued, joins the thread, drops
 *   unpolled results; *launches (may be NULL) = launches made.
 */
prrtc_status prrtc_serve_start(prrtc_ctx *ctx, const prrtc_plan_params *params, int32_t slots,
                               int32_t max_pending, int64_t memory_budget, int32_t path_cap);
prrtc_status prrtc_submit(prrtc_ctx *ctx, const prrtc_query *query, uint64_t *ticket);
prrtc_status prrtc_poll(prrtc_ctx *ctx, uint64_t ticket, prrtc_query_result *result, float *path,
                        int32_t path_cap);
prrtc_status prrtc_serve_stop(prrtc_ctx *ctx, int64_t *launches);

/*
 * Learned sampling proposal (not in the paper, which samples uniformly; an
 * addition whose definition follows).  A 16^3 occupancy grid of the scene
 * (cells of 0.1 m over [-0.8, 0.8]^3; a cell is occupied iff an obstacle lies
 * closer than its half diagonal to its centre) is embedded linearly to 256
 * values; with the start and goal scaled to [-1, 1] by the joint limits it
 * feeds three Linear(256) + GELU layers and a head giving an 8-component
 * diagonal Gaussian mixture over scaled configurations: per sample
 * [8 logits | 8 x dof means | 8 x dof log sigmas clamped to [-5, 2]].
 * Every matrix product rounds its operands to bfloat16 (nearest even) and
 * accumulates in FP32 on the matrix cores.
 *
 * Blob layout (little endian): header {uint32 magic 0x31505250 "PRP1",
 * uint32 version 1, int32 dof, int32 hidden 256, int32 components 8,
 * int32 voxels per side 16, int64 adam steps, int32 has_adam, int32 pad},
 * then the FP32 parameters W_v [4096][256], b_v, W_1 [2 dof + 256][256], b_1,
 * W_2 [256][256], b_2, W_3, b_3, W_4 [256][8 (1 + 2 dof)], b_4 (weights
 * [in][out] row-major), then, if has_adam, Adam's first and second moments
 * in the same layout.
 */
/* Copy a proposal to the device.  Non-finite weights are accepted (plans
 * with such a model fall back to uniform sampling). */
prrtc_status prrtc_load_proposal(prrtc_ctx *ctx, const void *blob, size_t bytes, int32_t *model_id);
/* Write the model (with Adam state) to blob.  E_CAPACITY if cap is too small;
 * *bytes is always set to the size needed.  Synchronises the device. */
prrtc_status prrtc_save_proposal(prrtc_ctx *ctx, int32_t model_id, void *blob, size_t cap, size_t *bytes);
/* Occupancy grid of a scene: vox = device uint8 [4096], x fastest.  Async. */
prrtc_status prrtc_voxelize(prrtc_ctx *ctx, int32_t scene_id, uint8_t *vox, void *stream);
/* Mixture parameters for n (start, goal) pairs: vox device uint8 [n_scenes][4096],
 * scene_of device int32 [n] (row of vox per sample), start/goal device float32
 * [n][dof] in joint units (scaled with robot_id's limits), gmm device float32
 * [n][8 (1 + 2 dof)].  Async on stream. */
prrtc_status prrtc_proposal_forward(prrtc_ctx *ctx, int32_t model_id, int32_t robot_id, const uint8_t *vox,
                                    int32_t n_scenes, const int32_t *scene_of, const float *start,
                                    const float *goal, int32_t n, float *gmm, void *stream);

/*
 * prrtc_proposal_forward for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, kernels and results, but the activations live
 * in a fixed device array of about 3.3 MiB that each GPU the library runs on
 * holds until the process ends.  No allocation, no synchronisation.
 * Limits: n <= 256 samples and n_scenes <= 256 scenes, else E_ARG (before
 * any work).  Every call on one device shares that array: calls that overlap
 * on one GPU (other streams, other contexts or threads) race and must be
 * serialised by the caller.  Nothing in the array needs clearing between
 * calls.
 */
prrtc_status prrtc_proposal_forward_noalloc(prrtc_ctx *ctx, int32_t model_id, int32_t robot_id,
                                            const uint8_t *vox, int32_t n_scenes, const int32_t *scene_of,
                                            const float *start, const float *goal, int32_t n, float *gmm,
                                            void *stream);

/* One training step on a batch whose samples are grouped by scene: samples
 * scene_start[s] .. scene_start[s+1]-1 belong to scene s (scene_of repeats
 * that mapping per sample).  All pointers are device memory; waypoint is the
 * target configuration (joint units). */
typedef struct {
    const uint8_t *vox;         /* [n_scenes][4096] */
    int32_t n_scenes;
    const int32_t *scene_start; /* [n_scenes + 1] */
    const int32_t *scene_of;    /* [n] */
    const float *start, *goal, *waypoint; /* [n][dof] */
    int32_t n;
} prrtc_train_batch;

/*
 * Drawing from a mixture (the planner's learned RANDOM_CONFIG).  All
 * uniforms are Philox4x32-10 words (key = seed) with counter
 * (c0, worker, round, query), c0 = 0x80000000 | attempt << 8 | slot, a
 * range the uniform sampler never uses; u(x) = (x >> 8) 2^-24.  Slot 255:
 * word 0 decides mixture vs uniform (u < mix, taken at attempt 4t for the
 * t-th draw of a round) and word 1 picks the component by inverse CDF of
 * softmax(logits); slot 1 + j/2 gives Box-Muller normals for joints j, j+1
 * (u1 = ((x >> 8) + 1) 2^-24, u2 = u(y); z = sqrt(-2 ln u1) cos or sin
 * (2 pi u2) for even or odd j).  Scaled draw x = mu + exp(log sigma) z,
 * q = lo + (x + 1)(hi - lo) / 2.  The planner tries attempts 4t..4t+3 and
 * keeps the first draw inside the joint limits, else draws uniformly.
 *
 * Test hook: n draws of one (query, round, attempt), draw i as worker i.
 * gmm: device float32 [8 (1 + 2 dof)] (one row of prrtc_proposal_forward's
 * output); q: device float32 [n][dof]; inside: device uint8 [n], 1 iff the
 * draw lies inside the limits.  attempt < 2^23.  Async on stream.
 */
prrtc_status prrtc_proposal_sample(prrtc_ctx *ctx, int32_t robot_id, const float *gmm, uint64_t seed,
                                   uint32_t query, uint32_t round, uint32_t attempt, int32_t n, float *q,
                                   uint8_t *inside, void *stream);

/* Forward, backward of the batch-mean negative log-likelihood and one Adam
 * step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr.  loss:
 * device float32 [1], the batch-mean NLL before the step.  Async; one model
 * must not be trained on two streams at once. */
prrtc_status prrtc_train_proposal(prrtc_ctx *ctx, int32_t model_id, int32_t robot_id,
                                  const prrtc_train_batch *batch, float lr, float *loss, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PRRTC_H */
