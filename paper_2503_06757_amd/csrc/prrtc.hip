// prrtc.hip -- libprrtc.so: C ABI, resident robot/scene tables and kernel launches.
//
// The entry points are declared (with their contracts) in include/prrtc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <fstream>
#include <map>
#include <sstream>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "prrtc.h"
#include "prrtc_device.h"
#include "prrtc_planner.h"
#include "prrtc_proposal.h"

using namespace prrtc;

// ----------------------------------------------------------------------------
// Kernels
// ----------------------------------------------------------------------------

// check_edges: one wavefront per workgroup.  Collision-free edges cost far
// more than colliding ones, so large batches are handed out dynamically: the
// batch is split into one contiguous range per XCD (workgroup ids are dealt
// to the 8 XCDs round-robin) and each wave takes chunks of `chunk` edges from
// its XCD's counter, keeping the atomics off a single shared address; the
// last wave to finish resets the counters for the next launch.  Batches of
// at most kEdgeStatic edges per resident wave take chunk = 0: wave b checks
// edges b, b + grid, b + 2 grid, ... with no atomics at all (there, the
// counters' serialised atomics, thousands per address, cost more than the
// imbalance: 4096 edges 122 -> 36 us, 131072 edges 305 -> 249 us).  The next
// edge's endpoints are fetched while the current edge is checked.
#ifndef PRRTC_EDGE_CHUNK
#define PRRTC_EDGE_CHUNK 8
#endif
#ifndef PRRTC_EDGE_WAVES
#define PRRTC_EDGE_WAVES 6
#endif
#ifndef PRRTC_EDGE_STATIC
#define PRRTC_EDGE_STATIC 48
#endif
constexpr int kEdgeChunk = PRRTC_EDGE_CHUNK;
constexpr long long kEdgeStatic = PRRTC_EDGE_STATIC;
constexpr int kXcds = 8;

struct EdgeCounter {
    unsigned long long next[kXcds * 8];  // one 64-byte line per XCD
    unsigned int done;
    unsigned int pad[15];
};

// Waves per SIMD: the one-stage kernels are held to 80 VGPRs, which keeps 6
// waves resident per SIMD instead of 5 with no spills (the wait for LDS and
// scalar loads in the obstacle loop is hidden better: 6% faster on the
// 7-DoF arm among 64 obstacles); the two-stage kernels would spill there.
template <int TP, int B, bool BOX_FIRST, bool TWO>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(TWO ? 1 : PRRTC_EDGE_WAVES)))
void k_check_edges(RobotArgs R, SceneArgs S,
                                                       const float* __restrict__ A,
                                                       const float* __restrict__ Bv,
                                                       long long n_edges, float res,
                                                       uint8_t* __restrict__ valid,
                                                       EdgeCounter* ctr, int chunk) {
    extern __shared__ float4 lds4[];
    const int lane = threadIdx.x;
    const int dof = R.dof;
    float4* sph = lds4;
    int* slot3 = reinterpret_cast<int*>(sph + R.n_move);
    WaveWs ws;
    ws.frames = reinterpret_cast<float4*>(slot3 + ((R.n_move + 3) & ~3));
    ws.sph = sph;
    ws.slot3 = slot3;
    float* wp = reinterpret_cast<float*>(ws.frames + TP * 3 * R.n_slots);
    ws.pk = reinterpret_cast<int*>(wp + 2 * kMaxDof);
    ws.sub_n = ws.pk + TP;
    ws.sub_off = ws.sub_n + 2;
    int* chunk_n = ws.sub_off + 2;   // point counts of the current chunk's edges
    two_stage_ws(R, TP, chunk_n + kEdgeChunk, ws);
    ws.shared = nullptr;   // single-wave checks share nothing
    stage_spheres(R, sph, slot3);
    load_bounds(S, ws);
    const bool fixed_hit = static_collision(R, S);
    __syncthreads();
    const bool dyn = chunk > 0;
    const int xcd = blockIdx.x % kXcds;
    const long long lo = dyn ? n_edges * xcd / kXcds : 0;
    const long long end = dyn ? n_edges * (xcd + 1) / kXcds : n_edges;
    const long long step = dyn ? chunk : 1;
    unsigned long long* my_ctr = &ctr->next[xcd * 8];
    long long cursor = blockIdx.x;
    auto grab = [&]() -> long long {
        if (dyn) {
            unsigned long long v = 0;
            if (lane == 0) v = atomicAdd(my_ctr, (unsigned long long)chunk);
            return lo + (long long)__shfl(v, 0, kWave);
        }
        const long long v = cursor;
        cursor += gridDim.x;
        return v;
    };
    long long c0 = grab();
    float ra = 0.0f, rb = 0.0f;
    if (c0 < end && lane < dof) {
        ra = A[c0 * dof + lane];
        rb = Bv[c0 * dof + lane];
    }
    while (c0 < end) {
        const long long c1 = grab();
        const long long cend = min(c0 + step, end);
        // the chunk's point counts, one edge per lane (lane l: edge c0 + l),
        // instead of the whole wave computing each edge's count in turn
        if (lane < cend - c0) chunk_n[lane] = edge_count_f32(A + (c0 + lane) * dof, Bv + (c0 + lane) * dof, dof, res);
        for (long long e = c0; e < cend; ++e) {
            if (lane < dof) {
                wp[lane] = ra;
                wp[dof + lane] = rb;
            }
            // prefetch the next edge (next in this chunk, else the next chunk's first)
            const long long nx = e + 1 < cend ? e + 1 : c1;
            if (nx < end && lane < dof) {
                ra = A[nx * dof + lane];
                rb = Bv[nx * dof + lane];
            }
            __syncthreads();
            const int n_e = chunk_n[e - c0];
            const int ok =
                fixed_hit ? 0 : (wave_check<TP, B, false, 1, BOX_FIRST, TWO>(R, S, wp, 1, 0, res, ws, 0, 1, n_e) == 1);
            if (lane == 0) valid[e] = (uint8_t)ok;
            __syncthreads();
        }
        c0 = c1;
    }
    if (dyn && lane == 0) {
        __threadfence();
        if (atomicAdd(&ctr->done, 1u) == gridDim.x - 1) {
            for (int x = 0; x < kXcds; ++x) atomicExch(&ctr->next[x * 8], 0ull);
            atomicExch(&ctr->done, 0u);
        }
    }
}

// FK entry point: the collision kernels' four-lanes-per-configuration FK
// (16 configurations per wave, every frame staged in LDS), then one lane per
// (configuration, sphere).
constexpr int kFkPerBlock = kWave / 4;

__global__ __launch_bounds__(kWave) void k_fk_spheres(RobotArgs R, const float* __restrict__ q,
                                                      long long n, float* __restrict__ xyz) {
    extern __shared__ float4 lds4[];
    const int lane = threadIdx.x;
    const long long c0 = (long long)blockIdx.x * kFkPerBlock;
    const int slot = lane >> 2;
    if (c0 + slot < n) {   // whole quads
        const float* qc = q + (c0 + slot) * R.dof;
        fk_rows<true>(R, [&](int j) { return qc[j]; }, lds4 + slot * 3 * R.n_frames, lane & 3);
    }
    __syncthreads();
    const int ns = R.n_move + R.n_static;
    const int m = (int)min((long long)kFkPerBlock, n - c0);
    for (int it = lane; it < m * ns; it += kWave) {
        const int p = it / ns, s = it - p * ns;
        const float4 loc = R.sph[s];
        const float3 c = frame_apply(lds4 + p * 3 * R.n_frames + 3 * R.sph_frame[s], loc.x, loc.y, loc.z);
        float* o = xyz + ((c0 + p) * ns + R.desc_index[s]) * 3;
        o[0] = c.x;
        o[1] = c.y;
        o[2] = c.z;
    }
}

// ESDF grid of a scene's primitives: each node's signed distance to their
// union (the least signed distance; +inf with none), one thread per node.
__global__ void k_esdf_build(SceneArgs S, float ox, float oy, float oz, float h, int nx, int ny, int nz,
                             float* __restrict__ out) {
    const long long at = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (at >= (long long)nx * ny * nz) return;
    const int i = (int)(at % nx), j = (int)((at / nx) % ny), k = (int)(at / ((long long)nx * ny));
    const float x = fmaf(h, (float)i, ox), y = fmaf(h, (float)j, oy), z = fmaf(h, (float)k, oz);
    float m = __builtin_inff();
    for (int o = 0; o < S.n_sph; ++o) m = fminf(m, sd_sphere(x, y, z, ld_sph(S, o)));
    for (int o = 0; o < S.n_box; ++o) m = fminf(m, sd_box(x, y, z, ld_box(S, o)));
    for (int o = 0; o < S.n_cyl; ++o) m = fminf(m, sd_cyl(x, y, z, ld_cyl(S, o)));
    out[at] = m;
}

// ----------------------------------------------------------------------------
// Host side
// ----------------------------------------------------------------------------
namespace {

struct RobotRec {
    RobotArgs args{};
    RobotArgs* dev_args = nullptr;  // copy of args in device memory
    void* mem = nullptr;
    int dof = 0, n_spheres = 0;
};

struct SceneRec {
    SceneArgs args{};
    SceneArgs* dev_args = nullptr;  // copy of args in device memory
    void* mem = nullptr;
    uint8_t* vox = nullptr;         // occupancy grid, made by the first learned plan
    float* emb = nullptr;           // [kHidden] the grid's embedding under the model stamped emb_stamp
    uint64_t emb_stamp = 0;
    std::unordered_map<int, int> edge_schedule;   // robot id -> timed check_edges schedule
    int n = 0;
    void* esdf_mem = nullptr;       // node values of an attached ESDF grid
};

}  // namespace

namespace {

constexpr uint32_t kPropMagic = 0x31505250u;  // "PRP1"
constexpr uint32_t kPropVersion = 1;

struct PropHeader {
    uint32_t magic, version;
    int32_t dof, hidden, n_comp, vox;
    int64_t adam_t;
    int32_t has_adam, pad;
};

enum { pWv, pbv, pW1, pb1, pW2, pb2, pW3, pb3, pW4, pb4, pCount };

struct PropLayout {
    size_t off[pCount + 1];
    int dof, D0, Cw;
};

PropLayout prop_layout(int dof) {
    PropLayout L{};
    L.dof = dof;
    L.D0 = 2 * dof + kHidden;
    L.Cw = kComp * (1 + 2 * dof);
    const size_t sz[pCount] = {(size_t)kVoxCells * kHidden, kHidden, (size_t)L.D0 * kHidden, kHidden,
                               (size_t)kHidden * kHidden, kHidden, (size_t)kHidden * kHidden, kHidden,
                               (size_t)kHidden * L.Cw, (size_t)L.Cw};
    L.off[0] = 0;
    for (int i = 0; i < pCount; ++i) L.off[i + 1] = L.off[i] + sz[i];
    return L;
}

}  // namespace

struct ModelRec {
    PropLayout L{};
    float* mem = nullptr;      // params | grads | adam m | adam v, each L.off[pCount] floats
    long long adam_t = 0;
    uint64_t stamp = 0;        // changes whenever the parameters change (context-wide counter)
    void* ws = nullptr;        // activation workspace
    size_t ws_bytes = 0;
    size_t n() const { return L.off[pCount]; }
    float* p(int i) { return mem + L.off[i]; }
    float* g(int i) { return mem + n() + L.off[i]; }
};


// Offsets of a learned launch's tables from one base (see learned_tables).
struct LearnedLayout {
    size_t mdev = 0, emb = 0, vox = 0, part = 0, end = 0;
    int n_scenes = 0, n_models = 0;
    // query (scene row si, model row mi): its embedding
    size_t emb_at(int si, int mi) const { return emb + sizeof(float) * kHidden * ((size_t)mi * n_scenes + si); }
};

// Device buffers of one worker group (reused by every query the group runs).
struct GroupLayout {
    size_t qa, pa, ba, ra, qb, pb, bb, rb, bar, stage, st, path, path_idx, bytes;
};

// Serving state of a context (see prrtc_serve_start).
struct ServeDone {
    prrtc_query_result res;
    std::vector<float> path;   // [path_len][dof]
};

struct Server {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    prrtc_plan_params params{};
    int slots = 0, max_pending = 0, path_cap = 0;
    int64_t budget = 0;
    uint64_t next_ticket = 1;
    std::deque<std::pair<uint64_t, prrtc_query>> queue;
    std::unordered_map<uint64_t, int> running;
    std::unordered_map<uint64_t, ServeDone> done;
    long long launches = 0;
    size_t in_flight() const { return queue.size() + running.size() + done.size(); }
    // persistent mode: one long launch takes queries as they are published
    // into a ring (see k_serve)
    bool persistent = false;
    int ring = 0, path_stride = 0, groups = 0, W = 0;
    size_t lds = 0;
    const void* kernel = nullptr;
    void* host_mem = nullptr;        // pinned: args ring | result words | paths | control words
    PlanArgs* host_args = nullptr;
    int* host_ctl = nullptr;
    float* host_path = nullptr;
    int* host_ctrl = nullptr;        // [0] published, [32] drain
    void* dev_mem = nullptr;         // groups | args ring | words | paths | counter | ServeArgs
    char* dev_groups = nullptr;
    ServeArgs* dev_sa = nullptr;
    ServeArgs sa{};
    GroupLayout L{};
    int tree_cap = 0;
    // learned sampling: every loaded (scene, model) pair's grid embedding, made
    // when serving starts (nothing can be loaded while serving)
    LearnedLayout LL{};
    std::vector<int> scene_row;      // scene id -> row of the tables (-1: not loaded)
    float* dev_gmm = nullptr;        // [ring][kComp (1 + 2 kMaxDof)] the queries' mixtures
    char* ring_base = nullptr;       // device: what the ring's and tables' offsets count from
};

struct prrtc_ctx {
    int device = 0;
    int n_cu = 256;
    double wall_khz = 100000.0;  // GPU wall-clock ticks per millisecond
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<RobotRec> robots;
    std::vector<SceneRec> scenes;
    PlannerBuffers plan;               // single-query launches
    PlannerBuffers batch;              // batched launches
    std::vector<float> stage_host;     // host staging of batched proposal inputs
    std::vector<ModelRec> models;
    uint64_t model_stamp = 0;         // last stamp given to a model's parameters
    EdgeCounter* counters = nullptr;  // kCounterSlots self-resetting work counters
    unsigned counter_next = 0;
    std::unordered_map<uint64_t, int> plan_per_cu;   // resident planner workgroups per CU by (waves, tile, LDS bytes)
    std::string arch;                  // device architecture name (gcnArchName), part of the tuning keys
    std::map<std::string, std::string> tuning;   // tuning records: key -> value (see prrtc_tuning_save)
    int edge_grid[4] = {0, 0, 0, 0};   // resident workgroups of each k_check_edges kernel (cached)
    size_t edge_grid_lds[4] = {0, 0, 0, 0};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float* pinned = nullptr;           // kPinnedFloats of pinned host staging
    float* scratch = nullptr;          // this device's address of the static scratch array
    std::unique_ptr<struct Server> server;
    std::atomic<bool> serving{false};  // while set, only submit/poll/serve_stop are accepted
    std::atomic<std::thread::id> serve_tid{};   // the serving thread: it never writes err
};

constexpr int kPinnedFloats = 1024;

namespace {
inline hipStream_t stream_of(const prrtc_ctx* ctx, void* stream) {
    return stream ? static_cast<hipStream_t>(stream) : ctx->stream;
}
}  // namespace

constexpr int kCounterSlots = 256;

namespace {

// The message of the caller's last failure.  The serving thread records
// none: its queries' outcomes come back as statuses, and the user's thread
// may read the message meanwhile.
bool records_errors(const prrtc_ctx* ctx) { return ctx && std::this_thread::get_id() != ctx->serve_tid.load(); }

prrtc_status fail(prrtc_ctx* ctx, prrtc_status st, const char* fmt, ...) {
    if (records_errors(ctx)) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

#define PRRTC_HIP(ctx, call)                                                                  \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), PRRTC_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Entry points other than submit / poll / serve_stop are refused while the
// context's serving thread owns its stream and buffers.
#define PRRTC_NOT_SERVING(ctx)                                                          \
    do {                                                                                \
        if ((ctx)->serving.load()) return fail((ctx), PRRTC_E_STATE, "context is serving"); \
    } while (0)

bool finite_all(const float* p, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

bool orthonormal(const float* m, int stride) {  // rows of a 3x3 with the given row stride
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += (double)m[k * stride + i] * (double)m[k * stride + j];
            if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-5) return false;
        }
    return true;
}

template <class T>
size_t align_up(size_t x) {
    return (x + 255) & ~size_t(255);
}

}  // namespace

namespace {
// The stream an asynchronous call enqueues on: the caller's, or for NULL the
// context's own stream.
inline hipStream_t stream_of(const prrtc_ctx* ctx, void* stream);
void serve_shutdown(prrtc_ctx* ctx);   // stops and joins a context's serving thread
hipError_t scratch_address(int device, float** out);   // the static scratch array on a device
}  // namespace

extern "C" {

prrtc_status prrtc_create(prrtc_ctx** out, int device) {
    if (!out) return PRRTC_E_ARG;
    *out = nullptr;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev) return PRRTC_E_ARG;
    std::unique_ptr<prrtc_ctx> ctx(new prrtc_ctx());
    ctx->device = device;
    PRRTC_HIP(ctx.get(), hipSetDevice(device));
    hipDeviceProp_t prop;
    PRRTC_HIP(ctx.get(), hipGetDeviceProperties(&prop, device));
    ctx->n_cu = prop.multiProcessorCount;
    ctx->arch = prop.gcnArchName;
    ctx->arch = ctx->arch.substr(0, ctx->arch.find(':'));   // "gfx950", without the target features
    int wall_khz = 0;
    if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && wall_khz > 0)
        ctx->wall_khz = (double)wall_khz;
    PRRTC_HIP(ctx.get(), hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    PRRTC_HIP(ctx.get(), hipMalloc(&ctx->counters, sizeof(EdgeCounter) * kCounterSlots));
    PRRTC_HIP(ctx.get(), hipMemset(ctx->counters, 0, sizeof(EdgeCounter) * kCounterSlots));
    PRRTC_HIP(ctx.get(), hipEventCreate(&ctx->ev0));
    PRRTC_HIP(ctx.get(), hipEventCreate(&ctx->ev1));
    PRRTC_HIP(ctx.get(), hipHostMalloc(reinterpret_cast<void**>(&ctx->pinned), sizeof(float) * kPinnedFloats));
    PRRTC_HIP(ctx.get(), scratch_address(device, &ctx->scratch));   // with `device` current
    *out = ctx.release();
    return PRRTC_OK;
}

void prrtc_destroy(prrtc_ctx* ctx) {
    if (!ctx) return;
    serve_shutdown(ctx);
    hipSetDevice(ctx->device);
    if (ctx->stream) hipStreamSynchronize(ctx->stream);
    for (auto& r : ctx->robots) {
        hipFree(r.mem);
        hipFree(r.dev_args);
    }
    for (auto& s : ctx->scenes) {
        if (!s.mem) continue;
        hipFree(s.mem);
        hipFree(s.dev_args);
        if (s.vox) hipFree(s.vox);
        if (s.emb) hipFree(s.emb);
        if (s.esdf_mem) hipFree(s.esdf_mem);
    }
    planner_free(ctx->plan);
    planner_free(ctx->batch);
    for (auto& m : ctx->models) {
        hipFree(m.mem);
        if (m.ws) hipFree(m.ws);
    }
    if (ctx->counters) hipFree(ctx->counters);
    if (ctx->ev0) hipEventDestroy(ctx->ev0);
    if (ctx->ev1) hipEventDestroy(ctx->ev1);
    if (ctx->pinned) hipHostFree(ctx->pinned);
    if (ctx->stream) hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char* prrtc_last_error(const prrtc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

prrtc_status prrtc_load_robot(prrtc_ctx* ctx, const prrtc_robot_desc* d, int32_t* robot_id) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (!d || !robot_id) return fail(ctx, PRRTC_E_ARG, "null descriptor or id");
    if (d->n_chains < 1 || d->n_chains > PRRTC_MAX_CHAINS)
        return fail(ctx, PRRTC_E_ARG, "n_chains must be 1 or 2");
    int dof = 0, n_frames = 0;
    int chain_f0[2] = {0, 0}, chain_q0[2] = {0, 0};
    for (int c = 0; c < d->n_chains; ++c) {
        if (d->chain_dof[c] < 1) return fail(ctx, PRRTC_E_ARG, "chain %d has no joints", c);
        chain_q0[c] = dof;
        chain_f0[c] = n_frames;
        dof += d->chain_dof[c];
        n_frames += d->chain_dof[c] + 1;
        if (!finite_all(d->base_pose[c], 12) || !orthonormal(d->base_pose[c], 4))
            return fail(ctx, PRRTC_E_ARG, "base pose of chain %d not finite/orthonormal", c);
    }
    if (dof > PRRTC_MAX_DOF) return fail(ctx, PRRTC_E_ARG, "dof %d exceeds %d", dof, PRRTC_MAX_DOF);
    if (!d->dh || !d->q_lo || !d->q_hi || !finite_all(d->dh, 3 * dof) || !finite_all(d->q_lo, dof) ||
        !finite_all(d->q_hi, dof))
        return fail(ctx, PRRTC_E_ARG, "DH table or limits missing or not finite");
    for (int j = 0; j < dof; ++j)
        if (!(d->q_lo[j] < d->q_hi[j])) return fail(ctx, PRRTC_E_ARG, "joint %d: lo >= hi", j);
    const int ns = d->n_spheres;
    if (ns < 1 || ns > PRRTC_MAX_SPHERES || !d->sphere_frame || !d->sphere_xyzr)
        return fail(ctx, PRRTC_E_ARG, "n_spheres must be in 1..%d", PRRTC_MAX_SPHERES);
    for (int k = 0; k < ns; ++k) {
        if (d->sphere_frame[k] < 0 || d->sphere_frame[k] >= n_frames)
            return fail(ctx, PRRTC_E_ARG, "sphere %d: frame id out of range", k);
        if (!finite_all(d->sphere_xyzr + 4 * k, 4) || !(d->sphere_xyzr[4 * k + 3] > 0.0f))
            return fail(ctx, PRRTC_E_ARG, "sphere %d: not finite or radius <= 0", k);
    }
    // coarse spheres (two-stage checks): each fine sphere names one on its
    // own frame that encloses it
    const int nc = d->n_coarse;
    if (nc < 0 || nc > PRRTC_MAX_SPHERES || (nc > 0 && (!d->coarse_frame || !d->coarse_xyzr || !d->sphere_coarse)))
        return fail(ctx, PRRTC_E_ARG, "n_coarse must be in 0..%d with its tables", PRRTC_MAX_SPHERES);
    for (int c = 0; c < nc; ++c)
        if (d->coarse_frame[c] < 0 || d->coarse_frame[c] >= n_frames || !finite_all(d->coarse_xyzr + 4 * c, 4) ||
            !(d->coarse_xyzr[4 * c + 3] > 0.0f))
            return fail(ctx, PRRTC_E_ARG, "coarse sphere %d: bad frame, not finite or radius <= 0", c);
    for (int k = 0; nc > 0 && k < ns; ++k) {
        const int c = d->sphere_coarse[k];
        if (c < 0 || c >= nc || d->coarse_frame[c] != d->sphere_frame[k])
            return fail(ctx, PRRTC_E_ARG, "sphere %d: coarse sphere out of range or on another frame", k);
        const float* f = d->sphere_xyzr + 4 * k;
        const float* g = d->coarse_xyzr + 4 * c;
        const double dist = std::sqrt(((double)f[0] - g[0]) * ((double)f[0] - g[0]) +
                                      ((double)f[1] - g[1]) * ((double)f[1] - g[1]) +
                                      ((double)f[2] - g[2]) * ((double)f[2] - g[2]));
        if (dist + (double)f[3] > (double)g[3] * (1.0 + 1e-6) + 1e-7)
            return fail(ctx, PRRTC_E_ARG, "sphere %d is not inside its coarse sphere %d", k, c);
    }
    const int np = d->n_self_pairs;
    if (np < 0 || np > PRRTC_MAX_SELF_PAIRS || (np > 0 && !d->self_pairs))
        return fail(ctx, PRRTC_E_ARG, "n_self_pairs must be in 0..%d", PRRTC_MAX_SELF_PAIRS);
    for (int p = 0; p < np; ++p) {
        const int i = d->self_pairs[2 * p], j = d->self_pairs[2 * p + 1];
        if (i < 0 || j < 0 || i >= ns || j >= ns || i == j)
            return fail(ctx, PRRTC_E_ARG, "self pair %d invalid", p);
    }
    // re-order: moving spheres (frame > chain base) sorted by frame, most distal first
    auto is_fixed = [&](int k) {
        for (int c = 0; c < d->n_chains; ++c)
            if (d->sphere_frame[k] == chain_f0[c]) return true;
        return false;
    };
    std::vector<int> order;
    for (int k = 0; k < ns; ++k)
        if (!is_fixed(k)) order.push_back(k);
    // (with coarse spheres: the fine spheres of one coarse sphere side by side)
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (d->sphere_frame[x] != d->sphere_frame[y]) return d->sphere_frame[x] > d->sphere_frame[y];
        return nc > 0 && d->sphere_coarse[x] < d->sphere_coarse[y];
    });
    const int n_move = (int)order.size();
    for (int k = 0; k < ns; ++k)
        if (is_fixed(k)) order.push_back(k);
    std::vector<int> new_of(ns);
    for (int k = 0; k < ns; ++k) new_of[order[k]] = k;
    // LDS slots for the frames that carry moving spheres
    int frame_slot[kMaxFrames];
    for (int f = 0; f < kMaxFrames; ++f) frame_slot[f] = -1;
    int n_slots = 0;
    for (int k = 0; k < n_move; ++k) {
        const int f = d->sphere_frame[order[k]];
        if (frame_slot[f] < 0) frame_slot[f] = n_slots++;
    }
    std::vector<float4> sph(ns);
    std::vector<int> frame(ns), desc(ns), slot3(ns, 0);
    for (int k = 0; k < ns; ++k) {
        const float* p = d->sphere_xyzr + 4 * order[k];
        sph[k] = make_float4(p[0], p[1], p[2], p[3]);
        frame[k] = d->sphere_frame[order[k]];
        desc[k] = order[k];
        if (k < n_move) slot3[k] = 3 * frame_slot[frame[k]];
    }
    std::vector<int2> pairs, spairs;
    for (int p = 0; p < np; ++p) {
        const int i = new_of[d->self_pairs[2 * p]], j = new_of[d->self_pairs[2 * p + 1]];
        if (i >= n_move && j >= n_move) spairs.push_back(make_int2(i, j));
        else pairs.push_back(make_int2(i, j));
    }
    // Is the whole pair list the complete bipartite set A x B of two disjoint
    // sphere groups?  Then the kernels test it group against group.
    std::vector<int> bip_a, bip_b;
    {
        std::vector<char> in_a(ns, 0), in_b(ns, 0);
        std::vector<std::pair<int, int>> all;
        for (int p = 0; p < np; ++p) {
            const int i = new_of[d->self_pairs[2 * p]], j = new_of[d->self_pairs[2 * p + 1]];
            in_a[i] = 1;
            in_b[j] = 1;
            all.emplace_back(i, j);
        }
        std::sort(all.begin(), all.end());
        const bool unique = std::adjacent_find(all.begin(), all.end()) == all.end();
        bool disjoint = true;
        for (int k = 0; k < ns; ++k) {
            if (in_a[k] && in_b[k]) disjoint = false;
            if (in_a[k]) bip_a.push_back(k);
            if (in_b[k]) bip_b.push_back(k);
        }
        if (!(np > 0 && unique && disjoint && (size_t)np == bip_a.size() * bip_b.size())) {
            bip_a.clear();
            bip_b.clear();
        } else {
            pairs.clear();  // covered group against group
        }
    }
    // coarse spheres on moving frames, in the order of their fine runs
    std::vector<float4> csph;
    std::vector<int> cslot3, cfirst;
    if (nc > 0) {
        for (int k = 0; k < n_move; ++k) {
            const int c = d->sphere_coarse[order[k]];
            if (k == 0 || c != d->sphere_coarse[order[k - 1]]) {
                const float* g = d->coarse_xyzr + 4 * c;
                csph.push_back(make_float4(g[0], g[1], g[2], g[3] + kCoarseMargin));
                cslot3.push_back(3 * frame_slot[d->coarse_frame[c]]);
                cfirst.push_back(k);
            }
        }
        cfirst.push_back(n_move);
    }
    const size_t o_sph = 0;
    const size_t o_frame = align_up<int>(o_sph + sizeof(float4) * ns);
    const size_t o_slot = align_up<int>(o_frame + sizeof(int) * ns);
    const size_t o_desc = align_up<int>(o_slot + sizeof(int) * ns);
    const size_t o_pairs = align_up<int>(o_desc + sizeof(int) * ns);
    const size_t o_spairs = align_up<int>(o_pairs + sizeof(int2) * pairs.size());
    const size_t o_bipa = align_up<int>(o_spairs + sizeof(int2) * spairs.size());
    const size_t o_bipb = align_up<int>(o_bipa + sizeof(int) * bip_a.size());
    const size_t o_csph = align_up<int>(o_bipb + sizeof(int) * bip_b.size());
    const size_t o_cslot = align_up<int>(o_csph + sizeof(float4) * csph.size());
    const size_t o_cfirst = align_up<int>(o_cslot + sizeof(int) * cslot3.size());
    const size_t bytes = align_up<int>(o_cfirst + sizeof(int) * cfirst.size());
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    RobotRec rec;
    PRRTC_HIP(ctx, hipMalloc(&rec.mem, bytes));
    char* base = static_cast<char*>(rec.mem);
    std::vector<char> host(bytes, 0);
    memcpy(host.data() + o_sph, sph.data(), sizeof(float4) * ns);
    memcpy(host.data() + o_frame, frame.data(), sizeof(int) * ns);
    memcpy(host.data() + o_slot, slot3.data(), sizeof(int) * ns);
    memcpy(host.data() + o_desc, desc.data(), sizeof(int) * ns);
    if (!pairs.empty()) memcpy(host.data() + o_pairs, pairs.data(), sizeof(int2) * pairs.size());
    if (!spairs.empty()) memcpy(host.data() + o_spairs, spairs.data(), sizeof(int2) * spairs.size());
    if (!bip_a.empty()) memcpy(host.data() + o_bipa, bip_a.data(), sizeof(int) * bip_a.size());
    if (!bip_b.empty()) memcpy(host.data() + o_bipb, bip_b.data(), sizeof(int) * bip_b.size());
    if (!csph.empty()) memcpy(host.data() + o_csph, csph.data(), sizeof(float4) * csph.size());
    if (!cslot3.empty()) memcpy(host.data() + o_cslot, cslot3.data(), sizeof(int) * cslot3.size());
    if (!cfirst.empty()) memcpy(host.data() + o_cfirst, cfirst.data(), sizeof(int) * cfirst.size());
    hipError_t e = hipMemcpy(rec.mem, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(rec.mem);
        return fail(ctx, PRRTC_E_HIP, "hipMemcpy robot: %s", hipGetErrorString(e));
    }
    RobotArgs& A = rec.args;
    A.n_chains = d->n_chains;
    A.dof = dof;
    A.n_frames = n_frames;
    A.n_slots = n_slots;
    for (int f = 0; f < kMaxFrames; ++f) A.frame_slot[f] = frame_slot[f];
    A.n_move = n_move;
    A.n_static = ns - n_move;
    A.n_pairs = (int)pairs.size();
    A.n_static_pairs = (int)spairs.size();
    for (int c = 0; c < kMaxChains; ++c) {
        A.chain_dof[c] = c < d->n_chains ? d->chain_dof[c] : 0;
        A.chain_q0[c] = chain_q0[c];
        A.chain_f0[c] = chain_f0[c];
        for (int i = 0; i < 12; ++i) A.base[c][i] = c < d->n_chains ? d->base_pose[c][i] : 0.0f;
    }
    for (int j = 0; j < kMaxDof; ++j) {
        const bool in = j < dof;
        const double alpha = in ? (double)d->dh[3 * j + 0] : 0.0;
        A.ca[j] = (float)std::cos(alpha);
        A.sa[j] = (float)std::sin(alpha);
        A.a[j] = in ? d->dh[3 * j + 1] : 0.0f;
        A.d[j] = in ? d->dh[3 * j + 2] : 0.0f;
        A.lo[j] = in ? d->q_lo[j] : 0.0f;
        A.hi[j] = in ? d->q_hi[j] : 0.0f;
    }
    A.sph = reinterpret_cast<const float4*>(base + o_sph);
    A.sph_frame = reinterpret_cast<const int*>(base + o_frame);
    A.sph_slot = reinterpret_cast<const int*>(base + o_slot);
    A.desc_index = reinterpret_cast<const int*>(base + o_desc);
    A.pairs = reinterpret_cast<const int2*>(base + o_pairs);
    A.static_pairs = reinterpret_cast<const int2*>(base + o_spairs);
    A.n_bip_a = (int)bip_a.size();
    A.n_bip_b = (int)bip_b.size();
    A.bip_a = reinterpret_cast<const int*>(base + o_bipa);
    A.bip_b = reinterpret_cast<const int*>(base + o_bipb);
    A.n_cmove = (int)csph.size();
    A.csph = reinterpret_cast<const float4*>(base + o_csph);
    A.cslot3 = reinterpret_cast<const int*>(base + o_cslot);
    A.cfirst = reinterpret_cast<const int*>(base + o_cfirst);
    rec.dof = dof;
    rec.n_spheres = ns;
    e = hipMalloc(&rec.dev_args, sizeof(RobotArgs));
    if (e == hipSuccess) e = hipMemcpy(rec.dev_args, &rec.args, sizeof(RobotArgs), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(rec.mem);
        hipFree(rec.dev_args);
        return fail(ctx, PRRTC_E_HIP, "robot tables: %s", hipGetErrorString(e));
    }
    ctx->robots.push_back(rec);
    *robot_id = (int32_t)ctx->robots.size() - 1;
    return PRRTC_OK;
}

prrtc_status prrtc_load_scene(prrtc_ctx* ctx, const prrtc_prim* p, int32_t n, int32_t* scene_id) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (!scene_id || n < 0 || n > PRRTC_MAX_PRIMS || (n > 0 && !p))
        return fail(ctx, PRRTC_E_ARG, "bad scene arguments (n must be in 0..%d)", PRRTC_MAX_PRIMS);
    std::vector<float4> sph, sph_b, box_b, cyl_b, box_e, cyl_e;
    std::vector<float> box, cyl;
    const float margin = 1e-4f;
    auto bound = [&](const prrtc_prim& q, double rad) {
        return make_float4(q.c[0], q.c[1], q.c[2], (float)(rad * (1.0 + 1e-6)) + margin);
    };
    // A world-axis box is worth its extra test when it is much thinner than
    // the bounding sphere along some axis (boards, rods): counted per type,
    // and the boxes are used for a type when a quarter of it is so.
    int box_thin = 0, cyl_thin = 0;
    auto extent = [&](const double* e, double rad, int& thin) {
        if (std::min(e[0], std::min(e[1], e[2])) < 0.5 * rad) ++thin;
        return make_float4((float)(e[0] * (1.0 + 1e-6)) + margin, (float)(e[1] * (1.0 + 1e-6)) + margin,
                           (float)(e[2] * (1.0 + 1e-6)) + margin, 0.0f);
    };
    for (int i = 0; i < n; ++i) {
        const prrtc_prim& q = p[i];
        if (!finite_all(q.c, 3) || !finite_all(q.rot, 9) || !finite_all(q.dims, 3))
            return fail(ctx, PRRTC_E_ARG, "primitive %d not finite", i);
        if (q.type == 0) {
            if (!(q.dims[0] > 0.0f)) return fail(ctx, PRRTC_E_ARG, "primitive %d: radius <= 0", i);
            sph.push_back(make_float4(q.c[0], q.c[1], q.c[2], q.dims[0]));
            sph_b.push_back(bound(q, q.dims[0]));
        } else if (q.type == 1 || q.type == 2) {
            if (!orthonormal(q.rot, 3)) return fail(ctx, PRRTC_E_ARG, "primitive %d: rotation not orthonormal", i);
            if (q.type == 1) {
                if (!(q.dims[0] > 0.0f && q.dims[1] > 0.0f && q.dims[2] > 0.0f))
                    return fail(ctx, PRRTC_E_ARG, "primitive %d: half-extent <= 0", i);
                // axis k is column k of rot; the record keeps -(axis_k . c)
                double off[3];
                for (int k = 0; k < 3; ++k)
                    off[k] = -((double)q.rot[k] * q.c[0] + (double)q.rot[3 + k] * q.c[1] +
                               (double)q.rot[6 + k] * q.c[2]);
                const float rec[16] = {(float)off[0], (float)off[1], (float)off[2], 0.0f,
                                       q.rot[0], q.rot[3], q.rot[6],
                                       q.rot[1], q.rot[4], q.rot[7],
                                       q.rot[2], q.rot[5], q.rot[8],
                                       q.dims[0], q.dims[1], q.dims[2]};
                box.insert(box.end(), rec, rec + 16);
                const double rad = std::sqrt((double)q.dims[0] * q.dims[0] + (double)q.dims[1] * q.dims[1] +
                                             (double)q.dims[2] * q.dims[2]);
                box_b.push_back(bound(q, rad));
                // world half-size along axis i: sum over k of |axis_k[i]| h_k
                double e[3];
                for (int i = 0; i < 3; ++i)
                    e[i] = std::fabs((double)q.rot[3 * i]) * q.dims[0] + std::fabs((double)q.rot[3 * i + 1]) * q.dims[1] +
                           std::fabs((double)q.rot[3 * i + 2]) * q.dims[2];
                box_e.push_back(extent(e, rad, box_thin));
            } else {
                if (!(q.dims[0] > 0.0f && q.dims[1] > 0.0f))
                    return fail(ctx, PRRTC_E_ARG, "primitive %d: cylinder radius/half-height <= 0", i);
                const float rec[8] = {q.c[0], q.c[1], q.c[2], q.rot[2], q.rot[5], q.rot[8], q.dims[0], q.dims[1]};
                cyl.insert(cyl.end(), rec, rec + 8);
                const double rad = std::sqrt((double)q.dims[0] * q.dims[0] + (double)q.dims[1] * q.dims[1]);
                cyl_b.push_back(bound(q, rad));
                // along world axis i: |a_i| h + r sqrt(1 - a_i^2) (the end discs' reach)
                double e[3];
                for (int i = 0; i < 3; ++i) {
                    const double a = q.rot[3 * i + 2];
                    e[i] = std::fabs(a) * q.dims[1] + q.dims[0] * std::sqrt(std::max(0.0, 1.0 - a * a));
                }
                cyl_e.push_back(extent(e, rad, cyl_thin));
            }
        } else {
            return fail(ctx, PRRTC_E_ARG, "primitive %d: unknown type %d", i, q.type);
        }
    }
    const size_t o_sph = 0;
    const size_t o_box = align_up<int>(sizeof(float4) * sph.size());
    const size_t o_cyl = align_up<int>(o_box + sizeof(float) * box.size());
    // one bounds table and one world-box table over all types, spheres,
    // cuboids, cylinders (a type's boxes are used when a quarter of it is
    // thin; 3e38 half-sizes keep everything else)
    const bool use_box_e = PRRTC_EXT_CULL && box_thin > 0 && 4 * box_thin >= (int)box_e.size();
    const bool use_cyl_e = PRRTC_EXT_CULL && cyl_thin > 0 && 4 * cyl_thin >= (int)cyl_e.size();
    const float4 wide = make_float4(3.0e38f, 3.0e38f, 3.0e38f, 0.0f);
    std::vector<float4> bnd(sph_b), ext(sph_b.size(), wide);
    bnd.insert(bnd.end(), box_b.begin(), box_b.end());
    bnd.insert(bnd.end(), cyl_b.begin(), cyl_b.end());
    for (const float4& e : box_e) ext.push_back(use_box_e ? e : wide);
    for (const float4& e : cyl_e) ext.push_back(use_cyl_e ? e : wide);
    if (bnd.empty()) {   // an empty scene keeps one zero entry of each
        bnd.push_back(make_float4(0.0f, 0.0f, 0.0f, 0.0f));
        ext.push_back(make_float4(0.0f, 0.0f, 0.0f, 0.0f));
    }
    const size_t o_bnd = align_up<int>(o_cyl + sizeof(float) * cyl.size());
    const size_t o_ext = align_up<int>(o_bnd + sizeof(float4) * bnd.size());
    const size_t bytes = std::max<size_t>(256, align_up<int>(o_ext + sizeof(float4) * ext.size()));
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    SceneRec rec;
    PRRTC_HIP(ctx, hipMalloc(&rec.mem, bytes));
    std::vector<char> host(bytes, 0);
    if (!sph.empty()) memcpy(host.data() + o_sph, sph.data(), sizeof(float4) * sph.size());
    if (!box.empty()) memcpy(host.data() + o_box, box.data(), sizeof(float) * box.size());
    if (!cyl.empty()) memcpy(host.data() + o_cyl, cyl.data(), sizeof(float) * cyl.size());
    if (!bnd.empty()) memcpy(host.data() + o_bnd, bnd.data(), sizeof(float4) * bnd.size());
    if (!ext.empty()) memcpy(host.data() + o_ext, ext.data(), sizeof(float4) * ext.size());
    hipError_t e = hipMemcpy(rec.mem, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(rec.mem);
        return fail(ctx, PRRTC_E_HIP, "hipMemcpy scene: %s", hipGetErrorString(e));
    }
    char* base = static_cast<char*>(rec.mem);
    rec.args.n_sph = (int)sph.size();
    rec.args.n_box = (int)(box.size() / 16);
    rec.args.n_cyl = (int)(cyl.size() / 8);
    rec.args.sph = reinterpret_cast<const float4*>(base + o_sph);
    rec.args.box = reinterpret_cast<const float*>(base + o_box);
    rec.args.cyl = reinterpret_cast<const float*>(base + o_cyl);
    rec.args.bnd = reinterpret_cast<const float4*>(base + o_bnd);
    rec.args.ext = reinterpret_cast<const float4*>(base + o_ext);
    rec.args.ext_cull = use_box_e || use_cyl_e;
    rec.n = n;
    e = hipMalloc(&rec.dev_args, sizeof(SceneArgs));
    if (e == hipSuccess) e = hipMemcpy(rec.dev_args, &rec.args, sizeof(SceneArgs), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(rec.mem);
        hipFree(rec.dev_args);
        return fail(ctx, PRRTC_E_HIP, "scene tables: %s", hipGetErrorString(e));
    }
    ctx->scenes.push_back(rec);
    *scene_id = (int32_t)ctx->scenes.size() - 1;
    return PRRTC_OK;
}

prrtc_status prrtc_unload_scene(prrtc_ctx* ctx, int32_t scene_id) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].mem)
        return fail(ctx, PRRTC_E_STATE, "unknown or unloaded scene id %d", scene_id);
    SceneRec& rec = ctx->scenes[scene_id];
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    PRRTC_HIP(ctx, hipDeviceSynchronize());
    PRRTC_HIP(ctx, hipFree(rec.mem));
    PRRTC_HIP(ctx, hipFree(rec.dev_args));
    if (rec.vox) PRRTC_HIP(ctx, hipFree(rec.vox));
    if (rec.emb) PRRTC_HIP(ctx, hipFree(rec.emb));
    if (rec.esdf_mem) PRRTC_HIP(ctx, hipFree(rec.esdf_mem));
    rec = SceneRec{};
    return PRRTC_OK;
}

namespace {
bool esdf_geometry_ok(prrtc_ctx* ctx, const float origin[3], float voxel, const int32_t dims[3]) {
    if (!finite_all(origin, 3) || !(voxel > 0.0f) || !std::isfinite(voxel)) {
        fail(ctx, PRRTC_E_ARG, "ESDF origin must be finite and voxel > 0");
        return false;
    }
    long long total = 1;
    for (int a = 0; a < 3; ++a) {
        if (dims[a] < 2 || dims[a] > 1024) {
            fail(ctx, PRRTC_E_ARG, "ESDF dims must be in 2..1024");
            return false;
        }
        total *= dims[a];
    }
    if (total > (1LL << 27)) {
        fail(ctx, PRRTC_E_ARG, "ESDF of %lld nodes exceeds 2^27", total);
        return false;
    }
    return true;
}
}  // namespace

prrtc_status prrtc_scene_set_esdf(prrtc_ctx* ctx, int32_t scene_id, const prrtc_esdf_desc* d) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].mem)
        return fail(ctx, PRRTC_E_STATE, "unknown or unloaded scene id %d", scene_id);
    SceneRec& rec = ctx->scenes[scene_id];
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    void* mem = nullptr;
    SceneArgs args = rec.args;
    if (d) {
        if (!esdf_geometry_ok(ctx, d->origin, d->voxel, d->dims)) return PRRTC_E_ARG;
        if (!d->values) return fail(ctx, PRRTC_E_ARG, "null ESDF values");
        const size_t n = (size_t)d->dims[0] * d->dims[1] * d->dims[2];
        for (size_t k = 0; k < n; ++k)
            if (std::isnan(d->values[k])) return fail(ctx, PRRTC_E_ARG, "ESDF value %zu is NaN", k);
        PRRTC_HIP(ctx, hipMalloc(&mem, sizeof(float) * n));
        hipError_t e = hipMemcpy(mem, d->values, sizeof(float) * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(mem);
            return fail(ctx, PRRTC_E_HIP, "ESDF upload: %s", hipGetErrorString(e));
        }
        args.esdf = static_cast<const float*>(mem);
        for (int a = 0; a < 3; ++a) {
            args.esdf_o[a] = d->origin[a];
            args.esdf_n[a] = d->dims[a];
        }
        args.esdf_ih = 1.0f / d->voxel;
        // Lipschitz bound of the interpolated field: per axis the largest
        // difference of neighbouring nodes over the spacing
        double lip2 = 0.0;
        const int nx = d->dims[0], ny = d->dims[1], nz = d->dims[2];
        for (int a = 0; a < 3; ++a) {
            const size_t step = a == 0 ? 1 : (a == 1 ? (size_t)nx : (size_t)nx * ny);
            double m = 0.0;
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        if ((a == 0 && i == nx - 1) || (a == 1 && j == ny - 1) || (a == 2 && k == nz - 1)) continue;
                        const size_t at = ((size_t)k * ny + j) * nx + i;
                        const double diff = std::fabs((double)d->values[at + step] - (double)d->values[at]);
                        if (!(diff <= m)) m = diff;   // also takes an infinite difference
                    }
            const double l = m / (double)d->voxel;
            lip2 += l * l;
        }
        args.esdf_gate = (float)std::max(1.0, std::sqrt(lip2) * (1.0 + 1e-6));
    } else {
        args.esdf = nullptr;
    }
    // the device copy of the tables changes: wait for work that may read it
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(rec.dev_args, &args, sizeof(SceneArgs), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (mem) (void)hipFree(mem);
        return fail(ctx, PRRTC_E_HIP, "scene tables: %s", hipGetErrorString(e));
    }
    if (rec.esdf_mem) (void)hipFree(rec.esdf_mem);
    rec.esdf_mem = mem;
    rec.args = args;
    rec.edge_schedule.clear();   // the check_edges schedules are timed again
    return PRRTC_OK;
}

prrtc_status prrtc_esdf_from_scene(prrtc_ctx* ctx, int32_t scene_id, const float origin[3], float voxel,
                                   const int32_t dims[3], float* values, void* stream) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].mem)
        return fail(ctx, PRRTC_E_STATE, "unknown or unloaded scene id %d", scene_id);
    if (!origin || !dims || !values) return fail(ctx, PRRTC_E_ARG, "null argument");
    if (!esdf_geometry_ok(ctx, origin, voxel, dims)) return PRRTC_E_ARG;
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    const long long n = (long long)dims[0] * dims[1] * dims[2];
    hipLaunchKernelGGL(k_esdf_build, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream_of(ctx, stream),
                       ctx->scenes[scene_id].args, origin[0], origin[1], origin[2], voxel, dims[0], dims[1], dims[2],
                       values);
    PRRTC_HIP(ctx, hipGetLastError());
    return PRRTC_OK;
}

}  // extern "C"

namespace {

#ifndef PRRTC_EDGE_TILE
#define PRRTC_EDGE_TILE 16
#endif
#ifndef PRRTC_EDGE_ITEMS
#define PRRTC_EDGE_ITEMS 3
#endif
constexpr int kEdgeTile = PRRTC_EDGE_TILE;
constexpr int kEdgeItems = PRRTC_EDGE_ITEMS;

// The check_edges schedules: bit 0 picks (items per lane, cuboids swept
// first) = (3, no) or (2, yes); bit 1, for robots with coarse spheres, adds
// the two-stage pass (schedules 2 and 3).  They return the same verdicts;
// which is faster depends on the robot and scene (measured: 2 items with
// cuboids first is 9% faster on the 7-DoF arm among 64 mixed obstacles, 3
// items with spheres first 3% faster on the dual arm in the shelf; the
// two-stage pass is 15% faster on the 7-DoF arm among 12 obstacles and 2x
// slower among 64), so the first large batch on a (robot, scene) pair times
// every schedule the robot has.
const void* edge_kernel(int schedule) {
    static const void* k[4] = {reinterpret_cast<const void*>(&k_check_edges<kEdgeTile, kEdgeItems, false, false>),
                               reinterpret_cast<const void*>(&k_check_edges<kEdgeTile, 2, true, false>),
                               reinterpret_cast<const void*>(&k_check_edges<kEdgeTile, kEdgeItems, false, true>),
                               reinterpret_cast<const void*>(&k_check_edges<kEdgeTile, 2, true, true>)};
    return k[schedule];
}
int edge_schedules(const RobotArgs& R) { return R.n_cmove > 0 ? 4 : 2; }
constexpr long long kEdgeTuneMin = 8192;      // batches at least this large pick the schedule
constexpr long long kEdgeTuneEdges = 1 << 20;  // edges timed per schedule (at most): small prefixes
                                               // mostly time the launch's tail, not the schedule

size_t sphere_lds_bytes(const RobotArgs& R) {
    return sizeof(float4) * R.n_move + sizeof(int) * ((R.n_move + 3) & ~3);
}

// two: a two-stage schedule (its flag and item tables are only needed then)
size_t check_lds_bytes(const RobotArgs& R, int tp, bool two) {
    return sphere_lds_bytes(R) + sizeof(float4) * tp * 3 * R.n_slots + sizeof(float) * 2 * kMaxDof +
           sizeof(int) * (tp + 4 + kEdgeChunk) + (two ? two_stage_lds_bytes(R, tp) : 0);
}

// Tuning records are keyed by what decides the timing: the device, and the
// robot's and scene's shape with counts in power-of-two buckets.
int bucket(int n) {
    int b = 0;
    while (n > 0) {
        ++b;
        n >>= 1;
    }
    return b;
}

std::string edge_tuning_key(const prrtc_ctx* ctx, int32_t robot_id, int32_t scene_id) {
    const RobotArgs& R = ctx->robots[robot_id].args;
    const SceneArgs& S = ctx->scenes[scene_id].args;
    std::ostringstream k;
    k << "edge " << ctx->arch << " dof=" << R.dof << " moving=" << bucket(R.n_move) << " coarse=" << (R.n_cmove > 0)
      << " pairs=" << bucket(R.n_pairs + R.n_bip_a * R.n_bip_b) << " spheres=" << bucket(S.n_sph)
      << " cuboids=" << bucket(S.n_box) << " cylinders=" << bucket(S.n_cyl) << " esdf=" << (S.esdf != nullptr);
    return k.str();
}

// A (robot, scene) pair without a schedule takes a stored record's.
void adopt_tuned_schedule(prrtc_ctx* ctx, int32_t robot_id, int32_t scene_id) {
    auto& m = ctx->scenes[scene_id].edge_schedule;
    if (m.count(robot_id) || ctx->tuning.empty()) return;
    auto t = ctx->tuning.find(edge_tuning_key(ctx, robot_id, scene_id));
    if (t == ctx->tuning.end() || t->second.size() != 1) return;
    const int v = t->second[0] - '0';
    if (v >= 0 && v < edge_schedules(ctx->robots[robot_id].args)) m[robot_id] = v;
}

std::string launch_tuning_key(const prrtc_ctx* ctx, const prrtc_query* q, int n, const int32_t* workers,
                              int n_workers, const int32_t* tiles, int n_tiles) {
    std::map<int, int> dofs;
    int obstacles = 0;
    for (int i = 0; i < n; ++i) {
        if (q[i].robot_id < 0 || q[i].robot_id >= (int)ctx->robots.size()) continue;
        dofs[ctx->robots[q[i].robot_id].dof] = 1;
        if (q[i].scene_id >= 0 && q[i].scene_id < (int)ctx->scenes.size())
            obstacles = std::max(obstacles, ctx->scenes[q[i].scene_id].n);
    }
    std::ostringstream k;
    k << "launch " << ctx->arch << " dofs=";
    for (const auto& d : dofs) k << d.first << ",";
    k << " obstacles=" << bucket(obstacles) << " workers=";
    for (int i = 0; i < n_workers; ++i) k << workers[i] << ",";
    k << " tiles=";
    for (int i = 0; i < n_tiles; ++i) k << tiles[i] << ",";
    return k.str();
}

prrtc_status lookup(prrtc_ctx* ctx, int32_t robot_id, int32_t scene_id, const RobotRec** r,
                    const SceneRec** s) {
    if (robot_id < 0 || robot_id >= (int32_t)ctx->robots.size())
        return fail(ctx, PRRTC_E_STATE, "unknown robot id %d", robot_id);
    *r = &ctx->robots[robot_id];
    if (s) {
        if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].mem)
            return fail(ctx, PRRTC_E_STATE, "unknown or unloaded scene id %d", scene_id);
        *s = &ctx->scenes[scene_id];
    }
    return PRRTC_OK;
}

}  // namespace

extern "C" {

prrtc_status prrtc_check_edges(prrtc_ctx* ctx, int32_t robot_id, int32_t scene_id, const float* a,
                               const float* b, int64_t n_edges, float res, uint8_t* valid,
                               void* stream) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    const RobotRec* r = nullptr;
    const SceneRec* s = nullptr;
    prrtc_status st = lookup(ctx, robot_id, scene_id, &r, &s);
    if (st != PRRTC_OK) return st;
    if (n_edges < 0) return fail(ctx, PRRTC_E_ARG, "n_edges < 0");
    if (!(res > 0.0f) || !std::isfinite(res)) return fail(ctx, PRRTC_E_ARG, "res must be finite and > 0");
    if (n_edges == 0) return PRRTC_OK;
    if (!a || !b || !valid) return fail(ctx, PRRTC_E_ARG, "null buffer");
    hipStream_t sm = stream_of(ctx, stream);
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    auto launch = [&](int schedule, long long n) -> prrtc_status {
        const int kk = schedule;
        const size_t lds = check_lds_bytes(r->args, kEdgeTile, schedule >= 2);
        if (ctx->edge_grid[kk] == 0 || ctx->edge_grid_lds[kk] != lds) {
            int per_cu = 0;
            PRRTC_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, edge_kernel(schedule), kWave, lds));
            ctx->edge_grid[kk] = std::max(1, per_cu) * ctx->n_cu;
            ctx->edge_grid_lds[kk] = lds;
        }
        // at least one workgroup per XCD range (empty ranges exit at once);
        // chunks of up to kEdgeChunk edges, at least four per resident wave;
        // small batches: the static interleave (chunk 0)
        const long long grid = std::max<long long>(std::min<long long>(n, ctx->edge_grid[kk]), kXcds);
        int chunk = n <= kEdgeStatic * ctx->edge_grid[kk]
                        ? 0
                        : (int)std::min<long long>(kEdgeChunk, std::max<long long>(1, n / (4LL * ctx->edge_grid[kk])));
        EdgeCounter* ctr = ctx->counters + (ctx->counter_next++ % kCounterSlots);
        RobotArgs ra = r->args;
        SceneArgs sa = s->args;
        const float* pa = a;
        const float* pb = b;
        float fres = res;
        uint8_t* pv = valid;
        void* kargs[] = {&ra, &sa, &pa, &pb, &n, &fres, &pv, &ctr, &chunk};
        PRRTC_HIP(ctx, hipLaunchKernel(edge_kernel(schedule), dim3((unsigned)grid), dim3(kWave), kargs, lds, sm));
        return PRRTC_OK;
    };
    SceneRec& sr = ctx->scenes[scene_id];
    adopt_tuned_schedule(ctx, robot_id, scene_id);
    auto it = sr.edge_schedule.find(robot_id);
    const int n_sched = edge_schedules(r->args);
    int schedule = it == sr.edge_schedule.end() ? n_sched - 2 : it->second;   // untimed: two-stage if it has it
    if (it == sr.edge_schedule.end() && n_edges >= kEdgeTuneMin) {
        // time every schedule on (a prefix of) this batch, twice in turn,
        // keeping each one's faster run (schedules within a few percent of
        // each other would otherwise be picked by the noise of one run);
        // its verdicts are written again by the launch below.  Synchronises
        // this once.
        const long long m = std::min<long long>(n_edges, kEdgeTuneEdges);
        float best = 0.0f;
        for (int k = 0; k < n_sched; ++k) {
            st = launch(k, kEdgeTuneMin);   // warm-up
            if (st != PRRTC_OK) return st;
        }
        for (int rep = 0; rep < 2; ++rep) {
            for (int k = 0; k < n_sched; ++k) {
                PRRTC_HIP(ctx, hipEventRecord(ctx->ev0, sm));
                st = launch(k, m);
                if (st != PRRTC_OK) return st;
                PRRTC_HIP(ctx, hipEventRecord(ctx->ev1, sm));
                PRRTC_HIP(ctx, hipEventSynchronize(ctx->ev1));
                float ms = 0.0f;
                PRRTC_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
                if ((rep == 0 && k == 0) || ms < best) {
                    best = ms;
                    schedule = k;
                }
            }
        }
        sr.edge_schedule[robot_id] = schedule;
        ctx->tuning[edge_tuning_key(ctx, robot_id, scene_id)] = std::to_string(schedule);
    }
    return launch(schedule, n_edges);
}

prrtc_status prrtc_edge_schedule(prrtc_ctx* ctx, int32_t robot_id, int32_t scene_id, int32_t set,
                                 int32_t* schedule) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    const RobotRec* r = nullptr;
    const SceneRec* s = nullptr;
    prrtc_status st = lookup(ctx, robot_id, scene_id, &r, &s);
    if (st != PRRTC_OK) return st;
    if (set < -2 || set >= edge_schedules(r->args))
        return fail(ctx, PRRTC_E_ARG, "schedule must be -2, -1, 0 or 1 (2 or 3 with coarse spheres)");
    if (set == -2) adopt_tuned_schedule(ctx, robot_id, scene_id);
    auto& m = ctx->scenes[scene_id].edge_schedule;
    if (set >= 0) m[robot_id] = set;
    if (set == -1) {   // timed again by the next large batch
        m.erase(robot_id);
        ctx->tuning.erase(edge_tuning_key(ctx, robot_id, scene_id));
    }
    if (schedule) {
        auto it = m.find(robot_id);
        *schedule = it == m.end() ? -1 : it->second;
    }
    return PRRTC_OK;
}

prrtc_status prrtc_fk_spheres(prrtc_ctx* ctx, int32_t robot_id, const float* q, int64_t n, float* xyz,
                              void* stream) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    const RobotRec* r = nullptr;
    prrtc_status st = lookup(ctx, robot_id, 0, &r, nullptr);
    if (st != PRRTC_OK) return st;
    if (n < 0) return fail(ctx, PRRTC_E_ARG, "n < 0");
    if (n == 0) return PRRTC_OK;
    if (!q || !xyz) return fail(ctx, PRRTC_E_ARG, "null buffer");
    hipStream_t sm = stream_of(ctx, stream);
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    const long long blocks = (n + kFkPerBlock - 1) / kFkPerBlock;
    if (blocks > 0x7fffffffLL) return fail(ctx, PRRTC_E_ARG, "n too large for one launch");
    const size_t lds = sizeof(float4) * kFkPerBlock * 3 * r->args.n_frames;
    hipLaunchKernelGGL(k_fk_spheres, dim3((unsigned)blocks), dim3(kWave), lds, sm, r->args, q, (long long)n, xyz);
    PRRTC_HIP(ctx, hipGetLastError());
    return PRRTC_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// plan
// ----------------------------------------------------------------------------
namespace {

// Planner launch shapes: the collision checks' FK tile (configurations per
// tile), items per lane and waves per worker.  Four waves sharing a
// 64-configuration tile cut the latency of a query's long connect checks; a
// one-wave worker with a 16-configuration tile needs a quarter of the LDS and
// a quarter of the waves, so more worker groups fit in batched launches.
#ifndef PRRTC_PLAN_WAVES
#define PRRTC_PLAN_WAVES 4
#endif
// kernel[1] / serve[1]: with the two-stage pass (robots with coarse spheres).
struct PlanShape {
    int tile, items, waves;
    const void* kernel[2];
    const void* serve[2];   // the persistent serving kernels of the same shape
};

const PlanShape* plan_shape(int tile) {
    static const PlanShape shapes[] = {
        {64, 6, PRRTC_PLAN_WAVES,
         {reinterpret_cast<const void*>(&k_plan<64, 6, PRRTC_PLAN_WAVES, 2, false>),
          reinterpret_cast<const void*>(&k_plan<64, 6, PRRTC_PLAN_WAVES, 2, true>)},
         {reinterpret_cast<const void*>(&k_serve<64, 6, PRRTC_PLAN_WAVES, 2, false>),
          reinterpret_cast<const void*>(&k_serve<64, 6, PRRTC_PLAN_WAVES, 2, true>)}},
        {16, 3, 1,
         {reinterpret_cast<const void*>(&k_plan<16, 3, 1, 3, false>),
          reinterpret_cast<const void*>(&k_plan<16, 3, 1, 3, true>)},
         {reinterpret_cast<const void*>(&k_serve<16, 3, 1, 3, false>),
          reinterpret_cast<const void*>(&k_serve<16, 3, 1, 3, true>)}},
    };
    if (tile == 0) return &shapes[0];
    for (const PlanShape& sh : shapes)
        if (sh.tile == tile) return &sh;
    return nullptr;
}

// Single plans of tile 64 (or the default) run workers of eight waves when
// all of them can be resident (up to one workgroup per CU), else the
// four-wave shape above.  Eight waves split a check's FK tile and item blocks
// and the nearest-neighbour scans twice as finely: on the dual arm in the
// shelf the median query takes 17% less time (its slowest 1% about 8% more).
// Results do not depend on the shape.
const PlanShape* plan_shape_wide() {
    static const PlanShape wide = {64, 6, 8,
                                   {reinterpret_cast<const void*>(&k_plan<64, 6, 8, 2, false>),
                                    reinterpret_cast<const void*>(&k_plan<64, 6, 8, 2, true>)},
                                   {nullptr, nullptr}};
    return &wide;
}


GroupLayout group_layout(int dof, int cap, int W, int stage_cap) {
    GroupLayout L{};
    size_t o = 0;
    auto take = [&](size_t n) { const size_t at = o; o = align_up<int>(o + n); return at; };
    const int path_cap = 2 * cap;
    L.qa = take(sizeof(float) * (size_t)dof * cap);
    L.pa = take(sizeof(int) * (size_t)cap);
    L.ba = take((size_t)cap);
    L.ra = take(sizeof(float) * (size_t)cap);
    L.qb = take(sizeof(float) * (size_t)dof * cap);
    L.pb = take(sizeof(int) * (size_t)cap);
    L.bb = take((size_t)cap);
    L.rb = take(sizeof(float) * (size_t)cap);
    L.bar = take(sizeof(int) * ((size_t)kBarWords + W));
    L.stage = take(sizeof(float) * 2 * (size_t)W * stage_cap * dof);   // two round parities
    L.st = take(sizeof(int) * 2 * 5 * (size_t)W);
    L.path = take(sizeof(float) * (size_t)path_cap * dof);
    L.path_idx = take(sizeof(int) * (size_t)path_cap);
    L.bytes = o;
    return L;
}

void group_args(PlanArgs& A, char* m, const GroupLayout& L, int W, int cap) {
    A.qa = reinterpret_cast<float*>(m + L.qa);
    A.pa = reinterpret_cast<int*>(m + L.pa);
    A.ba = reinterpret_cast<unsigned char*>(m + L.ba);
    A.ra = reinterpret_cast<float*>(m + L.ra);
    A.qb = reinterpret_cast<float*>(m + L.qb);
    A.pb = reinterpret_cast<int*>(m + L.pb);
    A.bb = reinterpret_cast<unsigned char*>(m + L.bb);
    A.rb = reinterpret_cast<float*>(m + L.rb);
    A.bar = reinterpret_cast<int*>(m + L.bar);
    A.stage = reinterpret_cast<float*>(m + L.stage);
    int* sti = reinterpret_cast<int*>(m + L.st);
    A.st_count = sti;
    A.st_nn = sti + W;
    A.st_other = sti + 2 * W;
    A.st_conn = sti + 3 * W;
    A.st_fail = sti + 4 * W;
    A.path = reinterpret_cast<float*>(m + L.path);
    A.path_idx = reinterpret_cast<int*>(m + L.path_idx);
    A.path_cap = 2 * cap;
}

// Longest greedy connect, ceil(|hi - lo| / delta) steps (+ margin for
// rounding); -1 if it exceeds the staging limit.
int stage_cap_for(const RobotArgs& RA, float delta) {
    double diag = 0.0;
    for (int j = 0; j < RA.dof; ++j) diag += (double)(RA.hi[j] - RA.lo[j]) * (double)(RA.hi[j] - RA.lo[j]);
    const int sc = (int)std::ceil(std::sqrt(diag) / (double)delta * (1.0 + 1e-6)) + 2;
    return sc > 4096 ? -1 : sc;
}

// Spheres, then the FK tile, query vectors and sub-edge tables; the tile's
// region also holds the input of a learned query's mixture before the rounds.
size_t plan_lds_bytes(const RobotArgs& RA, int stage_cap, int dof, int tile) {
    const size_t body = sizeof(float4) * tile * 3 * RA.n_slots +
                        sizeof(float) * (4 * kMaxDof + (size_t)(stage_cap + 1) * dof) +
                        sizeof(int) * (tile + 2 * (stage_cap + 2)) + two_stage_lds_bytes(RA, tile);
    return sphere_lds_bytes(RA) + std::max(body, sizeof(float) * kMlpInFloats);
}

prrtc_status check_plan_params(prrtc_ctx* ctx, const prrtc_plan_params& p) {
    if (p.workers < 1 || p.workers > 4096) return fail(ctx, PRRTC_E_ARG, "workers must be in 1..4096");
    if (!(p.delta > 0.0f) || !std::isfinite(p.delta)) return fail(ctx, PRRTC_E_ARG, "delta must be > 0");
    if (!(p.res > 0.0f) || !std::isfinite(p.res)) return fail(ctx, PRRTC_E_ARG, "res must be > 0");
    if (p.max_rounds < 0) return fail(ctx, PRRTC_E_ARG, "max_rounds < 0");
    if (p.tree_capacity < 2 || p.tree_capacity > (1 << 24))
        return fail(ctx, PRRTC_E_ARG, "tree_capacity must be in 2..2^24");
    if (p.validate_factor < 0 || p.validate_factor > 1024)
        return fail(ctx, PRRTC_E_ARG, "validate_factor must be in 0..1024");
    if (!(p.dds_radius >= 0.0f) || !std::isfinite(p.dds_radius))
        return fail(ctx, PRRTC_E_ARG, "dds_radius must be finite and >= 0");
    if (p.dds_tries < 1 || p.dds_tries > 64) return fail(ctx, PRRTC_E_ARG, "dds_tries must be in 1..64");
    if (p.sampler < 0 || p.sampler > 2) return fail(ctx, PRRTC_E_ARG, "sampler must be 0, 1 or 2");
    if (!plan_shape(p.tile)) return fail(ctx, PRRTC_E_ARG, "tile must be 0, 16 or 64");
    if (p.sampler == 1) {
        if (!(p.mix >= 0.0f && p.mix <= 1.0f)) return fail(ctx, PRRTC_E_ARG, "mix must be in [0, 1]");
        if (p.model_id < 0 || p.model_id >= (int32_t)ctx->models.size())
            return fail(ctx, PRRTC_E_STATE, "unknown model id %d", p.model_id);
    }
    return PRRTC_OK;
}

// Per-query fields of A (everything but the group buffers, ctl and out_path).
void query_args(prrtc_ctx* ctx, PlanArgs& A, const prrtc_plan_params& p, const RobotRec& r, const SceneRec& s,
                const float* start, const float* goal, uint64_t seed, uint32_t query, int stage_cap) {
    const int dof = r.dof;
    A.R = r.dev_args;
    A.S = s.dev_args;
    for (int j = 0; j < kMaxDof; ++j) {
        A.start[j] = j < dof ? start[j] : 0.0f;
        A.goal[j] = j < dof ? goal[j] : 0.0f;
    }
    A.seed = seed;
    A.query = query;
    A.W = p.workers;
    A.delta = p.delta;
    A.res = p.res;
    A.res_v = p.res * (float)p.validate_factor;
    A.max_rounds = p.max_rounds;
    A.cap = p.tree_capacity;
    A.stage_cap = stage_cap;
    A.validate = p.validate_factor;
    A.dds_radius = p.dds_radius;
    A.dds_tries = p.dds_tries;
    A.halton = p.sampler == 2;
    A.gmm = nullptr;
    A.model = nullptr;
    A.emb = nullptr;
    A.mix = p.mix;
    A.budget_ticks = p.time_budget_ms > 0.0f ? (long long)((double)p.time_budget_ms * ctx->wall_khz) : 0;
}

prrtc_status endpoints_ok(prrtc_ctx* ctx, const RobotArgs& RA, const float* start, const float* goal) {
    if (!finite_all(start, RA.dof) || !finite_all(goal, RA.dof))
        return fail(ctx, PRRTC_E_ARG, "start/goal not finite");
    for (int j = 0; j < RA.dof; ++j)
        if (!(start[j] >= RA.lo[j] && start[j] <= RA.hi[j] && goal[j] >= RA.lo[j] && goal[j] <= RA.hi[j]))
            return fail(ctx, PRRTC_E_INVALID_ENDPOINT, "start/goal joint %d outside the limits", j);
    return PRRTC_OK;
}

void fill_stats(const int* c, float ms, prrtc_plan_stats* st) {
    st->rounds = c[kRounds];
    st->nodes_a = c[kSizeA];
    st->nodes_b = c[kSizeB];
    st->edges_checked =
        (int64_t)((unsigned long long)(unsigned)c[kEdgesLo] | ((unsigned long long)(unsigned)c[kEdgesHi] << 32));
    st->validation_failures = c[kValFails];
    st->connect_worker = c[kStatus] == kStOk ? c[kConnWorker] : -1;
    st->gpu_ms = ms;
    st->fallback = c[kFallback];
    st->learned_samples =
        (int64_t)((unsigned long long)(unsigned)c[kLearnedLo] | ((unsigned long long)(unsigned)c[kLearnedHi] << 32));
}

prrtc_status status_of(int device_status) {
    switch (device_status) {
        case kStOk: return PRRTC_OK;
        case kStInvalidEndpoint: return PRRTC_E_INVALID_ENDPOINT;
        case kStNoSolution: return PRRTC_E_NO_SOLUTION;
        default: return PRRTC_E_HIP;
    }
}

// Mixture of the learned proposal for one (scene, start, goal): the scene's
// occupancy grid (made once per scene) and a batch-of-one forward pass, all
// enqueued on sm.  qin: device staging of [start | goal] and scene row 0.
prrtc_status plan_proposal(prrtc_ctx* ctx, int32_t model_id, const RobotRec& r, SceneRec& s, const float* start,
                           const float* goal, float* qin, float* gmm, hipStream_t sm);

// Device tables of a learned batched or served launch, where each worker
// group computes its query's mixture itself (mixture_in_block): the models'
// parameter pointers and the grid embedding of every (scene, model) pair of
// the given scenes and models, at offsets from one base.
LearnedLayout learned_layout(size_t base, int n_scenes, int n_models);
// Enqueue the tables on sm (the caller synchronises before the host vectors
// go out of scope): occupancy grids, then k_embed_partial / k_embed_reduce
// over up to kSmallRows scenes at a time -- the kernels and order of a single
// plan's cached embedding, so the mixtures equal a single plan's.
prrtc_status learned_tables(prrtc_ctx* ctx, hipStream_t sm, char* m, const LearnedLayout& L,
                            const std::vector<int>& scenes, const std::vector<int>& models,
                            std::vector<ModelDev>& host_mdev);

}  // namespace

extern "C" {

void prrtc_plan_params_default(prrtc_plan_params* p) {
    if (!p) return;
    p->seed = 1;
    p->query = 0;
    p->workers = 256;
    p->delta = 0.5f;
    p->res = 32.0f;
    p->max_rounds = 1000;
    p->tree_capacity = 65536;
    p->time_budget_ms = 0.0f;
    p->validate_factor = 4;
    p->dds_radius = 0.0f;
    p->dds_tries = 1;
    p->sampler = 0;
    p->model_id = -1;
    p->mix = 0.5f;
    p->tile = 0;
}

prrtc_status prrtc_plan(prrtc_ctx* ctx, int32_t robot_id, int32_t scene_id, const float* start,
                        const float* goal, const prrtc_plan_params* prm, float* path, int32_t path_cap,
                        int32_t* path_len, prrtc_plan_stats* stats) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (path_len) *path_len = 0;
    if (stats) memset(stats, 0, sizeof *stats);
    const RobotRec* r = nullptr;
    const SceneRec* s = nullptr;
    prrtc_status st = lookup(ctx, robot_id, scene_id, &r, &s);
    if (st != PRRTC_OK) return st;
    if (!start || !goal || !prm || !path_len) return fail(ctx, PRRTC_E_ARG, "null argument");
    if (path_cap < 0 || (path_cap > 0 && !path)) return fail(ctx, PRRTC_E_ARG, "bad path buffer");
    const prrtc_plan_params& p = *prm;
    st = check_plan_params(ctx, p);
    if (st != PRRTC_OK) return st;
    if (p.sampler == 1 && ctx->models[p.model_id].L.dof != r->dof)
        return fail(ctx, PRRTC_E_ARG, "model dof %d != robot dof %d", ctx->models[p.model_id].L.dof, r->dof);
    st = endpoints_ok(ctx, r->args, start, goal);
    if (st != PRRTC_OK) return st;
    const int dof = r->dof;
    const int stage_cap = stage_cap_for(r->args, p.delta);
    if (stage_cap < 0) return fail(ctx, PRRTC_E_ARG, "delta too small for the joint range");
    const int W = p.workers, cap = p.tree_capacity;
    const GroupLayout L = group_layout(dof, cap, W, stage_cap);
    // after the group: query words, the query's arguments, proposal staging
    // after the group: the query's words followed directly by its path (one
    // copy brings both back), its arguments, proposal staging
    const size_t o_ctl = L.bytes;
    const size_t o_out = o_ctl + sizeof(int) * kCtlWords;
    const size_t o_args = align_up<int>(o_out + sizeof(float) * (size_t)2 * cap * dof);
    const size_t o_qin = align_up<int>(o_args + sizeof(PlanArgs));
    const size_t o_gmm = align_up<int>(o_qin + sizeof(float) * 2 * kMaxDof + sizeof(int));
    const size_t bytes = align_up<int>(o_gmm + sizeof(float) * kComp * (1 + 2 * kMaxDof));
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    if (ctx->plan.bytes < bytes) {
        planner_free(ctx->plan);
        PRRTC_HIP(ctx, hipMalloc(&ctx->plan.mem, bytes));
        ctx->plan.bytes = bytes;
    }
    char* m = static_cast<char*>(ctx->plan.mem);
    PlanArgs A{};
    query_args(ctx, A, p, *r, *s, start, goal, p.seed, p.query, stage_cap);
    group_args(A, m, L, W, cap);
    A.ctl = reinterpret_cast<int*>(m + o_ctl);
    A.out_path = reinterpret_cast<float*>(m + o_out);
    A.out_path_cap = A.path_cap;
    PlanArgs* Pq = reinterpret_cast<PlanArgs*>(m + o_args);
    // the cooperative launch needs every worker resident at once (residency
    // cached per kernel and LDS size); the first shape that fits is taken
    const PlanShape* cands[2] = {plan_shape(p.tile), nullptr};
    if (p.tile == 0 || p.tile == 64) {
        cands[1] = cands[0];
        cands[0] = plan_shape_wide();
    }
    const int two = r->args.n_cmove > 0 ? 1 : 0;
    const PlanShape* chosen = nullptr;
    size_t lds = 0;
    int fit = 0;
    for (const PlanShape* c : cands) {
        if (!c) continue;
        const size_t l = plan_lds_bytes(r->args, stage_cap, dof, c->tile);
        int& per_cu = ctx->plan_per_cu[((uint64_t)c->waves << 48) | ((uint64_t)c->tile << 40) | ((uint64_t)two << 39) |
                                       (uint64_t)l];
        if (per_cu == 0)
            PRRTC_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, c->kernel[two], kWave * c->waves, l));
        fit = std::max(fit, per_cu * ctx->n_cu);
        if ((long long)per_cu * ctx->n_cu >= W) {
            chosen = c;
            lds = l;
            break;
        }
    }
    if (!chosen)
        return fail(ctx, PRRTC_E_CAPACITY, "%d workers do not fit on the device at once (%d with tile %d)", W, fit,
                    cands[1] ? cands[1]->tile : cands[0]->tile);
    const PlanShape& shape = *chosen;
    hipStream_t sm = ctx->stream;
    PRRTC_HIP(ctx, hipEventRecord(ctx->ev0, sm));
    if (p.sampler == 1) {
        float* gmm = reinterpret_cast<float*>(m + o_gmm);
        st = plan_proposal(ctx, p.model_id, *r, ctx->scenes[scene_id], start, goal,
                           reinterpret_cast<float*>(m + o_qin), gmm, sm);
        if (st != PRRTC_OK) return st;
        A.gmm = gmm;
    }
    const int bar_words = kBarWords + W;
    hipLaunchKernelGGL(k_plan_init, dim3((unsigned)((std::max(bar_words, 256) + 255) / 256)), dim3(256), 0, sm, A.bar,
                       1, bar_words, (size_t)0, A.ctl, 1, A, Pq, (int*)nullptr);
    PRRTC_HIP(ctx, hipGetLastError());
    int n_q = 1, n_g = 1;
    void* kargs[] = {&Pq, &n_q, &n_g};
    PRRTC_HIP(ctx, hipLaunchCooperativeKernel(shape.kernel[two], dim3(W), dim3(kWave * shape.waves), kargs,
                                              (unsigned)lds, sm));
    PRRTC_HIP(ctx, hipEventRecord(ctx->ev1, sm));
    // the words and the first nodes of the path in one copy to pinned memory
    const int prefix = std::min(std::min(path_cap, 2 * cap), (kPinnedFloats - kCtlWords) / dof);
    PRRTC_HIP(ctx, hipMemcpyAsync(ctx->pinned, A.ctl, sizeof(int) * kCtlWords + sizeof(float) * (size_t)prefix * dof,
                                  hipMemcpyDeviceToHost, sm));
    PRRTC_HIP(ctx, hipStreamSynchronize(sm));
    int ctl[kCtlWords];
    memcpy(ctl, ctx->pinned, sizeof ctl);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    if (stats) fill_stats(ctl, ms, stats);
    const int status = ctl[kStatus];
    if (status == kStInternal) {
        int code = 0;
        (void)hipMemcpy(&code, A.bar + kAbort, sizeof code, hipMemcpyDeviceToHost);
        return fail(ctx, PRRTC_E_HIP, "planner aborted on the device (%s)",
                    code == 1 ? "a group barrier waited more than 2 s"
                    : code == 2 ? "connect steps beyond the staging capacity"
                    : code == 3 ? "a parent chain longer than its tree" : "unknown cause");
    }
    if (status == kStInvalidEndpoint) return fail(ctx, PRRTC_E_INVALID_ENDPOINT, "start or goal in collision");
    if (status == kStNoSolution) return fail(ctx, PRRTC_E_NO_SOLUTION, "no connection within the round/time budget");
    const int len = ctl[kPathLen];
    *path_len = len;
    if (len > path_cap) return fail(ctx, PRRTC_E_CAPACITY, "path needs %d nodes, buffer holds %d", len, path_cap);
    if (len <= prefix) {
        memcpy(path, ctx->pinned + kCtlWords, sizeof(float) * (size_t)len * dof);
    } else {
        PRRTC_HIP(ctx, hipMemcpyAsync(path, A.out_path, sizeof(float) * (size_t)len * dof, hipMemcpyDeviceToHost, sm));
        PRRTC_HIP(ctx, hipStreamSynchronize(sm));
    }
    return PRRTC_OK;
}

namespace {

// The proposal model of a learned query (its own, else the parameters'),
// checked against its robot; -1 with *status set when it cannot be used.
int query_model(prrtc_ctx* ctx, const prrtc_query& q, const prrtc_plan_params& p, const RobotRec& r,
                int32_t* status) {
    const int m = q.model_id >= 0 ? q.model_id : p.model_id;
    if (m < 0 || m >= (int)ctx->models.size()) {
        *status = fail(ctx, PRRTC_E_STATE, "unknown model id %d", m);
        return -1;
    }
    if (ctx->models[m].L.dof != r.dof) {
        *status = fail(ctx, PRRTC_E_ARG, "model dof %d != robot dof %d", ctx->models[m].L.dof, r.dof);
        return -1;
    }
    return m;
}

}  // namespace

static prrtc_status plan_batch_impl(prrtc_ctx* ctx, const prrtc_query* queries, int32_t n,
                                    const prrtc_plan_params* prm, int32_t groups, int64_t memory_budget,
                                    float* paths, int32_t path_cap, prrtc_query_result* results,
                                    int32_t* groups_used) {
    if (records_errors(ctx)) ctx->err.clear();
    if (groups_used) *groups_used = 0;
    if (n < 0 || !prm || (n > 0 && (!queries || !results)) || path_cap < 0 || (path_cap > 0 && !paths) ||
        groups < 0 || memory_budget < 0)
        return fail(ctx, PRRTC_E_ARG, "bad batch arguments");
    if (n == 0) return PRRTC_OK;
    const prrtc_plan_params& p = *prm;
    prrtc_status st = check_plan_params(ctx, p);
    if (st != PRRTC_OK) return st;
    const int W = p.workers, cap = p.tree_capacity;
    // host-side checks per query; rejected queries are not launched
    std::vector<int> live;
    std::vector<int> model_of(n, -1);
    int dof_max = 1, stage_max = 1;
    size_t lds = 0;
    for (int k = 0; k < n; ++k) {
        prrtc_query_result& res = results[k];
        memset(&res, 0, sizeof res);
        const RobotRec* r = nullptr;
        const SceneRec* s = nullptr;
        res.status = lookup(ctx, queries[k].robot_id, queries[k].scene_id, &r, &s);
        if (res.status == PRRTC_OK) res.status = endpoints_ok(ctx, r->args, queries[k].start, queries[k].goal);
        if (res.status == PRRTC_OK && p.sampler == 1) {
            model_of[k] = query_model(ctx, queries[k], p, *r, &res.status);
        }
        int sc = 0;
        if (res.status == PRRTC_OK) {
            sc = stage_cap_for(r->args, p.delta);
            if (sc < 0) res.status = fail(ctx, PRRTC_E_ARG, "delta too small for the joint range");
        }
        if (res.status != PRRTC_OK) continue;
        live.push_back(k);
        dof_max = std::max(dof_max, r->dof);
        stage_max = std::max(stage_max, sc);
        lds = std::max(lds, plan_lds_bytes(r->args, sc, r->dof, plan_shape(p.tile)->tile));
    }
    if (records_errors(ctx)) ctx->err.clear();
    const int n_live = (int)live.size();
    if (n_live == 0) return PRRTC_OK;
    const GroupLayout L = group_layout(dof_max, cap, W, stage_max);
    // the two-stage kernel when any launched query's robot has coarse spheres
    int two = 0;
    for (int k : live) two |= ctx->robots[queries[k].robot_id].args.n_cmove > 0 ? 1 : 0;
    const void* kernel = plan_shape(p.tile)->kernel[two];
    // co-residency bound of the cooperative launch, then the memory budget
    int per_cu = 0;
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    PRRTC_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave * plan_shape(p.tile)->waves,
                                                                lds));
    const int g_resident = per_cu * ctx->n_cu / W;
    if (g_resident < 1) return fail(ctx, PRRTC_E_CAPACITY, "%d workers do not fit on the device at once", W);
    int G = groups > 0 ? groups : std::min(n_live, g_resident);
    if (G > g_resident) return fail(ctx, PRRTC_E_CAPACITY, "%d groups of %d workers exceed the %d resident",
                                    G, W, g_resident);
    G = std::min(G, n_live);
    const size_t per_query = align_up<int>(sizeof(int) * kCtlWords) + sizeof(PlanArgs) +
                             sizeof(float) * (size_t)path_cap * kMaxDof;
    if (memory_budget > 0) {
        const long long fit = (memory_budget - (long long)(per_query * n_live)) / (long long)L.bytes;
        if (fit < 1) return fail(ctx, PRRTC_E_CAPACITY, "memory budget below one worker group");
        G = (int)std::min<long long>(G, fit);
    }
    if (groups_used) *groups_used = G;
    // learned queries: the distinct scenes and models, whose embeddings the
    // groups start from
    std::vector<int> scenes_used, models_used, scene_row(n_live, -1), model_row(n_live, -1);
    if (p.sampler == 1) {
        auto row_of = [](std::vector<int>& v, int x) {
            for (size_t t = 0; t < v.size(); ++t)
                if (v[t] == x) return (int)t;
            v.push_back(x);
            return (int)v.size() - 1;
        };
        for (int i = 0; i < n_live; ++i) {
            scene_row[i] = row_of(scenes_used, queries[live[i]].scene_id);
            model_row[i] = row_of(models_used, model_of[live[i]]);
        }
    }
    // device memory: groups | query words | arguments | paths | learned tables | mixtures
    const int Cw = kComp * (1 + 2 * kMaxDof);
    const size_t o_ctl = (size_t)G * L.bytes;
    const size_t o_next = align_up<int>(o_ctl + sizeof(int) * kCtlWords * (size_t)n_live);
    const size_t o_args = align_up<int>(o_next + sizeof(int));
    const size_t o_path = align_up<int>(o_args + sizeof(PlanArgs) * (size_t)n_live);
    const size_t o_learn = align_up<int>(o_path + sizeof(float) * (size_t)path_cap * kMaxDof * n_live);
    const LearnedLayout LL = learned_layout(o_learn, (int)scenes_used.size(), (int)models_used.size());
    const size_t o_gmm = align_up<int>(LL.end);
    const size_t bytes = align_up<int>(o_gmm + (p.sampler == 1 ? sizeof(float) * Cw * (size_t)n_live : 0));
    if (ctx->batch.bytes < bytes) {
        planner_free(ctx->batch);
        PRRTC_HIP(ctx, hipMalloc(&ctx->batch.mem, bytes));
        ctx->batch.bytes = bytes;
    }
    char* m = static_cast<char*>(ctx->batch.mem);
    hipStream_t sm = ctx->stream;
    PRRTC_HIP(ctx, hipEventRecord(ctx->ev0, sm));
    float* gmm = reinterpret_cast<float*>(m + o_gmm);
    std::vector<ModelDev> host_mdev;
    if (p.sampler == 1) {
        st = learned_tables(ctx, sm, m, LL, scenes_used, models_used, host_mdev);
        if (st != PRRTC_OK) return st;
    }
    std::vector<PlanArgs> args(n_live);
    for (int i = 0; i < n_live; ++i) {
        const prrtc_query& q = queries[live[i]];
        const RobotRec& r = ctx->robots[q.robot_id];
        PlanArgs& A = args[i];
        query_args(ctx, A, p, r, ctx->scenes[q.scene_id], q.start, q.goal, q.seed, q.query,
                   stage_cap_for(r.args, p.delta));
        group_args(A, m, L, W, cap);   // group 0; the group that takes the query adds its offset
        A.group_bytes = L.bytes;
        A.next = reinterpret_cast<int*>(m + o_next);
        A.ctl = reinterpret_cast<int*>(m + o_ctl) + (size_t)kCtlWords * i;
        A.out_path = reinterpret_cast<float*>(m + o_path) + (size_t)path_cap * kMaxDof * i;
        A.out_path_cap = path_cap;
        if (p.sampler == 1) {
            A.gmm = gmm + (size_t)Cw * i;
            A.model = reinterpret_cast<const ModelDev*>(m + LL.mdev) + model_row[i];
            A.emb = reinterpret_cast<const float*>(m + LL.emb_at(scene_row[i], model_row[i]));
        }
    }
    PlanArgs* Pq = reinterpret_cast<PlanArgs*>(m + o_args);
    PRRTC_HIP(ctx, hipMemcpyAsync(Pq, args.data(), sizeof(PlanArgs) * n_live, hipMemcpyHostToDevice, sm));
    // every group's barrier words (blocks L.bytes apart) and every query's words
    const int bar_words = kBarWords + W;
    const int init_threads = std::max(bar_words * G, kCtlWords * n_live);
    hipLaunchKernelGGL(k_plan_init, dim3((unsigned)((init_threads + 255) / 256)), dim3(256), 0, sm, args[0].bar, G,
                       bar_words, L.bytes / sizeof(int), args[0].ctl, n_live, args[0], (PlanArgs*)nullptr,
                       args[0].next);
    PRRTC_HIP(ctx, hipGetLastError());
    int n_q = n_live, n_g = G;
    void* kargs[] = {&Pq, &n_q, &n_g};
    PRRTC_HIP(ctx, hipLaunchCooperativeKernel(kernel, dim3((unsigned)(G * W)),
                                              dim3(kWave * plan_shape(p.tile)->waves), kargs, (unsigned)lds, sm));
    PRRTC_HIP(ctx, hipEventRecord(ctx->ev1, sm));
    std::vector<int> ctl((size_t)kCtlWords * n_live);
    PRRTC_HIP(ctx, hipMemcpyAsync(ctl.data(), args[0].ctl, sizeof(int) * ctl.size(), hipMemcpyDeviceToHost, sm));
    PRRTC_HIP(ctx, hipStreamSynchronize(sm));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    // paths: one copy of the whole block when every query was launched (the
    // host and device layouts then agree), else one copy per solved query
    const bool bulk = n_live == n && n > 64 && path_cap > 0;
    if (bulk)
        PRRTC_HIP(ctx, hipMemcpyAsync(paths, m + o_path, sizeof(float) * (size_t)path_cap * kMaxDof * n,
                                      hipMemcpyDeviceToHost, sm));
    for (int i = 0; i < n_live; ++i) {
        const int* c = ctl.data() + (size_t)kCtlWords * i;
        prrtc_query_result& res = results[live[i]];
        fill_stats(c, ms, &res.stats);
        res.status = status_of(c[kStatus]);
        if (res.status == PRRTC_OK) {
            res.path_len = c[kPathLen];
            if (res.path_len > path_cap) {
                res.status = PRRTC_E_CAPACITY;
            } else if (!bulk) {
                const int dof = ctx->robots[queries[live[i]].robot_id].dof;
                PRRTC_HIP(ctx, hipMemcpyAsync(paths + (size_t)live[i] * path_cap * kMaxDof, args[i].out_path,
                                              sizeof(float) * (size_t)res.path_len * dof, hipMemcpyDeviceToHost, sm));
            }
        }
    }
    PRRTC_HIP(ctx, hipStreamSynchronize(sm));
    return PRRTC_OK;
}

prrtc_status prrtc_plan_batch(prrtc_ctx* ctx, const prrtc_query* queries, int32_t n,
                              const prrtc_plan_params* prm, int32_t groups, int64_t memory_budget,
                              float* paths, int32_t path_cap, prrtc_query_result* results,
                              int32_t* groups_used) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    return plan_batch_impl(ctx, queries, n, prm, groups, memory_budget, paths, path_cap, results, groups_used);
}

prrtc_status prrtc_tune_launch(prrtc_ctx* ctx, const prrtc_query* queries, int32_t n,
                               const prrtc_plan_params* params, const int32_t* workers, int32_t n_workers,
                               const int32_t* tiles, int32_t n_tiles, int64_t memory_budget, float* rates,
                               int32_t* best_workers, int32_t* best_tile) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (n < 1 || !queries || !params || !workers || n_workers < 1 || !tiles || n_tiles < 1 || !best_workers ||
        !best_tile || memory_budget < 0)
        return fail(ctx, PRRTC_E_ARG, "bad tuning arguments");
    for (int t = 0; t < n_tiles; ++t)
        if (!plan_shape(tiles[t])) return fail(ctx, PRRTC_E_ARG, "tile must be 0, 16 or 64");
    std::vector<prrtc_query_result> res(n);
    std::vector<float> path((size_t)n * kMaxDof);
    float best_rate = -1.0f;
    *best_workers = 0;
    *best_tile = 0;
    for (int c = 0; c < n_workers; ++c)
        for (int t = 0; t < n_tiles; ++t) {
            prrtc_plan_params p = *params;
            p.workers = workers[c];
            p.tile = tiles[t];
            const auto t0 = std::chrono::steady_clock::now();
            const prrtc_status st =
                plan_batch_impl(ctx, queries, n, &p, 0, memory_budget, path.data(), 1, res.data(), nullptr);
            const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            const float rate = st == PRRTC_OK ? (float)(n / sec) : 0.0f;   // a shape that cannot launch rates 0
            if (rates) rates[c * n_tiles + t] = rate;
            if (rate > best_rate) {
                best_rate = rate;
                *best_workers = workers[c];
                *best_tile = plan_shape(tiles[t])->tile;
            }
        }
    ctx->err.clear();
    if (best_rate <= 0.0f) return fail(ctx, PRRTC_E_CAPACITY, "no candidate could launch");
    ctx->tuning[launch_tuning_key(ctx, queries, n, workers, n_workers, tiles, n_tiles)] =
        std::to_string(*best_workers) + " " + std::to_string(*best_tile);
    return PRRTC_OK;
}

prrtc_status prrtc_tuned_launch(prrtc_ctx* ctx, const prrtc_query* queries, int32_t n, const int32_t* workers,
                                int32_t n_workers, const int32_t* tiles, int32_t n_tiles, int32_t* best_workers,
                                int32_t* best_tile) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    if (n < 1 || !queries || !workers || n_workers < 1 || !tiles || n_tiles < 1 || !best_workers || !best_tile)
        return fail(ctx, PRRTC_E_ARG, "bad tuning arguments");
    auto t = ctx->tuning.find(launch_tuning_key(ctx, queries, n, workers, n_workers, tiles, n_tiles));
    if (t == ctx->tuning.end()) return fail(ctx, PRRTC_E_STATE, "no tuning record for these queries and candidates");
    std::istringstream v(t->second);
    if (!(v >> *best_workers >> *best_tile)) return fail(ctx, PRRTC_E_STATE, "malformed tuning record");
    return PRRTC_OK;
}

prrtc_status prrtc_tuning_save(prrtc_ctx* ctx, const char* path) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    if (!path) return fail(ctx, PRRTC_E_ARG, "null path");
    std::ofstream f(path);
    if (!f) return fail(ctx, PRRTC_E_ARG, "cannot write %s", path);
    f << "# prrtc tuning records v1: key | value\n";
    for (const auto& kv : ctx->tuning) f << kv.first << " | " << kv.second << "\n";
    if (!f) return fail(ctx, PRRTC_E_ARG, "cannot write %s", path);
    return PRRTC_OK;
}

prrtc_status prrtc_tuning_load(prrtc_ctx* ctx, const char* path) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    if (!path) return fail(ctx, PRRTC_E_ARG, "null path");
    std::ifstream f(path);
    if (!f) return fail(ctx, PRRTC_E_ARG, "cannot read %s", path);
    std::string line;
    std::map<std::string, std::string> add;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        const size_t bar = line.find(" | ");
        if (bar == std::string::npos) return fail(ctx, PRRTC_E_ARG, "malformed tuning line: %s", line.c_str());
        add[line.substr(0, bar)] = line.substr(bar + 3);
    }
    for (const auto& kv : add) ctx->tuning[kv.first] = kv.second;
    return PRRTC_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Serving: a thread owned by the context gathers submitted queries into
// batched launches (continuous batching at launch granularity).
// ----------------------------------------------------------------------------
namespace {

void serve_loop(prrtc_ctx* ctx) {
    Server& S = *ctx->server;
    ctx->serve_tid.store(std::this_thread::get_id());
    (void)hipSetDevice(ctx->device);
    std::vector<prrtc_query> qs;
    std::vector<uint64_t> tickets;
    std::vector<prrtc_query_result> res;
    std::vector<float> paths;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S.mu);
            S.cv.wait(lk, [&] { return S.stop || !S.queue.empty(); });
            if (S.queue.empty()) return;   // stop requested and drained
            qs.clear();
            tickets.clear();
            while (!S.queue.empty() && (int)qs.size() < S.slots) {
                tickets.push_back(S.queue.front().first);
                qs.push_back(S.queue.front().second);
                S.queue.pop_front();
            }
            for (uint64_t t : tickets) S.running[t] = 1;
        }
        const int n = (int)qs.size();
        res.assign(n, prrtc_query_result{});
        paths.assign((size_t)n * S.path_cap * kMaxDof, 0.0f);
        const prrtc_status st = plan_batch_impl(ctx, qs.data(), n, &S.params, 0, S.budget, paths.data(), S.path_cap,
                                                res.data(), nullptr);
        std::lock_guard<std::mutex> lk(S.mu);
        for (int i = 0; i < n; ++i) {
            ServeDone d;
            d.res = res[i];
            if (st != PRRTC_OK) {
                d.res = prrtc_query_result{};
                d.res.status = st;
            }
            if (d.res.status == PRRTC_OK) {
                const int dof = ctx->robots[qs[i].robot_id].dof;
                const float* src = paths.data() + (size_t)i * S.path_cap * kMaxDof;
                d.path.assign(src, src + (size_t)d.res.path_len * dof);
            }
            S.done[tickets[i]] = std::move(d);
            S.running.erase(tickets[i]);
        }
        ++S.launches;
    }
}

// Persistent mode: one k_serve launch takes queries as they are published
// into the ring; results come back through host memory as each query ends.
// The launch closes once no group has claimed a query for kServeIdleMs
// (relaunched on the next submission) or, once the ring is used up, drains;
// the ring then starts again at slot 0 with the next launch.
constexpr double kServeIdleMs = 50.0;

void serve_result(prrtc_ctx* ctx, Server& S, uint64_t ticket, int k, const prrtc_query& q, double ms) {
    const int* c = S.host_ctl + (size_t)k * (kCtlWords + 1) + 1;
    ServeDone d;
    fill_stats(c, (float)ms, &d.res.stats);
    d.res.status = status_of(c[kStatus]);
    if (d.res.status == PRRTC_OK) {
        d.res.path_len = c[kPathLen];
        const int dof = ctx->robots[q.robot_id].dof;
        if (d.res.path_len > S.path_cap || (size_t)d.res.path_len * dof > (size_t)S.path_stride) {
            d.res.status = PRRTC_E_CAPACITY;
        } else {
            const float* src = S.host_path + (size_t)k * S.path_stride;
            d.path.assign(src, src + (size_t)d.res.path_len * dof);
        }
    }
    std::lock_guard<std::mutex> lk(S.mu);
    S.done[ticket] = std::move(d);
    S.running.erase(ticket);
}

void serve_loop_persistent(prrtc_ctx* ctx) {
    Server& S = *ctx->server;
    ctx->serve_tid.store(std::this_thread::get_id());
    (void)hipSetDevice(ctx->device);
    volatile int* published = S.host_ctrl;
    volatile int* drain = S.host_ctrl + 32;
    std::vector<uint64_t> ticket_of(S.ring);
    std::vector<prrtc_query> query_of(S.ring);
    std::vector<char> pending(S.ring, 0);
    std::vector<int> live;   // published slots whose result has not come back
    live.reserve(S.slots);
    std::vector<std::chrono::steady_clock::time_point> t_pub(S.ring);
    bool launched = false;
    int pub = 0, n_pending = 0;
    const prrtc_plan_params& p = S.params;
    const int bar_words = kBarWords + S.W;
    auto fail_pending = [&](prrtc_status st) {
        for (int k = 0; k < pub; ++k) {
            if (!pending[k]) continue;
            ServeDone d;
            d.res.status = st;
            std::lock_guard<std::mutex> lk(S.mu);
            S.done[ticket_of[k]] = std::move(d);
            S.running.erase(ticket_of[k]);
            pending[k] = 0;
        }
        n_pending = 0;
        live.clear();
    };
    for (;;) {
        bool busy = false;
        // 1. publish queued queries (host checks first; rejected ones answer at once)
        int pub0 = pub;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            if (!launched && S.queue.empty() && n_pending == 0) {
                if (S.stop) return;
                S.cv.wait_for(lk, std::chrono::milliseconds(5));
                if (S.queue.empty()) continue;
            }
            while (!S.queue.empty() && pub < S.ring && n_pending < S.slots && !(*drain && launched)) {
                const uint64_t t = S.queue.front().first;
                const prrtc_query q = S.queue.front().second;
                S.queue.pop_front();
                const RobotRec* r = nullptr;
                const SceneRec* sc = nullptr;
                prrtc_status st = lookup(ctx, q.robot_id, q.scene_id, &r, &sc);
                if (st == PRRTC_OK) st = endpoints_ok(ctx, r->args, q.start, q.goal);
                int stage_cap = 0;
                if (st == PRRTC_OK) {
                    stage_cap = stage_cap_for(r->args, p.delta);
                    if (stage_cap < 0) st = PRRTC_E_ARG;
                }
                int model = -1;
                if (st == PRRTC_OK && p.sampler == 1) {
                    int32_t mst = PRRTC_OK;
                    model = query_model(ctx, q, p, *r, &mst);
                    st = (prrtc_status)mst;
                }
                if (st != PRRTC_OK) {
                    ServeDone d;
                    d.res.status = st;
                    S.done[t] = std::move(d);
                    continue;
                }
                const int k = pub++;
                PlanArgs& A = S.host_args[k];
                A = PlanArgs{};
                query_args(ctx, A, p, *r, *sc, q.start, q.goal, q.seed, q.query, stage_cap);
                group_args(A, S.dev_groups, S.L, S.W, S.tree_cap);
                A.group_bytes = S.L.bytes;
                A.ctl = S.sa.dev_ctl + (size_t)k * kCtlWords;
                A.out_path = S.sa.dev_path + (size_t)k * S.path_stride;
                A.out_path_cap = S.path_stride / r->dof;
                if (p.sampler == 1) {
                    // the group computes the mixture (every model is a table row, by id)
                    A.gmm = S.dev_gmm + (size_t)k * kComp * (1 + 2 * kMaxDof);
                    A.model = reinterpret_cast<const ModelDev*>(S.ring_base + S.LL.mdev) + model;
                    A.emb = reinterpret_cast<const float*>(S.ring_base + S.LL.emb_at(S.scene_row[q.scene_id], model));
                }
                __atomic_store_n(S.host_ctl + (size_t)k * (kCtlWords + 1), 0, __ATOMIC_RELAXED);
                ticket_of[k] = t;
                query_of[k] = q;
                pending[k] = 1;
                live.push_back(k);
                t_pub[k] = std::chrono::steady_clock::now();
                ++n_pending;
                S.running[t] = 1;
            }
        }
        if (pub != pub0) {
            __atomic_store_n(published, pub, __ATOMIC_RELEASE);   // the arguments are written before
            busy = true;
        }
        // 2. a launch when work is waiting and none is running
        if (!launched && n_pending > 0) {
            *drain = 0;
            hipStream_t sm = ctx->stream;
            hipLaunchKernelGGL(k_plan_init, dim3((unsigned)((bar_words * S.groups + 255) / 256)), dim3(256), 0, sm,
                               reinterpret_cast<int*>(S.dev_groups + S.L.bar), S.groups, bar_words,
                               S.L.bytes / sizeof(int), (int*)nullptr, 0, PlanArgs{}, (PlanArgs*)nullptr, S.sa.next);
            void* kargs[] = {&S.dev_sa};
            hipError_t e = hipGetLastError();
            if (e == hipSuccess)
                e = hipLaunchCooperativeKernel(S.kernel, dim3((unsigned)(S.groups * S.W)),
                                               dim3(kWave * plan_shape(p.tile)->waves), kargs, (unsigned)S.lds, sm);
            if (e != hipSuccess) {
                fail_pending(PRRTC_E_HIP);
                pub = 0;
                continue;
            }
            launched = true;
            std::lock_guard<std::mutex> lk(S.mu);
            ++S.launches;
        }
        // 3. results of queries that have ended (only the live slots are scanned)
        for (size_t i = 0; i < live.size();) {
            const int k = live[i];
            if (__atomic_load_n(S.host_ctl + (size_t)k * (kCtlWords + 1), __ATOMIC_ACQUIRE) == 0) {
                ++i;
                continue;
            }
            const double ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_pub[k]).count();
            serve_result(ctx, S, ticket_of[k], k, query_of[k], ms);
            pending[k] = 0;
            --n_pending;
            live[i] = live.back();
            live.pop_back();
            busy = true;
        }
        // 4. the ring is used up, or the server stops: the launch drains
        bool stopping;
        {
            std::lock_guard<std::mutex> lk(S.mu);
            stopping = S.stop;
        }
        if (launched && (pub == S.ring || stopping)) *drain = 1;
        // 5. the launch has ended (idle, drained or aborted)
        if (launched && hipStreamQuery(ctx->stream) != hipErrorNotReady) {
            (void)hipStreamSynchronize(ctx->stream);
            for (int k : live)   // results that landed at the end
                if (pending[k] && __atomic_load_n(S.host_ctl + (size_t)k * (kCtlWords + 1), __ATOMIC_ACQUIRE)) {
                    serve_result(ctx, S, ticket_of[k], k, query_of[k], 0.0);
                    pending[k] = 0;
                    --n_pending;
                }
            // published after the groups had left (idle) or after an abort,
            // never claimed: queued again, in order, for the next launch
            int claimed = pub;
            if (hipMemcpy(&claimed, S.sa.next, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) claimed = pub;
            {
                std::lock_guard<std::mutex> lk(S.mu);
                for (int k = pub - 1; k >= std::max(claimed, 0); --k) {
                    if (!pending[k]) continue;
                    S.queue.emplace_front(ticket_of[k], query_of[k]);
                    S.running.erase(ticket_of[k]);
                    pending[k] = 0;
                    --n_pending;
                }
            }
            fail_pending(PRRTC_E_HIP);   // claimed by a group that aborted (as an aborted batch query)
            launched = false;
            pub = 0;
            __atomic_store_n(published, 0, __ATOMIC_RELEASE);
            busy = true;
        }
        if (!busy) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

#ifndef PRRTC_SERVE_PERSISTENT
#define PRRTC_SERVE_PERSISTENT 1   // servers run one persistent launch (0: launch-granular batches)
#endif
constexpr int kServeRingMax = 16384;  // queries per persistent launch before it drains (64 x slots, at most)

void serve_free_persistent(Server& S) {
    if (S.dev_mem) (void)hipFree(S.dev_mem);
    if (S.host_mem) (void)hipHostFree(S.host_mem);
    S.dev_mem = nullptr;
    S.host_mem = nullptr;
}

// Buffers and launch shape of the persistent mode.  Group buffers are sized
// for the largest robot loaded now (robots cannot be loaded while serving).
prrtc_status serve_setup_persistent(prrtc_ctx* ctx, Server& S) {
    const prrtc_plan_params& p = S.params;
    const PlanShape& shape = *plan_shape(p.tile);
    int dof_max = 0, stage_max = 1, two = 0;
    size_t lds = 0;
    for (const RobotRec& r : ctx->robots) {
        if (!r.dev_args) continue;
        const int sc = stage_cap_for(r.args, p.delta);
        if (sc < 0) return fail(ctx, PRRTC_E_ARG, "delta too small for a loaded robot's joint range");
        two |= r.args.n_cmove > 0 ? 1 : 0;
        dof_max = std::max(dof_max, r.dof);
        stage_max = std::max(stage_max, sc);
        lds = std::max(lds, plan_lds_bytes(r.args, sc, r.dof, shape.tile));
    }
    if (dof_max == 0) return fail(ctx, PRRTC_E_STATE, "load the robots before serving");
    S.W = p.workers;
    S.tree_cap = p.tree_capacity;
    S.L = group_layout(dof_max, p.tree_capacity, S.W, stage_max);
    S.lds = lds;
    S.kernel = shape.serve[two];
    S.path_stride = S.path_cap * dof_max;
    // ring entries: 64 x slots, at most kServeRingMax and about 256 MiB of
    // pinned host memory (arguments, words and path of each entry)
    const size_t entry = sizeof(PlanArgs) + sizeof(int) * (kCtlWords + 1) + sizeof(float) * S.path_stride;
    const int by_memory = (int)std::max<size_t>(32, (size_t(256) << 20) / entry);
    S.ring = std::min({kServeRingMax, std::max(32, 64 * S.slots), by_memory});
    int per_cu = 0;
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    PRRTC_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, S.kernel, kWave * shape.waves, lds));
    int G = per_cu * ctx->n_cu / S.W;
    if (G < 1) return fail(ctx, PRRTC_E_CAPACITY, "%d workers do not fit on the device at once", S.W);
    const size_t R = (size_t)S.ring;
    const size_t o_args = align_up<int>(0);
    const size_t o_ctl = align_up<int>(o_args + sizeof(PlanArgs) * R);
    const size_t o_path = align_up<int>(o_ctl + sizeof(int) * kCtlWords * R);
    const size_t o_next = align_up<int>(o_path + sizeof(float) * S.path_stride * R);
    const size_t o_sa = align_up<int>(o_next + 256);
    std::vector<int> scenes_used, models_used;
    if (p.sampler == 1) {
        S.scene_row.assign(ctx->scenes.size(), -1);
        for (size_t i = 0; i < ctx->scenes.size(); ++i)
            if (ctx->scenes[i].mem) {
                S.scene_row[i] = (int)scenes_used.size();
                scenes_used.push_back((int)i);
            }
        for (size_t i = 0; i < ctx->models.size(); ++i) models_used.push_back((int)i);
    }
    S.LL = learned_layout(align_up<int>(o_sa + sizeof(ServeArgs)), (int)scenes_used.size(), (int)models_used.size());
    const size_t o_gmm = align_up<int>(S.LL.end);
    const size_t ring_bytes =
        align_up<int>(o_gmm + (p.sampler == 1 ? sizeof(float) * kComp * (1 + 2 * kMaxDof) * R : 0));
    if (S.budget > 0) {
        const long long fit = (S.budget - (long long)ring_bytes) / (long long)S.L.bytes;
        if (fit < 1) return fail(ctx, PRRTC_E_CAPACITY, "memory budget below one worker group");
        G = (int)std::min<long long>(G, fit);
    }
    G = std::min(G, S.slots);
    S.groups = G;
    S.persistent = true;
    const size_t groups_bytes = align_up<int>((size_t)G * S.L.bytes);
    PRRTC_HIP(ctx, hipMalloc(&S.dev_mem, groups_bytes + ring_bytes));
    char* d = static_cast<char*>(S.dev_mem);
    S.dev_groups = d;
    char* dr = d + groups_bytes;
    const size_t h_args = 0;
    const size_t h_ctl = align_up<int>(h_args + sizeof(PlanArgs) * R);
    const size_t h_path = align_up<int>(h_ctl + sizeof(int) * (kCtlWords + 1) * R);
    const size_t h_ctrl = align_up<int>(h_path + sizeof(float) * S.path_stride * R);
    const size_t host_bytes = h_ctrl + 256;
    hipError_t e = hipHostMalloc(&S.host_mem, host_bytes, hipHostMallocCoherent);
    if (e != hipSuccess) {
        serve_free_persistent(S);
        return fail(ctx, PRRTC_E_HIP, "serving ring: %s", hipGetErrorString(e));
    }
    char* h = static_cast<char*>(S.host_mem);
    memset(h, 0, host_bytes);
    S.host_args = reinterpret_cast<PlanArgs*>(h + h_args);
    S.host_ctl = reinterpret_cast<int*>(h + h_ctl);
    S.host_path = reinterpret_cast<float*>(h + h_path);
    S.host_ctrl = reinterpret_cast<int*>(h + h_ctrl);
    ServeArgs& A = S.sa;
    A.host_args = S.host_args;
    A.dev_args = reinterpret_cast<PlanArgs*>(dr + o_args);
    A.dev_ctl = reinterpret_cast<int*>(dr + o_ctl);
    A.dev_path = reinterpret_cast<float*>(dr + o_path);
    A.host_ctl = S.host_ctl;
    A.host_path = S.host_path;
    A.published = S.host_ctrl;
    A.drain = S.host_ctrl + 32;
    A.next = reinterpret_cast<int*>(dr + o_next);
    A.bar0 = reinterpret_cast<int*>(d + S.L.bar);
    A.group_bytes = S.L.bytes;
    A.idle_ticks = (long long)(kServeIdleMs * ctx->wall_khz);
    A.cap = S.ring;
    A.W = S.W;
    A.path_stride = S.path_stride;
    S.dev_sa = reinterpret_cast<ServeArgs*>(dr + o_sa);
    e = hipMemcpy(S.dev_sa, &A, sizeof A, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        serve_free_persistent(S);
        return fail(ctx, PRRTC_E_HIP, "serving arguments: %s", hipGetErrorString(e));
    }
    S.ring_base = dr;
    if (p.sampler == 1) {
        // the LearnedLayout offsets count from the ring's base
        S.dev_gmm = reinterpret_cast<float*>(dr + o_gmm);
        std::vector<ModelDev> host_mdev;
        prrtc_status st = learned_tables(ctx, ctx->stream, dr, S.LL, scenes_used, models_used, host_mdev);
        if (st == PRRTC_OK && hipStreamSynchronize(ctx->stream) != hipSuccess)
            st = fail(ctx, PRRTC_E_HIP, "serving: grid embeddings failed");
        if (st != PRRTC_OK) {
            serve_free_persistent(S);
            return st;
        }
    }
    return PRRTC_OK;
}

void serve_shutdown(prrtc_ctx* ctx) {
    if (!ctx->server) return;
    {
        std::lock_guard<std::mutex> lk(ctx->server->mu);
        ctx->server->stop = true;
    }
    ctx->server->cv.notify_all();
    if (ctx->server->th.joinable()) ctx->server->th.join();
    Server& S = *ctx->server;
    if (S.persistent) {
        (void)hipStreamSynchronize(ctx->stream);   // the launch has drained before its buffers go
        serve_free_persistent(S);
    }
    ctx->server.reset();
    ctx->serve_tid.store(std::thread::id());
    ctx->serving.store(false);
}

}  // namespace

extern "C" {

prrtc_status prrtc_serve_start(prrtc_ctx* ctx, const prrtc_plan_params* params, int32_t slots, int32_t max_pending,
                               int64_t memory_budget, int32_t path_cap) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (!params || slots < 1 || slots > 65536 || max_pending < slots || memory_budget < 0 || path_cap < 1 ||
        path_cap > (1 << 20))
        return fail(ctx, PRRTC_E_ARG, "bad serving arguments");
    prrtc_status st = check_plan_params(ctx, *params);
    if (st != PRRTC_OK) return st;
    std::unique_ptr<Server> S(new Server());
    S->params = *params;
    S->slots = slots;
    S->max_pending = max_pending;
    S->budget = memory_budget;
    S->path_cap = path_cap;
    if (PRRTC_SERVE_PERSISTENT) {
        st = serve_setup_persistent(ctx, *S);
        if (st != PRRTC_OK) return st;
    }
    ctx->server = std::move(S);
    ctx->serving.store(true);
    try {
        ctx->server->th = std::thread(ctx->server->persistent ? serve_loop_persistent : serve_loop, ctx);
    } catch (...) {
        serve_free_persistent(*ctx->server);
        ctx->server.reset();
        ctx->serving.store(false);
        return fail(ctx, PRRTC_E_STATE, "cannot start the serving thread");
    }
    return PRRTC_OK;
}

prrtc_status prrtc_submit(prrtc_ctx* ctx, const prrtc_query* query, uint64_t* ticket) {
    if (!ctx || !query || !ticket) return PRRTC_E_ARG;
    if (!ctx->serving.load() || !ctx->server) return PRRTC_E_STATE;
    Server& S = *ctx->server;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        if ((int)S.in_flight() >= S.max_pending) return PRRTC_E_BUSY;
        *ticket = S.next_ticket++;
        S.queue.emplace_back(*ticket, *query);
    }
    S.cv.notify_one();
    return PRRTC_OK;
}

prrtc_status prrtc_poll(prrtc_ctx* ctx, uint64_t ticket, prrtc_query_result* result, float* path,
                        int32_t path_cap) {
    if (!ctx || !result || path_cap < 0 || (path_cap > 0 && !path)) return PRRTC_E_ARG;
    if (!ctx->serving.load() || !ctx->server) return PRRTC_E_STATE;
    Server& S = *ctx->server;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.done.find(ticket);
    if (it == S.done.end()) {
        if (S.running.count(ticket)) return PRRTC_E_BUSY;
        for (const auto& q : S.queue)
            if (q.first == ticket) return PRRTC_E_BUSY;
        return PRRTC_E_STATE;
    }
    *result = it->second.res;
    if (result->status == PRRTC_OK) {
        const int dof = (int)(it->second.path.size() / std::max(1, result->path_len));
        if (result->path_len > path_cap) return PRRTC_E_CAPACITY;   // kept: poll again with a larger buffer
        if (!it->second.path.empty()) memcpy(path, it->second.path.data(), sizeof(float) * it->second.path.size());
        (void)dof;
    }
    S.done.erase(it);
    return PRRTC_OK;
}

prrtc_status prrtc_serve_stop(prrtc_ctx* ctx, int64_t* launches) {
    if (!ctx) return PRRTC_E_ARG;
    if (!ctx->serving.load() || !ctx->server) return PRRTC_E_STATE;
    if (launches) {
        std::lock_guard<std::mutex> lk(ctx->server->mu);
        *launches = ctx->server->launches;
    }
    serve_shutdown(ctx);
    return PRRTC_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Learned sampling proposal: model storage, forward, training
// ----------------------------------------------------------------------------
struct PropWs {
    float *E, *dE, *X0, *dX0, *Z1, *H1, *Z2, *H2, *Z3, *H3, *O, *dO, *dZ, *dH, *qh, *nll, *part;
};

// Activations of prrtc_proposal_forward_noalloc, for callers that cannot
// allocate: a fixed device array sized for kNoAllocRows samples over
// kNoAllocScenes scenes at the largest DoF.  Each device keeps its own copy
// for the life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (scratch_address).
constexpr int kNoAllocRows = 256, kNoAllocScenes = 256;
constexpr size_t kNoAllocFloats =
    (size_t)kNoAllocScenes * kHidden +                               // E
    (size_t)kNoAllocRows * (2 * kMaxDof + kHidden) +                 // X0
    (size_t)6 * kNoAllocRows * kHidden +                             // Z1 H1 Z2 H2 Z3 H3
    (size_t)kNoAllocRows * kComp * (1 + 2 * kMaxDof) +               // O
    (size_t)kEmbedSlices * kSmallRows * kHidden;                     // partial embeddings
static_assert(kNoAllocScenes * kHidden % 64 == 0 && kNoAllocRows % 64 == 0 && kSmallRows * kHidden % 64 == 0,
              "every scratch region starts on a 256-byte boundary");
static __device__ __align__(256) float scratch[kNoAllocFloats];

namespace {

// Device address of `scratch` on `device`, which must be the current device.
// Looked up once per device and kept.
hipError_t scratch_address(int device, float** out) {
    static std::mutex mu;
    static std::unordered_map<int, float*> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        it = addr.emplace(device, static_cast<float*>(p)).first;
    }
    *out = it->second;
    return hipSuccess;
}

// The forward pass's buffers carved out of the scratch array (training-only
// buffers stay null: the forward kernels never touch them without a target).
// Nothing in them needs clearing: every kernel writes each value it later reads.
PropWs noalloc_workspace(float* base, int n, int S, int dof) {
    PropWs W{};
    float* p = base;
    W.E = p;
    p += (size_t)S * kHidden;
    W.X0 = p;
    p += (size_t)n * (2 * dof + kHidden);
    float** hid[6] = {&W.Z1, &W.H1, &W.Z2, &W.H2, &W.Z3, &W.H3};
    for (float** h : hid) {
        *h = p;
        p += (size_t)n * kHidden;
    }
    W.O = p;
    p += (size_t)n * kComp * (1 + 2 * dof);
    W.part = p;
    return W;
}

std::vector<ModelRec>& models_of(prrtc_ctx* ctx) { return ctx->models; }

prrtc_status prop_workspace(prrtc_ctx* ctx, ModelRec& M, int n, int S, PropWs& W) {
    const PropLayout& L = M.L;
    size_t o = 0;
    size_t offs[17];
    const size_t cnt[17] = {(size_t)S * kHidden, (size_t)S * kHidden, (size_t)n * L.D0, (size_t)n * L.D0,
                            (size_t)n * kHidden, (size_t)n * kHidden, (size_t)n * kHidden, (size_t)n * kHidden,
                            (size_t)n * kHidden, (size_t)n * kHidden, (size_t)n * L.Cw, (size_t)n * L.Cw,
                            (size_t)n * kHidden, (size_t)n * kHidden, (size_t)n * L.dof, (size_t)n,
                            (size_t)kEmbedSlices * kSmallRows * kHidden};
    for (int i = 0; i < 17; ++i) {
        offs[i] = o;
        o = align_up<int>(o + sizeof(float) * cnt[i]);
    }
    if (M.ws_bytes < o) {
        if (M.ws) (void)hipFree(M.ws);
        M.ws = nullptr;
        M.ws_bytes = 0;
        PRRTC_HIP(ctx, hipMalloc(&M.ws, o));
        M.ws_bytes = o;
    }
    char* b = static_cast<char*>(M.ws);
    float** f[17] = {&W.E, &W.dE, &W.X0, &W.dX0, &W.Z1, &W.H1, &W.Z2, &W.H2, &W.Z3, &W.H3, &W.O, &W.dO,
                     &W.dZ, &W.dH, &W.qh, &W.nll, &W.part};
    for (int i = 0; i < 17; ++i) *f[i] = reinterpret_cast<float*>(b + offs[i]);
    return PRRTC_OK;
}

inline unsigned blocks(size_t n, int t) { return (unsigned)((n + t - 1) / t); }

// With a partials buffer (part_floats floats), a product of fewer than 64
// output tiles and K >= 1024 is split along K (deterministic: the partials
// are added in order by k_split_sum).
template <typename TA, bool TA_, bool TB_, bool GELU>
void gemm(hipStream_t sm, const TA* A, int lda, const float* B, int ldb, const float* bias, float* C, float* Z,
          int ldc, int M, int N, int K, float* part = nullptr, size_t part_floats = 0) {
    dim3 grid(blocks(N, kGemmBN), blocks(M, kGemmBM));
    const int tiles = (int)(grid.x * grid.y);
    if (!GELU && part && tiles < 64 && K >= 1024 && ldc == N) {
        int ks = std::min<int>((128 + tiles - 1) / tiles, K / 256);
        ks = std::min<int>(ks, (int)(part_floats / ((size_t)M * N)));
        if (ks >= 2) {
            const int chunk = (int)((((K + ks - 1) / ks) + kGemmBK - 1) / kGemmBK * kGemmBK);
            ks = (K + chunk - 1) / chunk;
            hipLaunchKernelGGL((k_gemm_bf16<TA, TA_, TB_, false>), dim3(grid.x, grid.y, ks), dim3(256), 0, sm, A, lda,
                               B, ldb, nullptr, part, nullptr, ldc, M, N, K, chunk);
            hipLaunchKernelGGL(k_split_sum, dim3(blocks((size_t)M * N, 256)), dim3(256), 0, sm, part, ks, M, N, ldc,
                               bias, C);
            return;
        }
    }
    hipLaunchKernelGGL((k_gemm_bf16<TA, TA_, TB_, GELU>), grid, dim3(256), 0, sm, A, lda, B, ldb, bias, C, Z, ldc, M,
                       N, K, 0);
}

// Forward pass for n samples over S scenes; with q (training) also the NLL
// and the head gradient.  Returns the mixture in W.O.
void prop_forward(hipStream_t sm, ModelRec& M, const PropWs& W, const RobotArgs* R_dev, const uint8_t* vox, int S,
                  const int* scene_of, const float* s, const float* g, const float* q, int n, float* gmm_out) {
    const PropLayout& L = M.L;
    // the joint limits inside the device copy of the robot's arguments
    const char* rb = reinterpret_cast<const char*>(R_dev);
    const float* lo = reinterpret_cast<const float*>(rb + offsetof(RobotArgs, lo));
    const float* hi = reinterpret_cast<const float*>(rb + offsetof(RobotArgs, hi));
    if (!q && n <= kSmallRows && S <= kSmallRows) {
        // a few queries: split embedding and one workgroup per row
        hipLaunchKernelGGL(k_embed_partial, dim3(kEmbedSlices), dim3(256), 0, sm, vox, S, M.p(pWv), W.part);
        hipLaunchKernelGGL(k_embed_reduce, dim3(S), dim3(256), 0, sm, W.part, M.p(pbv), W.E);
        hipLaunchKernelGGL(k_mlp_rows, dim3(n), dim3(kRowThreads), 0, sm, s, g, scene_of, W.E, lo, hi, L.dof, M.p(pW1),
                           M.p(pb1), M.p(pW2), M.p(pb2), M.p(pW3), M.p(pb3), M.p(pW4), M.p(pb4), gmm_out);
        return;
    }
    // few scenes and K = 4096: split K, the partials in W.part
    gemm<uint8_t, false, false, false>(sm, vox, kVoxCells, M.p(pWv), kHidden, M.p(pbv), W.E, nullptr, kHidden, S,
                                       kHidden, kVoxCells, W.part, (size_t)kEmbedSlices * kSmallRows * kHidden);
    hipLaunchKernelGGL(k_build_x0, dim3(blocks((size_t)n * L.D0, 256)), dim3(256), 0, sm, s, g, q, scene_of, W.E,
                       lo, hi, n, L.dof, W.X0, W.qh);
    gemm<float, false, false, true>(sm, W.X0, L.D0, M.p(pW1), kHidden, M.p(pb1), W.H1, W.Z1, kHidden, n, kHidden, L.D0);
    gemm<float, false, false, true>(sm, W.H1, kHidden, M.p(pW2), kHidden, M.p(pb2), W.H2, W.Z2, kHidden, n, kHidden,
                                    kHidden);
    gemm<float, false, false, true>(sm, W.H2, kHidden, M.p(pW3), kHidden, M.p(pb3), W.H3, W.Z3, kHidden, n, kHidden,
                                    kHidden);
    gemm<float, false, false, false>(sm, W.H3, kHidden, M.p(pW4), L.Cw, M.p(pb4), W.O, nullptr, L.Cw, n, L.Cw,
                                     kHidden);
    hipLaunchKernelGGL(k_gmm_head, dim3(blocks(n, 128)), dim3(128), 0, sm, W.O, n, L.dof, q ? W.qh : nullptr,
                       gmm_out, W.nll, W.dO, 1.0f / (float)n);
}

void prop_backward(hipStream_t sm, ModelRec& M, const PropWs& W, const uint8_t* vox, int S, const int* scene_start,
                   int n) {
    const PropLayout& L = M.L;
    // head
    gemm<float, true, false, false>(sm, W.H3, kHidden, W.dO, L.Cw, nullptr, M.g(pW4), nullptr, L.Cw, kHidden, L.Cw, n);
    hipLaunchKernelGGL(k_col_sum, dim3(blocks(L.Cw, 64)), dim3(kColGroups * 64), 0, sm, W.dO, n, L.Cw, L.Cw, 0,
                       M.g(pb4));
    gemm<float, false, true, false>(sm, W.dO, L.Cw, M.p(pW4), L.Cw, nullptr, W.dH, nullptr, kHidden, n, kHidden, L.Cw);
    // hidden layers 3, 2
    const float* Zs[3] = {W.Z1, W.Z2, W.Z3};
    const float* Hin[3] = {W.X0, W.H1, W.H2};
    const int pw[3] = {pW1, pW2, pW3}, pb[3] = {pb1, pb2, pb3};
    for (int l = 2; l >= 0; --l) {
        hipLaunchKernelGGL(k_gelu_bwd, dim3(blocks((size_t)n * kHidden, 256)), dim3(256), 0, sm, W.dH, Zs[l], W.dZ,
                           n * kHidden);
        const int din = l == 0 ? L.D0 : kHidden;
        gemm<float, true, false, false>(sm, Hin[l], din, W.dZ, kHidden, nullptr, M.g(pw[l]), nullptr, kHidden, din,
                                        kHidden, n);
        hipLaunchKernelGGL(k_col_sum, dim3(blocks(kHidden, 64)), dim3(kColGroups * 64), 0, sm, W.dZ, n, kHidden, kHidden, 0,
                           M.g(pb[l]));
        float* dIn = l == 0 ? W.dX0 : W.dH;
        gemm<float, false, true, false>(sm, W.dZ, kHidden, M.p(pw[l]), kHidden, nullptr, dIn, nullptr, din, n, din,
                                        kHidden);
    }
    // embedding of the voxel grid
    hipLaunchKernelGGL(k_scene_sum, dim3(blocks((size_t)S * kHidden, 256)), dim3(256), 0, sm, W.dX0, L.D0, 2 * L.dof,
                       scene_start, S, W.dE);
    gemm<uint8_t, true, false, false>(sm, vox, kVoxCells, W.dE, kHidden, nullptr, M.g(pWv), nullptr, kHidden,
                                      kVoxCells, kHidden, S);
    hipLaunchKernelGGL(k_col_sum, dim3(blocks(kHidden, 64)), dim3(kColGroups * 64), 0, sm, W.dE, S, kHidden, kHidden, 0,
                       M.g(pbv));
}

prrtc_status plan_proposal(prrtc_ctx* ctx, int32_t model_id, const RobotRec& r, SceneRec& s, const float* start,
                           const float* goal, float* qin, float* gmm, hipStream_t sm) {
    ModelRec& M = ctx->models[model_id];
    const int dof = r.dof;
    if (!s.vox) {
        PRRTC_HIP(ctx, hipMalloc(&s.vox, kVoxCells));
        hipLaunchKernelGGL(k_voxelize, dim3(blocks(kVoxCells, 256)), dim3(256), 0, sm, s.args, s.vox);
    }
    PropWs W;
    prrtc_status st = prop_workspace(ctx, M, 1, 1, W);
    if (st != PRRTC_OK) return st;
    float* host = ctx->pinned;   // the plan synchronises before the staging is reused
    for (int j = 0; j < dof; ++j) {
        host[j] = start[j];
        host[dof + j] = goal[j];
    }
    const int zero = 0;
    memcpy(&host[2 * dof], &zero, sizeof zero);
    PRRTC_HIP(ctx, hipMemcpyAsync(qin, host, sizeof(float) * (2 * dof + 1), hipMemcpyHostToDevice, sm));
    // the grid's embedding depends on the scene and the parameters only: kept
    // per scene and recomputed when the model (or its parameters) change
    if (!s.emb) PRRTC_HIP(ctx, hipMalloc(&s.emb, sizeof(float) * kHidden));
    if (s.emb_stamp != M.stamp) {
        hipLaunchKernelGGL(k_embed_partial, dim3(kEmbedSlices), dim3(256), 0, sm, s.vox, 1, M.p(pWv), W.part);
        hipLaunchKernelGGL(k_embed_reduce, dim3(1), dim3(256), 0, sm, W.part, M.p(pbv), s.emb);
        s.emb_stamp = M.stamp;
    }
    const char* rb = reinterpret_cast<const char*>(r.dev_args);
    const float* lo = reinterpret_cast<const float*>(rb + offsetof(RobotArgs, lo));
    const float* hi = reinterpret_cast<const float*>(rb + offsetof(RobotArgs, hi));
    const PropLayout& L = M.L;
    hipLaunchKernelGGL(k_mlp_rows, dim3(1), dim3(kRowThreads), 0, sm, qin, qin + dof,
                       reinterpret_cast<const int*>(qin + 2 * dof), s.emb, lo, hi, L.dof, M.p(pW1), M.p(pb1),
                       M.p(pW2), M.p(pb2), M.p(pW3), M.p(pb3), M.p(pW4), M.p(pb4), gmm);
    PRRTC_HIP(ctx, hipGetLastError());
    return PRRTC_OK;
}

LearnedLayout learned_layout(size_t base, int n_scenes, int n_models) {
    LearnedLayout L;
    L.n_scenes = n_scenes;
    L.n_models = n_models;
    if (n_scenes == 0 || n_models == 0) {
        L.mdev = L.emb = L.vox = L.part = L.end = base;
        return L;
    }
    L.mdev = align_up<int>(base);
    L.emb = align_up<int>(L.mdev + sizeof(ModelDev) * (size_t)n_models);
    L.vox = align_up<int>(L.emb + sizeof(float) * kHidden * (size_t)n_scenes * n_models);
    L.part = align_up<int>(L.vox + (size_t)kVoxCells * n_scenes);
    L.end = align_up<int>(L.part + sizeof(float) * (size_t)kEmbedSlices * kSmallRows * kHidden);
    return L;
}

prrtc_status learned_tables(prrtc_ctx* ctx, hipStream_t sm, char* m, const LearnedLayout& L,
                            const std::vector<int>& scenes, const std::vector<int>& models,
                            std::vector<ModelDev>& host_mdev) {
    if (scenes.empty() || models.empty()) return PRRTC_OK;
    host_mdev.resize(models.size());
    for (size_t i = 0; i < models.size(); ++i) {
        ModelRec& M = ctx->models[models[i]];
        host_mdev[i] = ModelDev{M.p(pW1), M.p(pb1), M.p(pW2), M.p(pb2), M.p(pW3), M.p(pb3), M.p(pW4), M.p(pb4),
                                M.L.dof, 0};
    }
    PRRTC_HIP(ctx, hipMemcpyAsync(m + L.mdev, host_mdev.data(), sizeof(ModelDev) * host_mdev.size(),
                                  hipMemcpyHostToDevice, sm));
    uint8_t* vox = reinterpret_cast<uint8_t*>(m + L.vox);
    for (size_t si = 0; si < scenes.size(); ++si)
        hipLaunchKernelGGL(k_voxelize, dim3(blocks(kVoxCells, 256)), dim3(256), 0, sm, ctx->scenes[scenes[si]].args,
                           vox + si * kVoxCells);
    float* part = reinterpret_cast<float*>(m + L.part);
    for (size_t mi = 0; mi < models.size(); ++mi) {
        ModelRec& M = ctx->models[models[mi]];
        for (int s0 = 0; s0 < L.n_scenes; s0 += kSmallRows) {
            const int S = std::min(kSmallRows, L.n_scenes - s0);
            hipLaunchKernelGGL(k_embed_partial, dim3(kEmbedSlices), dim3(256), 0, sm, vox + (size_t)s0 * kVoxCells, S,
                               M.p(pWv), part);
            hipLaunchKernelGGL(k_embed_reduce, dim3(S), dim3(256), 0, sm, part, M.p(pbv),
                               reinterpret_cast<float*>(m + L.emb_at(s0, (int)mi)));
        }
    }
    PRRTC_HIP(ctx, hipGetLastError());
    return PRRTC_OK;
}

}  // namespace

extern "C" {

prrtc_status prrtc_load_proposal(prrtc_ctx* ctx, const void* blob, size_t bytes, int32_t* model_id) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (!blob || !model_id || bytes < sizeof(PropHeader)) return fail(ctx, PRRTC_E_ARG, "blob too small");
    PropHeader h;
    memcpy(&h, blob, sizeof h);
    if (h.magic != kPropMagic || h.version != kPropVersion) return fail(ctx, PRRTC_E_ARG, "not a proposal blob");
    if (h.hidden != kHidden || h.n_comp != kComp || h.vox != kVox || h.dof < 1 || h.dof > PRRTC_MAX_DOF)
        return fail(ctx, PRRTC_E_ARG, "unsupported proposal dimensions");
    ModelRec M;
    M.L = prop_layout(h.dof);
    const size_t n = M.n();
    const size_t need = sizeof(PropHeader) + sizeof(float) * n * (h.has_adam ? 3 : 1);
    if (bytes < need) return fail(ctx, PRRTC_E_ARG, "blob holds %zu bytes, needs %zu", bytes, need);
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    PRRTC_HIP(ctx, hipMalloc(&M.mem, sizeof(float) * n * 4));
    const char* src = static_cast<const char*>(blob) + sizeof(PropHeader);
    hipError_t e = hipMemcpy(M.mem, src, sizeof(float) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(M.mem + n, 0, sizeof(float) * n * 3);
    if (e == hipSuccess && h.has_adam)
        e = hipMemcpy(M.mem + 2 * n, src + sizeof(float) * n, sizeof(float) * n * 2, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(M.mem);
        return fail(ctx, PRRTC_E_HIP, "proposal upload: %s", hipGetErrorString(e));
    }
    M.adam_t = h.has_adam ? h.adam_t : 0;
    M.stamp = ++ctx->model_stamp;
    models_of(ctx).push_back(M);
    *model_id = (int32_t)models_of(ctx).size() - 1;
    return PRRTC_OK;
}

prrtc_status prrtc_save_proposal(prrtc_ctx* ctx, int32_t model_id, void* blob, size_t cap, size_t* bytes) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (model_id < 0 || model_id >= (int32_t)models_of(ctx).size())
        return fail(ctx, PRRTC_E_STATE, "unknown model id %d", model_id);
    if (!bytes) return fail(ctx, PRRTC_E_ARG, "null size");
    ModelRec& M = models_of(ctx)[model_id];
    const size_t n = M.n();
    *bytes = sizeof(PropHeader) + sizeof(float) * n * 3;
    if (!blob || cap < *bytes) return fail(ctx, PRRTC_E_CAPACITY, "blob needs %zu bytes", *bytes);
    PropHeader h{kPropMagic, kPropVersion, M.L.dof, kHidden, kComp, kVox, M.adam_t, 1, 0};
    memcpy(blob, &h, sizeof h);
    char* dst = static_cast<char*>(blob) + sizeof h;
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    PRRTC_HIP(ctx, hipDeviceSynchronize());
    PRRTC_HIP(ctx, hipMemcpy(dst, M.mem, sizeof(float) * n, hipMemcpyDeviceToHost));
    PRRTC_HIP(ctx, hipMemcpy(dst + sizeof(float) * n, M.mem + 2 * n, sizeof(float) * n * 2, hipMemcpyDeviceToHost));
    return PRRTC_OK;
}

prrtc_status prrtc_voxelize(prrtc_ctx* ctx, int32_t scene_id, uint8_t* vox, void* stream) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].mem)
        return fail(ctx, PRRTC_E_STATE, "unknown or unloaded scene id %d", scene_id);
    if (!vox) return fail(ctx, PRRTC_E_ARG, "null buffer");
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_voxelize, dim3(blocks(kVoxCells, 256)), dim3(256), 0, stream_of(ctx, stream),
                       ctx->scenes[scene_id].args, vox);
    PRRTC_HIP(ctx, hipGetLastError());
    return PRRTC_OK;
}

static prrtc_status prop_common(prrtc_ctx* ctx, int32_t model_id, int32_t robot_id, ModelRec** M,
                                const RobotArgs** R) {
    if (model_id < 0 || model_id >= (int32_t)models_of(ctx).size())
        return fail(ctx, PRRTC_E_STATE, "unknown model id %d", model_id);
    if (robot_id < 0 || robot_id >= (int32_t)ctx->robots.size())
        return fail(ctx, PRRTC_E_STATE, "unknown robot id %d", robot_id);
    *M = &models_of(ctx)[model_id];
    *R = &ctx->robots[robot_id].args;
    if ((*R)->dof != (*M)->L.dof) return fail(ctx, PRRTC_E_ARG, "model dof %d != robot dof %d", (*M)->L.dof, (*R)->dof);
    return PRRTC_OK;
}

prrtc_status prrtc_proposal_forward(prrtc_ctx* ctx, int32_t model_id, int32_t robot_id, const uint8_t* vox,
                                    int32_t n_scenes, const int32_t* scene_of, const float* start,
                                    const float* goal, int32_t n, float* gmm, void* stream) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    ModelRec* M;
    const RobotArgs* R;
    prrtc_status st = prop_common(ctx, model_id, robot_id, &M, &R);
    if (st != PRRTC_OK) return st;
    if (n < 0 || n_scenes < 1) return fail(ctx, PRRTC_E_ARG, "bad sizes");
    if (n == 0) return PRRTC_OK;
    if (!vox || !scene_of || !start || !goal || !gmm) return fail(ctx, PRRTC_E_ARG, "null buffer");
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t sm = stream_of(ctx, stream);
    PropWs W;
    st = prop_workspace(ctx, *M, n, n_scenes, W);
    if (st != PRRTC_OK) return st;
    prop_forward(sm, *M, W, ctx->robots[robot_id].dev_args, vox, n_scenes, scene_of, start, goal, nullptr, n, gmm);
    PRRTC_HIP(ctx, hipGetLastError());
    return PRRTC_OK;
}

prrtc_status prrtc_proposal_forward_noalloc(prrtc_ctx* ctx, int32_t model_id, int32_t robot_id, const uint8_t* vox,
                                            int32_t n_scenes, const int32_t* scene_of, const float* start,
                                            const float* goal, int32_t n, float* gmm, void* stream) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    ModelRec* M;
    const RobotArgs* R;
    prrtc_status st = prop_common(ctx, model_id, robot_id, &M, &R);
    if (st != PRRTC_OK) return st;
    if (n < 0 || n_scenes < 1) return fail(ctx, PRRTC_E_ARG, "bad sizes");
    if (n > kNoAllocRows || n_scenes > kNoAllocScenes)
        return fail(ctx, PRRTC_E_ARG, "%d samples over %d scenes exceed the static scratch (at most %d samples, %d scenes)",
                    n, n_scenes, kNoAllocRows, kNoAllocScenes);
    if (n == 0) return PRRTC_OK;
    if (!vox || !scene_of || !start || !goal || !gmm) return fail(ctx, PRRTC_E_ARG, "null buffer");
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    const PropWs W = noalloc_workspace(ctx->scratch, n, n_scenes, M->L.dof);
    prop_forward(stream_of(ctx, stream), *M, W, ctx->robots[robot_id].dev_args, vox, n_scenes, scene_of,
                 start, goal, nullptr, n, gmm);
    PRRTC_HIP(ctx, hipGetLastError());
    return PRRTC_OK;
}

prrtc_status prrtc_proposal_sample(prrtc_ctx* ctx, int32_t robot_id, const float* gmm, uint64_t seed,
                                   uint32_t query, uint32_t round, uint32_t attempt, int32_t n, float* q,
                                   uint8_t* inside, void* stream) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    if (robot_id < 0 || robot_id >= (int32_t)ctx->robots.size())
        return fail(ctx, PRRTC_E_STATE, "unknown robot id %d", robot_id);
    if (n < 0 || attempt > 0x7FFFFFu) return fail(ctx, PRRTC_E_ARG, "bad sizes");
    if (n == 0) return PRRTC_OK;
    if (!gmm || !q || !inside) return fail(ctx, PRRTC_E_ARG, "null buffer");
    const RobotRec& r = ctx->robots[robot_id];
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_gmm_sample, dim3((unsigned)n), dim3(kWave), 0, stream_of(ctx, stream), gmm,
                       r.dev_args, seed, query, round, attempt, n, q, inside);
    PRRTC_HIP(ctx, hipGetLastError());
    return PRRTC_OK;
}

prrtc_status prrtc_train_proposal(prrtc_ctx* ctx, int32_t model_id, int32_t robot_id, const prrtc_train_batch* b,
                                  float lr, float* loss, void* stream) {
    if (!ctx) return PRRTC_E_ARG;
    ctx->err.clear();
    PRRTC_NOT_SERVING(ctx);
    ModelRec* M;
    const RobotArgs* R;
    prrtc_status st = prop_common(ctx, model_id, robot_id, &M, &R);
    if (st != PRRTC_OK) return st;
    if (!b || b->n < 1 || b->n_scenes < 1 || !b->vox || !b->scene_start || !b->scene_of || !b->start || !b->goal ||
        !b->waypoint || !loss)
        return fail(ctx, PRRTC_E_ARG, "bad training batch");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(ctx, PRRTC_E_ARG, "lr must be > 0");
    PRRTC_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t sm = stream_of(ctx, stream);
    PropWs W;
    st = prop_workspace(ctx, *M, b->n, b->n_scenes, W);
    if (st != PRRTC_OK) return st;
    prop_forward(sm, *M, W, ctx->robots[robot_id].dev_args, b->vox, b->n_scenes, b->scene_of, b->start, b->goal, b->waypoint, b->n, nullptr);
    prop_backward(sm, *M, W, b->vox, b->n_scenes, b->scene_start, b->n);
    hipLaunchKernelGGL(k_mean, dim3(1), dim3(kWave), 0, sm, W.nll, b->n, loss);
    M->adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)M->adam_t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)M->adam_t)));
    const size_t n = M->n();
    hipLaunchKernelGGL(k_adam, dim3(blocks(n, 256)), dim3(256), 0, sm, M->mem, M->mem + n, M->mem + 2 * n,
                       M->mem + 3 * n, n, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    PRRTC_HIP(ctx, hipGetLastError());
    M->stamp = ++ctx->model_stamp;
    return PRRTC_OK;
}

}  // extern "C"
