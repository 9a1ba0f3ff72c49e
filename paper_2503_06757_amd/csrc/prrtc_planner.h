// prrtc_planner.h -- persistent round-synchronous RRT-Connect (Alg. 1) on gfx950.
//
// One workgroup of one wavefront per parallel worker (the paper's "block");
// all workers stay resident for the whole query and meet at grid barriers.
// A round is:
//   A. every worker, against the same snapshot of both trees: RANDOM_CONFIG
//      (Philox), NEAREST_NEIGHBOR in the smaller tree (wave argmin), steer
//      by at most delta, check the edge (points i = 1..n), then greedy
//      CONNECT toward the nearest node of the other tree (all equal steps
//      checked together, the longest valid prefix kept).  New nodes are
//      staged per worker.
//   -- barrier --
//   B. every worker scans the staged counts, appends its own nodes at its
//      prefix offset (deterministic node ids), and all agree on the lowest
//      connected worker.
//   -- barrier --
//   C. (only when a connection exists) the path is extracted and each
//      segment re-checked at validate_factor x res by the workers in
//      parallel; an offending node is blocked and the rounds go on.
// The paper's blocks insert asynchronously with atomics; rounds trade that
// for reproducibility: a seed fixes the trees and the path.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "prrtc_device.h"
#include "prrtc_proposal.h"

namespace prrtc {

// Barrier words (int32) of one worker group in device memory, zeroed before
// each launch: arrival counter, generation and the group's sticky abort word
// on separate cache lines; kNext holds the query the group takes next.
enum Bar { kBarCount = 0, kBarGen = 32, kAbort = 64, kNext = 72, kBarWords = 96 };

// Control and result words (int32) of one query, set up before each launch
// (status = internal error, everything else 0).
enum Ctl {
    kSizeA = 0,
    kSizeB,
    kStatus,
    kPathLen,
    kRounds,
    kConnWorker,
    kValFails,
    kStop,
    kEndpointBad,
    kValBad,
    kNa,
    kFallback,         // 1: the mixture was not finite, uniform sampling used
    kEdgesLo,          // 64-bit edge counter (two words)
    kEdgesHi,
    kLearnedLo,        // 64-bit count of draws taken from the learned mixture
    kLearnedHi,
    kCtlWords = 32
};
static_assert(kEdgesLo % 2 == 0 && kLearnedLo % 2 == 0, "64-bit counters need 8-byte alignment");

// The final re-check splits every path segment's points into this many
// chunks, checked by different workers.
constexpr int kValChunks = 4;

// Status codes written by the kernel (mirror prrtc_status).
constexpr int kStOk = 0, kStNoSolution = -5, kStInvalidEndpoint = -4, kStInternal = -7;

// One query of a launch.  Trees, staging, path and barrier words belong to
// the worker group that runs the query (the pointers name group 0's memory;
// group g adds g * group_bytes); ctl and out_path belong to the query.
struct alignas(64) PlanArgs {   // whole cache lines: a slot never shares one with its neighbour
    const RobotArgs* R;       // device copies of the robot and scene tables
    const SceneArgs* S;
    float start[kMaxDof], goal[kMaxDof];
    unsigned long long seed;
    unsigned int query;
    int W;
    float delta, res, res_v;
    int max_rounds, cap, stage_cap, validate;
    float dds_radius;         // dynamic-domain radius after a failed extension (0: off)
    int dds_tries;            // samples per worker and round
    int halton;               // 1: RANDOM_CONFIG from Halton points instead of Philox draws
    const float* gmm;         // learned mixture [K (1 + 2 dof)] or null (uniform sampling)
    const ModelDev* model;    // non-null: the group computes the mixture into gmm itself
    const float* emb;         //   from this grid embedding [kHidden] of the scene
    float mix;                // probability of drawing from the mixture
    long long budget_ticks;   // <= 0: none
    float* qa; int* pa; unsigned char* ba; float* ra;
    float* qb; int* pb; unsigned char* bb; float* rb;
    int* bar;                 // group barrier words [kBarWords + W] (generation, abort, per-worker flags)
    int* ctl;                 // query words [kCtlWords]
    float* stage;             // [W][stage_cap][dof]
    int* st_count; int* st_nn; int* st_other; int* st_conn; int* st_fail;
    float* path;              // [path_cap][dof]
    int* path_idx;            // [path_cap] tree node index; tree = (k < na ? A : B)
    int path_cap;
    float* out_path;          // [out_path_cap][dof]: the query's path
    int out_path_cap;
    unsigned long long group_bytes;  // group g's memory = the pointers above + g * group_bytes
    int* next;                // launch-wide count of queries handed out (several queries per group)
};
static_assert(sizeof(PlanArgs) % sizeof(int) == 0 && sizeof(PlanArgs) <= 256 * sizeof(int),
              "k_plan_init copies PlanArgs with one block of 256 threads");

// Device memory owned by a context for planner launches (grown on demand).
struct PlannerBuffers {
    void* mem = nullptr;
    size_t bytes = 0;
};

inline void planner_free(PlannerBuffers& b) {
    if (b.mem) (void)hipFree(b.mem);
    b.mem = nullptr;
    b.bytes = 0;
}

// ----------------------------------------------------------------------------
// Grid barrier with a bounded wait.  Arrival counter + generation word; the
// generation is read before arriving, so a late reader cannot miss a release.
// A wait longer than ~2 s (the GPU wall clock) raises the abort word, and
// every workgroup leaves its round loop on abort, so the grid always drains.
// ----------------------------------------------------------------------------
__device__ inline bool grid_barrier(int* bar, int nblocks) {
    __shared__ int ok_s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned* cnt = reinterpret_cast<unsigned*>(bar + kBarCount);
        unsigned* gen = reinterpret_cast<unsigned*>(bar + kBarGen);
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned arrived = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == (unsigned)nblocks - 1u) {
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const unsigned long long t0 = wall_clock64();
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (__hip_atomic_load(bar + kAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() - t0 > 200000000ull) {  // 2 s at the 100 MHz wall clock
                    __hip_atomic_store(bar + kAbort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // pairs with the release that ended the wait
        __threadfence();
        if (__hip_atomic_load(bar + kAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        ok_s = ok;
    }
    __syncthreads();
    return ok_s != 0;
}

// Group barrier without a shared counter: every workgroup w > 0 publishes its
// arrival by storing the next generation number into its own flag word
// (flags = bar + kBarWords, one int per worker) and then waits for the
// generation word to advance; the first wave of workgroup 0 polls all flags
// and advances the generation once every flag shows it.  Release stores and
// acquire loads at agent scope carry each workgroup's earlier writes through
// workgroup 0 to everyone.  Flags and generation only grow, so nothing is
// reset between barriers, queries or rounds.  Waits are bounded as above.
// Waiting loops read with relaxed loads and take one acquire fence after the
// value they wait for appears: an acquire load in the loop would invalidate
// the caches on every poll, slowing the waiter and every wave sharing them.
#ifndef PRRTC_FLAG_BARRIER
#define PRRTC_FLAG_BARRIER 1
#endif
//
// With `next`, the barrier also hands out work: once every worker has
// arrived, workgroup 0 takes the next query index from the launch-wide
// counter and stores it in bar[kNext] before the release, so every worker
// reads the same index after the barrier.
//
// With `act`, the first wave of workgroup 0 runs act() (all its lanes) once
// every worker has arrived and before the release, so whatever act writes is
// visible to every worker after the barrier.
struct NoAct {
    __device__ void operator()() const {}
};

template <class Act = NoAct>
__device__ inline bool group_barrier(int* bar, int w, int nblocks, int* next = nullptr, const Act& act = Act()) {
#if PRRTC_FLAG_BARRIER
    __shared__ int ok_s;
    __syncthreads();
    unsigned* gen = reinterpret_cast<unsigned*>(bar + kBarGen);
    unsigned* flags = reinterpret_cast<unsigned*>(bar + kBarWords);
    int ok = 1;
    if (w == 0 && threadIdx.x < kWave) {
        // only wave 0 of workgroup 0 polls and releases: a second wave that
        // read the generation after the release would wait for the next one
        const int lane = threadIdx.x & (kWave - 1);
        // the group's current generation (workgroup 0 wrote it last; a
        // relaxed load of the same word returns it)
        const unsigned g = __shfl(lane == 0 ? __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u,
                                  0, kWave);
        const unsigned target = g + 1u;
        const unsigned long long t0 = wall_clock64();
        for (;;) {
            bool arrived = true;
            for (int i = 1 + lane; i < nblocks; i += kWave)
                arrived &= __hip_atomic_load(flags + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == target;
            if (__all(arrived)) break;
            __builtin_amdgcn_s_sleep(1);
            const bool abort = __hip_atomic_load(bar + kAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            const bool late = wall_clock64() - t0 > 200000000ull;   // 2 s at the 100 MHz wall clock
            if (abort || late) {
                if (late && threadIdx.x == 0) __hip_atomic_store(bar + kAbort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the flags' release stores happen before what follows
        if (ok) {
            act();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
        if (ok && threadIdx.x == 0) {
            if (next)
                __hip_atomic_store(bar + kNext,
                                   __hip_atomic_fetch_add(next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(gen, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (threadIdx.x == 0) {
        // the current generation: this workgroup saw the word reach it at the
        // end of the last barrier (or it is the launch's initial 0), and it
        // cannot advance before this workgroup arrives, so a relaxed load of
        // the same word returns it
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(flags + w, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long t0 = wall_clock64();
        while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
            __builtin_amdgcn_s_sleep(1);
            if (__hip_atomic_load(bar + kAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = 0;
                break;
            }
            if (wall_clock64() - t0 > 200000000ull) {
                __hip_atomic_store(bar + kAbort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // pairs with workgroup 0's release of gen
    }
    if (threadIdx.x == 0) {
        if (__hip_atomic_load(bar + kAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        ok_s = ok;
    }
    __syncthreads();
    return ok_s != 0;
#else
    if (next && w == 0 && threadIdx.x == 0)   // before arriving: nobody reads it until the release
        __hip_atomic_store(bar + kNext, __hip_atomic_fetch_add(next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!grid_barrier(bar, nblocks)) return false;
    if (std::is_same<Act, NoAct>::value) return true;
    if (w == 0 && threadIdx.x < kWave) act();   // everyone has arrived; a second barrier publishes it
    return grid_barrier(bar, nblocks);
#endif
}

// Nearest neighbour: the FP32 squared distance (in joint order, no FMA) to
// x, argmin over the non-blocked nodes of a tree, ties -> lowest index.  The
// scan keeps a per-lane best (distance, index, source); nearest_reduce makes
// it wave-wide.  source < 0: a node of the tree's [dof][cap] arrays; else the
// offset of a staged node's row in the staging buffers.
struct NearBest {
    float d;
    int i, src;
};

// Nodes 0..size-1 of the tree arrays.  Each lane takes U nodes per step and
// issues all their loads (D >= dof joints; the joints past dof load joint
// dof-1 and add an exact zero) before using any, so a step waits for one
// memory latency instead of one per joint and node.  Nodes are visited in
// increasing index order per lane and the strict compare keeps the first of
// equal distances.  With parts > 1 the caller's waves split the steps: wave
// `part` takes every parts-th one.
template <int D, int U>
__device__ inline void near_scan_t(const float* tq, const unsigned char* blocked, int cap, int size, const float* x,
                                   int dof, NearBest& b, int part, int parts) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & (kWave - 1);
    float xr[D];
#pragma unroll
    for (int j = 0; j < D; ++j) xr[j] = j < dof ? x[j] : 0.0f;
    for (int i0 = lane + part * kWave * U; i0 < size; i0 += kWave * U * parts) {
        float v[U][D];
        int idx[U];
        bool skip[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            idx[u] = i0 + u * kWave;
            const int ic = min(idx[u], size - 1);
            skip[u] = blocked[ic] != 0;
#pragma unroll
            for (int j = 0; j < D; ++j) v[u][j] = tq[(size_t)min(j, dof - 1) * cap + ic];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const float d = xr[j] - (j < dof ? v[u][j] : 0.0f);
                const float sq = d * d;
                s = s + sq;
            }
            if (idx[u] < size && !skip[u] && s < b.d) {
                b.d = s;
                b.i = idx[u];
                b.src = -1;
            }
        }
    }
}

__device__ inline void near_scan(const float* tq, const unsigned char* blocked, int cap, int size, const float* x,
                                 int dof, NearBest& b, int part = 0, int parts = 1) {
    if (dof <= 8)
        near_scan_t<8, 4>(tq, blocked, cap, size, x, dof, b, part, parts);
    else
        near_scan_t<kMaxDof, 2>(tq, blocked, cap, size, x, dof, b, part, parts);
}

// The previous round's staged nodes of a tree that are not yet guaranteed to
// be in its arrays: worker v's nodes k < cnt[v] are rows v stage_cap + k of
// `stage` ([.][dof]) with tree index first + (counts of workers < v) + k,
// kept below cap.  Lane l takes workers l, l + 64, ...; indices grow with
// the worker and k, and every one exceeds the tree-array indices, so the
// strict compare again keeps the lowest index of equal distances.  With
// parts > 1, wave `part` takes the nodes k = part, part + parts, ...
__device__ inline void near_scan_staged(const float* stage, int stage_cap, const int* cnt, int W, int first, int cap,
                                        const float* x, int dof, NearBest& b, int part = 0, int parts = 1) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & (kWave - 1);
    int running = first;
    for (int c0 = 0; c0 < W; c0 += kWave) {
        const int v = c0 + lane;
        const int c = v < W ? cnt[v] : 0;
        int incl = c;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int t = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += t;
        }
        const int base = running + incl - c;
        const int kept = max(0, min(c, cap - base));
        for (int k = part; k < kept; k += parts) {
            const float* row = stage + ((size_t)v * stage_cap + k) * dof;
            float s = 0.0f;
            for (int j = 0; j < dof; ++j) {
                const float d = x[j] - row[j];
                const float sq = d * d;
                s = s + sq;
            }
            if (s < b.d) {
                b.d = s;
                b.i = base + k;
                b.src = (int)(((size_t)v * stage_cap + k) * dof);
            }
        }
        running += __shfl(incl, kWave - 1, kWave);
    }
}

__device__ inline NearBest nearest_reduce(NearBest b) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float od = __shfl_xor(b.d, off, kWave);
        const int oi = __shfl_xor(b.i, off, kWave);
        const int os = __shfl_xor(b.src, off, kWave);
        if (od < b.d || (od == b.d && oi < b.i)) {
            b.d = od;
            b.i = oi;
            b.src = os;
        }
    }
    return b;
}

__device__ inline int wave_nearest(const float* tq, const unsigned char* blocked, int cap, int size,
                                   const float* x, int dof) {
    NearBest b{__builtin_inff(), 0x7fffffff, -1};
    near_scan(tq, blocked, cap, size, x, dof, b);
    b = nearest_reduce(b);
    return b.i == 0x7fffffff ? -1 : b.i;
}

// One query on the W workers of a group (worker w); false if the group
// aborted (a barrier timed out or an internal limit was hit).
// The query's arguments are read through the constant address space: they
// never change during the launch, so the compiler may reload them instead of
// keeping every field live in registers.
typedef __attribute__((address_space(4))) const PlanArgs CPlanArgs;

// A worker is a workgroup of NW waves: wave 0 ("lead") does the worker's
// scalar bookkeeping and writes its small LDS vectors; every wave computes the
// same samples, the waves split the nearest-neighbour scans and share the
// collision checks.
// The group's own memory: the query's group-0 pointers moved by goff bytes.
// Each pointer is formed where it is used (a scalar load and add), so the
// seventeen of them do not all stay live in registers.
template <class T>
__device__ inline T* moved(T* p, unsigned long long goff) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(p) + goff);
}

// The offset passes through an empty asm at every use, so the compiler does
// not hoist all the moved pointers out of the round loop (they would crowd
// out the scalar registers and spill).
__device__ inline unsigned long long opaque(unsigned long long v) {
    asm volatile("" : "+s"(v));
    return v;
}

struct GroupView {
    CPlanArgs& P;
    unsigned long long off_;
    __device__ unsigned long long off() const { return opaque(off_); }
    __device__ float* qa() const { return moved(P.qa, off()); }
    __device__ int* pa() const { return moved(P.pa, off()); }
    __device__ unsigned char* ba() const { return moved(P.ba, off()); }
    __device__ float* ra() const { return moved(P.ra, off()); }
    __device__ float* qb() const { return moved(P.qb, off()); }
    __device__ int* pb() const { return moved(P.pb, off()); }
    __device__ unsigned char* bb() const { return moved(P.bb, off()); }
    __device__ float* rb() const { return moved(P.rb, off()); }
    __device__ int* bar() const { return moved(P.bar, off()); }
    __device__ float* stage(int par, int dof) const {
        return moved(P.stage, off()) + (size_t)par * P.W * P.stage_cap * dof;
    }
    // per-round worker results and staged nodes, double-buffered by round
    // parity: [parity][count | nn | other | conn | fail][W] and
    // [parity][W][stage_cap][dof]
    __device__ int* st_count(int par) const { return moved(P.st_count, off()) + (size_t)par * 5 * P.W; }
    __device__ int* st_nn(int par) const { return moved(P.st_nn, off()) + (size_t)par * 5 * P.W; }
    __device__ int* st_other(int par) const { return moved(P.st_other, off()) + (size_t)par * 5 * P.W; }
    __device__ int* st_conn(int par) const { return moved(P.st_conn, off()) + (size_t)par * 5 * P.W; }
    __device__ int* st_fail(int par) const { return moved(P.st_fail, off()) + (size_t)par * 5 * P.W; }
    __device__ float* path() const { return moved(P.path, off()); }
    __device__ int* path_idx() const { return moved(P.path_idx, off()); }
};

template <int TP, int B, int NW, bool TWO>
__device__ __attribute__((always_inline)) bool plan_query(CPlanArgs& P, int w, float4* lds4,
                                                          unsigned long long goff) {
    const GroupView G{P, goff};
    const RobotArgs& R = *P.R;   // device memory: uniform reads are scalar loads
    const SceneArgs& S = *P.S;
    const int tid = threadIdx.x, nth = NW * kWave;
    const int lane = tid & (kWave - 1);
    const bool lead = tid < kWave;
    const int dof = R.dof;
    const int cap = P.cap;
    // ---- LDS carve-up
    float4* sph = lds4;
    int* slot3 = reinterpret_cast<int*>(sph + R.n_move);
    WaveWs ws;
    ws.frames = reinterpret_cast<float4*>(slot3 + ((R.n_move + 3) & ~3));
    ws.sph = sph;
    ws.slot3 = slot3;
    float* vec = reinterpret_cast<float*>(ws.frames + TP * 3 * R.n_slots);
    float* c_rand = vec;
    float* c_nn = vec + kMaxDof;
    float* c_new = vec + 2 * kMaxDof;
    float* c_nno = vec + 3 * kMaxDof;
    float* wp = vec + 4 * kMaxDof;                      // [(stage_cap + 1)][dof]
    ws.pk = reinterpret_cast<int*>(wp + (P.stage_cap + 1) * dof);
    ws.sub_n = ws.pk + TP;
    ws.sub_off = ws.sub_n + P.stage_cap + 2;
    two_stage_ws(R, TP, ws.sub_off + P.stage_cap + 2, ws);
    __shared__ int sh_i[8];
    __shared__ int sh_check[2];
    __shared__ NearBest sh_nb[NW];
    ws.shared = sh_check;
    int* ctl = P.ctl;
    long long my_edges = 0;
    long long my_learned = 0;
    __shared__ float gmm_s[kComp * (1 + 2 * kMaxDof)];

    // ---- prologue: roots, endpoint checks.  Every worker writes the roots
    // (the same values), so its own first round can read them without a
    // barrier; nothing else writes them before the first round's barrier.
    if (lead && lane < dof) {
        G.qa()[(size_t)lane * cap] = P.start[lane];
        G.qb()[(size_t)lane * cap] = P.goal[lane];
    }
    if (tid == 0) {
        G.pa()[0] = -1;
        G.pb()[0] = -1;
        G.ba()[0] = 0;
        G.bb()[0] = 0;
        G.ra()[0] = __builtin_inff();
        G.rb()[0] = __builtin_inff();
    }
    if (w == 0 && tid == 0) {
        ctl[kSizeA] = 1;
        ctl[kSizeB] = 1;
    }
    stage_spheres(R, sph, slot3);
    load_bounds(S, ws);
    const bool fixed_hit = static_collision(R, S);
    __syncthreads();
    const int n_end_workers = P.W > 1 ? 2 : 1;
    for (int e = w; e < 2; e += n_end_workers) {
        if (lead && lane < dof) {
            const float v = e == 0 ? P.start[lane] : P.goal[lane];
            wp[lane] = v;
            wp[dof + lane] = v;
        }
        __syncthreads();
        const bool ok = !fixed_hit && wave_check<TP, B, false, NW, false, TWO>(R, S, wp, 1, 0, P.res, ws) == 1;
        if (!ok && tid == 0) atomicOr(ctl + kEndpointBad, 1);
        __syncthreads();
    }
    // a learned query of a batched or served launch: one worker (not one of
    // the two endpoint checkers when there are more) computes the mixture
    // while the others check the endpoints; the LDS tile is free until the
    // barrier, and gmm_s serves as the layer output
    if (P.model && w == (P.W > 2 ? 2 : 0)) {
        __syncthreads();
        auto ends = [&](int c) { return c < dof ? P.start[c] : P.goal[c - dof]; };
        mixture_in_block(*P.model, P.emb, ends, R.lo, R.hi, reinterpret_cast<float*>(ws.frames), gmm_s,
                         const_cast<float*>(P.gmm));
    }
    // The endpoint verdict is read after the first barrier: the first round
    // runs meanwhile and is discarded if an endpoint collides.  Only a
    // mixture computed in this launch needs a barrier before the rounds.
    bool ends_checked = false;
    auto ends_bad = [&]() {
        ends_checked = true;
        if (__hip_atomic_load(ctl + kEndpointBad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return false;
        if (w == 0 && tid == 0) ctl[kStatus] = kStInvalidEndpoint;
        return true;
    };
    if (P.model) {
        if (!group_barrier(G.bar(), w, P.W)) return false;
        if (ends_bad()) return true;
    }
    bool use_gmm = false;
    if (P.gmm) {
        // atomic loads: vector loads from the coherent level (another
        // workgroup may have written the mixture in this launch)
        for (int t = tid; t < kComp * (1 + 2 * dof); t += nth)
            gmm_s[t] = __hip_atomic_load(P.gmm + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        use_gmm = gmm_finite(gmm_s, dof);
        if (!use_gmm && w == 0 && tid == 0) ctl[kFallback] = 1;
    }
    const unsigned long long t_start = wall_clock64();
    int status = kStNoSolution;
    int round = 0;
    // One group barrier per round.  A round's nodes are copied into the tree
    // arrays after its barrier, by their own workers, while faster workers may
    // already run the next round; that copy is only guaranteed visible after
    // the next round's barrier.  So every worker tracks the sizes itself, and
    // the next round reads the previous round's nodes (indices lr_first..) of
    // the tree that grew (lr_tree: 0 = A, 1 = B, -1 = none pending) from the
    // staging buffers, which are double-buffered by round parity.  Domain
    // shrinks of the previous round (its workers' failed extension starts,
    // lr_fail_tree) are taken from its fail words for the same reason.
    int na = 1, nb = 1;
    int lr_tree = -1, lr_first = 0, lr_fail_tree = -1;
    int par = 0;
    for (; round < P.max_rounds; ++round) {
        const bool s_is_a = na <= nb;
        const int ts = s_is_a ? 0 : 1;
        // arrays part (visible) and staged part of each tree
        const int vis_a = lr_tree == 0 ? lr_first : na, vis_b = lr_tree == 1 ? lr_first : nb;
        const int vis_s = s_is_a ? vis_a : vis_b, vis_o = s_is_a ? vis_b : vis_a;
        const bool staged_s = lr_tree == ts, staged_o = lr_tree == 1 - ts;
        const float* stage_prev = G.stage(par ^ 1, dof);
        const int* cnt_prev = G.st_count(par ^ 1);
        const int* fail_prev = G.st_fail(par ^ 1);
        // Nearest neighbour of x among a tree's visible nodes (and the previous
        // round's staged ones when that tree grew), the scan split over the
        // worker's waves and their results combined through LDS by the same
        // (distance, index) order as within a wave: the same node as one
        // wave scanning everything.
        auto nearest = [&](const float* tq, const unsigned char* bl, int vis, bool staged, const float* x) {
            const int part = NW > 1 ? tid / kWave : 0;
            NearBest b{__builtin_inff(), 0x7fffffff, -1};
            near_scan(tq, bl, cap, vis, x, dof, b, part, NW);
            if (staged) near_scan_staged(stage_prev, P.stage_cap, cnt_prev, P.W, lr_first, cap, x, dof, b, part, NW);
            b = nearest_reduce(b);
            if (NW > 1) {
                // the last reads of sh_nb were followed by a workgroup barrier
                if (lane == 0) sh_nb[part] = b;
                __syncthreads();
                b = sh_nb[0];
                for (int k = 1; k < NW; ++k) {
                    const NearBest o = sh_nb[k];
                    if (o.d < b.d || (o.d == b.d && o.i < b.i)) b = o;
                }
            }
            return b;
        };
        float* qs = s_is_a ? G.qa() : G.qb();
        int* ps = s_is_a ? G.pa() : G.pb();
        unsigned char* bs = s_is_a ? G.ba() : G.bb();
        float* rs = s_is_a ? G.ra() : G.rb();
        const float* qo = s_is_a ? G.qb() : G.qa();
        const unsigned char* bo = s_is_a ? G.bb() : G.ba();
        const int ns = s_is_a ? na : nb;
        // ===== phase A: sample, nearest, extend, connect
        int count = 0, nn = -1, other = -1, conn = 0, fail = -1;
        // RANDOM_CONFIG + NEAREST_NEIGHBOR; with dynamic-domain sampling a sample
        // farther from its nearest node than that node's radius is redrawn
        for (int t = 0; t < P.dds_tries; ++t) {
            // learned: with probability mix, up to 4 mixture draws (attempts
            // 4t..4t+3) until one lies inside the limits, else the uniform draw
            bool drawn = false;
            if (use_gmm && mix_uniform(P.seed, P.query, (unsigned)round, (unsigned)w, 4u * t) < P.mix) {
                const float lo_j = lane < dof ? pick(R.lo, lane) : 0.0f;
                const float hi_j = lane < dof ? pick(R.hi, lane) : 0.0f;
                for (int a = 0; a < 4 && !drawn; ++a) {
                    float v = 0.0f;
                    drawn = gmm_draw(gmm_s, dof, lo_j, hi_j, P.seed, P.query, (unsigned)round, (unsigned)w,
                                     4u * t + a, lane, &v);
                    if (drawn && lead && lane < dof) c_rand[lane] = v;
                }
                my_learned += drawn;
            }
            if (!drawn && lead && lane < dof)
                c_rand[lane] = P.halton ? halton_joint(P.seed, P.query, (unsigned)round, (unsigned)w, (unsigned)P.W,
                                                       (unsigned)P.dds_tries, (unsigned)t, lane, pick(R.lo, lane),
                                                       pick(R.hi, lane))
                                        : sample_joint(P.seed, P.query, (unsigned)round, (unsigned)w, (unsigned)t, dof,
                                                       lane, pick(R.lo, lane), pick(R.hi, lane));
            __syncthreads();
            const NearBest nb_s = nearest(qs, bs, vis_s, staged_s, c_rand);
            const int cand = nb_s.i == 0x7fffffff ? -1 : nb_s.i;
            if (cand < 0) break;
            if (lead && lane < dof)
                c_nn[lane] = nb_s.src < 0 ? qs[(size_t)lane * cap + cand] : stage_prev[nb_s.src + lane];
            __syncthreads();
            if (P.dds_radius > 0.0f) {
                // the node's domain: unbounded for the previous round's new
                // nodes, dds_radius if it failed an extension in the previous
                // round (its own write may not be visible yet), else its word
                float radius = __builtin_inff();
                if (nb_s.src < 0) {
                    radius = rs[cand];
                    if (lr_fail_tree == ts) {
                        bool hit = false;
                        for (int v = lane; v < P.W; v += kWave) hit |= fail_prev[v] == cand;
                        if (__any(hit)) radius = P.dds_radius;
                    }
                }
                if (!(norm_diff_f32(c_nn, c_rand, dof) <= radius)) continue;
            }
            nn = cand;
            break;
        }
        if (nn >= 0) {
            {
#pragma clang fp contract(off)
                const float L = norm_diff_f32(c_nn, c_rand, dof);
                if (lead && lane < dof) {
                    if (L <= P.delta) {
                        c_new[lane] = c_rand[lane];
                    } else {
                        const float k = P.delta / L;
                        c_new[lane] = fmaf(k, c_rand[lane] - c_nn[lane], c_nn[lane]);
                    }
                    wp[lane] = c_nn[lane];
                    wp[dof + lane] = c_new[lane];
                }
            }
            __syncthreads();
            const bool ext_ok = wave_check<TP, B, false, NW, false, TWO>(R, S, wp, 1, 1, P.res, ws) == 1;
            my_edges += 1;
            if (!ext_ok) fail = nn;
            if (ext_ok) {
                count = 1;
                const NearBest nb_o = nearest(qo, bo, vis_o, staged_o, c_new);
                other = nb_o.i == 0x7fffffff ? -1 : nb_o.i;
                if (other >= 0) {
                    if (lead && lane < dof)
                        c_nno[lane] = nb_o.src < 0 ? qo[(size_t)lane * cap + other] : stage_prev[nb_o.src + lane];
                    __syncthreads();
                    int n_ext;
                    {
#pragma clang fp contract(off)
                        const float L = norm_diff_f32(c_new, c_nno, dof);
                        const float ratio = L / P.delta;
                        const float xf = ceilf(ratio);
                        n_ext = xf >= 1.0f ? (int)fminf(xf, 1.0e9f) : 1;
                    }
                    if (n_ext > P.stage_cap) {
                        // cannot happen for nodes inside the joint limits
                        if (tid == 0) atomicExch(G.bar() + kAbort, 2);
                        n_ext = P.stage_cap;
                    }
                    // waypoints t_0 = c_new, t_k = fmaf(k / n_ext, c_nno - c_new, c_new), t_n = c_nno
                    for (int e = tid; e < (n_ext + 1) * dof; e += nth) {
                        const int k = e / dof, j = e - k * dof;
                        float v;
                        if (k == 0) v = c_new[j];
                        else if (k == n_ext) v = c_nno[j];
                        else {
#pragma clang fp contract(off)
                            const float t = (float)k / (float)n_ext;
                            v = fmaf(t, c_nno[j] - c_new[j], c_new[j]);
                        }
                        wp[e] = v;
                    }
                    __syncthreads();
                    const int K = wave_check<TP, B, true, NW, false, TWO>(R, S, wp, n_ext, 1, P.res, ws);
                    my_edges += min(K + 1, n_ext);
                    count = 1 + min(K, n_ext - 1);
                    conn = K == n_ext;
                }
                // stage c_new and the valid intermediate targets
                float* st = G.stage(par, dof) + (size_t)w * P.stage_cap * dof;
                for (int e = tid; e < count * dof; e += nth) st[e] = (e < dof) ? c_new[e] : wp[e];
            }
        }
        if (tid == 0) {
            G.st_count(par)[w] = count;
            G.st_nn(par)[w] = nn;
            G.st_other(par)[w] = other;
            G.st_conn(par)[w] = conn;
            G.st_fail(par)[w] = fail;
        }
        // the time budget is checked once every worker has arrived, so all of
        // them read the same stop word after the barrier
        auto budget = [&]() {
            if (lane == 0 && P.budget_ticks > 0 && (long long)(wall_clock64() - t_start) > P.budget_ticks)
                ctl[kStop] = 1;
        };
        if (!group_barrier(G.bar(), w, P.W, nullptr, budget)) break;
        if (!ends_checked && ends_bad()) return true;
        const bool stop = __hip_atomic_load(ctl + kStop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        // ===== phase B: ordered commit
        int running = 0, my_base = 0, first = 0x7fffffff, first_last = -1, first_other = -1, first_base = -1;
        for (int c0 = 0; c0 < P.W; c0 += kWave) {
            const int wi = c0 + lane;
            const int cnt = wi < P.W ? G.st_count(par)[wi] : 0;
            const int cn = wi < P.W ? G.st_conn(par)[wi] : 0;
            int incl = cnt;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int v = __shfl_up(incl, off, kWave);
                if (lane >= off) incl += v;
            }
            const int base_i = ns + running + incl - cnt;
            const bool fits = base_i + cnt <= cap;
            if (lead && wi == w) sh_i[0] = base_i;
            const int cand = wave_min_int((cn && fits) ? wi : 0x7fffffff);
            if (first == 0x7fffffff && cand != 0x7fffffff) {
                first = cand;
                const int src = cand - c0;
                const int fb = __shfl(base_i, src, kWave);
                const int fc = __shfl(cnt, src, kWave);
                first_last = fb + fc - 1;
                first_base = fb;
                first_other = G.st_other(par)[cand];
            }
            running += __shfl(incl, kWave - 1, kWave);
        }
        __syncthreads();
        my_base = sh_i[0];
        {
            const int c = max(0, min(count, cap - my_base));
            const float* st = G.stage(par, dof) + (size_t)w * P.stage_cap * dof;
            for (int e = tid; e < c * dof; e += nth) {
                const int k = e / dof, j = e - k * dof;
                qs[(size_t)j * cap + my_base + k] = st[e];
            }
            for (int k = tid; k < c; k += nth) {
                ps[my_base + k] = k == 0 ? nn : my_base + k - 1;
                bs[my_base + k] = 0;
                rs[my_base + k] = __builtin_inff();
            }
            // a failed extension shrinks its start node's domain (same value
            // from every worker, so the order of these writes does not matter)
            if (tid == 0 && fail >= 0 && P.dds_radius > 0.0f) rs[fail] = P.dds_radius;
        }
        const int new_size = min(cap, ns + running);
        if (w == 0 && tid == 0) ctl[s_is_a ? kSizeA : kSizeB] = new_size;   // for the statistics
        lr_tree = new_size > ns ? ts : -1;
        lr_first = ns;
        lr_fail_tree = ts;
        if (s_is_a) na = new_size; else nb = new_size;
        // ===== phase C: path and re-check
        if (first != 0x7fffffff) {
            lr_tree = -1;        // after this phase's barriers everything is visible,
            lr_fail_tree = -1;   // the domain shrinks included
            const int xa = s_is_a ? first_last : first_other;
            const int xb = s_is_a ? first_other : first_last;
            // The connecting worker's nodes of this round (first_base ..
            // first_last of tree s) may not be in the arrays yet: the walk
            // follows their chain itself (each node's parent is the one before,
            // the first one's is that worker's nn) and reads their coordinates
            // from its staging rows.  Everything older is in the arrays.
            const int first_nn = G.st_nn(par)[first];
            const float* first_rows = G.stage(par, dof) + (size_t)first * P.stage_cap * dof;
            auto fresh = [&](bool tree_a, int x) { return tree_a == s_is_a && x >= first_base; };
            if (w == 0) {
                if (tid == 0) {
                    // one walk per tree: A from the connection node up to its root
                    // (stored reversed, flipped below), B from its node up to its root
                    int bad = 0, la = 0, lb = 0, x = xa;
                    for (; x >= 0 && la < cap;
                         x = fresh(true, x) ? (x > first_base ? x - 1 : first_nn) : G.pa()[x]) {
                        G.path_idx()[la++] = x;
                        if (!fresh(true, x)) bad |= G.ba()[x];
                    }
                    int y = xb;
                    for (; y >= 0 && lb < cap;
                         y = fresh(false, y) ? (y > first_base ? y - 1 : first_nn) : G.pb()[y]) {
                        G.path_idx()[la + lb++] = y;
                        if (!fresh(false, y)) bad |= G.bb()[y];
                    }
                    int len = la + lb;
                    if (x >= 0 || y >= 0) {           // a parent chain longer than the tree
                        bad = 1;
                        len = P.path_cap + 1;
                        atomicExch(G.bar() + kAbort, 3);
                    }
                    if (P.validate <= 0) bad = len > P.path_cap;  // no re-check: blocked nodes cannot exist
                    ctl[kNa] = la;
                    ctl[kPathLen] = len;
                    ctl[kValBad] = bad;
                    __threadfence_block();
                    sh_i[1] = la;
                    sh_i[2] = len;
                    sh_i[3] = bad && len <= P.path_cap;   // block the ends after the barrier
                }
                __syncthreads();
                __threadfence_block();
                const int la = sh_i[1], len = sh_i[2];
                if (len <= P.path_cap) {
                    for (int m = tid; m < la / 2; m += nth) {
                        const int u = G.path_idx()[m], v = G.path_idx()[la - 1 - m];
                        G.path_idx()[m] = v;
                        G.path_idx()[la - 1 - m] = u;
                    }
                    __syncthreads();
                    __threadfence_block();
                    for (int e = tid; e < len * dof; e += nth) {
                        const int m = e / dof, j = e - m * dof;
                        const bool in_a = m < la;
                        const int x = G.path_idx()[m];
                        const float* q = in_a ? G.qa() : G.qb();
                        G.path()[e] = fresh(in_a, x) ? first_rows[(size_t)(x - first_base) * dof + j]
                                                     : q[(size_t)j * cap + x];
                    }
                }
            }
            if (!group_barrier(G.bar(), w, P.W)) break;
            // every worker's nodes of this round are in the arrays now
            if (w == 0 && tid == 0 && sh_i[3]) {
                if (xa != 0) G.ba()[xa] = 1;
                if (xb != 0) G.bb()[xb] = 1;
            }
            const int la = ctl[kNa], len = ctl[kPathLen];
            if (P.validate > 0) {
                // each segment's points in kValChunks chunks, one per worker
                for (int item = w; item < (len - 1) * kValChunks; item += P.W) {
                    const int k = item / kValChunks, c = item - k * kValChunks;
                    if (lead && lane < 2 * dof) wp[lane] = G.path()[(size_t)k * dof + lane];
                    __syncthreads();
                    const bool ok = wave_check<TP, B, false, NW, false, TWO>(R, S, wp, 1, 0, P.res_v, ws, c, kValChunks) == 1;
                    if (c == 0) my_edges += 1;
                    if (!ok && tid == 0) {
                        ctl[kValBad] = 1;
                        if (k + 1 < la) G.ba()[G.path_idx()[k + 1]] = 1;
                        else if (k + 1 == la) { if (s_is_a) G.ba()[xa] = 1; else G.bb()[xb] = 1; }
                        else G.bb()[G.path_idx()[k]] = 1;
                    }
                    __syncthreads();
                }
            }
            if (!group_barrier(G.bar(), w, P.W)) break;
            if (!ctl[kValBad]) {
                status = kStOk;
                if (w == 0 && tid == 0) ctl[kConnWorker] = first;
                ++round;
                break;
            }
            if (w == 0 && tid == 0) ctl[kValFails] += 1;
        }
        if (stop) {
            ++round;
            break;
        }
        par ^= 1;
    }
    // no round ran (max_rounds 0): the endpoint verdict still decides the
    // status, after a barrier of its own
    if (!ends_checked && P.max_rounds <= 0) {
        if (!group_barrier(G.bar(), w, P.W)) return false;
        if (ends_bad()) return true;
    }
    if (tid == 0 && my_edges) atomicAdd(reinterpret_cast<unsigned long long*>(ctl + kEdgesLo), (unsigned long long)my_edges);
    if (tid == 0 && my_learned)
        atomicAdd(reinterpret_cast<unsigned long long*>(ctl + kLearnedLo), (unsigned long long)my_learned);
    const bool aborted = __hip_atomic_load(G.bar() + kAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    if (w == 0) {
        // hand the path to the query's own buffer (the group's is reused)
        const int len = ctl[kPathLen];
        if (!aborted && status == kStOk && P.out_path != G.path() && len <= P.out_path_cap)
            for (int e = tid; e < len * dof; e += nth) P.out_path[e] = G.path()[e];
        if (tid == 0) {
            ctl[kRounds] = round;
            ctl[kStatus] = aborted ? kStInternal : status;
        }
    }
    return !aborted;
}

// Launch-wide words after the hand-out counter (next[0]), in the 128 bytes
// k_plan_init clears: the wall-clock tick of the last claim (serving) and the
// serving launch's closing flag.
constexpr int kNextLastClaim = 16;   // unsigned long long at next + 16
constexpr int kNextClosing = 24;
constexpr int kNextWords = 32;

// Prepare a launch: zero the barrier words (bar_words each) of n_groups groups
// (bar_stride ints apart), the kNextWords launch-wide words at next, and set
// every query's words to (status = internal error, rest 0); with Pq, the
// single query's arguments (by value) are stored there.
__global__ void k_plan_init(int* bar, int n_groups, int bar_words, size_t bar_stride, int* ctl, int n_queries,
                            PlanArgs one_query, PlanArgs* Pq, int* next) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_groups * bar_words) bar[(size_t)(t / bar_words) * bar_stride + t % bar_words] = 0;
    if (next && t < kNextWords) next[t] = 0;
    if (t < n_queries * kCtlWords) ctl[t] = (t % kCtlWords) == kStatus ? kStInternal : 0;
    if (Pq && t < (int)(sizeof(PlanArgs) / sizeof(int)))
        reinterpret_cast<int*>(Pq)[t] = reinterpret_cast<const int*>(&one_query)[t];
}

// Persistent planner: n_groups groups of W workgroups (NW waves each).  With
// no more queries than groups, group g runs query g.  Otherwise the groups
// take queries one at a time from a launch-wide counter (handed out at a
// group barrier), so a group whose queries end early takes more of them and
// the launch is not held to the unluckiest static share.  All queries of a
// launch share W.  A group that aborts stops taking queries; one it had
// taken is left at "internal".
// WPE: waves per SIMD the register allocation must allow.
template <int TP, int B, int NW, int WPE, bool TWO>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(WPE))) void k_plan(
    const PlanArgs* __restrict__ Pq, int n_queries, int n_groups) {
    extern __shared__ float4 lds4[];
    const int W = Pq[0].W;
    const int g = blockIdx.x / W;
    const int w = blockIdx.x - g * W;
    const unsigned long long goff = (unsigned long long)g * Pq[0].group_bytes;
    const bool handed_out = n_queries > n_groups;
    int k = g;
    for (;;) {
        if (handed_out) {
            int* bar = moved(Pq[0].bar, goff);
            if (!group_barrier(bar, w, W, Pq[0].next)) break;
            // one value for the whole workgroup: keeps the query's arguments
            // on scalar loads
            k = __builtin_amdgcn_readfirstlane(__hip_atomic_load(bar + kNext, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT));
        }
        if (k >= n_queries) break;
        if (!plan_query<TP, B, NW, TWO>(((CPlanArgs*)Pq)[k], w, lds4, goff) || !handed_out) break;
    }
}

// ----------------------------------------------------------------------------
// Persistent serving launch: queries are published while the kernel runs.
// The host writes query k's arguments into host memory (host_args[k]) and then
// raises *published past k; a group claims the next published index at its
// fetch barrier, copies the arguments into device memory (dev_args[k], read
// through the constant address space like a batch launch's) and plans it.  At
// its next fetch barrier the group copies the finished query's words and path
// into host memory (host_ctl[k], host_path[k]) and raises host_ctl[k][0].  A
// slot is written once per launch, so no cache holds an older copy of it.  The
// kernel ends when *drain is set and nothing is left to claim, or once the
// launch has been idle: a group that waits idle_ticks of the wall clock after
// the launch's last claim (by any group) closes the launch, and every group
// leaves at its next claim, so the launch never keeps a few groups for a
// later burst.
// ----------------------------------------------------------------------------
struct ServeArgs {
    const PlanArgs* host_args;    // [cap] host memory
    PlanArgs* dev_args;           // [cap]
    int* dev_ctl;                 // [cap][kCtlWords]
    float* dev_path;              // [cap][path_stride]
    int* host_ctl;                // [cap][kCtlWords + 1]: done flag, then the query's words
    float* host_path;             // [cap][path_stride]
    const int* published;         // host memory: queries published so far this launch
    const int* drain;             // host memory: 1 = leave once nothing is left to claim
    int* next;                    // device: claim counter, then the launch-wide words (kNextLastClaim, kNextClosing)
    int* bar0;                    // group 0's barrier words
    unsigned long long group_bytes;
    long long idle_ticks;
    int cap, W, path_stride, pad;
};

typedef __attribute__((address_space(4))) const ServeArgs CServeArgs;

template <int TP, int B, int NW, int WPE, bool TWO>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(WPE))) void k_serve(
    const ServeArgs* __restrict__ SAp) {
    extern __shared__ float4 lds4[];
    CServeArgs& SA = *(CServeArgs*)SAp;
    const int W = SA.W;
    const int g = blockIdx.x / W;
    const int w = blockIdx.x - g * W;
    const unsigned long long goff = (unsigned long long)g * SA.group_bytes;
    int* bar = moved(SA.bar0, goff);
    int prev = -1;
    for (;;) {
        // first wave of workgroup 0, everyone arrived: hand back the previous
        // query, claim the next, stage its arguments and words
        auto act = [&]() {
            const int lane = threadIdx.x & (kWave - 1);
            if (prev >= 0) {
                const int* c = SA.dev_ctl + (size_t)prev * kCtlWords;
                int* hc = SA.host_ctl + (size_t)prev * (kCtlWords + 1);
                if (lane < kCtlWords) hc[1 + lane] = __hip_atomic_load(c + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int len = c[kPathLen];
                const int dof = SA.dev_args[prev].R->dof;
                if (c[kStatus] == kStOk && len * dof <= SA.path_stride) {
                    const float* src = SA.dev_path + (size_t)prev * SA.path_stride;
                    float* dst = SA.host_path + (size_t)prev * SA.path_stride;
                    for (int e = lane; e < len * dof; e += kWave) dst[e] = src[e];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");   // system scope: the host reads these
                if (lane == 0) __hip_atomic_store(hc, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            int k = -1;
            if (lane == 0) {
                int* closing = SA.next + kNextClosing;
                unsigned long long* last = reinterpret_cast<unsigned long long*>(SA.next + kNextLastClaim);
                const unsigned long long t0 = wall_clock64();
                for (;;) {
                    if (__hip_atomic_load(closing, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                    const int pub = __hip_atomic_load(SA.published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    const int n = __hip_atomic_load(SA.next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (n < pub && n < SA.cap) {
                        int want = n;
                        if (__hip_atomic_compare_exchange_strong(SA.next, &want, n + 1, __ATOMIC_RELAXED,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            __hip_atomic_store(last, wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            // the host wrote the query's arguments before it raised `published`
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                            k = n;
                            break;
                        }
                        continue;
                    }
                    if (__hip_atomic_load(SA.drain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) break;
                    // idle since this wait began and since the launch's last claim
                    const unsigned long long lc = __hip_atomic_load(last, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((long long)(wall_clock64() - (lc > t0 ? lc : t0)) > SA.idle_ticks) {
                        __hip_atomic_store(closing, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            k = __shfl(k, 0, kWave);
            if (k >= 0) {
                // the host's copy of the arguments, then fresh query words
                const int* src = reinterpret_cast<const int*>(SA.host_args + k);
                int* dst = reinterpret_cast<int*>(SA.dev_args + k);
                constexpr int kWords = (int)(sizeof(PlanArgs) / sizeof(int));
                for (int e = lane; e < kWords; e += kWave)
                    dst[e] = __hip_atomic_load(src + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                int* c = SA.dev_ctl + (size_t)k * kCtlWords;
                if (lane < kCtlWords) c[lane] = lane == kStatus ? kStInternal : 0;
            }
            if (lane == 0) __hip_atomic_store(bar + kNext, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        };
        if (!group_barrier(bar, w, W, nullptr, act)) break;
        const int k = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(bar + kNext, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (k < 0) break;
        prev = k;
        if (!plan_query<TP, B, NW, TWO>(((CPlanArgs*)SA.dev_args)[k], w, lds4, goff)) break;
    }
}

}  // namespace prrtc
