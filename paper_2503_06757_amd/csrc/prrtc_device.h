// prrtc_device.h -- device-side tables and routines of the pRRTC hot path on gfx950.
//
// One wavefront (64 lanes) is the unit of work: it validates a list of
// consecutive sub-edges (a single edge for check_edges and pEXTEND, the equal
// steps of a greedy CONNECT, or the segments of a path), Alg. 2 / Sec. III-A.
// Its lanes first run forward kinematics for a tile of interpolated
// configurations (one configuration per lane, chain transforms in registers,
// the frames that carry moving spheres written to LDS), then sweep
// (configuration, sphere) items, configuration-major, against the obstacles.
// Obstacle records are indexed only by loop counters, so the compiler keeps
// them in scalar registers (wave-uniform operands of the vector ALU); a ballot
// after every obstacle ends the sweep at the first hit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace prrtc {

constexpr int kMaxDof = 16;
constexpr int kMaxChains = 2;
constexpr int kMaxFrames = kMaxDof + kMaxChains;
constexpr int kMaxSpheres = 256;
constexpr int kWave = 64;

#ifndef PRRTC_OBS_GROUP
#define PRRTC_OBS_GROUP 1   // obstacles tested between two ballots
#endif
#ifndef PRRTC_ITEM_ORDER
#define PRRTC_ITEM_ORDER 1  // 0: configuration-major items, 1: sphere-major
#endif
#ifndef PRRTC_EXT_CULL
#define PRRTC_EXT_CULL 1    // cuboids and cylinders also culled by their world-axis box (set on the host)
#endif
#ifndef PRRTC_CULL
#define PRRTC_CULL 1        // block bounding-box culling of obstacles
#endif

// Robot tables.  Spheres are re-ordered on load: spheres that move come
// first (their frame depends on some joint), spheres on a chain's base frame
// (which never move) after them.  Frames that carry a moving sphere get an
// LDS slot; the others are computed but never stored.
struct RobotArgs {
    int n_chains, dof, n_frames, n_slots;
    int n_move, n_static;          // spheres [0, n_move) move; [n_move, n_move + n_static) fixed
    int n_pairs, n_static_pairs;   // self pairs with a moving sphere / with two fixed spheres
    int chain_dof[kMaxChains], chain_q0[kMaxChains], chain_f0[kMaxChains];
    int frame_slot[kMaxFrames];    // LDS slot of a frame, -1 if it carries no moving sphere
    float base[kMaxChains][12];
    float ca[kMaxDof], sa[kMaxDof], a[kMaxDof], d[kMaxDof];  // cos/sin(alpha), a, d per joint
    float lo[kMaxDof], hi[kMaxDof];
    const float4* sph;        // local centre + radius, re-ordered
    const int* sph_frame;     // global frame id, re-ordered
    const int* sph_slot;      // 3 * frame slot of each moving sphere
    const int2* pairs;        // re-ordered indices
    const int2* static_pairs;
    const int* desc_index;    // re-ordered sphere -> descriptor order
    // Self pairs forming a complete bipartite set A x B (e.g. all pairs
    // between two arms) are kept as the two groups instead of a pair list.
    int n_bip_a, n_bip_b;
    const int* bip_a;         // re-ordered sphere indices of group A
    const int* bip_b;
    // Two-stage checks (Sec. III-A: a low-resolution sphere pass flags the
    // links that may collide, and only their fine spheres are checked): coarse
    // spheres on moving frames, coarse sphere c enclosing the moving fine
    // spheres cfirst[c] .. cfirst[c + 1] - 1.  n_cmove = 0: one stage.
    int n_cmove;
    const float4* csph;       // [n_cmove] local centre, radius + kCoarseMargin
    const int* cslot3;        // [n_cmove] 3 * frame slot
    const int* cfirst;        // [n_cmove + 1]
};

// Margin added to coarse radii: a fine sphere that the FP32 tests find
// colliding always lies in a coarse sphere that they find colliding too.
constexpr float kCoarseMargin = 1e-4f;

// Scene tables, one array per primitive type.
//   sph: (cx, cy, cz, R)
//   box: 16 floats: -(axis_k . c) for k = 0..2, pad, axis0(3), axis1(3),
//        axis2(3), half-extents(3) (box frame coordinates of a point p are
//        axis_k . p - axis_k . c, three FMAs each)
//   cyl: 8 floats: c(3), unit axis(3), R, half-height
//   bnd:   bounding sphere of every primitive, (centre, radius + 1e-4 m),
//          spheres first, then cuboids, then cylinders (n_sph + n_box + n_cyl)
//   ext:   half-sizes of the world-axis bounding box of every primitive
//          around the same centre (+ 1e-4 m), w unused, in bnd's order;
//          3e38 for the primitives of a type whose boxes would cull little
//          beyond the bounding spheres (all spheres); ext_cull = 0 when no
//          type's would (the boxes are then not tested)
//   Both tables hold at least one (zero) entry in an empty scene.
//   esdf:  node values [nz][ny][nx] (x fastest) of an attached signed
//          distance grid, node (i, j, k) at esdf_o + voxel (i, j, k), or null
struct SceneArgs {
    int n_sph, n_box, n_cyl;
    const float4* sph;
    const float* box;
    const float* cyl;
    const float4* bnd;
    const float4* ext;
    int ext_cull;
    const float* esdf;
    float esdf_o[3], esdf_ih;   // origin, 1 / voxel
    int esdf_n[3];              // nodes per axis, each >= 2
    float esdf_gate;            // max(1, Lipschitz bound of the interpolated field)
};

// ----------------------------------------------------------------------------
// FP32 contract helpers: sums in index order, no contraction, correctly
// rounded sqrt/division (the compiler default for HIP device code).
// ----------------------------------------------------------------------------
__device__ inline float norm_diff_f32(const float* a, const float* b, int dof) {
#pragma clang fp contract(off)
    float s = 0.0f;
    for (int j = 0; j < dof; ++j) {
        const float d = b[j] - a[j];
        const float sq = d * d;
        s = s + sq;
    }
    return sqrtf(s);
}

// n = max(1, ceil(res * L)), capped at 2^24.
__device__ inline int edge_count_f32(const float* a, const float* b, int dof, float res) {
#pragma clang fp contract(off)
    const float L = norm_diff_f32(a, b, dof);
    const float prod = res * L;
    const float x = ceilf(prod);
    if (!(x >= 1.0f)) return 1;
    if (x > 16777216.0f) return 16777216;
    return (int)x;
}

// Element `idx` (lane-varying) of a small kernel-argument array, through
// selects: indexing kernel arguments by a lane-varying value makes the
// compiler copy the whole argument block to private memory.
template <int N>
__device__ inline float pick(const float (&arr)[N], int idx) {
    float v = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) v = (i == idx) ? arr[i] : v;
    return v;
}

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).
// ----------------------------------------------------------------------------
__device__ inline uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k.x += 0x9E3779B9u;
            k.y += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    }
    return c;
}

// RANDOM_CONFIG joint j of sample `attempt`: counter (draw, worker, round,
// query) with draw = attempt * ceil(dof / 4) + j / 4, word j % 4,
// u = (word >> 8) * 2^-24, q_j = fmaf(u, hi_j - lo_j, lo_j).
__device__ inline float sample_joint(uint64_t seed, uint32_t query, uint32_t round, uint32_t worker,
                                     uint32_t attempt, int dof, int j, float lo, float hi) {
#pragma clang fp contract(off)
    const uint32_t draw = attempt * (uint32_t)((dof + 3) >> 2) + (uint32_t)(j >> 2);
    const uint4 w = philox4x32_10(make_uint4(draw, worker, round, query),
                                  make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
    const int m = j & 3;
    const uint32_t word = m == 0 ? w.x : (m == 1 ? w.y : (m == 2 ? w.z : w.w));
    const float u = (float)(word >> 8) * 0x1p-24f;
    const float span = hi - lo;
    return fmaf(u, span, lo);
}

// Halton RANDOM_CONFIG (Sec. IV-A: the paper's experiments sample from Halton
// sequences).  Point i = (low word of seed) + 65536 query + (round W + worker)
// tries + attempt + 1 (mod 2^32); joint j takes the radical inverse of i in
// the j-th prime base: with i's base-b digits d_0 (least significant) ..
// d_{m-1}, sum_k d_k b^-(k+1) = v / b^m exactly (v the reversed digits), which
// is rounded to FP64 by one division and then to FP32; q_j = fmaf(u, hi_j -
// lo_j, lo_j).  v < b^m <= 53^6 < 2^53, so both are exact doubles.
__device__ inline float radical_inverse(uint32_t i, uint32_t b) {
    uint64_t v = 0, bm = 1;
    for (uint32_t x = i; x > 0; x /= b) {
        v = v * b + x % b;
        bm *= b;
    }
    return (float)((double)v / (double)bm);
}

__device__ inline uint32_t halton_prime(int j) {
    constexpr uint32_t primes[kMaxDof] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53};
    uint32_t p = 2;
#pragma unroll
    for (int k = 0; k < kMaxDof; ++k) p = k == j ? primes[k] : p;
    return p;
}

__device__ inline float halton_joint(uint64_t seed, uint32_t query, uint32_t round, uint32_t worker,
                                     uint32_t workers, uint32_t tries, uint32_t attempt, int j, float lo, float hi) {
    const uint32_t i = (uint32_t)seed + 65536u * query + (round * workers + worker) * tries + attempt + 1u;
    return fmaf(radical_inverse(i, halton_prime(j)), hi - lo, lo);
}

// sin and cos of a joint angle for FK: the hardware's transcendental unit
// for angles within four turns (sphere centres within 5e-7 m of FP64 FK over
// 2^20 random configurations of the 7-DoF arm, against 3e-7 m with the
// library routine, and 3-8% less time per edge check), the accurate library
// routine beyond them or with PRRTC_FK_NATIVE_TRIG 0.
#ifndef PRRTC_FK_NATIVE_TRIG
#define PRRTC_FK_NATIVE_TRIG 1
#endif
__device__ inline void joint_sincos(float q, float* s, float* c) {
#if PRRTC_FK_NATIVE_TRIG
    if (fabsf(q) <= 25.0f) {
        *s = __sinf(q);
        *c = __cosf(q);
        return;
    }
#endif
    sincosf(q, s, c);
}

// ----------------------------------------------------------------------------
// Forward kinematics of one configuration (one lane).  Frame j+1 = frame j *
// Rx(alpha_j) Tx(a_j) Rz(q_j) Tz(d_j); a frame is three float4 rows [R | t].
// With M = R Rx(alpha):  M0 = R0, M1 = ca R1 + sa R2, M2 = ca R2 - sa R1;
// new R = (cq M0 + sq M1, cq M1 - sq M0, M2) and new t = t + a R0 + d M2.
// ALL = true stores every frame at 3 * f; otherwise only slotted frames, at
// 3 * slot.
// ----------------------------------------------------------------------------
template <bool ALL, class QF>
__device__ inline void fk_frames(const RobotArgs& R, QF qf, float4* out) {
    for (int c = 0; c < R.n_chains; ++c) {
        const float* B = R.base[c];
        float r00 = B[0], r01 = B[1], r02 = B[2], t0 = B[3];
        float r10 = B[4], r11 = B[5], r12 = B[6], t1 = B[7];
        float r20 = B[8], r21 = B[9], r22 = B[10], t2 = B[11];
        int f = R.chain_f0[c];
        auto store = [&](int fr) {
            const int at = ALL ? fr : R.frame_slot[fr];
            if (at >= 0) {
                out[3 * at + 0] = make_float4(r00, r01, r02, t0);
                out[3 * at + 1] = make_float4(r10, r11, r12, t1);
                out[3 * at + 2] = make_float4(r20, r21, r22, t2);
            }
        };
        store(f);
        const int q0 = R.chain_q0[c];
        for (int jj = 0; jj < R.chain_dof[c]; ++jj) {
            const int j = q0 + jj;
            float sq, cq;
            joint_sincos(qf(j), &sq, &cq);
            const float ca = R.ca[j], sa = R.sa[j], a = R.a[j], d = R.d[j];
            const float u0 = ca * r01 + sa * r02, u1 = ca * r11 + sa * r12, u2 = ca * r21 + sa * r22;
            const float m0 = ca * r02 - sa * r01, m1 = ca * r12 - sa * r11, m2 = ca * r22 - sa * r21;
            t0 += a * r00 + d * m0;
            t1 += a * r10 + d * m1;
            t2 += a * r20 + d * m2;
            const float n00 = cq * r00 + sq * u0, n10 = cq * r10 + sq * u1, n20 = cq * r20 + sq * u2;
            const float n01 = cq * u0 - sq * r00, n11 = cq * u1 - sq * r10, n21 = cq * u2 - sq * r20;
            r00 = n00; r10 = n10; r20 = n20;
            r01 = n01; r11 = n11; r21 = n21;
            r02 = m0; r12 = m1; r22 = m2;
            store(++f);
        }
    }
}

// The same recursion on four lanes (a quad) per configuration.  The rows of
// a frame evolve independently given the joint's (cos q, sin q), so lane r of
// the quad (r < 3) carries row r with exactly the arithmetic of fk_frames
// (bit-identical frames), and the trigonometry is shared: for joints
// j4..j4+3 of the chain, lane r takes sincos of joint j4 + r and each joint's
// pair is broadcast from the lane that made it (DPP within the quad).  ALL =
// true stores every frame at 3 * f; otherwise only slotted frames, at
// 3 * slot.  The whole quad must be active.  Chains c_lo..c_hi-1 only
// (each chain's frames depend on that chain alone).
#ifndef PRRTC_FK_QUAD
#define PRRTC_FK_QUAD 1
#endif
// Broadcast lane u of each quad to the whole quad (DPP quad_perm).
template <int U>
__device__ inline float quad_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), U * 0x55, 0xF, 0xF, false));
}

template <bool ALL, class QF>
__device__ inline void fk_rows(const RobotArgs& R, QF qf, float4* out, int r, int c_lo = 0, int c_hi = kMaxChains) {
    const int rr = r < 3 ? r : 2;   // lane 3 shadows row 2 and stores nothing
    for (int c = c_lo; c < min(c_hi, R.n_chains); ++c) {
        const float* B = R.base[c] + 4 * rr;
        float x = B[0], y = B[1], z = B[2], t = B[3];
        int f = R.chain_f0[c];
        auto store = [&](int fr) {
            const int at = ALL ? fr : R.frame_slot[fr];
            if (at >= 0 && r < 3) out[3 * at + r] = make_float4(x, y, z, t);
        };
        store(f);
        const int q0 = R.chain_q0[c], cd = R.chain_dof[c];
        for (int j4 = 0; j4 < cd; j4 += 4) {
            float sv = 0.0f, cv = 1.0f;
            if (j4 + r < cd) joint_sincos(qf(q0 + j4 + r), &sv, &cv);
            auto joint = [&](int jj, float sq, float cq) {
                const int j = q0 + jj;
                const float ca = R.ca[j], sa = R.sa[j], a = R.a[j], d = R.d[j];
                const float u = ca * y + sa * z;
                const float m = ca * z - sa * y;
                t += a * x + d * m;
                const float n0 = cq * x + sq * u;
                const float n1 = cq * u - sq * x;
                x = n0;
                y = n1;
                z = m;
                store(++f);
            };
            joint(j4, quad_bcast<0>(sv), quad_bcast<0>(cv));
            if (j4 + 1 < cd) joint(j4 + 1, quad_bcast<1>(sv), quad_bcast<1>(cv));
            if (j4 + 2 < cd) joint(j4 + 2, quad_bcast<2>(sv), quad_bcast<2>(cv));
            if (j4 + 3 < cd) joint(j4 + 3, quad_bcast<3>(sv), quad_bcast<3>(cv));
        }
    }
}

__device__ inline float3 frame_apply(const float4* fr, float x, float y, float z) {
    const float4 a = fr[0], b = fr[1], c = fr[2];
    return make_float3(a.x * x + a.y * y + a.z * z + a.w, b.x * x + b.y * y + b.z * z + b.w,
                       c.x * x + c.y * y + c.z * z + c.w);
}

// ----------------------------------------------------------------------------
// Penetration predicates in FP32: a sphere (centre c, radius r) collides with
// a primitive iff its centre lies strictly closer than r to the solid.
// ----------------------------------------------------------------------------
__device__ inline bool hit_sphere(float cx, float cy, float cz, float r, float4 o) {
    const float dx = cx - o.x, dy = cy - o.y, dz = cz - o.z;
    const float rr = r + o.w;
    return dx * dx + dy * dy + dz * dz < rr * rr;
}

// The scene tables are read-only for the whole launch: reading them through
// the constant address space lets wave-uniform reads become scalar loads.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(4))) const v4f cv4f;
__device__ inline float4 ld4(const void* base, int i) {
    const v4f v = ((cv4f*)base)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}
struct Box { float4 a, b, c, d; };   // see SceneArgs::box
struct Cyl { float4 a, b; };         // see SceneArgs::cyl
__device__ inline float4 ld_sph(const SceneArgs& S, int o) { return ld4(S.sph, o); }
__device__ inline Box ld_box(const SceneArgs& S, int o) {
    return Box{ld4(S.box, 4 * o), ld4(S.box, 4 * o + 1), ld4(S.box, 4 * o + 2), ld4(S.box, 4 * o + 3)};
}
__device__ inline Cyl ld_cyl(const SceneArgs& S, int o) { return Cyl{ld4(S.cyl, 2 * o), ld4(S.cyl, 2 * o + 1)}; }

__device__ inline bool hit_box(float cx, float cy, float cz, float r, const Box& o) {
    // o.a = (-ax0.c, -ax1.c, -ax2.c, pad), o.b = (ax0, ax1.x), o.c = (ax1.yz, ax2.xy),
    // o.d = (ax2.z, h)
    const float l0 = fmaf(o.b.x, cx, fmaf(o.b.y, cy, fmaf(o.b.z, cz, o.a.x)));
    const float l1 = fmaf(o.b.w, cx, fmaf(o.c.x, cy, fmaf(o.c.y, cz, o.a.y)));
    const float l2 = fmaf(o.c.z, cx, fmaf(o.c.w, cy, fmaf(o.d.x, cz, o.a.z)));
    const float e0 = fmaxf(fabsf(l0) - o.d.y, 0.0f);
    const float e1 = fmaxf(fabsf(l1) - o.d.z, 0.0f);
    const float e2 = fmaxf(fabsf(l2) - o.d.w, 0.0f);
    return e0 * e0 + e1 * e1 + e2 * e2 < r * r;
}

__device__ inline float sd_box(float x, float y, float z, const Box& o) {
    const float l0 = fmaf(o.b.x, x, fmaf(o.b.y, y, fmaf(o.b.z, z, o.a.x)));
    const float l1 = fmaf(o.b.w, x, fmaf(o.c.x, y, fmaf(o.c.y, z, o.a.y)));
    const float l2 = fmaf(o.c.z, x, fmaf(o.c.w, y, fmaf(o.d.x, z, o.a.z)));
    const float q0 = fabsf(l0) - o.d.y, q1 = fabsf(l1) - o.d.z, q2 = fabsf(l2) - o.d.w;
    const float e0 = fmaxf(q0, 0.0f), e1 = fmaxf(q1, 0.0f), e2 = fmaxf(q2, 0.0f);
    return sqrtf(e0 * e0 + e1 * e1 + e2 * e2) + fminf(fmaxf(q0, fmaxf(q1, q2)), 0.0f);
}

__device__ inline float sd_cyl(float x, float y, float z, const Cyl& o) {
    const float vx = x - o.a.x, vy = y - o.a.y, vz = z - o.a.z;
    const float h = o.a.w * vx + o.b.x * vy + o.b.y * vz;
    const float wx = vx - h * o.a.w, wy = vy - h * o.b.x, wz = vz - h * o.b.y;
    const float dr = sqrtf(wx * wx + wy * wy + wz * wz) - o.b.z;
    const float dz = fabsf(h) - o.b.w;
    const float er = fmaxf(dr, 0.0f), ez = fmaxf(dz, 0.0f);
    return sqrtf(er * er + ez * ez) + fminf(fmaxf(dr, dz), 0.0f);
}

__device__ inline bool hit_cyl(float cx, float cy, float cz, float r, const Cyl& o) {
    // o.a = (c, u.x), o.b = (u.yz, R, H)
    const float vx = cx - o.a.x, vy = cy - o.a.y, vz = cz - o.a.z;
    const float z = o.a.w * vx + o.b.x * vy + o.b.y * vz;
    const float wx = vx - z * o.a.w, wy = vy - z * o.b.x, wz = vz - z * o.b.y;
    const float rho = __builtin_amdgcn_sqrtf(wx * wx + wy * wy + wz * wz);
    const float dr = fmaxf(rho - o.b.z, 0.0f);
    const float dz = fmaxf(fabsf(z) - o.b.w, 0.0f);
    return dr * dr + dz * dz < r * r;
}

// ESDF grid (Sec. III-A: with camera-built maps the spheres are checked
// against a Euclidean signed distance field): trilinear interpolation of the
// node values, grid coordinates clamped to the grid's box (outside, the
// field continues as its value at the nearest point of the box).  A sphere
// collides iff the value at its centre is below its radius.
__device__ inline float esdf_value(const SceneArgs& S, float x, float y, float z) {
    const float p[3] = {x, y, z};
    int i[3];
    float t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float g = fminf(fmaxf((p[a] - S.esdf_o[a]) * S.esdf_ih, 0.0f), (float)(S.esdf_n[a] - 1));
        i[a] = min((int)g, S.esdf_n[a] - 2);
        t[a] = g - (float)i[a];
    }
    const size_t sy = (size_t)S.esdf_n[0], sz = sy * (size_t)S.esdf_n[1];
    const float* v = S.esdf + (size_t)i[2] * sz + (size_t)i[1] * sy + (size_t)i[0];
    const float c00 = fmaf(t[0], v[1] - v[0], v[0]);
    const float c10 = fmaf(t[0], v[sy + 1] - v[sy], v[sy]);
    const float c01 = fmaf(t[0], v[sz + 1] - v[sz], v[sz]);
    const float c11 = fmaf(t[0], v[sz + sy + 1] - v[sz + sy], v[sz + sy]);
    const float c0 = fmaf(t[1], c10 - c00, c00);
    const float c1 = fmaf(t[1], c11 - c01, c01);
    return fmaf(t[2], c1 - c0, c0);
}

__device__ inline bool hit_esdf(float cx, float cy, float cz, float r, const SceneArgs& S) {
    return esdf_value(S, cx, cy, cz) < r;
}

// Signed distances (negative inside) of a point to the primitives, for
// building a grid from a scene.
__device__ inline float sd_sphere(float x, float y, float z, float4 o) {
    const float dx = x - o.x, dy = y - o.y, dz = z - o.z;
    return sqrtf(dx * dx + dy * dy + dz * dz) - o.w;
}

__device__ inline bool hit_pair(float4 a, float4 b) {
    const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    const float rr = a.w + b.w;
    return dx * dx + dy * dy + dz * dz < rr * rr;
}

// Wave-wide min / max (all 64 lanes active), returned to every lane as a
// wave-uniform value.  Data-parallel-primitive (DPP) moves fuse into the
// min/max instructions: pairs and quads by quad permutes, rows of 16 by the
// half-row and row mirrors, then row broadcasts 15 and 31 carry the partial
// results up so that lane 63 holds the wave's value.
#ifndef PRRTC_FASTDIV
#define PRRTC_FASTDIV 1
#endif
#ifndef PRRTC_DPP_REDUCE
#define PRRTC_DPP_REDUCE 1
#endif
template <bool MAX>
__device__ inline float wave_reduce_f(float v) {
#if PRRTC_DPP_REDUCE
#define PRRTC_DPP(x, ctrl, rows) \
    __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), ctrl, rows, 0xF, false))
    auto op = [](float a, float b) { return MAX ? fmaxf(a, b) : fminf(a, b); };
    v = op(v, PRRTC_DPP(v, 0xB1, 0xF));    // quad_perm [1, 0, 3, 2]
    v = op(v, PRRTC_DPP(v, 0x4E, 0xF));    // quad_perm [2, 3, 0, 1]
    v = op(v, PRRTC_DPP(v, 0x141, 0xF));   // row_half_mirror
    v = op(v, PRRTC_DPP(v, 0x140, 0xF));   // row_mirror
    v = op(v, PRRTC_DPP(v, 0x142, 0xA));   // row_bcast:15 into rows 1 and 3
    v = op(v, PRRTC_DPP(v, 0x143, 0xC));   // row_bcast:31 into rows 2 and 3
#undef PRRTC_DPP
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
#else
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = MAX ? fmaxf(v, __shfl_xor(v, off, kWave)) : fminf(v, __shfl_xor(v, off, kWave));
    return v;
#endif
}

__device__ inline float wave_min_f(float v) { return wave_reduce_f<false>(v); }
__device__ inline float wave_max_f(float v) { return wave_reduce_f<true>(v); }

// Wave-wide minima of (lx, ly, lz) and maxima of (hx, hy, hz), returned in
// every lane: the same six DPP steps as wave_reduce_f, each a single
// v_min/v_max with the DPP operand (the compiler's form copies the value,
// moves it with DPP, quiets NaNs and then takes the min: four instructions a
// step).  The six reductions are interleaved, so each DPP read comes six
// instructions after the write it depends on (two wait states are needed);
// the leading and trailing s_nop cover the writes before and the reads after
// the block.  Needs every lane of the wave active and no NaN inputs.
#ifndef PRRTC_DPP_ASM
#define PRRTC_DPP_ASM 1
#endif
__device__ inline void wave_box(float& lx, float& ly, float& lz, float& hx, float& hy, float& hz) {
#if PRRTC_DPP_ASM
#define PRRTC_BOX_STEP(ctrl)                                  \
    "v_min_f32_dpp %0, %0, %0 " ctrl "\n"                     \
    "v_min_f32_dpp %1, %1, %1 " ctrl "\n"                     \
    "v_min_f32_dpp %2, %2, %2 " ctrl "\n"                     \
    "v_max_f32_dpp %3, %3, %3 " ctrl "\n"                     \
    "v_max_f32_dpp %4, %4, %4 " ctrl "\n"                     \
    "v_max_f32_dpp %5, %5, %5 " ctrl "\n"
    asm volatile("s_nop 1\n"
                 PRRTC_BOX_STEP("quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf")
                 PRRTC_BOX_STEP("quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf")
                 PRRTC_BOX_STEP("row_half_mirror row_mask:0xf bank_mask:0xf")
                 PRRTC_BOX_STEP("row_mirror row_mask:0xf bank_mask:0xf")
                 PRRTC_BOX_STEP("row_bcast:15 row_mask:0xa bank_mask:0xf")
                 PRRTC_BOX_STEP("row_bcast:31 row_mask:0xc bank_mask:0xf")
                 "s_nop 1"
                 : "+v"(lx), "+v"(ly), "+v"(lz), "+v"(hx), "+v"(hy), "+v"(hz));
#undef PRRTC_BOX_STEP
    auto last = [](float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kWave - 1)); };
    lx = last(lx); ly = last(ly); lz = last(lz);
    hx = last(hx); hy = last(hy); hz = last(hz);
#else
    lx = wave_min_f(lx); ly = wave_min_f(ly); lz = wave_min_f(lz);
    hx = wave_max_f(hx); hy = wave_max_f(hy); hz = wave_max_f(hz);
#endif
}

// Does an obstacle's bounding sphere b reach the box [lo, hi]?
__device__ inline bool sphere_meets_box(float4 b, float lx, float ly, float lz, float hx, float hy,
                                        float hz) {
    const float dx = fmaxf(fmaxf(lx - b.x, b.x - hx), 0.0f);
    const float dy = fmaxf(fmaxf(ly - b.y, b.y - hy), 0.0f);
    const float dz = fmaxf(fmaxf(lz - b.z, b.z - hz), 0.0f);
    return dx * dx + dy * dy + dz * dz < b.w * b.w;
}

// Wave-wide minimum of an integer.
__device__ inline int wave_min_int(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
    return v;
}

// World position (+ radius) of a sphere on a chain's base frame.
// (The chain is selected per lane without indexing the kernel-argument
// tables by a lane-varying value, which would force a private copy.)
__device__ inline float4 fixed_world(const RobotArgs& R, int s) {
    const int f = R.sph_frame[s];
    const bool c1 = R.n_chains > 1 && f >= R.chain_f0[1];
    float B[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) B[i] = c1 ? R.base[1][i] : R.base[0][i];
    const float4 p = R.sph[s];
    return make_float4(B[0] * p.x + B[1] * p.y + B[2] * p.z + B[3],
                       B[4] * p.x + B[5] * p.y + B[6] * p.z + B[7],
                       B[8] * p.x + B[9] * p.y + B[10] * p.z + B[11], p.w);
}

// Does any fixed sphere (or fixed-fixed self pair) collide?  Evaluated once
// per wave: those spheres are at the same place in every configuration.
__device__ inline bool static_collision(const RobotArgs& R, const SceneArgs& S) {
    const int lane = threadIdx.x & (kWave - 1);
    auto world = [&](int s) { return fixed_world(R, s); };
    bool hit = false;
    for (int k = lane; k < R.n_static; k += kWave) {
        const float4 c = world(R.n_move + k);
        for (int o = 0; o < S.n_sph; ++o) hit |= hit_sphere(c.x, c.y, c.z, c.w, ld_sph(S, o));
        for (int o = 0; o < S.n_box; ++o) hit |= hit_box(c.x, c.y, c.z, c.w, ld_box(S, o));
        for (int o = 0; o < S.n_cyl; ++o) hit |= hit_cyl(c.x, c.y, c.z, c.w, ld_cyl(S, o));
        if (S.esdf) hit |= hit_esdf(c.x, c.y, c.z, c.w, S);
    }
    for (int k = lane; k < R.n_static_pairs; k += kWave) {
        const int2 pr = R.static_pairs[k];
        hit |= hit_pair(world(pr.x), world(pr.y));
    }
    return __any(hit);
}

// ----------------------------------------------------------------------------
// Wave-level check of a waypoint list.
//
// Sub-edge k joins waypoint k to k+1 (wp is LDS, row-major [n_sub + 1][dof]).
// Its points are i = i_first..n_k with n_k from edge_count_f32 and
// q = fmaf((float)i / (float)n_k, w_{k+1} - w_k, w_k).  Returns the index of
// the first sub-edge with a colliding point, or n_sub when none collides.
// MULTI = false specialises the single-sub-edge case (any hit ends the call).
//
// Workspace (LDS, per wave): frames [TP][n_slots][3] float4, the moving
// spheres' local records and slot offsets, pk [TP], sub_n / sub_off
// [n_sub + 1].
// ----------------------------------------------------------------------------
struct WaveWs {
    float4* frames;
    const float4* sph;   // [n_move]
    const int* slot3;    // [n_move] 3 * frame slot
    int* pk;
    int* sub_n;
    int* sub_off;
    int* shared;         // two ints: running minimum and stop flag (multi-wave checks only)
    float4 bnd0, ext0;   // per lane: bounding sphere and world box of obstacle `lane`
    // two-stage checks: flags of the tile's (coarse sphere, configuration)
    // items [n_cmove][TP], the fine items they let through [TP n_move] as
    // (sphere << 8 | configuration), and that list's length
    unsigned char* cflag;
    int* list;
    int* list_n;
};

// LDS of the two-stage tables for a tile of tp configurations (none for a
// one-stage robot): flags, item list, list length.
__host__ __device__ inline size_t two_stage_lds_bytes(const RobotArgs& R, int tp) {
    if (R.n_cmove == 0) return 0;
    return sizeof(int) * (1 + (size_t)R.n_move * tp) + (((size_t)R.n_cmove * tp + 3) & ~(size_t)3);
}

// Carve the two-stage tables out of LDS at `at` (ints).
__device__ inline void two_stage_ws(const RobotArgs& R, int tp, int* at, WaveWs& ws) {
    ws.list_n = at;
    ws.list = at + 1;
    ws.cflag = reinterpret_cast<unsigned char*>(ws.list + (size_t)R.n_move * tp);
}

// Load each lane's first-chunk obstacle bounds (kept in registers).
__device__ inline void load_bounds(const SceneArgs& S, WaveWs& ws) {
    const int lane = threadIdx.x & (kWave - 1);
    // lanes past the last obstacle load the last one (or the zero entry of
    // an empty scene); the sweeps never keep them
    const int i = min(lane, max(S.n_sph + S.n_box + S.n_cyl - 1, 0));
    ws.bnd0 = S.bnd[i];
    ws.ext0 = S.ext[i];
}

// Bits lo..hi-1 of a wave mask (lo and hi clamped to 0..64).
__device__ inline unsigned long long lane_bits(int lo, int hi) {
    lo = max(lo, 0);
    hi = min(hi, kWave);
    if (hi <= lo) return 0ull;
    const unsigned long long below_hi = hi >= kWave ? ~0ull : (1ull << hi) - 1ull;
    return below_hi & ~((1ull << lo) - 1ull);
}

// Culling of every obstacle against a world box [l, h]: one obstacle per
// lane over chunks of 64 (all types in one table), each lane's obstacle kept
// when its bounding sphere, and its world box where the scene has them,
// reach [l, h].  The survivors go to sph(o) / box(o) / cyl(o) (o: index in
// the type's own table), cuboids first when BOX_FIRST; a call that returns
// true ends the sweep.
template <bool BOX_FIRST, class FS, class FB, class FC>
__device__ __attribute__((always_inline)) bool cull_sweep(const SceneArgs& S, float4 bnd0, float4 ext0, float lx,
                                                          float ly, float lz, float hx, float hy, float hz, FS&& sph,
                                                          FB&& box, FC&& cyl) {
    const int lane = threadIdx.x & (kWave - 1);
    const int n_all = S.n_sph + S.n_box + S.n_cyl;
    for (int c0 = 0; c0 < n_all; c0 += kWave) {
        const int o = c0 + lane;
        bool keep = false;
        if (o < n_all) {
            const float4 b = c0 == 0 ? bnd0 : S.bnd[o];
            keep = sphere_meets_box(b, lx, ly, lz, hx, hy, hz);
            if (S.ext_cull && keep) {
                const float4 e = c0 == 0 ? ext0 : S.ext[o];
                keep = b.x - e.x <= hx && b.x + e.x >= lx && b.y - e.y <= hy && b.y + e.y >= ly &&
                       b.z - e.z <= hz && b.z + e.z >= lz;
            }
        }
        const unsigned long long m = __ballot(keep);
        if (!m) continue;
        const int e1 = S.n_sph - c0, e2 = e1 + S.n_box;   // type boundaries within the chunk
        auto run = [&](unsigned long long mt, int first, auto&& f) -> bool {
            while (mt) {
                const int oi = c0 + (int)__builtin_ctzll(mt) - first;
                mt &= mt - 1;
                if (f(oi)) return true;
            }
            return false;
        };
        const unsigned long long ms = m & lane_bits(0, e1), mb = m & lane_bits(e1, e2), mc = m & lane_bits(e2, kWave);
        if (BOX_FIRST) {
            if (run(mb, S.n_sph, box) || run(ms, 0, sph)) return true;
        } else {
            if (run(ms, 0, sph) || run(mb, S.n_sph, box)) return true;
        }
        if (run(mc, S.n_sph + S.n_box, cyl)) return true;
    }
    return false;
}

// ceil(2^20 / n) for the item decode's multiply-and-shift division by the
// tile's configuration count n = 1..64: a table lookup instead of an integer
// division per tile.
struct FastDivTable {
    unsigned m[kWave + 1];
    constexpr FastDivTable() : m{} {
        for (int n = 1; n <= kWave; ++n) m[n] = ((1u << 20) + (unsigned)n - 1u) / (unsigned)n;
    }
};
__device__ constexpr FastDivTable kFastDiv{};

// Stage the moving spheres' records in LDS (once per workgroup).
__device__ inline void stage_spheres(const RobotArgs& R, float4* sph, int* slot3) {
    for (int s = threadIdx.x; s < R.n_move; s += blockDim.x) {
        sph[s] = R.sph[s];
        slot3[s] = R.sph_slot[s];
    }
}

// With n_chunks > 1 (one sub-edge only) the points i_first..n are split into
// n_chunks equal runs and only run `chunk` is checked.  n_known >= 0 (one
// sub-edge): the edge's point count, already computed by the caller from the
// same endpoints (edge_count_f32).
//
// BOX_FIRST: cuboids are swept before spheres (the first hit ends the
// check, so the order only changes the time; check_edges picks it by timing).
//
// TWO: the kernel includes the two-stage pass for robots with coarse spheres
// (without it, a robot's coarse spheres are ignored: one stage).
//
// NW > 1: the NW waves of a workgroup check together.  Every wave runs the
// same tile loop; the tile's FK is split into TP / NW configurations per
// wave, its item blocks are dealt to the waves in turn, and at the end of
// the tile the waves' results meet in LDS (ws.shared[0]: least colliding
// sub-edge; ws.shared[1]: a wave found a hit, single sub-edge).
template <int TP, int B, bool MULTI, int NW = 1, bool BOX_FIRST = false, bool TWO = false>
__device__ __attribute__((always_inline)) int wave_check(const RobotArgs& R, const SceneArgs& S, const float* wp, int n_sub,
                          int i_first, float res, const WaveWs& ws, int chunk = 0, int n_chunks = 1,
                          int n_known = -1) {
    static_assert(TP >= 1 && TP <= kWave, "one configuration per lane in the FK tile");
    static_assert(NW >= 1 && TP % NW == 0, "the FK tile splits evenly over the waves");
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = NW > 1 ? (int)(threadIdx.x / kWave) : 0;
    volatile int* shared = ws.shared;
    const int dof = R.dof;
    const int fstride = 3 * R.n_slots;
    // point counts and prefix offsets, in chunks of 64 sub-edges (one
    // sub-edge: every lane computes the same count from the same LDS words)
    int total = 0;
    if (!MULTI) {
        const int n = n_known >= 0 ? n_known : edge_count_f32(wp, wp + dof, dof, res);
        int cnt = n - i_first + 1, lo = 0;
        if (n_chunks > 1) {
            lo = cnt * chunk / n_chunks;
            cnt = cnt * (chunk + 1) / n_chunks - lo;
        }
        if (wave == 0 && lane == 0) {
            ws.sub_n[0] = n;
            ws.sub_off[0] = -lo;
        }
        total = cnt;
    }
    for (int k0 = 0; MULTI && k0 < n_sub; k0 += kWave) {
        const int k = k0 + lane;
        int cnt = 0, lo = 0;
        if (k < n_sub) {
            const int n = edge_count_f32(wp + k * dof, wp + (k + 1) * dof, dof, res);
            if (wave == 0) ws.sub_n[k] = n;
            cnt = n - i_first + 1;
            if (n_chunks > 1) {
                lo = cnt * chunk / n_chunks;
                cnt = cnt * (chunk + 1) / n_chunks - lo;
            }
        }
        int incl = cnt;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int v = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += v;
        }
        if (k < n_sub && wave == 0) ws.sub_off[k] = total + incl - cnt - lo;   // point i = i_first + g - sub_off
        total += __shfl(incl, kWave - 1, kWave);
    }
    if (NW > 1 && threadIdx.x == 0) {
        shared[0] = n_sub;
        shared[1] = 0;
    }
    __syncthreads();
    int kmin = n_sub;
    const int S_move = R.n_move;
    for (int g0 = 0; g0 < total; g0 += TP) {
        const int np = min(TP, total - g0);
        // ---- FK of the tile's configurations: slot wave * TP / NW + lane / LPC
        // takes point g0 + slot, on LPC lanes (a quad when the wave's share of
        // the tile leaves room for it)
        constexpr int CPW = TP / NW;
        constexpr int LPC = (PRRTC_FK_QUAD && 4 * CPW <= kWave) ? 4 : 1;
        // a tile that fits half the waves' shares, of a two-chain robot: the
        // first half of the waves takes chain 0 of the configurations, the
        // second half chain 1 (the FK's latency halves; the waves past the
        // configurations would idle anyway)
        constexpr int HALF = NW >= 2 ? NW / 2 : 1;
        const bool by_chain = NW >= 2 && LPC == 4 && R.n_chains == 2 && np <= CPW * HALF;
        const int chain = wave / HALF;
        const int slot = (by_chain ? (wave % HALF) : wave) * CPW + lane / LPC;
        if (lane < CPW * LPC && slot < np) {
            const int g = g0 + slot;
            int k = 0;
            if (MULTI)
                while (k + 1 < n_sub && ws.sub_off[k + 1] <= g) ++k;
            const int i = i_first + (g - ws.sub_off[k]);
            const float t = (float)i / (float)ws.sub_n[k];
            const float* w0 = wp + k * dof;
            const float* w1 = w0 + dof;
            if (lane % LPC == 0) ws.pk[slot] = k;
            auto qf = [&](int j) { return fmaf(t, w1[j] - w0[j], w0[j]); };
            if (LPC == 4)
                fk_rows<false>(R, qf, ws.frames + slot * fstride, lane & 3, by_chain ? chain : 0,
                               by_chain ? chain + 1 : kMaxChains);
            else
                fk_frames<false>(R, qf, ws.frames + slot * fstride);
        }
        __syncthreads();
        // ---- two-stage checks, stage 1: every (coarse sphere, configuration)
        // item against the obstacles, no early exit; a flagged item lets its
        // fine spheres through to the (point, sphere) pass below
        const bool two = TWO && R.n_cmove > 0;   // TWO: compiled with the two-stage pass
        int nitems = np * S_move;
        if (two) {
            const int n1 = np * R.n_cmove;
            for (int base = wave * kWave * B; base < n1; base += NW * kWave * B) {
                float cx[B], cy[B], cz[B], cr[B];
                bool hit[B];
                float lx = 3.0e38f, ly = 3.0e38f, lz = 3.0e38f, hx = -3.0e38f, hy = -3.0e38f, hz = -3.0e38f;
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int it = min(base + lane + kWave * b, n1 - 1);
                    const int c = it / np, p = it - c * np;
                    const float4 loc = R.csph[c];
                    const float3 w = frame_apply(ws.frames + p * fstride + R.cslot3[c], loc.x, loc.y, loc.z);
                    cx[b] = w.x; cy[b] = w.y; cz[b] = w.z; cr[b] = loc.w;
                    hit[b] = false;
                    lx = fminf(lx, w.x - loc.w); hx = fmaxf(hx, w.x + loc.w);
                    ly = fminf(ly, w.y - loc.w); hy = fmaxf(hy, w.y + loc.w);
                    lz = fminf(lz, w.z - loc.w); hz = fmaxf(hz, w.z + loc.w);
                }
                wave_box(lx, ly, lz, hx, hy, hz);
                auto gate = [&](auto&& exact) {
#pragma unroll
                    for (int b = 0; b < B; ++b) hit[b] |= exact(cx[b], cy[b], cz[b], cr[b]);
                    return false;   // no early exit: every flag is needed
                };
                cull_sweep<BOX_FIRST>(
                    S, ws.bnd0, ws.ext0, lx, ly, lz, hx, hy, hz,
                    [&](int oi) { return gate([&](float x, float y, float z, float r) { return hit_sphere(x, y, z, r, ld_sph(S, oi)); }); },
                    [&](int oi) { return gate([&](float x, float y, float z, float r) { return hit_box(x, y, z, r, ld_box(S, oi)); }); },
                    [&](int oi) { return gate([&](float x, float y, float z, float r) { return hit_cyl(x, y, z, r, ld_cyl(S, oi)); }); });
                // the interpolated field changes by at most esdf_gate per metre
                // (>= 1), so a fine sphere that meets it lies in a coarse
                // sphere whose radius, scaled by esdf_gate, meets it
#pragma unroll
                for (int b = 0; b < B; ++b)
                    if (S.esdf) hit[b] |= hit_esdf(cx[b], cy[b], cz[b], S.esdf_gate * cr[b] + kCoarseMargin, S);
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int it = base + lane + kWave * b;
                    if (it < n1) ws.cflag[it] = hit[b] ? 1 : 0;
                }
            }
            __syncthreads();
            // the fine items of the flagged coarse items, coarse-major
            if (wave == 0) {
                int total2 = 0;
                for (int b0 = 0; b0 < n1; b0 += kWave) {
                    const int it = b0 + lane;
                    int cnt = 0, f0 = 0, p = 0;
                    if (it < n1 && ws.cflag[it]) {
                        const int c = it / np;
                        p = it - c * np;
                        f0 = R.cfirst[c];
                        cnt = R.cfirst[c + 1] - f0;
                    }
                    int incl = cnt;
#pragma unroll
                    for (int off = 1; off < kWave; off <<= 1) {
                        const int v = __shfl_up(incl, off, kWave);
                        if (lane >= off) incl += v;
                    }
                    const int at = total2 + incl - cnt;
                    for (int k = 0; k < cnt; ++k) ws.list[at + k] = ((f0 + k) << 8) | p;
                    total2 += __shfl(incl, kWave - 1, kWave);
                }
                if (lane == 0) *ws.list_n = total2;
            }
            __syncthreads();
            nitems = *ws.list_n;
        }
        // ---- (point, sphere) items, against the obstacles

        // it / np as a multiply and shift: with m = ceil(2^20 / np), (it m) >> 20
        // equals floor(it / np) for it < np * 256 and np <= 64 (the rounding
        // excess it (m - 2^20 / np) / 2^20 stays below 1/64 <= 1/np), and
        // it m < 2^32
        const unsigned div_m = kFastDiv.m[np];
        bool stop = false;
        for (int base = wave * kWave * B; base < nitems && !stop; base += NW * kWave * B) {
            if (NW > 1 && !MULTI && shared[1]) break;   // another wave found a hit
            float cx[B], cy[B], cz[B], cr[B];
            int ck[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int it = min(base + lane + kWave * b, nitems - 1);
#if PRRTC_ITEM_ORDER == 1
#if PRRTC_FASTDIV
                // sphere-major; the low 20 bits of it m are (it mod np) / np
                // in 2^-20 units plus less than it / 2^20 < 1 / np, so
                // scaling them by np and dropping 20 bits gives it mod np
                const unsigned itm = (unsigned)it * div_m;
                int s = (int)(itm >> 20);
                int p = (int)(__umul24(itm & 0xFFFFFu, (unsigned)np) >> 20);
#else
                int s = it / np;
                int p = it - s * np;
#endif
#else
                int p = it / S_move;      // point-major
                int s = it - p * S_move;
#endif
                if (two) {
                    const int e = ws.list[it];
                    s = e >> 8;
                    p = e & 255;
                }
                const float4 loc = ws.sph[s];
                const float3 c = frame_apply(ws.frames + __umul24((unsigned)p, (unsigned)fstride) + ws.slot3[s], loc.x,
                                             loc.y, loc.z);
                cx[b] = c.x; cy[b] = c.y; cz[b] = c.z; cr[b] = loc.w;
                ck[b] = MULTI ? ws.pk[p] : 0;
            }
            if (MULTI) {
                bool alive = false;
#pragma unroll
                for (int b = 0; b < B; ++b) alive |= ck[b] < kmin;
                if (!__any(alive)) continue;
            }
            // One obstacle against the lane's B items.  Returns true when the
            // block (single sub-edge: the whole check) is decided.
            auto test = [&](auto&& hit) -> bool {
                // one vote per item slot, OR-ed as wave masks (the compares'
                // own masks, no per-lane boolean to re-vote)
                unsigned long long votes = 0;
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const bool h = hit(cx[b], cy[b], cz[b], cr[b]);
                    votes |= __ballot(MULTI ? (h && ck[b] < kmin) : h);
                }
                if (!votes) return false;
                if (!MULTI) return true;
                int mk = 0x7fffffff;
#pragma unroll
                for (int b = 0; b < B; ++b)
                    if (ck[b] < kmin && hit(cx[b], cy[b], cz[b], cr[b])) mk = min(mk, ck[b]);
                kmin = min(kmin, wave_min_int(mk));
                bool alive = false;
#pragma unroll
                for (int b = 0; b < B; ++b) alive |= ck[b] < kmin;
                return !__any(alive);
            };
#if PRRTC_CULL
            // Axis-aligned box around the block's item spheres; every lane
            // tests one obstacle's bounding sphere against it, and only the
            // obstacles that reach the box get exact tests.  The 1e-4 m margin
            // on the bounding radii keeps culling from changing any verdict.
            float lx = 3.0e38f, ly = 3.0e38f, lz = 3.0e38f;
            float hx = -3.0e38f, hy = -3.0e38f, hz = -3.0e38f;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (!MULTI || ck[b] < kmin) {
                    lx = fminf(lx, cx[b] - cr[b]); hx = fmaxf(hx, cx[b] + cr[b]);
                    ly = fminf(ly, cy[b] - cr[b]); hy = fmaxf(hy, cy[b] + cr[b]);
                    lz = fminf(lz, cz[b] - cr[b]); hz = fmaxf(hz, cz[b] + cr[b]);
                }
            }
            wave_box(lx, ly, lz, hx, hy, hz);
            // Cuboids and cylinders must also reach the block's box with
            // their own world-axis box where the scene keeps them (far
            // tighter than the bounding sphere for flat or long ones, such as
            // shelf boards).
            bool done = cull_sweep<BOX_FIRST>(
                S, ws.bnd0, ws.ext0, lx, ly, lz, hx, hy, hz,
                [&](int oi) { return test([&](float x, float y, float z, float r) { return hit_sphere(x, y, z, r, ld_sph(S, oi)); }); },
                [&](int oi) { return test([&](float x, float y, float z, float r) { return hit_box(x, y, z, r, ld_box(S, oi)); }); },
                [&](int oi) { return test([&](float x, float y, float z, float r) { return hit_cyl(x, y, z, r, ld_cyl(S, oi)); }); });
            // an attached ESDF grid: every item, one interpolated lookup each
            if (S.esdf && !done) done = test([&](float x, float y, float z, float r) { return hit_esdf(x, y, z, r, S); });
#else
            // obstacles in groups of U between ballots (a tail group re-tests
            // its last obstacle, which cannot change the verdict)
            constexpr int U = PRRTC_OBS_GROUP;
            bool done = false;
            for (int o = 0; o < S.n_sph && !done; o += U) {
                float4 ob[U];
#pragma unroll
                for (int u = 0; u < U; ++u) ob[u] = ld_sph(S, min(o + u, S.n_sph - 1));
                done = test([&](float x, float y, float z, float r) {
                    bool h = false;
#pragma unroll
                    for (int u = 0; u < U; ++u) h |= hit_sphere(x, y, z, r, ob[u]);
                    return h;
                });
            }
            for (int o = 0; o < S.n_box && !done; o += U) {
                Box ob[U];
#pragma unroll
                for (int u = 0; u < U; ++u) ob[u] = ld_box(S, min(o + u, S.n_box - 1));
                done = test([&](float x, float y, float z, float r) {
                    bool h = false;
#pragma unroll
                    for (int u = 0; u < U; ++u) h |= hit_box(x, y, z, r, ob[u]);
                    return h;
                });
            }
            if (S.esdf && !done) done = test([&](float x, float y, float z, float r) { return hit_esdf(x, y, z, r, S); });
            for (int o = 0; o < S.n_cyl && !done; o += U) {
                Cyl ob[U];
#pragma unroll
                for (int u = 0; u < U; ++u) ob[u] = ld_cyl(S, min(o + u, S.n_cyl - 1));
                done = test([&](float x, float y, float z, float r) {
                    bool h = false;
#pragma unroll
                    for (int u = 0; u < U; ++u) h |= hit_cyl(x, y, z, r, ob[u]);
                    return h;
                });
            }
#endif
            if (!MULTI && done) {
                kmin = 0;
                stop = true;
                if (NW > 1 && lane == 0) shared[1] = 1;
            }
        }
        // ---- self collision, bipartite groups: per configuration, lanes
        // hold group A's spheres; group B's spheres (one per lane) are culled
        // against A's bounding box and the survivors tested against all of A.
        if (R.n_bip_a > 0 && (MULTI || kmin == n_sub)) {
            for (int p = wave; p < np; p += NW) {
                if (NW > 1 && !MULTI && shared[1]) break;
                const int k = MULTI ? ws.pk[p] : 0;
                if (k >= kmin) continue;
                const float4* fp = ws.frames + p * fstride;
                auto centre = [&](int s) {
                    if (s >= S_move) return fixed_world(R, s);
                    const float4 l = ws.sph[s];
                    const float3 c = frame_apply(fp + ws.slot3[s], l.x, l.y, l.z);
                    return make_float4(c.x, c.y, c.z, l.w);
                };
                bool hit = false;
                for (int a0 = 0; a0 < R.n_bip_a && !hit; a0 += kWave) {
                    const bool va = a0 + lane < R.n_bip_a;
                    const float4 ca = va ? centre(R.bip_a[a0 + lane]) : make_float4(0.f, 0.f, 0.f, 0.f);
                    float lx = va ? ca.x - ca.w : 3.0e38f, ly = va ? ca.y - ca.w : 3.0e38f;
                    float lz = va ? ca.z - ca.w : 3.0e38f, hx = va ? ca.x + ca.w : -3.0e38f;
                    float hy = va ? ca.y + ca.w : -3.0e38f, hz = va ? ca.z + ca.w : -3.0e38f;
                    wave_box(lx, ly, lz, hx, hy, hz);
                    for (int b0 = 0; b0 < R.n_bip_b && !hit; b0 += kWave) {
                        const bool vb = b0 + lane < R.n_bip_b;
                        const float4 cb = vb ? centre(R.bip_b[b0 + lane]) : make_float4(0.f, 0.f, 0.f, 0.f);
                        const bool keep =
                            vb && sphere_meets_box(make_float4(cb.x, cb.y, cb.z, cb.w + 1e-4f), lx, ly, lz, hx, hy, hz);
                        unsigned long long m = __ballot(keep);
                        while (m && !hit) {
                            const int j = (int)__builtin_ctzll(m);
                            m &= m - 1;
                            const float4 c = make_float4(__shfl(cb.x, j, kWave), __shfl(cb.y, j, kWave),
                                                         __shfl(cb.z, j, kWave), __shfl(cb.w, j, kWave));
                            hit = __any(va && hit_pair(ca, c));
                        }
                    }
                }
                if (hit) {
                    kmin = k;
                    if (!MULTI) {
                        if (NW > 1 && lane == 0) shared[1] = 1;
                        break;
                    }
                }
            }
        }
        // ---- self-collision pairs: (point, pair) items, point-major
        if (R.n_pairs > 0 && (MULTI || kmin == n_sub)) {
            const int npi = np * R.n_pairs;
            for (int base = wave * kWave; base < npi; base += NW * kWave) {
                const int it = min(base + lane, npi - 1);
                const int p = it / R.n_pairs;
                const int pr_i = it - p * R.n_pairs;
                const int k = MULTI ? ws.pk[p] : 0;
                const int2 pr = R.pairs[pr_i];
                const float4* fp = ws.frames + p * fstride;
                auto centre = [&](int s) {
                    if (s >= S_move) return fixed_world(R, s);
                    const float4 l = ws.sph[s];
                    const float3 c = frame_apply(fp + ws.slot3[s], l.x, l.y, l.z);
                    return make_float4(c.x, c.y, c.z, l.w);
                };
                const float4 ca = centre(pr.x), cb = centre(pr.y);
                const bool h = hit_pair(ca, cb) && k < kmin;
                if (__any(h)) {
                    kmin = min(kmin, wave_min_int(h ? k : 0x7fffffff));
                    if (!MULTI) break;
                }
            }
        }
        if (NW > 1) {
            if (lane == 0 && kmin < n_sub) atomicMin((int*)&shared[0], kmin);
            __syncthreads();
            kmin = shared[0];
            __syncthreads();
        } else {
            __syncthreads();
        }
        if (kmin < n_sub) return kmin;
    }
    return kmin;
}

}  // namespace prrtc
