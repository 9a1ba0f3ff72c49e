// prrtc_proposal.h -- learned sampling proposal on gfx950: voxel grid, MLP
// with BF16 matrix-core products (FP32 accumulate), Gaussian-mixture head,
// training by backpropagation and Adam.
//
// Model: e = vox W_v + b_v (4096 -> 256); x0 = [s_hat, g_hat, e] (start and
// goal scaled to [-1, 1] by the joint limits); h_l = GELU(h_{l-1} W_l + b_l)
// for three layers of 256; o = h_3 W_4 + b_4 = K mixture logits, K x dof means
// and K x dof log standard deviations (clamped to [-5, 2]), K = 8.  Every
// matrix product rounds both operands to bfloat16 (nearest even) and
// accumulates in FP32.  Weights are stored [in][out], row-major, FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "prrtc_device.h"

namespace prrtc {

constexpr int kComp = 8;
constexpr int kHidden = 256;
constexpr int kVox = 16;
constexpr int kVoxCells = kVox * kVox * kVox;
constexpr float kLogSigLo = -5.0f, kLogSigHi = 2.0f;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f_acc __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even.
__device__ inline unsigned short bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ---------------------------------------------------------------------------
// Voxel grid: cell (x, y, z) has centre -0.8 + 0.1 (i + 0.5); it is occupied
// iff some obstacle is strictly closer than the half diagonal 0.05 sqrt(3).
// ---------------------------------------------------------------------------
__global__ void k_voxelize(SceneArgs S, uint8_t* __restrict__ vox) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kVoxCells) return;
    const int x = i % kVox, y = (i / kVox) % kVox, z = i / (kVox * kVox);
    const float cx = -0.8f + 0.1f * ((float)x + 0.5f);
    const float cy = -0.8f + 0.1f * ((float)y + 0.5f);
    const float cz = -0.8f + 0.1f * ((float)z + 0.5f);
    const float h = 0.086602540378443865f;
    bool occ = false;
    for (int o = 0; o < S.n_sph; ++o) occ |= hit_sphere(cx, cy, cz, h, ld_sph(S, o));
    for (int o = 0; o < S.n_box; ++o) occ |= hit_box(cx, cy, cz, h, ld_box(S, o));
    for (int o = 0; o < S.n_cyl; ++o) occ |= hit_cyl(cx, cy, cz, h, ld_cyl(S, o));
    vox[i] = occ ? 1 : 0;
}

// ---------------------------------------------------------------------------
// C[M][N] = op(A)[M][K] op(B)[K][N] (+ bias[N]); optional GELU epilogue that
// keeps the pre-activation in Z and writes GELU(Z) to C.  op(A) = A
// ([M][lda]) or A^T ([K][lda]); op(B) = B ([K][ldb]) or B^T ([N][ldb]).
// Block tile 64 x 64, K step 32, 256 threads; each wave owns a 32 x 32
// quarter as 2 x 2 tiles of gfx950's v_mfma_f32_16x16x32_bf16 (lane l holds
// row / column l % 16 and k = 8 (l / 16) .. 8 (l / 16) + 7 of its operands).
// Operands are rounded to bfloat16 while staged into LDS; the next K step's
// global values are loaded into registers while the current one multiplies.
// With k_chunk > 0 (split K, for shapes with few output tiles and a long K)
// blockIdx.z takes k = z k_chunk .. (z + 1) k_chunk - 1 and writes its plain
// partial product to C + z M ldc (no bias or GELU); k_split_sum adds the
// partials in order.
// ---------------------------------------------------------------------------
constexpr int kGemmBM = 64, kGemmBN = 64, kGemmBK = 32;
constexpr int kGemmLd = kGemmBK + 8;   // LDS row: 80 bytes, 16-byte aligned fragments

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <typename TA, bool TRANS_A, bool TRANS_B, bool GELU>
__global__ __launch_bounds__(256) void k_gemm_bf16(const TA* __restrict__ A, int lda,
                                                   const float* __restrict__ Bm, int ldb,
                                                   const float* __restrict__ bias,
                                                   float* __restrict__ C, float* __restrict__ Z, int ldc,
                                                   int M, int N, int K, int k_chunk) {
    __shared__ __attribute__((aligned(16))) unsigned short As[kGemmBM][kGemmLd];   // [row][k]
    __shared__ __attribute__((aligned(16))) unsigned short Bt[kGemmBN][kGemmLd];   // [col][k]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int row0 = blockIdx.y * kGemmBM, col0 = blockIdx.x * kGemmBN;
    const int wr = wave >> 1, wc = wave & 1;
    v4f_acc acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = v4f_acc{0.f, 0.f, 0.f, 0.f};
    // staging: 64 x 32 of A and 32 x 64 of B, 8 elements per thread each.
    // Element e of thread t, idx = t + 256 e, is (row or column, k) =
    // (idx / 32, idx % 32) when the operand is contiguous along k, else
    // (idx % 64, idx / 64): consecutive threads read consecutive addresses.
    auto rk = [](int idx, bool along_k, int& r, int& k) {
        if (along_k) {
            r = idx / kGemmBK;
            k = idx % kGemmBK;
        } else {
            r = idx % kGemmBM;
            k = idx / kGemmBM;
        }
    };
    const int kb = k_chunk > 0 ? (int)blockIdx.z * k_chunk : 0;
    const int ke = k_chunk > 0 ? min(K, kb + k_chunk) : K;
    float ra[8], rb[8];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = tid + 256 * e;
            int r, k;
            rk(idx, !TRANS_A, r, k);
            const int gr = row0 + r, gka = k0 + k;
            ra[e] = (gr < M && gka < ke) ? (float)(TRANS_A ? A[(size_t)gka * lda + gr] : A[(size_t)gr * lda + gka])
                                        : 0.0f;
            rk(idx, TRANS_B, r, k);
            const int gc = col0 + r, gkb = k0 + k;
            rb[e] = (gc < N && gkb < ke) ? (TRANS_B ? Bm[(size_t)gc * ldb + gkb] : Bm[(size_t)gkb * ldb + gc]) : 0.0f;
        }
    };
    fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += kGemmBK) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = tid + 256 * e;
            int r, k;
            rk(idx, !TRANS_A, r, k);
            As[r][k] = bf16_bits(ra[e]);
            rk(idx, TRANS_B, r, k);
            Bt[r][k] = bf16_bits(rb[e]);
        }
        __syncthreads();
        if (k0 + kGemmBK < ke) fetch(k0 + kGemmBK);   // in flight during the products
        const int kk = 8 * (lane >> 4);
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
            const int ar = 32 * wr + 16 * mi + (lane & 15);
            const v8bf av = *reinterpret_cast<const v8bf*>(&As[ar][kk]);
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) {
                const int bc = 32 * wc + 16 * ni + (lane & 15);
                const v8bf bv = *reinterpret_cast<const v8bf*>(&Bt[bc][kk]);
                acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[mi][ni], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // lane holds rows 4 (lane / 16) + i, column lane % 16 of each 16 x 16 tile
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = row0 + 32 * wr + 16 * mi + 4 * (lane >> 4) + i;
                const int c = col0 + 32 * wc + 16 * ni + (lane & 15);
                if (r < M && c < N && k_chunk > 0) {
                    C[(size_t)blockIdx.z * M * ldc + (size_t)r * ldc + c] = acc[mi][ni][i];
                } else if (r < M && c < N) {
                    float v = acc[mi][ni][i] + (bias ? bias[c] : 0.0f);
                    if (GELU) {
                        Z[(size_t)r * ldc + c] = v;
                        v = 0.5f * v * (1.0f + erff(v * 0.70710678118654752f));
                    }
                    C[(size_t)r * ldc + c] = v;
                }
            }
}

// C[r][c] = bias[c] + the ks split-K partials P[z][r][c] (ld = ldc), added in
// z order.
__global__ void k_split_sum(const float* __restrict__ P, int ks, int M, int N, int ldc, const float* __restrict__ bias,
                            float* __restrict__ C) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * N) return;
    const int r = i / N, c = i - r * N;
    float v = 0.0f;
    for (int z = 0; z < ks; ++z) v += P[(size_t)z * M * ldc + (size_t)r * ldc + c];
    C[(size_t)r * ldc + c] = v + (bias ? bias[c] : 0.0f);
}

// x0[b] = [s_hat, g_hat, E[scene_of[b]]]; q_hat likewise when q is given.
__global__ void k_build_x0(const float* __restrict__ s, const float* __restrict__ g,
                           const float* __restrict__ q, const int* __restrict__ scene_of,
                           const float* __restrict__ E, const float* __restrict__ lo,
                           const float* __restrict__ hi, int n, int dof, float* __restrict__ x0,
                           float* __restrict__ q_hat) {
    const int D = 2 * dof + kHidden;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * D) return;
    const int b = i / D, c = i - b * D;
    float v;
    if (c < 2 * dof) {
        const int j = c % dof;
        const float x = c < dof ? s[b * dof + j] : g[b * dof + j];
        v = 2.0f * (x - lo[j]) / (hi[j] - lo[j]) - 1.0f;
    } else {
        v = E[(size_t)scene_of[b] * kHidden + (c - 2 * dof)];
    }
    x0[i] = v;
    if (q && c < dof) q_hat[b * dof + c] = 2.0f * (q[b * dof + c] - lo[c]) / (hi[c] - lo[c]) - 1.0f;
}

// Mixture head, one thread per sample: clamps log sigma, writes the mixture
// (logits, means, clamped log sigmas) and, given a target, its NLL and the
// gradient of the batch-mean NLL with respect to the head output.
__global__ void k_gmm_head(const float* __restrict__ O, int n, int dof, const float* __restrict__ q_hat,
                           float* __restrict__ gmm, float* __restrict__ nll, float* __restrict__ dO,
                           float inv_batch) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const int Cw = kComp * (1 + 2 * dof);
    const float* o = O + (size_t)b * Cw;
    float* out = gmm ? gmm + (size_t)b * Cw : nullptr;
    float lmax = -3.0e38f;
    for (int k = 0; k < kComp; ++k) lmax = fmaxf(lmax, o[k]);
    float lse = 0.0f;
    for (int k = 0; k < kComp; ++k) lse += expf(o[k] - lmax);
    lse = lmax + logf(lse);
    if (out) {
        for (int k = 0; k < kComp; ++k) out[k] = o[k];
        for (int t = kComp; t < kComp * (1 + dof); ++t) out[t] = o[t];
        for (int t = kComp * (1 + dof); t < Cw; ++t) out[t] = fminf(fmaxf(o[t], kLogSigLo), kLogSigHi);
    }
    if (!q_hat) return;
    const float* q = q_hat + (size_t)b * dof;
    float a[kComp];
    float amax = -3.0e38f;
    for (int k = 0; k < kComp; ++k) {
        float s = o[k] - lse;
        for (int j = 0; j < dof; ++j) {
            const float ls = fminf(fmaxf(o[kComp * (1 + dof) + k * dof + j], kLogSigLo), kLogSigHi);
            const float z = (q[j] - o[kComp + k * dof + j]) * expf(-ls);
            s += -0.5f * z * z - ls - 0.91893853320467274f;
        }
        a[k] = s;
        amax = fmaxf(amax, s);
    }
    float den = 0.0f;
    for (int k = 0; k < kComp; ++k) den += expf(a[k] - amax);
    nll[b] = -(amax + logf(den));
    float* d = dO + (size_t)b * Cw;
    for (int k = 0; k < kComp; ++k) {
        const float r = expf(a[k] - amax) / den;
        d[k] = (expf(o[k] - lse) - r) * inv_batch;
        for (int j = 0; j < dof; ++j) {
            const float raw = o[kComp * (1 + dof) + k * dof + j];
            const float ls = fminf(fmaxf(raw, kLogSigLo), kLogSigHi);
            const float isg = expf(-ls);
            const float z = (q[j] - o[kComp + k * dof + j]) * isg;
            d[kComp + k * dof + j] = -r * z * isg * inv_batch;
            const bool inside = raw >= kLogSigLo && raw <= kLogSigHi;
            d[kComp * (1 + dof) + k * dof + j] = inside ? -r * (z * z - 1.0f) * inv_batch : 0.0f;
        }
    }
}

// ---------------------------------------------------------------------------
// Inference for a handful of queries (planning): the matrix-core GEMM's
// 64-row tiles would be almost empty, and the 4096-deep embedding would run
// on four workgroups.  Instead:
//   k_embed_partial: grid (kEmbedSlices), 256 threads (one per output
//     column); slice z sums bf16(W_v[k][col]) over its 64 cells k that are
//     occupied, for every scene row (at most kSmallRows);
//   k_embed_reduce: E[s][col] = b_v[col] + the slices' partial sums, in
//     slice order;
//   k_mlp_rows: one workgroup per query row, activations in LDS, each layer
//     a BF16-operand FP32-accumulate dot product per output column (k split
//     four ways, the quarters added in order), GELU, and the mixture head
//     (log sigma clamped).
// Same arithmetic as the GEMM path (BF16 operands, FP32 sums); only the
// order of the sums differs.
// ---------------------------------------------------------------------------
constexpr int kEmbedSlices = 64;
constexpr int kSmallRows = 16;

__device__ inline float bf16_round(float x) { return __uint_as_float((unsigned)bf16_bits(x) << 16); }

__global__ __launch_bounds__(256) void k_embed_partial(const uint8_t* __restrict__ vox, int S,
                                                       const float* __restrict__ Wv, float* __restrict__ part) {
    const int z = blockIdx.x, col = threadIdx.x;
    constexpr int kCells = kVoxCells / kEmbedSlices;
    float acc[kSmallRows];
#pragma unroll
    for (int r = 0; r < kSmallRows; ++r) acc[r] = 0.0f;
    for (int c = 0; c < kCells; ++c) {
        const int k = z * kCells + c;
        const float w = bf16_round(Wv[(size_t)k * kHidden + col]);
#pragma unroll
        for (int r = 0; r < kSmallRows; ++r)
            if (r < S && vox[(size_t)r * kVoxCells + k]) acc[r] += w;
    }
    for (int r = 0; r < S; ++r) part[((size_t)z * kSmallRows + r) * kHidden + col] = acc[r];
}

__global__ __launch_bounds__(256) void k_embed_reduce(const float* __restrict__ part, const float* __restrict__ bv,
                                                      float* __restrict__ E) {
    const int r = blockIdx.x, col = threadIdx.x;
    float e = 0.0f;
    for (int z = 0; z < kEmbedSlices; ++z) e += part[((size_t)z * kSmallRows + r) * kHidden + col];
    E[(size_t)r * kHidden + col] = e + bv[col];
}

// out[col] = act(sum_k bf16(x[k]) bf16(W[k][col]) + b[col]) for col < N <= kHidden.
// kRowSplit groups of kHidden threads each sum a quarter of k (loads issued
// eight at a time), and the quarters are added in order: a short dependent
// chain per thread instead of one K-long chain of loads.
constexpr int kRowSplit = 4;
constexpr int kRowThreads = kRowSplit * kHidden;

template <bool GELU>
__device__ inline void row_layer(const float* __restrict__ x, int K, const float* __restrict__ W, int N,
                                 const float* __restrict__ b, float* __restrict__ out, float* red) {
    const int c = threadIdx.x % kHidden, part = threadIdx.x / kHidden;
    const int k0 = K * part / kRowSplit, k1 = K * (part + 1) / kRowSplit;
    for (int c0 = 0; c0 < N; c0 += kHidden) {   // uniform: every thread takes each pass
        const int col = c0 + c;
        float acc = 0.0f;
        if (col < N) {
            int k = k0;
            for (; k + 8 <= k1; k += 8) {
                float w[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) w[u] = bf16_round(W[(size_t)(k + u) * N + col]);
#pragma unroll
                for (int u = 0; u < 8; ++u) acc = fmaf(x[k + u], w[u], acc);
            }
            for (; k < k1; ++k) acc = fmaf(x[k], bf16_round(W[(size_t)k * N + col]), acc);
        }
        red[part * kHidden + c] = acc;
        __syncthreads();
        if (part == 0 && col < N) {
            float v = red[c];
#pragma unroll
            for (int q = 1; q < kRowSplit; ++q) v += red[q * kHidden + c];
            v += b[col];
            if (GELU) v = 0.5f * v * (1.0f + erff(v * 0.70710678118654752f));
            out[col] = v;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kRowThreads) void k_mlp_rows(const float* __restrict__ s, const float* __restrict__ g,
                                                          const int* __restrict__ scene_of, const float* __restrict__ E,
                                                          const float* __restrict__ lo, const float* __restrict__ hi,
                                                          int dof, const float* __restrict__ W1,
                                                          const float* __restrict__ b1, const float* __restrict__ W2,
                                                          const float* __restrict__ b2, const float* __restrict__ W3,
                                                          const float* __restrict__ b3, const float* __restrict__ W4,
                                                          const float* __restrict__ b4, float* __restrict__ gmm) {
    __shared__ float xa[2 * kMaxDof + kHidden];
    __shared__ float xb[kComp * (1 + 2 * kMaxDof) > kHidden ? kComp * (1 + 2 * kMaxDof) : kHidden];
    __shared__ float red[kRowThreads];
    const int row = blockIdx.x, t = threadIdx.x;
    const int D0 = 2 * dof + kHidden, Cw = kComp * (1 + 2 * dof);
    for (int c = t; c < D0; c += blockDim.x) {
        float v;
        if (c < 2 * dof) {
            const int j = c % dof;
            const float x = c < dof ? s[row * dof + j] : g[row * dof + j];
            v = 2.0f * (x - lo[j]) / (hi[j] - lo[j]) - 1.0f;
        } else {
            v = E[(size_t)scene_of[row] * kHidden + (c - 2 * dof)];
        }
        xa[c] = bf16_round(v);
    }
    __syncthreads();
    row_layer<true>(xa, D0, W1, kHidden, b1, xb, red);
    __syncthreads();
    for (int c = t; c < kHidden; c += blockDim.x) xa[c] = bf16_round(xb[c]);
    __syncthreads();
    row_layer<true>(xa, kHidden, W2, kHidden, b2, xb, red);
    __syncthreads();
    for (int c = t; c < kHidden; c += blockDim.x) xa[c] = bf16_round(xb[c]);
    __syncthreads();
    row_layer<true>(xa, kHidden, W3, kHidden, b3, xb, red);
    __syncthreads();
    for (int c = t; c < kHidden; c += blockDim.x) xa[c] = bf16_round(xb[c]);
    __syncthreads();
    row_layer<false>(xa, kHidden, W4, Cw, b4, xb, red);
    __syncthreads();
    float* out = gmm + (size_t)row * Cw;
    for (int c = t; c < Cw; c += blockDim.x)
        out[c] = c < kComp * (1 + dof) ? xb[c] : fminf(fmaxf(xb[c], kLogSigLo), kLogSigHi);
}

// ---------------------------------------------------------------------------
// The mixture of one query computed by one planner workgroup inside a
// persistent launch (batched and served learned queries), from the scene's
// grid embedding.  Same operands, rounding and order of every sum as
// k_mlp_rows: each output column is kRowSplit sequential FMA chains over the
// quarters of k, added in order, then the bias; so the mixture equals the one
// a single plan computes with k_mlp_rows.
// ---------------------------------------------------------------------------
struct ModelDev {
    const float *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
    int dof, pad;
};

constexpr int kMlpInFloats = 2 * kMaxDof + kHidden;                 // LDS: layer input
constexpr int kMlpOutFloats = kComp * (1 + 2 * kMaxDof) > kHidden ? kComp * (1 + 2 * kMaxDof) : kHidden;

template <bool GELU>
__device__ inline void block_layer(const float* x, int K, const float* __restrict__ W, int N,
                                   const float* __restrict__ b, float* out) {
    for (int col = threadIdx.x; col < N; col += blockDim.x) {
        int k0[kRowSplit], k1[kRowSplit];
        float acc[kRowSplit];
#pragma unroll
        for (int p = 0; p < kRowSplit; ++p) {
            k0[p] = K * p / kRowSplit;
            k1[p] = K * (p + 1) / kRowSplit;
            acc[p] = 0.0f;
        }
        // the chains side by side; each stays in order of k
        const int steps = k1[kRowSplit - 1] - k0[kRowSplit - 1];   // the longest quarter
        for (int i = 0; i < steps; ++i) {
#pragma unroll
            for (int p = 0; p < kRowSplit; ++p) {
                const int k = k0[p] + i;
                if (k < k1[p]) acc[p] = fmaf(x[k], bf16_round(W[(size_t)k * N + col]), acc[p]);
            }
        }
        float v = acc[0];
#pragma unroll
        for (int p = 1; p < kRowSplit; ++p) v += acc[p];
        v += b[col];
        if (GELU) v = 0.5f * v * (1.0f + erff(v * 0.70710678118654752f));
        out[col] = v;
    }
}

// x: LDS [kMlpInFloats], y: LDS [kMlpOutFloats]; ends(c): the query's start
// (c < dof) then goal (c - dof); lo, hi: the robot's limits; emb: the scene's
// embedding [kHidden]; out: the mixture [kComp (1 + 2 dof)] in global memory.
// Every thread of the workgroup must call it.
template <class Ends>
__device__ inline void mixture_in_block(const ModelDev& M, const float* __restrict__ emb, Ends ends,
                                        const float* lo, const float* hi, float* x, float* y,
                                        float* __restrict__ out) {
    const int dof = M.dof;
    const int D0 = 2 * dof + kHidden, Cw = kComp * (1 + 2 * dof);
    for (int c = threadIdx.x; c < D0; c += blockDim.x) {
        float v;
        if (c < 2 * dof) {
            const int j = c % dof;
            const float q = ends(c);
            v = 2.0f * (q - lo[j]) / (hi[j] - lo[j]) - 1.0f;
        } else {
            v = emb[c - 2 * dof];
        }
        x[c] = bf16_round(v);
    }
    __syncthreads();
    block_layer<true>(x, D0, M.W1, kHidden, M.b1, y);
    __syncthreads();
    for (int c = threadIdx.x; c < kHidden; c += blockDim.x) x[c] = bf16_round(y[c]);
    __syncthreads();
    block_layer<true>(x, kHidden, M.W2, kHidden, M.b2, y);
    __syncthreads();
    for (int c = threadIdx.x; c < kHidden; c += blockDim.x) x[c] = bf16_round(y[c]);
    __syncthreads();
    block_layer<true>(x, kHidden, M.W3, kHidden, M.b3, y);
    __syncthreads();
    for (int c = threadIdx.x; c < kHidden; c += blockDim.x) x[c] = bf16_round(y[c]);
    __syncthreads();
    block_layer<false>(x, kHidden, M.W4, Cw, M.b4, y);
    __syncthreads();
    for (int c = threadIdx.x; c < Cw; c += blockDim.x)
        out[c] = c < kComp * (1 + dof) ? y[c] : fminf(fmaxf(y[c], kLogSigLo), kLogSigHi);
}

// dZ = dH * GELU'(Z)
__global__ void k_gelu_bwd(const float* __restrict__ dH, const float* __restrict__ Z, float* __restrict__ dZ,
                           int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = Z[i];
    const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
    dZ[i] = dH[i] * (cdf + x * pdf);
}

// db[c] = sum over rows of D[r][c] (ld), fixed order: a workgroup of
// kColGroups x 64 threads takes 64 columns; thread (g, c) adds rows g,
// g + kColGroups, ... in order, and the group sums are added in g order.
constexpr int kColGroups = 16;
__global__ __launch_bounds__(kColGroups * 64) void k_col_sum(const float* __restrict__ D, int rows, int N, int ld,
                                                              int col_off, float* __restrict__ out) {
    __shared__ float part[kColGroups][64];
    const int cl = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cl;
    float s = 0.0f;
    if (c < N)
        for (int r = g; r < rows; r += kColGroups) s += D[(size_t)r * ld + col_off + c];
    part[g][cl] = s;
    __syncthreads();
    if (g == 0 && c < N) {
        float t = part[0][cl];
        for (int k = 1; k < kColGroups; ++k) t += part[k][cl];
        out[c] = t;
    }
}

// dE[s][c] = sum of dX0[b][2 dof + c] over the samples b of scene s
// (contiguous rows scene_start[s] .. scene_start[s + 1]), fixed order.
__global__ void k_scene_sum(const float* __restrict__ dX0, int ld, int off, const int* __restrict__ scene_start,
                            int n_scenes, float* __restrict__ dE) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_scenes * kHidden) return;
    const int s = i / kHidden, c = i - s * kHidden;
    float v = 0.0f;
    for (int b = scene_start[s]; b < scene_start[s + 1]; ++b) v += dX0[(size_t)b * ld + off + c];
    dE[i] = v;
}

// Adam: c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Mean of n values (one wave).
__global__ void k_mean(const float* __restrict__ x, int n, float* __restrict__ out) {
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += kWave) s += x[i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (threadIdx.x == 0) out[0] = s / (float)n;
}

// ---------------------------------------------------------------------------
// Sampling the mixture inside the planner.  All uniforms come from Philox4x32-10
// with counter (word0, worker, round, query), word0 in a range the uniform
// sampler never uses: 0x80000000 | attempt << 8 | slot.  Slot 255 holds the
// (mix, component) uniforms, slot 1 + j/2 the Box-Muller pair of joints j, j+1.
// Lane j produces joint j; every lane evaluates the component choice itself.
// Returns, uniformly across the wave, whether the draw lies inside the limits.
// ---------------------------------------------------------------------------
__device__ inline float philox_unit(uint32_t word) { return (float)(word >> 8) * 0x1p-24f; }

__device__ inline float mix_uniform(uint64_t seed, uint32_t query, uint32_t round, uint32_t worker,
                                    uint32_t attempt) {
    const uint4 w = philox4x32_10(make_uint4(0x80000000u | (attempt << 8) | 255u, worker, round, query),
                                  make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
    return philox_unit(w.x);
}

__device__ inline bool gmm_draw(const float* gmm, int dof, float lo_j, float hi_j, uint64_t seed, uint32_t query,
                                uint32_t round, uint32_t worker, uint32_t attempt, int j, float* out_j) {
    const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
    const uint4 wc = philox4x32_10(make_uint4(0x80000000u | (attempt << 8) | 255u, worker, round, query), key);
    const float uc = philox_unit(wc.y);
    float lmax = -3.0e38f;
    for (int k = 0; k < kComp; ++k) lmax = fmaxf(lmax, gmm[k]);
    float tot = 0.0f;
    for (int k = 0; k < kComp; ++k) tot += expf(gmm[k] - lmax);
    const float target = uc * tot;
    int comp = kComp - 1;
    float acc = 0.0f;
    for (int k = 0; k < kComp; ++k) {
        acc += expf(gmm[k] - lmax);
        if (target < acc) {
            comp = k;
            break;
        }
    }
    bool inside = true;
    if (j < dof) {
        const uint4 wn = philox4x32_10(
            make_uint4(0x80000000u | (attempt << 8) | (uint32_t)(1 + (j >> 1)), worker, round, query), key);
        const float u1 = ((float)(wn.x >> 8) + 1.0f) * 0x1p-24f;   // (0, 1]
        const float u2 = philox_unit(wn.y);
        const float rad = sqrtf(-2.0f * logf(u1));
        float sn, cs;
        sincosf(6.28318530717958648f * u2, &sn, &cs);
        const float z = (j & 1) ? rad * sn : rad * cs;
        const float mu = gmm[kComp + comp * dof + j];
        const float ls = gmm[kComp * (1 + dof) + comp * dof + j];
        const float xh = mu + expf(ls) * z;
        const float q = lo_j + 0.5f * (xh + 1.0f) * (hi_j - lo_j);
        *out_j = q;
        inside = q >= lo_j && q <= hi_j;
    }
    return !__any(!inside);
}

// Are all mixture parameters finite?  (wave-uniform)
__device__ inline bool gmm_finite(const float* gmm, int dof) {
    const int lane = threadIdx.x & (kWave - 1);
    bool ok = true;
    for (int t = lane; t < kComp * (1 + 2 * dof); t += kWave) ok &= isfinite(gmm[t]);
    return !__any(!ok);
}

// n mixture draws of one (query, round, attempt); draw i acts as worker i.
// One wave per draw.
__global__ void k_gmm_sample(const float* __restrict__ gmm, const RobotArgs* __restrict__ Rp, uint64_t seed,
                             uint32_t query, uint32_t round, uint32_t attempt, int n, float* __restrict__ out,
                             unsigned char* __restrict__ inside) {
    const RobotArgs& R = *Rp;
    const int i = blockIdx.x;
    const int j = threadIdx.x;
    const int dof = R.dof;
    if (i >= n) return;
    float v = 0.0f;
    const bool ok = gmm_draw(gmm, dof, j < dof ? pick(R.lo, j) : 0.0f, j < dof ? pick(R.hi, j) : 0.0f, seed, query,
                             round, (uint32_t)i, attempt, j, &v);
    if (j < dof) out[(size_t)i * dof + j] = v;
    if (j == 0) inside[i] = ok;
}

}  // namespace prrtc
