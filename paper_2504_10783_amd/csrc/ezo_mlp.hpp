// ezo_mlp.hpp -- kernels of the learned self-collision screen: a multilayer
// perceptron dof -> H -> H -> H -> 1 with SiLU activations that predicts a
// configuration's minimum self-collision signed distance from x = q / pi.
//
// Parameters (FP32 master copy, one flat vector):
//   W1[H][D] b1[H] W2[H][H] b2[H] W3[H][H] b3[H] W4[H] b4[1]   (z = W a + b)
// BF16 copies of W2 and W3 feed the MFMA GEMMs (FP32 accumulation); the
// first and last layers (K = dof and N = 1) run on the vector ALUs.
// Activations between layers are BF16; pre-activations kept for the
// backward pass are FP32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ezo_screen.hpp"

namespace ezo {

__device__ __forceinline__ const float* row_ptr(const RowSource& s, int64_t r, int64_t* stride) {
    r += s.rbase;
    int64_t cfg = s.idx ? (int64_t)s.idx[r] : r;
    const float* base = s.q;
    if (s.rows_per_batch > 0) {
        base += (r / s.rows_per_batch) * s.qb;
        cfg = r % s.rows_per_batch;
    }
    *stride = s.sd;
    return base + cfg * s.sn;
}

// Row r of this launch is inactive: past the valid rows, or in a batch
// (edge) whose status is final.
__device__ __forceinline__ bool row_inactive(const RowSource& s, int64_t r, const int* status) {
    if (r >= s.rows) return true;
    return status && s.rows_per_batch > 0 && status[(r + s.rbase) / s.rows_per_batch] >= 0;
}

// Layer 1 on the VALUs: z1 = W1 (q / pi) + b1; h1 = bf16(silu(z1)); z1 kept
// (FP32) when z1out != NULL.  One thread per (row, unit).
__global__ void __launch_bounds__(256) k_mlp_layer1(RowSource src, int64_t rows, int D, int H,
                                                    const float* __restrict__ P, float* __restrict__ z1out,
                                                    __bf16* __restrict__ h1, const int* __restrict__ status) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * H) return;
    const int64_t r = t / H;
    const int i = (int)(t % H);
    if (row_inactive(src, r, status)) {
        if (z1out) z1out[t] = 0.f;
        h1[t] = (__bf16)0.f;
        return;
    }
    const MlpOffsets o = mlp_offsets(D, H);
    int64_t sd;
    const float* x = row_ptr(src, r, &sd);
    float z = P[o.b1 + i];
    for (int j = 0; j < D; ++j) z = fmaf(P[o.W1 + (int64_t)i * D + j], x[j * sd] * kInvPi, z);
    if (z1out) z1out[t] = z;
    h1[t] = (__bf16)siluf(z);
}

// Output layer on the VALUs: y = W4 . h3 + b4, one thread per row.
__global__ void __launch_bounds__(256) k_mlp_out(RowSource src, int64_t rows, int D, int H, const float* __restrict__ P,
                                                 const __bf16* __restrict__ h3, float* __restrict__ y,
                                                 const int* __restrict__ status) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows || row_inactive(src, r, status)) return;
    const MlpOffsets o = mlp_offsets(D, H);
    const bf16x8* h = reinterpret_cast<const bf16x8*>(h3 + r * H);
    float s = P[o.b4];
    for (int k = 0; k < H / 8; ++k) {
        const bf16x8 v = h[k];
#pragma unroll
        for (int e = 0; e < 8; ++e) s = fmaf(P[o.W4 + 8 * k + e], (float)v[e], s);
    }
    y[r] = s;
}

// ---------------------------------------------------------------------------
// BF16 MFMA GEMM  C[M][N] = sum_k A(m, k) B(k, n)
// A(m, k) = A[m*sam + k*sak] with AK: sak == 1 (K contiguous) else sam == 1
// (M contiguous); B(k, n) = B[k*sbk + n*sbn] with BK: sbk == 1 else sbn == 1.
// M, N multiples of 64, K a multiple of 32, contiguous runs 16-byte aligned.
// Workgroup: 64x64 output tile, 4 waves of 32x32, each a 2x2 grid of
// v_mfma_f32_16x16x32_bf16.  Staging: every thread loads one 16-byte vector
// of A and one of B per K step (eight consecutive elements along the
// contiguous dimension) into LDS tiles held K-major ([row][k], 8-element
// pad).  Fragment layout (16x16x32): lane l holds A[row l%16][k 8(l/16)..+7],
// B[k 8(l/16)..+7][col l%16] and returns C[rows 4(l/16)..+3][col l%16].
// Split K: blockIdx.z takes K steps [z kc, (z + 1) kc); with gridDim.z > 1
// only GEMM_STORE is allowed and slice z writes C + z M ldc (partial sums,
// reduced by k_sum_slices).
// Epilogues: STORE C = acc (FP32); FWD z = acc + bias[n] -> C (optional),
// Hout = bf16(silu(z)); BWD Hout = bf16(acc * silu'(Z[m][n])).
// ---------------------------------------------------------------------------
enum { GEMM_STORE = 0, GEMM_FWD = 1, GEMM_BWD = 2 };

template <int EPI, bool AK, bool BK>
__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, int kc, const __bf16* __restrict__ A,
                                                   int64_t sam, int64_t sak, const __bf16* __restrict__ B,
                                                   int64_t sbk, int64_t sbn, float* __restrict__ C, int64_t ldc,
                                                   const float* __restrict__ bias, __bf16* __restrict__ Hout,
                                                   int64_t ldh, const float* __restrict__ Z, int64_t ldz,
                                                   const int* __restrict__ status, int64_t rows_per_batch,
                                                   int64_t rbase) {
    __shared__ __attribute__((aligned(16))) __bf16 As[64][40];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[64][40];
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    if (m0 >= M || n0 >= N) return;
    // tiles of finished edges are skipped (rows_per_batch is a multiple of 64)
    if (status && rows_per_batch > 0 && status[(m0 + rbase) / rows_per_batch] >= 0) return;
    const int kb0 = blockIdx.z * kc, kb1 = min(K, kb0 + kc);
    if (gridDim.z > 1) C += (int64_t)blockIdx.z * M * ldc;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    // this thread's staging vector: (row, k) of its eight elements
    const int ar = AK ? (tid >> 2) : ((tid & 7) * 8), ak = AK ? ((tid & 3) * 8) : (tid >> 3);
    const int br = BK ? (tid >> 2) : ((tid & 7) * 8), bk = BK ? ((tid & 3) * 8) : (tid >> 3);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb0; k0 < kb1; k0 += 32) {
        const bf16x8 av = *reinterpret_cast<const bf16x8*>(A + (int64_t)(m0 + ar) * sam + (int64_t)(k0 + ak) * sak);
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(B + (int64_t)(k0 + bk) * sbk + (int64_t)(n0 + br) * sbn);
        if (AK) {
            *reinterpret_cast<bf16x8*>(&As[ar][ak]) = av;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) As[ar + e][ak] = av[e];
        }
        if (BK) {
            *reinterpret_cast<bf16x8*>(&Bs[br][bk]) = bv;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) Bs[br + e][bk] = bv[e];
        }
        __syncthreads();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * i + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * j + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * j + (lane & 15);
                const float v = acc[i][j][r];
                if (EPI == GEMM_STORE) {
                    C[(int64_t)m * ldc + n] = v;
                } else if (EPI == GEMM_FWD) {
                    const float z = v + bias[n];
                    if (C) C[(int64_t)m * ldc + n] = z;
                    Hout[(int64_t)m * ldh + n] = (__bf16)siluf(z);
                } else {
                    Hout[(int64_t)m * ldh + n] = (__bf16)(v * silu_gradf(Z[(int64_t)m * ldz + n]));
                }
            }
}

// out[i] = sum_z part[z n + i] (z < slices), a fixed order: deterministic.
__global__ void __launch_bounds__(256) k_sum_slices(const float* __restrict__ part, int slices, int64_t n,
                                                    float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int z = 0; z < slices; ++z) s += part[(int64_t)z * n + i];
    out[i] = s;
}

// ---------------------------------------------------------------------------
// Training pieces
// ---------------------------------------------------------------------------
// Output layer backward for a batch of B rows with targets t (clipped):
// dy = huber'(y - t) / B;  dz3[r][i] = dy W4[i] silu'(z3[r][i]) (BF16);
// row r's Huber loss to row_loss[r] (summed by k_colsum).
__global__ void __launch_bounds__(256) k_mlp_out_back(int64_t B, int D, int H, const float* __restrict__ P,
                                                      const float* __restrict__ y, const float* __restrict__ t,
                                                      const int* __restrict__ tidx, float huber, float clip_lo,
                                                      float clip_hi, const float* __restrict__ z3,
                                                      float* __restrict__ dy_out, __bf16* __restrict__ dz3,
                                                      float* __restrict__ row_loss) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const MlpOffsets o = mlp_offsets(D, H);
    if (q >= B * H) return;
    const int64_t r = q / H;
    const int i = (int)(q % H);
    const float tv = fminf(fmaxf(t[tidx ? tidx[r] : r], clip_lo), clip_hi);
    const float res = y[r] - tv;
    const float g = (fabsf(res) <= huber ? res : (res > 0.f ? huber : -huber)) / (float)B;
    if (i == 0) {
        dy_out[r] = g;
        row_loss[r] = fabsf(res) <= huber ? 0.5f * res * res : huber * (fabsf(res) - 0.5f * huber);
    }
    dz3[q] = (__bf16)(g * P[o.W4 + i] * silu_gradf(z3[q]));
}

// Single-launch batch reductions.  Every block of a group (blockIdx.x) sums
// one slice of rows (blockIdx.y) into part[slice][...]; then the block that
// finishes last in its group (the counter cnt[group] reaches the number of
// slices) adds the slices in slice order -- deterministic, whichever block
// that is -- and resets the counter: cnt[] is zero before and after a launch.
// Called by every thread after its slice sums are written.
__device__ inline bool last_slice(unsigned* cnt) {
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        last = atomicAdd(&cnt[blockIdx.x], 1u) == gridDim.y - 1 ? 1 : 0;
        if (last) cnt[blockIdx.x] = 0u;       // every block of the group has counted
    }
    __syncthreads();
    if (last) __threadfence();
    return last != 0;
}

// sum over the slices z < gridDim.y of part[z stride + i], in slice order;
// the acquire fence in last_slice makes the other blocks' sums visible to
// these plain loads (issued eight at a time)
__device__ inline float sum_slices_of(const float* part, int64_t stride, int64_t i) {
    float tot = 0.f;
    const int nz = (int)gridDim.y;
    int z = 0;
    for (; z + 8 <= nz; z += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(z + u) * stride + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) tot += v[u];
    }
    for (; z < nz; ++z) tot += part[(int64_t)z * stride + i];
    return tot;
}

// Column sums: out[j] = sum_r w[r] X[r][j] (plus out[j] when accumulate),
// j < ncol, w NULL -> 1, X BF16 [B][ncol] or FP32 Xf.  blockIdx.x = a group
// of 64 columns, blockIdx.y = a slice of kColRows rows, four row groups of
// one wave each summed in a fixed order.
constexpr int kColRows = 256;

__global__ void __launch_bounds__(256) k_colsum(int64_t B, int ncol, const float* __restrict__ w,
                                                const __bf16* __restrict__ X, const float* __restrict__ Xf,
                                                float* __restrict__ part, unsigned* __restrict__ cnt,
                                                float* __restrict__ out, int accumulate) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    const int64_t r0 = (int64_t)blockIdx.y * kColRows, r1 = min(B, r0 + kColRows);
    float s = 0.f;
    if (j < ncol) {
#pragma unroll 8
        for (int64_t r = r0 + g; r < r1; r += 4) {
            const float x = X ? (float)X[r * ncol + j] : Xf[r * ncol + j];
            s = fmaf(w ? w[r] : 1.f, x, s);
        }
    }
    red[g][lane] = s;
    __syncthreads();
    if (g == 0 && j < ncol)
        part[(int64_t)blockIdx.y * ncol + j] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    if (!last_slice(cnt)) return;
    if (g == 0 && j < ncol) {
        const float tot = sum_slices_of(part, ncol, j);
        out[j] = accumulate ? out[j] + tot : tot;
    }
}

// dW1[i][j] = sum_r dz1[r][i] * x[r][j] / pi -> out[i D + j]: one thread
// per (i, j), blockIdx.y = a slice of rs <= kGradW1Rows rows whose inputs
// (x / pi) the block first gathers into LDS, slices summed as in k_colsum.
constexpr int kGradW1Rows = 64;

__global__ void __launch_bounds__(256) k_mlp_grad_w1(RowSource src, int64_t B, int D, int H, int64_t rs,
                                                     const __bf16* __restrict__ dz1, float* __restrict__ part,
                                                     unsigned* __restrict__ cnt, float* __restrict__ out) {
    __shared__ float xs[kGradW1Rows][kMaxDof];
    const int64_t r0 = (int64_t)blockIdx.y * rs, r1 = min(B, r0 + rs);
    const int nr = (int)(r1 - r0);
    for (int q = threadIdx.x; q < nr * D; q += blockDim.x) {
        const int rr = q / D, j = q % D;
        int64_t sd;
        const float* x = row_ptr(src, r0 + rr, &sd);
        xs[rr][j] = x[j * sd] * kInvPi;
    }
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = t < H * D;
    if (ok) {
        const int i = t / D, j = t % D;
        float s = 0.f;
#pragma unroll 8
        for (int r = 0; r < nr; ++r) s = fmaf((float)dz1[(r0 + r) * H + i], xs[r][j], s);
        part[(int64_t)blockIdx.y * H * D + t] = s;
    }
    if (!last_slice(cnt)) return;
    if (ok) out[t] = sum_slices_of(part, (int64_t)H * D, t);
}

// Adam step with bias correction on the flat parameter vector; refreshes
// the BF16 copies of W2 and W3.
__global__ void __launch_bounds__(256) k_adam(int64_t n, float* __restrict__ P, const float* __restrict__ G,
                                              float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                              float b2, float eps, float c1, float c2, int D, int H,
                                              __bf16* __restrict__ W2b, __bf16* __restrict__ W3b) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float g = G[k];
    const float mk = b1 * m[k] + (1.f - b1) * g;
    const float vk = b2 * v[k] + (1.f - b2) * g * g;
    m[k] = mk;
    v[k] = vk;
    const float p = P[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    P[k] = p;
    const MlpOffsets o = mlp_offsets(D, H);
    if (k >= o.W2 && k < o.W2 + (int64_t)H * H) W2b[k - o.W2] = (__bf16)p;
    if (k >= o.W3 && k < o.W3 + (int64_t)H * H) W3b[k - o.W3] = (__bf16)p;
}

// BF16 copies of W2, W3 from the master parameters.
__global__ void __launch_bounds__(256) k_mlp_cast(int D, int H, const float* __restrict__ P, __bf16* __restrict__ W2b,
                                                  __bf16* __restrict__ W3b) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const MlpOffsets o = mlp_offsets(D, H);
    if (k >= (int64_t)H * H) return;
    W2b[k] = (__bf16)P[o.W2 + k];
    W3b[k] = (__bf16)P[o.W3 + k];
}

__global__ void __launch_bounds__(256) k_fill(float* __restrict__ p, int64_t n, float v) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// Counts of {pred >= m} among configurations with target < 0, for a set of
// candidate margins (calibration by bisection on the host).
__global__ void __launch_bounds__(256) k_count_above(int64_t n, const float* __restrict__ pred,
                                                     const float* __restrict__ target, float m,
                                                     unsigned long long* __restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool colliding = r < n && target[r] < 0.f;
    const bool above = colliding && pred[r] >= m;
    const unsigned long long a = __ballot(above), c = __ballot(colliding);
    if ((threadIdx.x & 63) == 0) {
        if (a) atomicAdd(&out[0], (unsigned long long)__popcll(a));
        if (c) atomicAdd(&out[1], (unsigned long long)__popcll(c));
    }
}

}  // namespace ezo
