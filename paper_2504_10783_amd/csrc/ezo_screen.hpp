// ezo_screen.hpp -- the learned self-collision screen's network as seen by
// the hot-path kernels: parameter layout, activations, and a whole forward
// pass of up to 16 FR rows inside one workgroup (BF16 MFMA hidden layers,
// FP32 accumulation), used by the fused screening kernel and by the
// bisection's screened tile checks.
//
// Network: x = q / pi -> H -> H -> H -> 1, SiLU; parameters (FP32 master,
// one flat vector) W1[H][D] b1[H] W2[H][H] b2[H] W3[H][H] b3[H] W4[H] b4[1]
// (z = W a + b); BF16 copies of W2 and W3 feed the MFMA layers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ezo {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr float kInvPi = 0.318309886183790671538f;

__device__ __forceinline__ float sigmoidf_(float z) { return 1.f / (1.f + __expf(-z)); }
__device__ __forceinline__ float siluf(float z) { return z * sigmoidf_(z); }
__device__ __forceinline__ float silu_gradf(float z) {
    const float s = sigmoidf_(z);
    return s * (1.f + z * (1.f - s));
}

struct MlpOffsets {
    int64_t W1, b1, W2, b2, W3, b3, W4, b4, total;
};

__host__ __device__ inline MlpOffsets mlp_offsets(int D, int H) {
    MlpOffsets o;
    o.W1 = 0;
    o.b1 = o.W1 + (int64_t)H * D;
    o.W2 = o.b1 + H;
    o.b2 = o.W2 + (int64_t)H * H;
    o.W3 = o.b2 + H;
    o.b3 = o.W3 + (int64_t)H * H;
    o.W4 = o.b3 + H;
    o.b4 = o.W4 + H;
    o.total = o.b4 + 1;
    return o;
}

// A screen as the kernels read it.  P == nullptr: no screen.
struct MlpView {
    int D, H;                  // H a multiple of 16, at most kMlpMaxH
    const float* P;            // FP32 parameters (W1, b1, b2, b3, W4, b4 read here)
    const __bf16* W2b;         // BF16 W2 [H][H], row n = unit n
    const __bf16* W3b;
    float margin;              // skip exact self pairs iff prediction >= margin
};

constexpr int kMlpMaxH = 256;
constexpr int kMlpPad = 8;     // BF16 elements of padding per activation row (LDS banks)

// LDS bytes of mlp_forward_tile<FR>: one activation buffer [16 FR][H + pad].
__host__ __device__ constexpr size_t mlp_tile_smem_bytes(int FR) {
    return sizeof(__bf16) * (size_t)16 * FR * (kMlpMaxH + kMlpPad);
}

// Forward pass of rows r < 16 FR of a workgroup of at least MINW waves
// (MINW >= 2; every thread must call it).  q(r, j) = q[r * q_stride + j] (LDS or global; rows
// >= nrows are not read and give unspecified outputs); h: LDS activation
// buffer of mlp_tile_smem_bytes(FR); y[r] (r < 16 FR) receives the
// prediction.  Starts and ends with a barrier.
//
// Layer 1 and the output layer run on the vector ALUs.  The hidden layers
// are v_mfma_f32_16x16x32_bf16 products: the waves split the H output units
// into 16-wide column tiles; for a tile, lane l reads the A fragment
// h[row 16 f + l % 16][k0 + 8 (l / 16) .. + 7] from LDS and the B fragment
// W[n0 + l % 16][k0 + 8 (l / 16) .. + 7] (16 contiguous bytes of the
// row-major BF16 weights) from global memory, and receives C[rows 4 (l / 16)
// .. + 3][column l % 16].  Each B fragment is used by all FR row fragments.
// The layer's outputs stay in registers until every wave has read the layer's
// inputs, then overwrite them in the same buffer.
template <int FR, int MINW>
__device__ inline void mlp_forward_tile(const MlpView& m, const float* q, int q_stride, int nrows, __bf16* h,
                                        float* y) {
    static_assert(MINW >= 2 && (kMlpMaxH / 16) % MINW == 0, "waves of the forward pass");
    constexpr int kMlpTilesPerWave = kMlpMaxH / 16 / MINW;    // 16-wide column tiles per wave
    constexpr int ROWS = 16 * FR;
    constexpr int LD = kMlpMaxH + kMlpPad;
    const int H = m.H, D = m.D;
    const int tid = threadIdx.x, lane = tid & 63;
    const int nw = blockDim.x >> 6, w = tid >> 6;
    const MlpOffsets o = mlp_offsets(D, H);
    __syncthreads();
    // layer 1: h = bf16(silu(W1 (q / pi) + b1))
    for (int idx = tid; idx < ROWS * H; idx += blockDim.x) {
        const int r = idx / H, i = idx - r * H;
        float z = m.P[o.b1 + i];
        if (r < nrows)
            for (int j = 0; j < D; ++j) z = fmaf(m.P[o.W1 + (int64_t)i * D + j], q[r * q_stride + j] * kInvPi, z);
        h[r * LD + i] = (__bf16)siluf(z);
    }
    __syncthreads();
    const int ntiles = H / 16;
    // hidden layers 2 and 3; wave w takes column tiles w, w + nw, ... (at
    // most kMlpTilesPerWave of them: nw >= MINW)
    for (int layer = 0; layer < 2; ++layer) {
        const __bf16* Wb = layer == 0 ? m.W2b : m.W3b;
        const float* bias = m.P + (layer == 0 ? o.b2 : o.b3);
        f32x4 acc[kMlpTilesPerWave][FR];
#pragma unroll
        for (int tt = 0; tt < kMlpTilesPerWave; ++tt) {
            const int tcol = w + tt * nw;
#pragma unroll
            for (int f = 0; f < FR; ++f) acc[tt][f] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (tcol < ntiles) {
                const int n = tcol * 16 + (lane & 15);
                const __bf16* wrow = Wb + (int64_t)n * H + 8 * (lane >> 4);
                for (int k0 = 0; k0 < H; k0 += 32) {
                    const bf16x8 b = *reinterpret_cast<const bf16x8*>(wrow + k0);
#pragma unroll
                    for (int f = 0; f < FR; ++f) {
                        const bf16x8 a =
                            *reinterpret_cast<const bf16x8*>(&h[(16 * f + (lane & 15)) * LD + k0 + 8 * (lane >> 4)]);
                        acc[tt][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[tt][f], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();                                  // every wave has read this layer's inputs
#pragma unroll
        for (int tt = 0; tt < kMlpTilesPerWave; ++tt) {
            const int tcol = w + tt * nw;
            if (tcol < ntiles) {
                const int n = tcol * 16 + (lane & 15);
                const float bn = bias[n];
#pragma unroll
                for (int f = 0; f < FR; ++f)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        h[(16 * f + 4 * (lane >> 4) + r) * LD + n] = (__bf16)siluf(acc[tt][f][r] + bn);
            }
        }
        __syncthreads();
    }
    // output layer: y = W4 . h + b4, one wave per row, lanes over the units
    for (int r = w; r < ROWS; r += nw) {
        float s = 0.f;
        for (int i = lane; i < H; i += 64) s = fmaf(m.P[o.W4 + i], (float)h[r * LD + i], s);
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) y[r] = s + m.P[o.b4];
    }
    __syncthreads();
}

}  // namespace ezo
