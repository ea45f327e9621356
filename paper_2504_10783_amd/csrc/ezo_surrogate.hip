// ezo_surrogate.hip -- the learned self-collision screen: creation, training
// (forward, backward and Adam, all in this library's kernels), prediction,
// calibration of the screening margin, and the chunked forward pass used by
// the inflation loop.
#include "ezo_internal.hpp"
#include "ezo_mlp.hpp"

using namespace ezo;

namespace {

constexpr int64_t kChunkRows = 262144;  // rows per forward chunk (multiple of 64)

int64_t round64(int64_t x) { return (x + 63) / 64 * 64; }

uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double unit(uint64_t& s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

// Training batch buffers: z1 z2 z3 (FP32), h1 h2 h3 d3 d2 d1 (BF16) of
// [B][H]; y dy rl (FP32 [B], rl = each row's loss); idx (int [B]); loss
// (FP32); the column sums' counters (zero between launches).
struct TrainBufs {
    float *z1, *z2, *z3, *y, *dy, *rl, *loss;
    __bf16 *h1, *h2, *h3, *d3, *d2, *d1;
    int* idx;
    unsigned* cnt;
    float* part;        // partial sums of the batch reductions
};

constexpr int kColGroups = 128;         // groups of k_colsum (H / 64) and k_mlp_grad_w1 (H D / 256)

TrainBufs carve(void* base, int B, int H) {
    TrainBufs t;
    char* p = reinterpret_cast<char*>(base);
    auto take = [&](size_t bytes) {
        char* q = p;
        p += (bytes + 255) & ~(size_t)255;
        return q;
    };
    const size_t bh = (size_t)B * H;
    t.cnt = (unsigned*)take(sizeof(unsigned) * kColGroups);     // first: the same place for every B
    t.z1 = (float*)take(4 * bh);
    t.z2 = (float*)take(4 * bh);
    t.z3 = (float*)take(4 * bh);
    t.h1 = (__bf16*)take(2 * bh);
    t.h2 = (__bf16*)take(2 * bh);
    t.h3 = (__bf16*)take(2 * bh);
    t.d3 = (__bf16*)take(2 * bh);
    t.d2 = (__bf16*)take(2 * bh);
    t.d1 = (__bf16*)take(2 * bh);
    t.y = (float*)take(4 * (size_t)B);
    t.dy = (float*)take(4 * (size_t)B);
    t.rl = (float*)take(4 * (size_t)B);
    t.idx = (int*)take(4 * (size_t)B);
    t.loss = (float*)take(256);
    t.part = (float*)take(0);
    return t;
}

// Row slices of dW1's batch reduction (summed in the same launch, like the
// column sums) and K slices of the weight-gradient GEMMs (K = batch rows,
// summed in a fixed order by k_sum_slices).
constexpr int kRowsPerSlice = kGradW1Rows;
constexpr int kGradSplitK = 16;

size_t partial_floats(int B, int H, int D) {
    const size_t slices = (size_t)(B + kRowsPerSlice - 1) / kRowsPerSlice;
    const size_t col_slices = (size_t)(B + kColRows - 1) / kColRows;
    return std::max({(size_t)kGradSplitK * H * H, slices * H * std::max(D, 1), col_slices * H});
}

size_t train_bytes(int B, int H, int D) {
    const size_t bh = (size_t)B * H;
    return 3 * (((4 * bh) + 255) & ~(size_t)255) + 6 * (((2 * bh) + 255) & ~(size_t)255) +
           4 * ((4 * (size_t)B + 255) & ~(size_t)255) + 256 + 512 + ((4 * partial_floats(B, H, D) + 255) & ~(size_t)255);
}

// C = A B with the strides' contiguous dimensions picking the staging; split
// > 1 (GEMM_STORE only) writes partial products over slices of about K /
// split rows (a multiple of 32) to C + z M ldc.  Returns the slice count.
template <int EPI>
int gemm(hipStream_t st, int M, int N, int K, const __bf16* A, int64_t sam, int64_t sak, const __bf16* B, int64_t sbk,
          int64_t sbn, float* C, int64_t ldc, const float* bias, __bf16* Hout, int64_t ldh, const float* Z, int64_t ldz,
          const int* status = nullptr, int64_t rpb = 0, int64_t rbase = 0, int split = 1) {
    const int kc = (K / split + 31) / 32 * 32;
    dim3 grid((unsigned)(N / 64), (unsigned)(M / 64), (unsigned)((K + kc - 1) / kc)), block(256);
    const bool ak = sak == 1, bk = sbk == 1;
#define EZO_GEMM(AKV, BKV)                                                                                          \
    hipLaunchKernelGGL((k_gemm_bf16<EPI, AKV, BKV>), grid, block, 0, st, M, N, K, kc, A, sam, sak, B, sbk, sbn, C, ldc, \
                       bias, Hout, ldh, Z, ldz, status, rpb, rbase)
    if (ak && bk) EZO_GEMM(true, true);
    else if (ak) EZO_GEMM(true, false);
    else if (bk) EZO_GEMM(false, true);
    else EZO_GEMM(false, false);
#undef EZO_GEMM
    return (int)grid.z;
}

// sum of the row slices of a batch reduction into out[n]
void sum_slices(hipStream_t st, const float* part, int slices, int64_t n, float* out) {
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, slices, n, out);
}

// out[j] (+)= sum_r w[r] X[r][j] over the batch, one launch
void colsum(hipStream_t st, int64_t B, int ncol, const float* w, const __bf16* X, const float* Xf, const TrainBufs& t,
            float* out, int accumulate = 0) {
    const int slices = (int)((B + kColRows - 1) / kColRows);
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((ncol + 63) / 64), (unsigned)slices), dim3(256), 0, st, B, ncol, w, X,
                       Xf, t.part, t.cnt, out, accumulate);
}

// batch row indices: an affine permutation of [0, n) per epoch
__global__ void k_batch_idx(int* __restrict__ idx, int B, int64_t start, int64_t n, uint64_t a, uint64_t c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const uint64_t k = (uint64_t)((start + i) % n);
    idx[i] = (int)((a % (uint64_t)n * k + c) % (uint64_t)n);
}

uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) {
        uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// One forward + backward pass over a batch of B rows (src.idx gathers them);
// leaves the gradient in s->G and adds the summed loss to t.loss.
ezo_status forward_backward(ezo_ctx* c, ezo_surrogate* s, const RowSource& src, const float* target, int B,
                            const ezo_train_params* hp, const TrainBufs& t, hipStream_t st) {
    const int D = s->D, H = s->H;
    const MlpOffsets o = mlp_offsets(D, H);
    float* G = s->G;
    const float* P = s->P;
    const int64_t BH = (int64_t)B * H;
    hipLaunchKernelGGL(k_mlp_layer1, dim3((unsigned)((BH + 255) / 256)), dim3(256), 0, st, src, (int64_t)B, D, H, P,
                       t.z1, t.h1, (const int*)nullptr);
    gemm<GEMM_FWD>(st, B, H, H, t.h1, H, 1, s->W2b, 1, H, t.z2, H, P + o.b2, t.h2, H, nullptr, 0);
    gemm<GEMM_FWD>(st, B, H, H, t.h2, H, 1, s->W3b, 1, H, t.z3, H, P + o.b3, t.h3, H, nullptr, 0);
    RowSource plain{};
    plain.rows = B;
    hipLaunchKernelGGL(k_mlp_out, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, plain, (int64_t)B, D, H, P, t.h3,
                       t.y, (const int*)nullptr);
    hipLaunchKernelGGL(k_mlp_out_back, dim3((unsigned)((BH + 255) / 256)), dim3(256), 0, st, (int64_t)B, D, H, P, t.y,
                       target, (const int*)src.idx, (float)hp->huber_delta, (float)hp->clip_lo, (float)hp->clip_hi,
                       t.z3, t.dy, t.d3, t.rl);
    float* part = t.part;
    colsum(st, B, H, t.dy, t.h3, nullptr, t, G + o.W4);
    colsum(st, B, 1, nullptr, nullptr, t.dy, t, G + o.b4);
    colsum(st, B, 1, nullptr, nullptr, t.rl, t, t.loss, 1);
    colsum(st, B, H, nullptr, t.d3, nullptr, t, G + o.b3);
    int ks = gemm<GEMM_STORE>(st, H, H, B, t.d3, 1, H, t.h2, H, 1, part, H, nullptr, nullptr, 0, nullptr, 0, nullptr,
                              0, 0, kGradSplitK);
    sum_slices(st, part, ks, (int64_t)H * H, G + o.W3);
    gemm<GEMM_BWD>(st, B, H, H, t.d3, H, 1, s->W3b, H, 1, nullptr, 0, nullptr, t.d2, H, t.z2, H);
    colsum(st, B, H, nullptr, t.d2, nullptr, t, G + o.b2);
    ks = gemm<GEMM_STORE>(st, H, H, B, t.d2, 1, H, t.h1, H, 1, part, H, nullptr, nullptr, 0, nullptr, 0, nullptr, 0, 0,
                          kGradSplitK);
    sum_slices(st, part, ks, (int64_t)H * H, G + o.W2);
    gemm<GEMM_BWD>(st, B, H, H, t.d2, H, 1, s->W2b, H, 1, nullptr, 0, nullptr, t.d1, H, t.z1, H);
    colsum(st, B, H, nullptr, t.d1, nullptr, t, G + o.b1);
    {
        const int slices = (B + kRowsPerSlice - 1) / kRowsPerSlice;
        hipLaunchKernelGGL(k_mlp_grad_w1, dim3((unsigned)((H * D + 255) / 256), (unsigned)slices), dim3(256), 0, st,
                           src, (int64_t)B, D, H, (int64_t)kRowsPerSlice, (const __bf16*)t.d1, part, t.cnt, G + o.W1);
    }
    HIP_TRY(c, hipGetLastError());
    return EZO_OK;
}

bool valid_train(const ezo_train_params* hp) {
    return hp && hp->epochs >= 0 && hp->batch >= 64 && hp->batch % 64 == 0 && hp->lr > 0 && hp->beta1 >= 0 &&
           hp->beta1 < 1 && hp->beta2 >= 0 && hp->beta2 < 1 && hp->adam_eps > 0 && hp->huber_delta > 0 &&
           hp->clip_lo < hp->clip_hi;
}

ezo_status ensure_train_bufs(ezo_ctx* c, ezo_surrogate* s, int B) {
    if (s->tb && s->batch >= B) return EZO_OK;
    if (s->tb) {
        (void)hipFree(s->tb);
        s->tb = nullptr;
    }
    if (hipMalloc(&s->tb, train_bytes(B, s->H, s->D)) != hipSuccess) return ezo_fail(c, EZO_E_NOMEM, "training buffers");
    s->batch = B;
    HIP_TRY(c, hipMemset(carve(s->tb, B, s->H).cnt, 0, sizeof(unsigned) * kColGroups));
    return EZO_OK;
}

}  // namespace

ezo_status ezo_surrogate_reserve(ezo_ctx* c, const ezo_surrogate* s, int64_t rows) {
    void *h1, *h2;
    const int64_t R = std::min<int64_t>(kChunkRows, round64(std::max<int64_t>(rows, 1)));
    ezo_status e;
    if ((e = ezo_ws_get(c, W_MLP_H1, sizeof(__bf16) * (size_t)R * s->H, &h1)) ||
        (e = ezo_ws_get(c, W_MLP_H2, sizeof(__bf16) * (size_t)R * s->H, &h2)))
        return e;
    return EZO_OK;
}

ezo_status ezo_surrogate_forward_rows(ezo_ctx* c, const ezo_surrogate* s, const RowSource& src, float* pred,
                                      const int* status, hipStream_t st) {
    const int D = s->D, H = s->H;
    void *h1, *h2;
    const int64_t R = std::min<int64_t>(kChunkRows, round64(std::max<int64_t>(src.rows, 1)));
    ezo_status e;
    if ((e = ezo_ws_get(c, W_MLP_H1, sizeof(__bf16) * (size_t)R * H, &h1)) ||
        (e = ezo_ws_get(c, W_MLP_H2, sizeof(__bf16) * (size_t)R * H, &h2)))
        return e;
    const MlpOffsets o = mlp_offsets(D, H);
    for (int64_t r0 = 0; r0 < src.rows; r0 += R) {
        RowSource cs = src;
        cs.rbase = src.rbase + r0;
        cs.rows = std::min<int64_t>(R, src.rows - r0);
        const int64_t M = round64(cs.rows);
        hipLaunchKernelGGL(k_mlp_layer1, dim3((unsigned)((M * H + 255) / 256)), dim3(256), 0, st, cs, M, D, H, s->P,
                           (float*)nullptr, (__bf16*)h1, status);
        gemm<GEMM_FWD>(st, (int)M, H, H, (const __bf16*)h1, H, 1, s->W2b, 1, H, nullptr, 0, s->P + o.b2, (__bf16*)h2, H,
                       nullptr, 0, status, src.rows_per_batch, cs.rbase);
        gemm<GEMM_FWD>(st, (int)M, H, H, (const __bf16*)h2, H, 1, s->W3b, 1, H, nullptr, 0, s->P + o.b3, (__bf16*)h1, H,
                       nullptr, 0, status, src.rows_per_batch, cs.rbase);
        hipLaunchKernelGGL(k_mlp_out, dim3((unsigned)((cs.rows + 255) / 256)), dim3(256), 0, st, cs, cs.rows, D, H,
                           s->P, (const __bf16*)h1, pred + r0, status);
    }
    HIP_TRY(c, hipGetLastError());
    return EZO_OK;
}

extern "C" {

int64_t ezo_surrogate_num_params(int32_t dof, int32_t hidden) { return mlp_offsets(dof, hidden).total; }

ezo_status ezo_surrogate_create(ezo_ctx* c, int32_t dof, int32_t hidden, uint64_t seed, ezo_surrogate** out) {
    if (!c || !out) return EZO_E_INVALID;
    *out = nullptr;
    if (dof < 1 || dof > EZO_MAX_DOF) return ezo_fail(c, EZO_E_UNSUPPORTED, "dof %d", dof);
    if (hidden < 64 || hidden % 64 != 0 || hidden > 4096)
        return ezo_fail(c, EZO_E_INVALID, "hidden width %d must be a multiple of 64 in [64, 4096]", hidden);
    HIP_TRY(c, hipSetDevice(c->device));
    ezo_surrogate* s = new ezo_surrogate();
    s->ctx = c;
    s->device = c->device;
    s->D = dof;
    s->H = hidden;
    const MlpOffsets o = mlp_offsets(dof, hidden);
    s->n_params = o.total;
    const size_t P = (size_t)o.total;
    if (hipMalloc((void**)&s->P, 4 * P) != hipSuccess || hipMalloc((void**)&s->G, 4 * P) != hipSuccess ||
        hipMalloc((void**)&s->m, 4 * P) != hipSuccess || hipMalloc((void**)&s->v, 4 * P) != hipSuccess ||
        hipMalloc((void**)&s->W2b, 2 * (size_t)hidden * hidden) != hipSuccess ||
        hipMalloc((void**)&s->W3b, 2 * (size_t)hidden * hidden) != hipSuccess) {
        ezo_surrogate_destroy(s);
        return ezo_fail(c, EZO_E_NOMEM, "surrogate allocation failed");
    }
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for every weight and bias
    std::vector<float> h(P);
    uint64_t st = seed ^ 0x5EED5EEDull;
    auto fill = [&](int64_t off, int64_t n, int fan_in) {
        const double b = 1.0 / std::sqrt((double)fan_in);
        for (int64_t k = 0; k < n; ++k) h[off + k] = (float)((2.0 * unit(st) - 1.0) * b);
    };
    fill(o.W1, (int64_t)hidden * dof, dof);
    fill(o.b1, hidden, dof);
    fill(o.W2, (int64_t)hidden * hidden, hidden);
    fill(o.b2, hidden, hidden);
    fill(o.W3, (int64_t)hidden * hidden, hidden);
    fill(o.b3, hidden, hidden);
    fill(o.W4, hidden, hidden);
    fill(o.b4, 1, hidden);
    ezo_status e = ezo_surrogate_set_params(s, h.data(), (int64_t)P);
    if (e) {
        ezo_surrogate_destroy(s);
        return e;
    }
    *out = s;
    return EZO_OK;
}

void ezo_surrogate_destroy(ezo_surrogate* s) {
    if (!s) return;
    hipError_t e = hipSetDevice(s->device);
    for (void* p : {(void*)s->P, (void*)s->G, (void*)s->m, (void*)s->v, (void*)s->W2b, (void*)s->W3b, s->tb})
        if (p) e = hipFree(p);
    (void)e;
    (void)hipGetLastError();
    delete s;
}

ezo_status ezo_surrogate_set_params(ezo_surrogate* s, const float* params, int64_t n) {
    if (!s || !params || n != s->n_params) return EZO_E_INVALID;
    ezo_ctx* c = s->ctx;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpy(s->P, params, 4 * (size_t)n, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemsetAsync(s->m, 0, 4 * (size_t)n, c->stream));
    HIP_TRY(c, hipMemsetAsync(s->v, 0, 4 * (size_t)n, c->stream));
    const int64_t HH = (int64_t)s->H * s->H;
    hipLaunchKernelGGL(k_mlp_cast, dim3((unsigned)((HH + 255) / 256)), dim3(256), 0, c->stream, s->D, s->H,
                       (const float*)s->P, s->W2b, s->W3b);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    s->adam_steps = 0;
    return EZO_OK;
}

ezo_status ezo_surrogate_get_params(const ezo_surrogate* s, float* params, int64_t n) {
    if (!s || !params || n != s->n_params) return EZO_E_INVALID;
    ezo_ctx* c = s->ctx;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(params, s->P, 4 * (size_t)n, hipMemcpyDeviceToHost));
    return EZO_OK;
}

ezo_status ezo_surrogate_loss_grad(ezo_ctx* c, ezo_surrogate* s, const float* q, const float* target, int64_t n,
                                   const ezo_train_params* hp, float* grad, double* loss, void* stream) {
    if (!c || !s || !q || !target || !grad || !valid_train(hp)) return c ? ezo_fail(c, EZO_E_INVALID, "bad argument") : EZO_E_INVALID;
    if (n < 64 || n % 64 != 0 || n > (1 << 20)) return ezo_fail(c, EZO_E_INVALID, "n must be a multiple of 64 in [64, 2^20]");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = c->stream;
    HIP_TRY(c, hipEventRecord(c->ev_in, as_stream(stream)));
    HIP_TRY(c, hipStreamWaitEvent(st, c->ev_in, 0));
    ezo_status e = ensure_train_bufs(c, s, (int)n);
    if (e) return e;
    TrainBufs t = carve(s->tb, (int)n, s->H);
    HIP_TRY(c, hipMemsetAsync(t.loss, 0, sizeof(float), st));
    RowSource src{};
    src.q = q;
    src.sn = s->D;
    src.sd = 1;
    src.rows = n;
    hipLaunchKernelGGL(k_batch_idx, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, t.idx, (int)n, (int64_t)0,
                       (int64_t)n, (uint64_t)1, (uint64_t)0);
    src.idx = t.idx;
    if ((e = forward_backward(c, s, src, target, (int)n, hp, t, st))) return e;
    float hl = 0.f;
    HIP_TRY(c, hipMemcpyAsync(grad, s->G, 4 * (size_t)s->n_params, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(&hl, t.loss, sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (loss) *loss = (double)hl / (double)n;
    return EZO_OK;
}

ezo_status ezo_surrogate_train(ezo_ctx* c, ezo_surrogate* s, const float* q, const float* target, int64_t n,
                               const ezo_train_params* hp, float* epoch_loss, void* stream) {
    if (!c || !s || !q || !target || !valid_train(hp)) return c ? ezo_fail(c, EZO_E_INVALID, "bad argument") : EZO_E_INVALID;
    if (n < hp->batch || n > INT32_MAX) return ezo_fail(c, EZO_E_INVALID, "need batch <= n < 2^31 rows");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = c->stream;
    HIP_TRY(c, hipEventRecord(c->ev_in, as_stream(stream)));
    HIP_TRY(c, hipStreamWaitEvent(st, c->ev_in, 0));
    const int B = hp->batch;
    ezo_status e = ensure_train_bufs(c, s, B);
    if (e) return e;
    TrainBufs t = carve(s->tb, B, s->H);
    RowSource src{};
    src.q = q;
    src.sn = s->D;
    src.sd = 1;
    src.idx = t.idx;
    src.rows = B;
    const int64_t steps_per_epoch = n / B;
    const int64_t total = steps_per_epoch * hp->epochs;
    uint64_t rs = hp->seed ^ 0xB47C5EEDull;
    int64_t step = 0;
    for (int ep = 0; ep < hp->epochs; ++ep) {
        // this epoch's order: k -> (a k + c) mod n with gcd(a, n) = 1
        uint64_t a = (splitmix64(rs) % (uint64_t)n) | 1ull;
        while (gcd64(a, (uint64_t)n) != 1) a += 2;
        const uint64_t cc = splitmix64(rs) % (uint64_t)n;
        HIP_TRY(c, hipMemsetAsync(t.loss, 0, sizeof(float), st));
        for (int64_t b = 0; b < steps_per_epoch; ++b, ++step) {
            hipLaunchKernelGGL(k_batch_idx, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, t.idx, B, b * B, n,
                               a, cc);
            if ((e = forward_backward(c, s, src, target, B, hp, t, st))) return e;
            const double lr = 0.5 * hp->lr * (1.0 + std::cos(3.14159265358979323846 * (double)step / (double)total));
            s->adam_steps++;
            const double c1 = 1.0 - std::pow(hp->beta1, (double)s->adam_steps);
            const double c2 = 1.0 - std::pow(hp->beta2, (double)s->adam_steps);
            hipLaunchKernelGGL(k_adam, dim3((unsigned)((s->n_params + 255) / 256)), dim3(256), 0, st, s->n_params, s->P,
                               (const float*)s->G, s->m, s->v, (float)lr, (float)hp->beta1, (float)hp->beta2,
                               (float)hp->adam_eps, (float)c1, (float)c2, s->D, s->H, s->W2b, s->W3b);
        }
        HIP_TRY(c, hipGetLastError());
        float hl = 0.f;
        HIP_TRY(c, hipMemcpyAsync(&hl, t.loss, sizeof(float), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        if (epoch_loss) epoch_loss[ep] = hl / (float)(steps_per_epoch * B);
    }
    HIP_TRY(c, hipStreamSynchronize(st));
    HIP_TRY(c, hipEventRecord(c->ev_out, st));
    HIP_TRY(c, hipStreamWaitEvent(as_stream(stream), c->ev_out, 0));
    return EZO_OK;
}

ezo_status ezo_surrogate_predict(ezo_ctx* c, const ezo_surrogate* s, const float* q, int64_t n, float* pred,
                                 void* stream) {
    if (!c || !s || n < 0) return EZO_E_INVALID;
    if (n == 0) return EZO_OK;
    if (!q || !pred) return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    HIP_TRY(c, hipSetDevice(c->device));
    RowSource src{};
    src.q = q;
    src.sn = s->D;
    src.sd = 1;
    src.rows = n;
    return ezo_surrogate_forward_rows(c, s, src, pred, nullptr, as_stream(stream));
}

// Fraction of configurations with target < 0 whose prediction is >= m.
static ezo_status count_above(ezo_ctx* c, const float* pred, const float* target, int64_t n, float m,
                              unsigned long long* cnt, hipStream_t st) {
    void* w;
    ezo_status e = ezo_ws_get(c, W_MLP_CNT, 2 * sizeof(unsigned long long), &w);
    if (e) return e;
    unsigned long long zero[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(w, zero, sizeof(zero), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_count_above, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, pred, target, m,
                       (unsigned long long*)w);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(cnt, w, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    return EZO_OK;
}

ezo_status ezo_surrogate_calibrate(ezo_ctx* c, ezo_surrogate* s, const float* q, const float* target, int64_t n,
                                   double alpha, double* margin_out, void* stream) {
    if (!c || !s || n <= 0 || !(alpha >= 0 && alpha < 1)) return c ? ezo_fail(c, EZO_E_INVALID, "bad argument") : EZO_E_INVALID;
    if (!q || !target) return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = c->stream;
    HIP_TRY(c, hipEventRecord(c->ev_in, as_stream(stream)));
    HIP_TRY(c, hipStreamWaitEvent(st, c->ev_in, 0));
    void* pred;
    ezo_status e = ezo_ws_get(c, W_PRED, sizeof(float) * (size_t)n, &pred);
    if (e) return e;
    RowSource src{};
    src.q = q;
    src.sn = s->D;
    src.sd = 1;
    src.rows = n;
    if ((e = ezo_surrogate_forward_rows(c, s, src, (float*)pred, nullptr, st))) return e;
    // smallest m with #{pred >= m | target < 0} <= alpha #{target < 0}, by bisection
    double lo = -16.0, hi = 16.0;
    unsigned long long cnt[2];
    if ((e = count_above(c, (const float*)pred, target, n, (float)hi, cnt, st))) return e;
    if (cnt[1] == 0) {
        s->margin = INFINITY;              // nothing colliding to calibrate on: screen nothing
        if (margin_out) *margin_out = INFINITY;
        return EZO_OK;
    }
    const double allowed = alpha * (double)cnt[1];
    for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if ((e = count_above(c, (const float*)pred, target, n, (float)mid, cnt, st))) return e;
        if ((double)cnt[0] <= allowed) hi = mid;
        else lo = mid;
    }
    s->margin = (float)hi;
    if (margin_out) *margin_out = hi;
    return EZO_OK;
}

ezo_status ezo_surrogate_set_margin(ezo_surrogate* s, double margin) {
    if (!s) return EZO_E_INVALID;
    s->margin = (float)margin;
    return EZO_OK;
}

ezo_status ezo_surrogate_set_scope(ezo_surrogate* s, int32_t scope) {
    if (!s || (scope & ~(EZO_SCREEN_SAMPLES | EZO_SCREEN_MIDPOINTS)) != 0) return EZO_E_INVALID;
    s->scope = scope;
    return EZO_OK;
}

ezo_status ezo_surrogate_miss_rate(ezo_ctx* c, const ezo_surrogate* s, const float* q, const float* target, int64_t n,
                                   double* miss_rate, double* screened_fraction, void* stream) {
    if (!c || !s || n <= 0 || !q || !target) return c ? ezo_fail(c, EZO_E_INVALID, "bad argument") : EZO_E_INVALID;
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = c->stream;
    HIP_TRY(c, hipEventRecord(c->ev_in, as_stream(stream)));
    HIP_TRY(c, hipStreamWaitEvent(st, c->ev_in, 0));
    void* pred;
    ezo_status e = ezo_ws_get(c, W_PRED, sizeof(float) * (size_t)n, &pred);
    if (e) return e;
    RowSource src{};
    src.q = q;
    src.sn = s->D;
    src.sd = 1;
    src.rows = n;
    if ((e = ezo_surrogate_forward_rows(c, s, src, (float*)pred, nullptr, st))) return e;
    unsigned long long cnt[2];
    if ((e = count_above(c, (const float*)pred, target, n, s->margin, cnt, st))) return e;
    if (miss_rate) *miss_rate = cnt[1] ? (double)cnt[0] / (double)cnt[1] : 0.0;
    if (screened_fraction) {
        // every configuration (target sign ignored): count with a target of -1
        unsigned long long all[2];
        void* neg;
        if ((e = ezo_ws_get(c, W_SCREENED, sizeof(float) * (size_t)n, &neg))) return e;
        hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (float*)neg, n, -1.f);
        if ((e = count_above(c, (const float*)pred, (const float*)neg, n, s->margin, all, st))) return e;
        *screened_fraction = (double)all[0] / (double)n;
    }
    return EZO_OK;
}

}  // extern "C"
