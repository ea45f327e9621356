// ezo_kernels.hpp -- the HIP kernels of the EI-ZO hot path (gfx950).
//
// Every kernel serves both the step-by-step entry points and the fused
// inflation loop.  In the fused loop, per-iteration quantities (iteration k,
// M_k, T_k, |S|) are read from device memory through IterArgs, so one
// captured hipGraph can be replayed for every iteration; edges whose status
// is final (>= 0) are skipped by every kernel.
#pragma once
#include "ezo_device.hpp"
#include "ezo_screen.hpp"

namespace ezo {

// Per-iteration constants: either given directly, or read from the loop's
// current row *cur = table[k] = (M_k, T_k, |S|_k, k), which k_init_edges sets
// to table[1] and k_advance moves to the next row (one load per kernel, issued
// with the edge's status).
struct IterArgs {
    const int4* cur;      // NULL => use k, M, T, nS below
    int k, M, T, nS;
};

struct IterVals { int k, M, T, nS; };

__device__ __forceinline__ IterVals resolve(const IterArgs& a) {
    IterVals v;
    if (a.cur) {
        const int4 e = *a.cur;
        v.k = e.w; v.M = e.x; v.T = e.y; v.nS = e.z;
    } else {
        v.k = a.k; v.M = a.M; v.T = a.T; v.nS = a.nS;
    }
    return v;
}

struct EdgeStatsDev {
    long long iterations, planes, final_m, test_collisions, samples, exact_checks, screened;
};

// Edge is still running (fused mode) -- or always, when no status array.
__device__ __forceinline__ bool edge_running(const int* status, int e) {
    return status == nullptr || status[e] < 0;
}

// ---------------------------------------------------------------------------
// Start of the fused loop for edge e: P_e = D (box rows: +e_j <= hi_j, then
// -e_j <= -lo_j), status RUNNING (-1), or INVALID (3) when a vertex is outside
// D or not finite, or CONTAINED (4) with no rows when skip[e]; statistics
// cleared.  Edge 0 also sets the loop's current row *cur = table[1]
// (iteration 1) and the running-edge count *active = n_edges.
// ---------------------------------------------------------------------------
struct EdgeInit {
    int dof;
    const float* q_lo;
    const float* q_hi;
    const float* edges;
    int n_edges;                       // 0: nothing to initialise
    float* A;
    float* bvec;
    int* n_faces;
    int cap;
    int* status;
    EdgeStatsDev* stats;
    uint8_t* proj_any;
    int4* cur;
    const int4* table;
    int* active;
    const uint8_t* skip;
};

__device__ inline void init_edge(const EdgeInit& a, int e) {
    const int dof = a.dof, cap = a.cap;
    if (e == 0) {
        *a.cur = a.table[1];
        *a.active = a.n_edges;
    }
    if (e >= a.n_edges) return;
    if (a.skip && a.skip[e]) {                  // not inflated: final from the start, no rows
        a.n_faces[e] = 0;
        a.status[e] = 4;                        // EZO_EDGE_CONTAINED
        a.stats[e] = EdgeStatsDev{0, 0, 0, 0, 0, 0, 0};
        a.proj_any[e] = 0;
        return;
    }
    float* Ae = a.A + (size_t)e * cap * dof;
    float* be = a.bvec + (size_t)e * cap;
    for (int f = 0; f < 2 * dof; ++f) {
        for (int j = 0; j < dof; ++j) Ae[(size_t)f * dof + j] = 0.f;
        if (f < dof) {
            Ae[(size_t)f * dof + f] = 1.f;
            be[f] = a.q_hi[f];
        } else {
            Ae[(size_t)f * dof + (f - dof)] = -1.f;
            be[f] = -a.q_lo[f - dof];
        }
    }
    a.n_faces[e] = 2 * dof;
    bool ok = true;
    const float* v = a.edges + (size_t)e * 2 * dof;
    for (int j = 0; j < 2 * dof; ++j) {
        const float x = v[j];
        const int jj = j % dof;
        if (!(x == x) || isinf(x) || x < a.q_lo[jj] || x > a.q_hi[jj]) ok = false;
    }
    a.status[e] = ok ? -1 : 3;
    a.stats[e] = EdgeStatsDev{0, 0, 0, 0, 0, 0, 0};
    a.proj_any[e] = 0;
}

// ---------------------------------------------------------------------------
// Obstacle preparation (workgroup 0): bounding box of the obstacle centres
// and largest obstacle radius; records (o', r) with o' = o - centre of the
// box; geometry of a G^3 grid over the box grown by
// r_sphere_max + r_obstacle_max + slack.
// ---------------------------------------------------------------------------
constexpr float kGridSlack = 1e-4f;

__global__ void __launch_bounds__(256) k_prep_obstacles(const float* __restrict__ obs, int n, float4* __restrict__ rec,
                                                        float4* __restrict__ centre, GridGeom* __restrict__ geom,
                                                        int G, float r_sphere_max, int* __restrict__ count,
                                                        int count_init, int clear_wg, EdgeInit ei) {
    // Workgroups 1 .. clear_wg set the grid's cell counts to count_init (0
    // before k_grid_scatter), the ones after them start the fused loop's edges
    // (independent work that would otherwise take launches of its own);
    // workgroup 0 does the rest (and the counts too when clear_wg is 0).
    const int cells = G * G * G;
    if (blockIdx.x > 0 && (int)blockIdx.x <= clear_wg) {
        for (int k = (blockIdx.x - 1) * blockDim.x + threadIdx.x; k < cells; k += clear_wg * blockDim.x)
            count[k] = count_init;
        return;
    }
    if ((int)blockIdx.x > clear_wg) {
        init_edge(ei, (int)((blockIdx.x - 1 - clear_wg) * blockDim.x + threadIdx.x));
        return;
    }
    if (clear_wg == 0)
        for (int k = threadIdx.x; k < cells; k += blockDim.x) count[k] = count_init;
    __shared__ float red[7][256];
    const int tid = threadIdx.x;
    float mn[3] = {kHuge, kHuge, kHuge}, mx[3] = {-kHuge, -kHuge, -kHuge}, rmax = 0.f;
    for (int o = tid; o < n; o += blockDim.x) {
        for (int k = 0; k < 3; ++k) {
            const float v = obs[4 * (size_t)o + k];
            mn[k] = fminf(mn[k], v);
            mx[k] = fmaxf(mx[k], v);
        }
        rmax = fmaxf(rmax, obs[4 * (size_t)o + 3]);
    }
    for (int k = 0; k < 3; ++k) { red[k][tid] = mn[k]; red[3 + k][tid] = mx[k]; }
    red[6][tid] = rmax;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
            for (int k = 0; k < 3; ++k) {
                red[k][tid] = fminf(red[k][tid], red[k][tid + s]);
                red[3 + k][tid] = fmaxf(red[3 + k][tid], red[3 + k][tid + s]);
            }
            red[6][tid] = fmaxf(red[6][tid], red[6][tid + s]);
        }
        __syncthreads();
    }
    float c[3] = {0.f, 0.f, 0.f}, half[3] = {0.f, 0.f, 0.f};
    if (n > 0)
        for (int k = 0; k < 3; ++k) {
            c[k] = 0.5f * (red[k][0] + red[3 + k][0]);
            half[k] = 0.5f * (red[3 + k][0] - red[k][0]);
        }
    if (tid == 0) {
        centre[0] = make_float4(c[0], c[1], c[2], 0.f);
        const float margin = r_sphere_max + red[6][0] + kGridSlack;
        GridGeom g;
        float h[3];
        for (int k = 0; k < 3; ++k) h[k] = 2.f * (half[k] + margin) / (float)G;
        g.ox = -half[0] - margin; g.oy = -half[1] - margin; g.oz = -half[2] - margin;
        g.hx = h[0]; g.hy = h[1]; g.hz = h[2];
        g.ihx = 1.f / h[0]; g.ihy = 1.f / h[1]; g.ihz = 1.f / h[2];
        g.reach = r_sphere_max + kGridSlack;
        geom[0] = g;
    }
    for (int o = tid; o < n; o += blockDim.x) {
        const float x = obs[4 * (size_t)o + 0] - c[0], y = obs[4 * (size_t)o + 1] - c[1], z = obs[4 * (size_t)o + 2] - c[2];
        const float r = obs[4 * (size_t)o + 3];
        rec[o] = make_float4(x, y, z, r);
    }
}

// Grid lists, built from the obstacles' side: one wave per obstacle, its
// lanes over the block of cells its reach can touch (the cell-index range of
// [o - R, o + R] widened by one cell on each side, R = r_o + reach), each
// cell kept by the same exact test of the distance from o to the cell's box;
// a kept obstacle takes the next slot of the cell by an atomic count
// (count[] must be zero on entry).  Which obstacles a cell lists is exactly
// what a cell-by-cell scan of all obstacles lists; their order within the
// list is whatever the atomics leave (the flags sweep only asks whether any
// of them collides).  A count above cap marks an overflowing cell (the sweep
// then scans every obstacle).
__global__ void __launch_bounds__(256) k_grid_scatter(const float4* __restrict__ rec, int n,
                                                      const GridGeom* __restrict__ geom, int G, int cap,
                                                      int* __restrict__ count, unsigned short* __restrict__ list) {
    const int o = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (o >= n) return;
    const GridGeom g = *geom;
    const float4 O = rec[o];
    const float R = O.w + g.reach;
    int lo[3], hi[3];
    const float oc[3] = {O.x, O.y, O.z}, orig[3] = {g.ox, g.oy, g.oz}, inv[3] = {g.ihx, g.ihy, g.ihz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {           // clamped in FP32 (an infinite reach covers the grid)
        lo[a] = (int)fmaxf(floorf((oc[a] - R - orig[a]) * inv[a]) - 1.f, 0.f);
        hi[a] = (int)fminf(floorf((oc[a] + R - orig[a]) * inv[a]) + 1.f, (float)(G - 1));
    }
    const int nx = hi[0] - lo[0] + 1, ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
    if (nx <= 0 || ny <= 0 || nz <= 0) return;
    const int total = nx * ny * nz;
    for (int k = lane; k < total; k += 64) {
        const int cx = lo[0] + k % nx, cy = lo[1] + (k / nx) % ny, cz = lo[2] + k / (nx * ny);
        const float lx = g.ox + cx * g.hx, ly = g.oy + cy * g.hy, lz = g.oz + cz * g.hz;
        const float ux = lx + g.hx, uy = ly + g.hy, uz = lz + g.hz;
        const float dx = fmaxf(fmaxf(lx - O.x, O.x - ux), 0.f);
        const float dy = fmaxf(fmaxf(ly - O.y, O.y - uy), 0.f);
        const float dz = fmaxf(fmaxf(lz - O.z, O.z - uz), 0.f);
        if (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < R * R) {
            const int cell = (cz * G + cy) * G + cx;
            const int pos = atomicAdd(&count[cell], 1);
            if (pos < cap) list[(size_t)cell * cap + pos] = (unsigned short)o;
        }
    }
}

// ---------------------------------------------------------------------------
// Batched collision check.  blockIdx.y = batch b (an edge in the fused loop),
// blockIdx.x = tile.  q_b = q + b * q_batch; flags_b = flags + b * out_batch.
// n = iteration's |S| when it.cur is set, else n_arg.
// ---------------------------------------------------------------------------
template <int T, bool SD, bool BOX>
__global__ void __launch_bounds__(1024) k_check(RobotView rb, ObsView ob, GridView gv, const float* __restrict__ q, int64_t n_arg,
                                                int64_t stride_n, int64_t stride_d, int64_t q_batch,
                                                uint8_t* __restrict__ flags, float* __restrict__ min_sd,
                                                float* __restrict__ min_sd_self, int64_t out_batch,
                                                const int* __restrict__ status, IterArgs it,
                                                const float* __restrict__ pred, float margin,
                                                EdgeStatsDev* __restrict__ stats) {
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.y;
    const IterVals iv = resolve(it);
    if (!edge_running(status, b)) return;
    int64_t n = n_arg, screen_from = n_arg;
    if (it.cur) {
        n = iv.nS;
        screen_from = iv.M;               // the unadaptive test's samples are never screened
    }
    const int64_t base = (int64_t)blockIdx.x * T;
    if (base >= n) return;
    const int nv = (int)((n - base) < T ? (n - base) : T);
    const int W = blockDim.x >> 6;
    TileSmem t = carve_tile(smem, T, tile_slots(rb.n_spheres, rb.n_boxes), W, SD ? 0 : ob.lds_n);
    if (!SD) stage_obstacles(ob, t);
    const float* qb = q + b * q_batch;
    for (int i = threadIdx.x; i < T * rb.dof; i += blockDim.x) {
        const int c = i % T, j = i / T;
        if (c < nv) t.q[c * kMaxDof + j] = qb[(base + c) * stride_n + j * stride_d];
    }
    if (threadIdx.x < (unsigned)T) {
        const int64_t g = base + threadIdx.x;
        const bool s = !SD && pred && threadIdx.x < (unsigned)nv && g >= screen_from && pred[b * out_batch + g] >= margin;
        t.scr[threadIdx.x] = s ? 1 : 0;
        if (s && stats) atomicAdd((unsigned long long*)&stats[b].screened, 1ull);
    }
    __syncthreads();
    const unsigned ntest = tile_check<SD, BOX>(rb, ob, gv, t, T, nv);
    if (gv.tests) flush_tests(gv.tests, ntest);
    if (threadIdx.x < (unsigned)nv) {
        const int64_t g = b * out_batch + base + threadIdx.x;
        flags[g] = (uint8_t)t.hit[threadIdx.x];
        if (SD) {
            if (min_sd) min_sd[g] = t.red[threadIdx.x];
            if (min_sd_self) min_sd_self[g] = t.red[W * T + threadIdx.x];
        }
    }
}

// Sphere centres in world coordinates, original sphere order.
template <int T>
__global__ void __launch_bounds__(256) k_centres(RobotView rb, ObsView ob, const int* __restrict__ sorted_to_orig,
                                                 const float* __restrict__ q, int64_t n, int64_t stride_n,
                                                 int64_t stride_d, float* __restrict__ out) {
    extern __shared__ __align__(16) char smem[];
    const int64_t base = (int64_t)blockIdx.x * T;
    if (base >= n) return;
    const int nv = (int)((n - base) < T ? (n - base) : T);
    TileSmem t = carve_tile(smem, T, tile_slots(rb.n_spheres, rb.n_boxes), blockDim.x >> 6);
    for (int i = threadIdx.x; i < T * rb.dof; i += blockDim.x) {
        const int c = i % T, j = i / T;
        if (c < nv) t.q[c * kMaxDof + j] = q[(base + c) * stride_n + j * stride_d];
    }
    __syncthreads();
    tile_fk<false>(rb, ob, t, T, nv);
    const float4 sh = ob.centre[0];
    const int S = rb.n_spheres;
    for (int i = threadIdx.x; i < nv * S; i += blockDim.x) {
        const int c = i / S, s = i % S;
        const float4 v = t.cen[s * T + c];
        float* o = out + ((base + c) * S + sorted_to_orig[s]) * 3;
        o[0] = v.x + sh.x;
        o[1] = v.y + sh.y;
        o[2] = v.z + sh.z;
    }
}

// ---------------------------------------------------------------------------
// Hit-and-run sampler.
//
// Step s of walk i (edge e, iteration k) draws Philox calls (i, e, k, 16 s + c),
// c < 3: words 2m, 2m+1 feed Box-Muller pair m (normals 2m, 2m+1 of the
// direction g ~ N(0, I)), word 2 ceil(dof/2) gives the chord position; u =
// g / |g|.  The chord through x along u is cut by every row of P.
//
// A walk is carried by a group of L lanes (L in {1, 2, 4, 8}) that all hold
// x; the rows of P (LDS, all walks of a workgroup belong to one edge =
// blockIdx.y) are split over the L lanes and the chord ends are combined with
// DPP min/max, which is exact, so the samples do not depend on L.
//   L <= 2: every lane draws each step's direction itself.
//   L >= 4: the directions of 2 L steps are drawn ahead, lane m of the group
//   drawing steps m and m + L, into LDS; the walk then reads them, so the
//   random draws are off the walk's step-to-step dependency chain.
// Rows stored as [F][D] normals plus b[F].
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int sample_chunk(int L) { return 2 * L; }        // steps drawn ahead (L >= 4)
__host__ __device__ constexpr int sample_dir_stride(int D) { return D + 4; }   // u[D], chord word, pad
// Words per walk group's block of drawn steps: one more than the steps' words,
// so that the groups of a wave, each reading its own block, start on distinct
// LDS banks (an even block size put them on the same banks).
__host__ __device__ constexpr int sample_group_words(int D, int L) { return sample_chunk(L) * sample_dir_stride(D) + 1; }

// LDS bytes of k_sample: rows, then (L >= 4) the drawn directions, sized for
// the most walk groups (L = 4) so that one size serves every L >= 4 (the fused
// loop's sampler picks L at run time).
__host__ __device__ inline size_t sample_smem_bytes(int D, int L, int cap, int threads) {
    const size_t rows = (sizeof(float) * (size_t)cap * (D + 1) + 15) & ~(size_t)15;
    return rows + (L >= 4 ? sizeof(float) * (size_t)(threads / 4) * sample_group_words(D, 4) : 0);
}
static_assert(16 * sample_group_words(7, 16) <= 64 * sample_group_words(7, 4) &&
              32 * sample_group_words(7, 8) <= 64 * sample_group_words(7, 4), "directions fit the L = 4 size");

// Normalised direction u (zero beyond dof) and chord word of one step.
template <int D>
__device__ __forceinline__ float draw_direction(int dof, uint32_t ii, uint32_t eid, uint32_t kk, uint32_t s, uint32_t key0,
                                       uint32_t key1, float (&u)[D]) {
    const int npair = (dof + 1) >> 1;
    const int tword = 2 * npair;
    const int ncall = (tword + 4) >> 2;
    // calls as separate values (an array indexed through a reference would
    // be kept in scratch memory)
    const U4 r0 = philox4x32_10(U4{ii, eid, kk, 16u * s}, key0, key1);
    U4 r1{0, 0, 0, 0}, r2{0, 0, 0, 0};
    if (ncall > 1) r1 = philox4x32_10(U4{ii, eid, kk, 16u * s + 1u}, key0, key1);
    if (ncall > 2) r2 = philox4x32_10(U4{ii, eid, kk, 16u * s + 2u}, key0, key1);
#pragma unroll
    for (int m = 0; m < (D + 1) / 2; ++m) {
        float ge = 0.f, go = 0.f;
        if (m < npair) {
            const U4 rm = (m >> 1) == 0 ? r0 : r1;
            const bool hi = (m & 1) != 0;
            const float ua = u01(hi ? rm.z : rm.x);
            const float ub = u01(hi ? rm.w : rm.y);
            // the chip's transcendental instructions: v_log_f32 (log2),
            // v_sqrt_f32, and v_sin_f32 / v_cos_f32, whose argument is in
            // revolutions (sin 2 pi ub directly); measured against FP64
            // over 2^24 arguments in (0, 1): 1.3e-7 absolute for sin and cos,
            // 1.6e-7 relative for log, about the libm FP32 functions' error
            const float rad = __builtin_amdgcn_sqrtf(-2.f * (__builtin_amdgcn_logf(ua) * 0.69314718055994531f));
            const float sn = __builtin_amdgcn_sinf(ub), cs = __builtin_amdgcn_cosf(ub);
            ge = rad * cs;
            go = rad * sn;
        }
        if (2 * m < D) u[2 * m] = (2 * m < dof) ? ge : 0.f;
        if (2 * m + 1 < D) u[2 * m + 1] = (2 * m + 1 < dof) ? go : 0.f;
    }
    float nrm = 0.f;
#pragma unroll
    for (int j = 0; j < D; ++j) nrm = fmaf(u[j], u[j], nrm);
    const float inv = __builtin_amdgcn_rsqf(nrm);          // v_rsq_f32: 9.4e-8 relative measured
#pragma unroll
    for (int j = 0; j < D; ++j) u[j] *= inv;
    const int tc = tword >> 2;
    const U4 rt = tc == 0 ? r0 : (tc == 1 ? r1 : r2);
    return u01(word_of(rt, tword & 3));
}

// The chord's ends are reduced with IEEE 754-2019 minimum / maximum
// (v_minimum3_f32 / v_maximum3_f32): a total order on the non-NaN values
// they see (-0 below +0), so a group's result does not depend on how its rows
// are split over lanes or on the order of the reduction, and, unlike fminf /
// fmaxf, the operands need no canonicalising instruction each.
__device__ __forceinline__ float tmin(float a, float b) { return __builtin_elementwise_minimum(a, b); }
__device__ __forceinline__ float tmax(float a, float b) { return __builtin_elementwise_maximum(a, b); }

// min / max over the L lanes of a group (groups aligned to L lanes): DPP
// quad permutations for lane distances 1 and 2, the half-row mirror (lane i
// with 7 - i) to join the two quads of an 8-lane group, the row mirror (lane
// i with 15 - i) to join the two halves of a 16-lane row.
template <int L>
__device__ __forceinline__ void group_minmax(float& lo_max, float& hi_min) {
    auto dpp = [](float v, int ctrl) -> float {
        const int b = __builtin_bit_cast(int, v);
        int r;
        switch (ctrl) {
            case 0: r = __builtin_amdgcn_mov_dpp(b, 0xB1, 0xF, 0xF, true); break;    // quad_perm [1,0,3,2]
            case 1: r = __builtin_amdgcn_mov_dpp(b, 0x4E, 0xF, 0xF, true); break;    // quad_perm [2,3,0,1]
            case 2: r = __builtin_amdgcn_mov_dpp(b, 0x141, 0xF, 0xF, true); break;   // row_half_mirror
            default: r = __builtin_amdgcn_mov_dpp(b, 0x140, 0xF, 0xF, true); break;  // row_mirror
        }
        return __builtin_bit_cast(float, r);
    };
    if constexpr (L >= 2) {
        hi_min = tmin(hi_min, dpp(hi_min, 0));
        lo_max = tmax(lo_max, dpp(lo_max, 0));
    }
    if constexpr (L >= 4) {
        hi_min = tmin(hi_min, dpp(hi_min, 1));
        lo_max = tmax(lo_max, dpp(lo_max, 1));
    }
    if constexpr (L >= 8) {
        hi_min = tmin(hi_min, dpp(hi_min, 2));
        lo_max = tmax(lo_max, dpp(lo_max, 2));
    }
    if constexpr (L >= 16) {
        hi_min = tmin(hi_min, dpp(hi_min, 3));
        lo_max = tmax(lo_max, dpp(lo_max, 3));
    }
}

// One hit-and-run step of the group's walk: chord of x along u through P
// (rows f = sub, sub + L, ... on this lane), x += t u with t = tlo + w (thi -
// tlo); t = 0 when rounding empties the chord.
// nbox = dof when the first 2 dof rows of P are the joint box (+e_j <= hi_j,
// then -e_j <= -lo_j), else 0.  Those rows' a^T u and a^T x are +-u_j and
// +-x_j exactly, so they are evaluated without the dot products (coordinates
// j = sub, sub + L, ... on this lane), with the same FP32 operations on the
// same values as the general rows: the chord ends are unchanged bit for bit.
template <int D, int L>
__device__ __forceinline__ void walk_step(const float* rowA, const float* rowb, int F, int sub, const float (&u)[D],
                                          float wt, float (&x)[D], int nbox) {
    float tlo = -INFINITY, thi = INFINITY;
    // coordinate j = m L + sub of this lane: its u_j and x_j picked from the
    // register arrays by selects (no divergent per-coordinate blocks)
#pragma unroll
    for (int m = 0; m * L < D; ++m) {
        float uj = 0.f, xj = 0.f;
#pragma unroll
        for (int s2 = 0; s2 < L && m * L + s2 < D; ++s2)
            if (s2 == sub) {
                uj = u[m * L + s2];
                xj = x[m * L + s2];
            }
        const int j = m * L + sub;
        if (j < nbox) {
            const float r = __builtin_amdgcn_rcpf(uj), rn = __builtin_amdgcn_rcpf(-uj);
            const float th = (rowb[j] - xj) * r;              // row +e_j <= hi_j
            const float tl = (rowb[nbox + j] - (-xj)) * rn;   // row -e_j <= -lo_j
            // branch-free: a row that does not bound this side offers +-inf
            const bool pos = uj > 0.f, neg = uj < 0.f;
            thi = tmin(thi, pos ? th : (neg ? tl : INFINITY));
            tlo = tmax(tlo, pos ? tl : (neg ? th : -INFINITY));
        }
    }
    for (int f = 2 * nbox + sub; f < F; f += L) {
        float den = 0.f, ax = 0.f;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const float a = rowA[f * D + j];
            den = fmaf(a, u[j], den);
            ax = fmaf(a, x[j], ax);
        }
        const float tt = (rowb[f] - ax) * __builtin_amdgcn_rcpf(den);
        thi = tmin(thi, den > 0.f ? tt : INFINITY);     // branch-free, as above
        tlo = tmax(tlo, den < 0.f ? tt : -INFINITY);
    }
    group_minmax<L>(tlo, thi);
    float tm = 0.f;
    if (thi >= tlo && tlo > -INFINITY && thi < INFINITY) tm = fmaf(wt, thi - tlo, tlo);
#pragma unroll
    for (int j = 0; j < D; ++j) x[j] = fmaf(tm, u[j], x[j]);
}

// The sampler's work for one workgroup with L lanes per walk; walk i =
// (blockIdx.x blockDim.x + threadIdx.x) / L of edge blockIdx.y.
template <int D, int L>
__device__ __forceinline__ void sample_block(char* smem, int dof, const float* __restrict__ A, const float* __restrict__ bvec,
                                    const int* __restrict__ n_faces, int cap, const float* __restrict__ edges,
                                    uint32_t key0, uint32_t key1, int64_t edge_id_base, int n_mix,
                                    float* __restrict__ S, int64_t stride, const IterVals& iv,
                                    const int* __restrict__ edge_ids = nullptr) {
    static_assert(L == 1 || L == 2 || L == 4 || L == 8 || L == 16, "lanes per walk");
    const int e = blockIdx.y;
    const int F = min(max(n_faces[e], 0), cap);
    float* rowA = reinterpret_cast<float*>(smem);        // [F][D]
    float* rowb = rowA + (size_t)F * D;                   // [F]
    const float* Ae = A + (size_t)e * cap * dof;
    for (int i = threadIdx.x; i < F * D; i += blockDim.x) {
        const int f = i / D, j = i % D;
        rowA[i] = j < dof ? Ae[(size_t)f * dof + j] : 0.f;
    }
    for (int f = threadIdx.x; f < F; f += blockDim.x) rowb[f] = bvec[(size_t)e * cap + f];
    __syncthreads();
    // the joint box as the first 2 dof rows?  (every polytope of the fused
    // loop starts so; a caller's P may not).  Used with at most four lanes
    // per walk: with more, a lane holds one or two rows of P and the box
    // rows' own path (a select of the lane's coordinate) is no cheaper.
    int nbox = 0;
    if (F >= 2 * dof) {                                   // uniform
        bool ok = true;
        for (int i = threadIdx.x; i < 2 * dof * dof; i += blockDim.x) {
            const int f = i / dof, j = i % dof;
            ok = ok && rowA[f * D + j] == (j == f % dof ? (f < dof ? 1.f : -1.f) : 0.f);
        }
        nbox = (__syncthreads_and(ok ? 1 : 0) && L <= 4) ? dof : 0;
    }
    const int lane = threadIdx.x & 63;
    const int sub = lane & (L - 1);                       // position in the walk's lane group
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) / L;
    // A group past the end still runs (it takes part in the workgroup's
    // barriers) but stores nothing; groups never straddle walks.
    const bool live = i < iv.nS;
    const float* v = edges + (size_t)e * 2 * dof;
    const uint32_t eid = (uint32_t)(edge_id_base + (edge_ids ? edge_ids[e] : e));
    const uint32_t ii = (uint32_t)i, kk = (uint32_t)iv.k;
    float x[D], u[D];
    {
        const U4 r = philox4x32_10(U4{ii, eid, kk, 0u}, key0, key1);
        const float w0 = u01(r.x);
#pragma unroll
        for (int j = 0; j < D; ++j) x[j] = j < dof ? fmaf(w0, v[dof + j] - v[j], v[j]) : 0.f;
    }
    if constexpr (L <= 2) {
        for (int s = 1; s <= n_mix; ++s) {
            const float wt = draw_direction<D>(dof, ii, eid, kk, (uint32_t)s, key0, key1, u);
            walk_step<D, L>(rowA, rowb, F, sub, u, wt, x, nbox);
        }
    } else {
        constexpr int SD = sample_dir_stride(D), CH = sample_chunk(L);
        float* dirs = reinterpret_cast<float*>(smem + sample_smem_bytes(D, 1, cap, 0)) +
                      (size_t)(threadIdx.x / L) * sample_group_words(D, L);
        for (int s0 = 1; s0 <= n_mix; s0 += CH) {
            const int ns = min(CH, n_mix - s0 + 1);
            // this lane's two steps of the chunk, drawn side by side (independent
            // chains the scheduler interleaves)
            {
                float u2[D];
                const int c0 = sub, c1 = sub + L;
                const float w0 = draw_direction<D>(dof, ii, eid, kk, (uint32_t)(s0 + c0), key0, key1, u);
                const float w1 = draw_direction<D>(dof, ii, eid, kk, (uint32_t)(s0 + c1), key0, key1, u2);
                if (c0 < ns) {
#pragma unroll
                    for (int j = 0; j < D; ++j) dirs[c0 * SD + j] = u[j];
                    dirs[c0 * SD + D] = w0;
                }
                if (c1 < ns) {
#pragma unroll
                    for (int j = 0; j < D; ++j) dirs[c1 * SD + j] = u2[j];
                    dirs[c1 * SD + D] = w1;
                }
            }
            __syncthreads();
            for (int c = 0; c < ns; ++c) {
#pragma unroll
                for (int j = 0; j < D; ++j) u[j] = dirs[c * SD + j];
                walk_step<D, L>(rowA, rowb, F, sub, u, dirs[c * SD + D], x, nbox);
            }
            __syncthreads();
        }
    }
    if (live) {
#pragma unroll
        for (int j = 0; j < D; ++j)
            if (j < dof && (j % L) == sub) S[((size_t)e * dof + j) * stride + i] = x[j];
    }
}

template <int D, int L>
__global__ void __launch_bounds__(256) k_sample(int dof, const float* __restrict__ A, const float* __restrict__ bvec,
                                                const int* __restrict__ n_faces, int cap,
                                                const float* __restrict__ edges, uint32_t key0, uint32_t key1,
                                                int64_t edge_id_base, int n_mix, float* __restrict__ S,
                                                int64_t stride, const int* __restrict__ status, IterArgs it) {
    extern __shared__ __align__(16) char smem[];
    const IterVals iv = resolve(it);
    if (!edge_running(status, blockIdx.y)) return;
    sample_block<D, L>(smem, dof, A, bvec, n_faces, cap, edges, key0, key1, edge_id_base, n_mix, S, stride, iv);
}

// The fused loop's sampler: launched with the grid of 16 lanes per walk, it
// picks the lanes per walk from the walks of all running edges (*active x
// |S|): 16 up to walks16, 4 up to walks4, else 1 (workgroups past the walks
// exit).  Few walks are latency-bound and gain from splitting the rows; many
// walks fill the chip either way and one lane per walk does the least work.
// Samples are identical in every mode.
template <int D>
__global__ void __launch_bounds__(256) k_sample_auto(int dof, const float* __restrict__ A,
                                                     const float* __restrict__ bvec, const int* __restrict__ n_faces,
                                                     int cap, const float* __restrict__ edges, uint32_t key0,
                                                     uint32_t key1, int64_t edge_id_base, int n_mix,
                                                     float* __restrict__ S, int64_t stride,
                                                     const int* __restrict__ status, IterArgs it,
                                                     const int* __restrict__ active, int64_t walks16, int64_t walks4,
                                                     const int* __restrict__ edge_ids) {
    extern __shared__ __align__(16) char smem[];
    const IterVals iv = resolve(it);
    if (!edge_running(status, blockIdx.y)) return;
    const int64_t walks = (int64_t)max(*active, 1) * iv.nS;
    const int64_t wg_first = (int64_t)blockIdx.x * blockDim.x;     // first thread of this workgroup
    if (walks <= walks16) {
        sample_block<D, 16>(smem, dof, A, bvec, n_faces, cap, edges, key0, key1, edge_id_base, n_mix, S, stride, iv,
                            edge_ids);
    } else if (walks <= walks4) {
        if (wg_first >= 4 * (int64_t)iv.nS) return;
        sample_block<D, 4>(smem, dof, A, bvec, n_faces, cap, edges, key0, key1, edge_id_base, n_mix, S, stride, iv,
                            edge_ids);
    } else {
        if (wg_first >= iv.nS) return;
        sample_block<D, 1>(smem, dof, A, bvec, n_faces, cap, edges, key0, key1, edge_id_base, n_mix, S, stride, iv,
                            edge_ids);
    }
}

// ---------------------------------------------------------------------------
// Learned screen of the loop's samples: the network's prediction for the
// samples that the screen may skip, rows M_k <= i < |S| of every running
// edge (the unadaptive test's first M_k samples are always checked exactly).
// One workgroup (4 waves) per 64 consecutive sample rows of one edge
// (blockIdx.y); the whole forward pass runs in the workgroup
// (mlp_forward_tile), so activations never leave LDS.  pred[e][i] is written
// for the rows of every tile that overlaps [M_k, |S|); others are untouched
// and never read.
// ---------------------------------------------------------------------------
constexpr int kScreenRows = 64;

__global__ void __launch_bounds__(256) k_screen_samples(MlpView mv, const float* __restrict__ S, int64_t stride,
                                                        int dof, float* __restrict__ pred,
                                                        const int* __restrict__ status, IterArgs it) {
    __shared__ __attribute__((aligned(16))) __bf16 h[kScreenRows * (kMlpMaxH + kMlpPad)];
    __shared__ float q[kScreenRows * kMaxDof];
    __shared__ float y[kScreenRows];
    const int e = blockIdx.y;
    const IterVals iv = resolve(it);
    if (!edge_running(status, e)) return;
    const int64_t r0 = (int64_t)blockIdx.x * kScreenRows;
    if (r0 + kScreenRows <= iv.M || r0 >= iv.nS) return;
    const int nr = (int)min<int64_t>(kScreenRows, iv.nS - r0);
    const float* Se = S + (size_t)e * dof * stride;
    for (int i = threadIdx.x; i < kScreenRows * dof; i += blockDim.x) {
        const int r = i % kScreenRows, j = i / kScreenRows;
        q[r * kMaxDof + j] = r < nr ? Se[(size_t)j * stride + r0 + r] : 0.f;
    }
    mlp_forward_tile<kScreenRows / 16, 4>(mv, q, kMaxDof, nr, h, y);
    if (threadIdx.x < (unsigned)nr) pred[(size_t)e * stride + r0 + threadIdx.x] = y[threadIdx.x];
}

// Sum over the wave: DPP quad permutations (lane distance 1, 2), the half-row
// and row mirrors (every lane of a 16-lane row ends with the row's sum), then
// the four rows' sums by readlane.  Every lane active.
__device__ __forceinline__ int wave_sum_i32(int v) {
    v += __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);    // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);    // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);   // row_half_mirror
    v += __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true);   // row_mirror
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) + __builtin_amdgcn_readlane(v, 32) +
           __builtin_amdgcn_readlane(v, 48);
}

// ---------------------------------------------------------------------------
// Unadaptive test + selection of the first N_p colliding samples.
// One workgroup (1024 threads) per edge.
// ---------------------------------------------------------------------------


__global__ void __launch_bounds__(1024) k_test_select(const uint8_t* __restrict__ flags, int64_t stride, int n_p,
                                                      int n_b, int* __restrict__ cand_idx, int cand_cap,
                                                      int* __restrict__ n_cands, uint8_t* __restrict__ accept_out,
                                                      int* __restrict__ count_out, int* __restrict__ status,
                                                      EdgeStatsDev* __restrict__ stats, IterArgs it) {
    __shared__ int wsum[16];
    __shared__ int s_base;
    const int e = blockIdx.x;
    const IterVals iv = resolve(it);
    if (!edge_running(status, e)) {
        if (threadIdx.x == 0 && n_cands) n_cands[e] = 0;
        return;
    }
    const uint8_t* fe = flags + (size_t)e * stride;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
    const int nt4 = 4 * (int)blockDim.x;
    // the thread's four consecutive flags of each of the first kTestPre
    // passes, loaded together up front (one memory latency instead of one per
    // pass); flag i of pass c is bit 8 (i - c nt4 - 4 tid) of pre[c]
    constexpr int kTestPre = 4;
    uint32_t pre[kTestPre];
    const bool words = (reinterpret_cast<uintptr_t>(fe) & 3) == 0;
#pragma unroll
    for (int c = 0; c < kTestPre; ++c) {
        const int i0 = c * nt4 + 4 * tid;
        pre[c] = 0;
        if (words && i0 + 4 <= iv.nS) {
            pre[c] = *reinterpret_cast<const uint32_t*>(fe + i0);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (i0 + q < iv.nS) pre[c] |= (uint32_t)fe[i0 + q] << (8 * q);
        }
    }
    auto flag_at = [&](int c, int i0, int q) -> bool {       // flag i0 + q of pass c (i0 + q < nS)
        return c < kTestPre ? ((pre[c] >> (8 * q)) & 0xFFu) != 0 : fe[i0 + q] != 0;
    };
    // count over the first M samples (four consecutive flags per thread)
    int cnt = 0;
    for (int i0 = 4 * tid, c = 0; i0 < iv.M; i0 += nt4, ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) cnt += (i0 + q < iv.M && flag_at(c, i0, q)) ? 1 : 0;
    cnt = wave_sum_i32(cnt);
    if (lane == 0) wsum[w] = cnt;
    __syncthreads();
    int total = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) total += k < nw ? wsum[k] : 0;
    const bool accept = total <= iv.T;
    __syncthreads();
    int taken = 0;
    if (!accept) {
        if (tid == 0) s_base = 0;
        __syncthreads();
        const unsigned long long lt = (1ull << lane) - 1ull;
        for (int c0 = 0, c = 0; c0 < iv.nS; c0 += nt4, ++c) {
            // flags i0 .. i0 + 3 of this thread; the wave's exclusive prefix of
            // the per-thread counts (0..4) from one ballot per count bit
            const int i0 = c0 + 4 * tid;
            bool f[4];
            int lc = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                f[q] = (i0 + q < iv.nS) && flag_at(c, i0, q);
                lc += f[q] ? 1 : 0;
            }
            const unsigned long long b0 = __ballot(lc & 1), b1 = __ballot(lc & 2), b2 = __ballot(lc & 4);
            const int before = __popcll(b0 & lt) + 2 * __popcll(b1 & lt) + 4 * __popcll(b2 & lt);
            if (lane == 0) wsum[w] = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
            __syncthreads();
            int off = s_base, chunk = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int c = k < nw ? wsum[k] : 0;
                chunk += c;
                off += k < w ? c : 0;
            }
            int pos = off + before;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (f[q]) {
                    if (pos < n_p) cand_idx[(size_t)e * cand_cap + pos] = i0 + q;
                    ++pos;
                }
            __syncthreads();
            if (tid == 0) s_base += chunk;
            __syncthreads();
            if (s_base >= n_p) break;
        }
        taken = s_base < n_p ? s_base : n_p;
    }
    if (tid == 0) {
        if (n_cands) n_cands[e] = taken;
        if (accept_out) accept_out[e] = accept ? 1 : 0;
        if (count_out) count_out[e] = total;
        if (stats) {
            EdgeStatsDev& s = stats[e];
            s.iterations = iv.k;
            s.final_m = iv.M;
            s.test_collisions = total;
            atomicAdd((unsigned long long*)&s.samples, (unsigned long long)iv.nS);
            atomicAdd((unsigned long long*)&s.exact_checks, (unsigned long long)iv.nS + (unsigned long long)taken * (1 + n_b));
        }
        if (status && accept) status[e] = 0;   // EZO_EDGE_CERTIFIED
    }
}

// ---------------------------------------------------------------------------
// Projection + fail-fast check + N_b bisection steps.  blockIdx.y = edge,
// blockIdx.x = a group of TC candidates; every check is a whole-workgroup
// tile check of up to TC (2^DEPTH - 1) configurations.  Candidate j of edge e
// is sample cand_idx[e][j], coordinate k at S[e s_edge + k stride + idx].
//
// The first check is the projections c_proj (fail-fast).  The bisection then
// runs DEPTH levels per round: a round checks, for every candidate, the
// 2^lev - 1 points of the next lev <= DEPTH levels of its bisection tree
// (heap order: node 1 = midpoint of [lo, hi]; the children of node i are the
// midpoints of its two halves), then walks the tree with the flags.  These
// are exactly the points, computed by the same FP32 operations, and the
// decisions of one-midpoint-at-a-time bisection, in ceil(N_b / DEPTH)
// dependent rounds instead of N_b.  Candidate state lives with the threads
// c < TC; configuration c (2^lev - 1) + i - 1 holds node i of candidate c.
// LDS: the tile, the staged obstacles (ob.lds_n records), then the robot
// tables (robot_stage_bytes), read by every one of the dependent checks.
// ---------------------------------------------------------------------------
template <int TC, int DEPTH, bool BOX, bool SCR = false>
__global__ void __launch_bounds__(1024) k_project_bisect(RobotView rg, ObsView ob, GridView gv, const float* __restrict__ edges,
                                                         const float* __restrict__ S, int64_t stride, int64_t s_edge,
                                                         const int* __restrict__ cand_idx,
                                                         const int* __restrict__ n_cands, int cand_cap, int n_b,
                                                         float* __restrict__ c_star, float* __restrict__ a_dir,
                                                         float* __restrict__ t_star,
                                                         uint8_t* __restrict__ proj_collides,
                                                         uint8_t* __restrict__ proj_any,
                                                         const int* __restrict__ status, MlpView mv,
                                                         EdgeStatsDev* __restrict__ stats) {
    static_assert(DEPTH >= 1 && DEPTH <= 3 && TC >= 1, "bisection depth per round");
    static_assert(!SCR || (DEPTH == 1 && TC <= 16), "the screened bisection checks at most 16 points per round");
    // (the screened form runs with at least four waves: the network's layers)
    constexpr int NODES = (1 << DEPTH) - 1;
    constexpr int T = TC * NODES;                   // configurations per tile check
    extern __shared__ __align__(16) char smem[];
    const int e = blockIdx.y;
    if (!edge_running(status, e)) return;
    const int nc = min(max(n_cands[e], 0), cand_cap);
    const int base = blockIdx.x * TC;
    if (base >= nc) return;
    const int nv = (nc - base) < TC ? (nc - base) : TC;
    const int dof = rg.dof;
    const int W = blockDim.x >> 6;
    const int slots = tile_slots(rg.n_spheres, rg.n_boxes);
    TileSmem t = carve_tile(smem, T, slots, W, ob.lds_n);
    char* rs_base = smem + tile_smem_bytes(T, slots, W) + 16 * (size_t)ob.lds_n;
    const RobotView rb = stage_robot(rg, rs_base);
    // screened form: the network's activations and predictions after the
    // staged robot tables
    __bf16* mlp_h = reinterpret_cast<__bf16*>(rs_base + robot_stage_bytes(slots, rg.n_self, rg.n_blocks));
    float* mlp_y = reinterpret_cast<float*>(reinterpret_cast<char*>(mlp_h) + mlp_tile_smem_bytes(1));
    stage_obstacles(ob, t);
    const int tid = threadIdx.x;
    const bool own = tid < nv;
    if (tid < T) t.scr[tid] = 0;          // the projections (fail-fast) are always checked exactly
    float lo[kMaxDof], hi[kMaxDof], cp[kMaxDof];
    const float* v = edges + (size_t)e * 2 * dof;
    if (own) {
        const int idx = min(max(cand_idx[(size_t)e * cand_cap + base + tid], 0), (int)(stride - 1));
        const float* Se = S + (size_t)e * s_edge;
        float num = 0.f, den = 0.f;
#pragma unroll
        for (int j = 0; j < kMaxDof; ++j) {
            hi[j] = j < dof ? Se[(size_t)j * stride + idx] : 0.f;
            const float dv = j < dof ? v[dof + j] - v[j] : 0.f;
            num = fmaf(hi[j] - (j < dof ? v[j] : 0.f), dv, num);
            den = fmaf(dv, dv, den);
        }
        float alpha = 0.f;
        if (den > 0.f) alpha = fminf(fmaxf(num / den, 0.f), 1.f);
        float nrm = 0.f;
#pragma unroll
        for (int j = 0; j < kMaxDof; ++j) {
            cp[j] = j < dof ? fmaf(alpha, v[dof + j], (1.f - alpha) * v[j]) : 0.f;
            lo[j] = cp[j];
            nrm = fmaf(hi[j] - cp[j], hi[j] - cp[j], nrm);
        }
        nrm = sqrtf(nrm);
        const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
        for (int j = 0; j < dof; ++j) {
            a_dir[((size_t)e * dof + j) * cand_cap + base + tid] = (hi[j] - cp[j]) * inv;
            t.q[tid * kMaxDof + j] = cp[j];
        }
    }
    __syncthreads();
    unsigned ntest = tile_check<false, BOX>(rb, ob, gv, t, T, nv);
    if (own) {
        const int h = t.hit[tid];
        proj_collides[(size_t)e * cand_cap + base + tid] = (uint8_t)h;
        if (h && proj_any) proj_any[e] = 1;
    }
    for (int done = 0; done < n_b;) {
        const int lev = min(DEPTH, n_b - done);
        const int npt = (1 << lev) - 1;
        __syncthreads();                  // the previous check's reads of t.q are done
        if (own) {
            float* q0 = t.q + (size_t)tid * npt * kMaxDof;
#pragma unroll
            for (int j = 0; j < kMaxDof; ++j) {
                if (j >= dof) break;
                // node i's interval [L_i, H_i]; L_2i = L_i, H_2i = p_i, L_2i+1 = p_i, H_2i+1 = H_i
                float Lv[NODES + 1], Hv[NODES + 1], pv[NODES + 1];
                Lv[1] = lo[j];
                Hv[1] = hi[j];
#pragma unroll
                for (int i = 1; i <= NODES; ++i) {
                    if (i > 1) {
                        Lv[i] = (i & 1) ? pv[i >> 1] : Lv[i >> 1];
                        Hv[i] = (i & 1) ? Hv[i >> 1] : pv[i >> 1];
                    }
                    pv[i] = 0.5f * (Lv[i] + Hv[i]);
                    if (i <= npt) q0[(i - 1) * kMaxDof + j] = pv[i];
                }
            }
        }
        __syncthreads();
        if constexpr (SCR) {
            // one-sided screen of the midpoints: exact self pairs are skipped
            // iff the predicted self distance is >= the margin, so a point
            // judged colliding is truly colliding and c* stays a collision
            mlp_forward_tile<1, 4>(mv, t.q, kMaxDof, nv, mlp_h, mlp_y);
            int screened = 0;
            if (tid < T) {
                const bool sc = tid < nv && mlp_y[tid] >= mv.margin;
                t.scr[tid] = sc ? 1 : 0;
                screened = sc ? 1 : 0;
            }
            if (stats && tid < 64) {
                const unsigned long long b = __ballot(screened != 0);
                if (tid == 0 && b) atomicAdd((unsigned long long*)&stats[e].screened, (unsigned long long)__popcll(b));
            }
        }
        ntest += tile_check<false, BOX>(rb, ob, gv, t, T, nv * npt);
        if (own) {
            const int* h = t.hit + tid * npt;
            const float* q0 = t.q + (size_t)tid * npt * kMaxDof;
            int node = 1;
            for (int d = 0; d < lev; ++d) {
                const bool hc = h[node - 1] != 0;
#pragma unroll
                for (int j = 0; j < kMaxDof; ++j) {
                    if (j < dof) {
                        const float m = q0[(node - 1) * kMaxDof + j];
                        if (hc) hi[j] = m;
                        else lo[j] = m;
                    }
                }
                node = 2 * node + (hc ? 0 : 1);
            }
        }
        done += lev;
    }
    if (own) {
        float ts = 0.f;
        for (int j = 0; j < dof; ++j) {
            c_star[((size_t)e * dof + j) * cand_cap + base + tid] = hi[j];
            ts = fmaf(hi[j] - cp[j], hi[j] - cp[j], ts);
        }
        t_star[(size_t)e * cand_cap + base + tid] = sqrtf(ts);
    }
    if (gv.tests) flush_tests(gv.tests, ntest);
}

// ---------------------------------------------------------------------------
// Ordering and placing hyperplanes: one workgroup (1024 threads) per edge,
// up to n_f rounds of (argmin over the alive candidates by (t*, index), the
// chosen candidate's row, discard of the candidates that row separates).
//
// Candidate j = tid + q blockDim with q < NQ keeps c* and t* in the thread's
// registers, and its direction a too when HOLD_A (NQ = kPlaceReg).  With more
// candidates, NQ = 2 kPlaceReg holds c* only and a chosen candidate's a is
// read from global memory (every candidate's a is loaded once at the start,
// so those reads hit L2).  Candidates past NQ blockDim (the tail) are read
// from global memory in every round, their alive flags in LDS.
// One barrier per round: each wave takes its smallest (t*, index) key by DPP
// and readlane, the lane holding that candidate publishes its c* and a in the
// wave's LDS slot, and after the barrier every wave reduces the slots' keys
// the same way (one slot per lane) and builds the row itself (the same FP32
// operations on the same values in every thread).  The chosen rows stay in
// LDS and are written to global memory once, after the last round.
// ---------------------------------------------------------------------------
constexpr int kPlaceReg = 4;       // candidates per thread held with their a
constexpr int kPlaceHist = 64;     // chosen rows kept in LDS until the end
constexpr int kPlaceWaves = 16;    // waves of the 1024-thread workgroup

struct PlaceSlot {                 // a wave's smallest candidate of one round
    float a[kMaxDof], c[kMaxDof];  // zero past dof
};

struct PlaceSmem {
    PlaceSlot slot[2][kPlaceWaves];                 // by round parity
    unsigned long long skey[2][kPlaceWaves];        // the slots' keys (~0: none)
    float hist_a[kPlaceHist][kMaxDof], hist_c[kPlaceHist][kMaxDof], hist_b[kPlaceHist];
    int hist_j[kPlaceHist];
    float sv[2][kMaxDof];                           // the edge's ends, zero past dof
};

// Upper bound of k_place's static LDS; the rest of the workgroup's LDS holds
// the tail's alive flags (one byte per candidate).
constexpr size_t kPlaceStaticLds = 8192;
static_assert(sizeof(PlaceSmem) + 256 <= kPlaceStaticLds, "k_place static LDS");

// Smallest value over the wave: DPP quad permutations (lane distance 1, 2),
// the half-row and row mirrors (every lane of a 16-lane row ends with the
// row's minimum), then the four rows' minima by readlane.  Every lane active.
__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
    v = min(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true));   // quad_perm [1,0,3,2]
    v = min(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true));   // quad_perm [2,3,0,1]
    v = min(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true));  // row_half_mirror
    v = min(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true));  // row_mirror
    const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
    const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
    const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
    const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
    return min(min(r0, r1), min(r2, r3));
}

__device__ __forceinline__ unsigned long long place_key(unsigned t_bits, int j) {
    return ((unsigned long long)t_bits << 32) | (unsigned)j;
}

// The placement rounds of edge e (n > 0 candidates); returns the rows placed.
template <int NQ, bool HOLD_A>
__device__ __forceinline__ int place_edge(PlaceSmem& sm, uint8_t* alive, int e, int dof, int n, int nf0,
                                          const float* __restrict__ cs, const float* __restrict__ ad,
                                          const float* __restrict__ ts, int cand_cap, int n_f, float step_back_max,
                                          float t_col, float* __restrict__ A, float* __restrict__ bvec, int cap,
                                          int* __restrict__ status, int* __restrict__ placed_idx,
                                          float* __restrict__ row_pts) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nt = blockDim.x, nw = nt >> 6;
    const int nreg = min(n, NQ * nt);
    float cx[NQ][kMaxDof];
    float ax[HOLD_A ? NQ : 1][kMaxDof];
    unsigned tk[NQ];
    bool al[NQ];
    // smallest (t*, index) key among this thread's alive candidates; after a
    // row is chosen the discard pass and the next round's scan are one pass
    unsigned long long best = ~0ull;
    float touch = 0.f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = tid + q * nt;
        al[q] = j < nreg;
        tk[q] = ~0u;
        if (al[q]) {
            tk[q] = __float_as_uint(ts[j]);
#pragma unroll
            for (int k = 0; k < kMaxDof; ++k) {
                cx[q][k] = k < dof ? cs[(size_t)k * cand_cap + j] : 0.f;
                const float a = k < dof ? ad[(size_t)k * cand_cap + j] : 0.f;
                if constexpr (HOLD_A) ax[q][k] = a;
                else touch += a;
            }
            const unsigned long long kj = place_key(tk[q], j);
            best = kj < best ? kj : best;
        }
    }
    if constexpr (!HOLD_A) asm volatile("" : : "v"(touch));   // keeps the loads that bring a into L2
    for (int j = nreg + tid; j < n; j += nt) {
        alive[j] = 1;
        const unsigned long long kj = place_key(__float_as_uint(ts[j]), j);
        best = kj < best ? kj : best;
    }
    int nf = nf0, placed = 0;
    for (int round = 0; round < n_f; ++round) {
        PlaceSlot* ps = sm.slot[round & 1];
        unsigned long long* pk = sm.skey[round & 1];
        // the wave's smallest key; the one lane holding it publishes c* and a
        const unsigned whi = wave_min_u32((unsigned)(best >> 32));
        const unsigned wlo = wave_min_u32((unsigned)(best >> 32) == whi ? (unsigned)best : ~0u);
        const unsigned long long wkey = place_key(whi, (int)wlo);
        if (lane == 0) pk[w] = wkey;
        if (wkey != ~0ull && best == wkey) {
            const int j = (int)wlo;
            if (j < nreg) {
                const int qb = j / nt;                    // j = tid + qb blockDim
#pragma unroll
                for (int k = 0; k < kMaxDof; ++k) {
                    float c = cx[0][k];
#pragma unroll
                    for (int q = 1; q < NQ; ++q)
                        if (q == qb) c = cx[q][k];
                    ps[w].c[k] = c;
                    if constexpr (HOLD_A) {
                        float a = ax[0][k];
#pragma unroll
                        for (int q = 1; q < NQ; ++q)
                            if (q == qb) a = ax[q][k];
                        ps[w].a[k] = a;
                    } else {
                        ps[w].a[k] = k < dof ? ad[(size_t)k * cand_cap + j] : 0.f;
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < kMaxDof; ++k) {
                    ps[w].a[k] = k < dof ? ad[(size_t)k * cand_cap + j] : 0.f;
                    ps[w].c[k] = k < dof ? cs[(size_t)k * cand_cap + j] : 0.f;
                }
            }
        }
        __syncthreads();
        // the workgroup's smallest key (the same in every thread) and its slot
        const unsigned long long kl = lane < nw ? pk[lane] : ~0ull;
        const unsigned bhi = wave_min_u32((unsigned)(kl >> 32));
        const unsigned blo = wave_min_u32((unsigned)(kl >> 32) == bhi ? (unsigned)kl : ~0u);
        const unsigned long long bk = place_key(bhi, (int)blo);
        if (bk == ~0ull) break;                           // no candidate left
        const int bw = __builtin_ctzll(__ballot(kl == bk));
        const int jb = (int)blo;
        if (__uint_as_float(bhi) <= t_col) {
            if (tid == 0) status[e] = 2;                  // EZO_EDGE_IN_COLLISION
            break;
        }
        if (nf >= cap) break;
        // the row a^T q <= b of candidate jb, with the relaxed step back.  The
        // sums run over all kMaxDof entries: the zero entries past dof add
        // +0, which can only turn a -0 sum into +0, and every sum below is
        // compared with or offset by a nonzero value, so the row, its bound
        // and every discard decision are those of the sums over dof entries.
        float rw[kMaxDof], rc[kMaxDof];
#pragma unroll
        for (int k = 0; k < kMaxDof; ++k) {
            rw[k] = ps[bw].a[k];
            rc[k] = ps[bw].c[k];
        }
        float bj = 0.f, av1 = 0.f, av2 = 0.f;
#pragma unroll
        for (int k = 0; k < kMaxDof; ++k) {
            bj = fmaf(rw[k], rc[k], bj);
            av1 = fmaf(rw[k], sm.sv[0][k], av1);
            av2 = fmaf(rw[k], sm.sv[1][k], av2);
        }
        const float r = fmaxf(av1, av2) - bj + step_back_max;
        const float delta = r > 0.f ? step_back_max - r : step_back_max;
        const float rhs = bj - delta;
        if (tid == 0) {
            if (placed < kPlaceHist) {
#pragma unroll
                for (int k = 0; k < kMaxDof; ++k) {
                    sm.hist_a[placed][k] = rw[k];
                    sm.hist_c[placed][k] = rc[k];
                }
                sm.hist_b[placed] = rhs;
                sm.hist_j[placed] = jb;
            } else {
                for (int k = 0; k < dof; ++k) {
                    A[((size_t)e * cap + nf) * dof + k] = rw[k];
                    if (row_pts) row_pts[((size_t)e * cap + nf) * dof + k] = rc[k];
                }
                bvec[(size_t)e * cap + nf] = rhs;
                if (placed_idx) placed_idx[(size_t)e * n_f + placed] = jb;
            }
        }
        ++nf;
        ++placed;
        best = ~0ull;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (!al[q]) continue;
            float ac = 0.f;
#pragma unroll
            for (int k = 0; k < kMaxDof; ++k) ac = fmaf(rw[k], cx[q][k], ac);   // zero past dof
            if (ac > rhs) {
                al[q] = false;
            } else {
                const unsigned long long kj = place_key(tk[q], tid + q * nt);
                best = kj < best ? kj : best;
            }
        }
        for (int j = nreg + tid; j < n; j += nt) {
            if (!alive[j]) continue;
            float ac = 0.f;
            for (int k = 0; k < dof; ++k) ac = fmaf(rw[k], cs[(size_t)k * cand_cap + j], ac);
            if (ac > rhs) {
                alive[j] = 0;
            } else {
                const unsigned long long kj = place_key(__float_as_uint(ts[j]), j);
                best = kj < best ? kj : best;
            }
        }
    }
    return placed;
}

// The end of a fused-loop iteration (the work of k_advance below) for a call
// with one edge, done by k_place's single workgroup after its own writes:
// at k == max_iters a running edge becomes MAX_ITERS (1); the running-edge
// count; the current row moves to table[k + 1]; the edge's statistics and
// the count for the host.  cur == NULL: k_advance does it.
struct IterEnd {
    int4* cur;
    const int4* table;
    int max_iters;
    int* active_count;
    int* host_active;                 // pinned, or NULL
    EdgeStatsDev* host_stats;         // pinned, or NULL
};

__global__ void __launch_bounds__(1024) k_place(int dof, const float* __restrict__ edges, const float* __restrict__ c_star,
                                                const float* __restrict__ a_dir, const float* __restrict__ t_star,
                                                const int* __restrict__ n_cands, int cand_cap, int n_f,
                                                float step_back_max, float t_col, float* __restrict__ A,
                                                float* __restrict__ bvec, int* __restrict__ n_faces, int cap,
                                                int* __restrict__ status, int* __restrict__ placed_idx,
                                                int* __restrict__ n_placed, const uint8_t* __restrict__ proj_any,
                                                EdgeStatsDev* __restrict__ stats, float* __restrict__ row_pts,
                                                IterEnd ie) {
    extern __shared__ __align__(16) char smem[];
    uint8_t* alive = reinterpret_cast<uint8_t*>(smem);                // [cand_cap]: tail candidates
    __shared__ PlaceSmem sm;
    const int e = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    // the edge's state, loaded together
    const int st = status[e];
    const int pany = proj_any ? proj_any[e] : 0;
    const int nc = n_cands[e], nfa = n_faces[e];
    int placed = 0;
    if (st < 0 && pany) {
        if (tid == 0) {
            status[e] = 2;   // EZO_EDGE_IN_COLLISION
            if (n_placed) n_placed[e] = 0;
        }
    } else if (st < 0) {
        const int n = min(max(nc, 0), cand_cap);
        const int nf0 = min(max(nfa, 0), cap);
        const float* v = edges + (size_t)e * 2 * dof;
        if (tid < 2 * kMaxDof) {
            const int end = tid / kMaxDof, k = tid % kMaxDof;
            sm.sv[end][k] = k < dof ? v[end * dof + k] : 0.f;
        }
        const float* cs = c_star + (size_t)e * dof * cand_cap;
        const float* ad = a_dir + (size_t)e * dof * cand_cap;
        const float* ts = t_star + (size_t)e * cand_cap;
        if (n <= kPlaceReg * nt)
            placed = place_edge<kPlaceReg, true>(sm, alive, e, dof, n, nf0, cs, ad, ts, cand_cap, n_f, step_back_max,
                                                 t_col, A, bvec, cap, status, placed_idx, row_pts);
        else
            placed = place_edge<2 * kPlaceReg, false>(sm, alive, e, dof, n, nf0, cs, ad, ts, cand_cap, n_f,
                                                      step_back_max, t_col, A, bvec, cap, status, placed_idx,
                                                      row_pts);
        __syncthreads();                                  // thread 0's rows in LDS
        const int nh = min(placed, kPlaceHist);
        for (int i = tid; i < nh * kMaxDof; i += nt) {
            const int rr = i / kMaxDof, k = i % kMaxDof;
            if (k >= dof) continue;
            A[((size_t)e * cap + nf0 + rr) * dof + k] = sm.hist_a[rr][k];
            if (row_pts) row_pts[((size_t)e * cap + nf0 + rr) * dof + k] = sm.hist_c[rr][k];
        }
        for (int rr = tid; rr < nh; rr += nt) {
            bvec[(size_t)e * cap + nf0 + rr] = sm.hist_b[rr];
            if (placed_idx) placed_idx[(size_t)e * n_f + rr] = sm.hist_j[rr];
        }
        if (tid == 0) {
            n_faces[e] = nf0 + placed;
            if (n_placed) n_placed[e] = placed;
            if (stats && !ie.cur) atomicAdd((unsigned long long*)&stats[e].planes, (unsigned long long)placed);
        }
    }
    if (ie.cur && tid == 0) {                 // one edge: every status write above was this thread's
        EdgeStatsDev s{};
        if (stats) {
            s = stats[e];
            s.planes += placed;
            if (placed) stats[e] = s;
        }
        if (ie.host_stats) ie.host_stats[e] = s;
        const int k = ie.cur->w;
        int running = 0;
        if (status[e] < 0) {
            if (k >= ie.max_iters) status[e] = 1;   // EZO_EDGE_MAX_ITERS
            else running = 1;
        }
        *ie.active_count = running;
        *ie.cur = ie.table[min(k + 1, ie.max_iters + 1)];
        if (ie.host_active) *ie.host_active = running;
    }
}

// ---------------------------------------------------------------------------
// Fused-loop bookkeeping
// ---------------------------------------------------------------------------
// P_e = D (box rows: +e_j <= hi_j, then -e_j <= -lo_j); status -1 (running) or
// INVALID (3) when a vertex is outside D or not finite.
// The autotuner's stand-in polytope: the joint box, its 2 dof rows repeated
// up to F rows (a typical face count of the loop; repeated rows leave the
// polytope unchanged).  One thread per edge.
__global__ void k_tune_polytope(int dof, const float* __restrict__ q_lo, const float* __restrict__ q_hi, int n_edges,
                                int cap, int F, float* __restrict__ A, float* __restrict__ bvec,
                                int* __restrict__ n_faces) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_edges) return;
    for (int f = 0; f < F; ++f) {
        const int g = f % (2 * dof), j0 = g % dof;
        for (int j = 0; j < dof; ++j) A[((size_t)e * cap + f) * dof + j] = j == j0 ? (g < dof ? 1.f : -1.f) : 0.f;
        bvec[(size_t)e * cap + f] = g < dof ? q_hi[j0] : -q_lo[j0];
    }
    n_faces[e] = F;
}

// The autotuner's lighter candidate counts: out[e] = min(in[e], cap).
__global__ void k_cap_counts(const int* __restrict__ in, int* __restrict__ out, int n, int cap) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = min(in[e], cap);
}

// The fused loop's start, one thread per edge (init_edge above).
__global__ void k_init_edges(EdgeInit ei) { init_edge(ei, blockIdx.x * blockDim.x + threadIdx.x); }

// End of an iteration: at k == max_iters every running edge becomes
// MAX_ITERS (1); count running edges; the current row moves to table[k + 1]
// (table[max_iters + 1] at most).  One workgroup.
__global__ void __launch_bounds__(256) k_advance(int4* __restrict__ cur, const int4* __restrict__ table, int max_iters,
                                                 int* __restrict__ status,
                                                 int n_edges, int* __restrict__ active_count,
                                                 int* __restrict__ host_active,
                                                 const EdgeStatsDev* __restrict__ stats,
                                                 EdgeStatsDev* __restrict__ host_stats) {
    // the edges' statistics after this iteration, for the host (pinned)
    if (host_stats)
        for (int e = threadIdx.x; e < n_edges; e += blockDim.x) host_stats[e] = stats[e];
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int k = cur->w;
    int local = 0;
    for (int e = threadIdx.x; e < n_edges; e += blockDim.x) {
        if (status[e] < 0) {
            if (k >= max_iters) status[e] = 1;   // EZO_EDGE_MAX_ITERS
            else ++local;
        }
    }
    atomicAdd(&cnt, local);
    __syncthreads();
    if (threadIdx.x == 0) {
        *active_count = cnt;
        *cur = table[min(k + 1, max_iters + 1)];
        if (host_active) *host_active = cnt;
    }
}

// Largest window of ezo_inflate_paths (edges of one path per round).
constexpr int kPathWindowMax = 1024;

// ---------------------------------------------------------------------------
// Inflation of piecewise-linear paths with the containment skip (Sec. V-A).
// Path p's edges are eoff[p] .. eoff[p+1]-1 (global numbering); its vertices
// start at eoff[p] + p, so edge g of path p runs from vertex g + p to g + p + 1.
// Round r takes the window of s edges at positions r s .. r s + s - 1 of every
// path; slot p s + i of the round holds position r s + i of path p.
// ---------------------------------------------------------------------------

// Smallest h in [h0, h1) whose set contains the segment v[0 .. 2 dof), or
// 0x7fffffff; set(h, &A_h, &b_h, &F) gives set h's rows and whether it counts
// (an inflated edge that ended CERTIFIED or MAX_ITERS).  Both ends satisfy
// every row a.v <= b (FP32, fmaf in index order).  One wave per candidate
// set, lanes over its rows; the whole workgroup calls it (it has barriers).
template <class SetFn>
__device__ inline int first_containing_set(int dof, const float* v, int h0, int h1, SetFn set, int* best) {
    if (threadIdx.x == 0) *best = 0x7fffffff;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    for (int h = h0 + wave; h < h1; h += n_waves) {
        const float* Ah;
        const float* bh;
        int F;
        if (!set(h, &Ah, &bh, &F) || F == 0) continue;        // uniform over the wave
        bool out = false;
        for (int f = lane; f < F; f += 64) {
            float a1 = 0.f, a2 = 0.f;
            for (int j = 0; j < dof; ++j) {
                const float a = Ah[(size_t)f * dof + j];
                a1 = fmaf(a, v[j], a1);
                a2 = fmaf(a, v[dof + j], a2);
            }
            out |= !(a1 <= bh[f] && a2 <= bh[f]);
        }
        if (__ballot(out) == 0 && lane == 0) atomicMin(best, h);
    }
    __syncthreads();
    return *best;
}

// One workgroup (256 threads) per path: the s slots of round r.  A slot past
// the path's end is skipped; an edge whose segment lies in a set of an
// earlier round is skipped too (covered_by = that set's edge); the others are
// inflated (covered_by = -1 for now).
__global__ void __launch_bounds__(256) k_path_round(int dof, const float* __restrict__ verts,
                                                    const int* __restrict__ eoff, int r, int s,
                                                    const float* __restrict__ A, const float* __restrict__ bvec,
                                                    const int* __restrict__ n_faces,
                                                    const int* __restrict__ status, int cap,
                                                    int* __restrict__ covered_by, float* __restrict__ round_edges,
                                                    int* __restrict__ round_ids, uint8_t* __restrict__ round_skip) {
    __shared__ int best;
    const int p = blockIdx.x;
    const int e0 = eoff[p], K = eoff[p + 1] - e0;
    for (int i = 0; i < s; ++i) {
        const int slot = p * s + i, k = r * s + i;
        float* re = round_edges + (size_t)slot * 2 * dof;
        if (k >= K) {
            if (threadIdx.x < 2 * dof) re[threadIdx.x] = 0.f;
            if (threadIdx.x == 0) {
                round_ids[slot] = e0;
                round_skip[slot] = 1;
            }
            continue;                                            // uniform over the workgroup
        }
        const int g = e0 + k;
        const float* v = verts + (size_t)(g + p) * dof;
        if (threadIdx.x < 2 * dof) re[threadIdx.x] = v[threadIdx.x];
        // sets of earlier rounds: final arrays, written by earlier kernels
        auto set = [&](int h, const float** Ah, const float** bh, int* F) {
            const int sh = status[h];
            *Ah = A + (size_t)h * cap * dof;
            *bh = bvec + (size_t)h * cap;
            *F = min(max(n_faces[h], 0), cap);
            return covered_by[h] == -1 && (sh == 0 || sh == 1);
        };
        const int h = first_containing_set(dof, v, e0, e0 + r * s, set, &best);
        if (threadIdx.x == 0) {
            const int c = h == 0x7fffffff ? -1 : h;
            covered_by[g] = c;
            round_ids[slot] = g;
            round_skip[slot] = c >= 0;
        }
    }
}

// One workgroup per path, the window's edges in path order: an inflated edge
// whose segment lies in the set of an earlier inflated edge of the same
// window is contained after all (covered_by = the first such edge, status
// CONTAINED, no rows); every other slot's rows, face count and status go to
// its global edge.  (Sets of earlier rounds were checked before inflation.)
__global__ void __launch_bounds__(256) k_path_resolve(int dof, const float* __restrict__ verts,
                                                      const int* __restrict__ eoff, int r, int s,
                                                      const float* __restrict__ rA, const float* __restrict__ rb,
                                                      const int* __restrict__ rnf, const int* __restrict__ rst,
                                                      int cap, float* __restrict__ A, float* __restrict__ bvec,
                                                      int* __restrict__ n_faces, int* __restrict__ status,
                                                      int* __restrict__ covered_by) {
    __shared__ int best;
    __shared__ uint8_t kept[kPathWindowMax];                     // window edge i holds its set
    const int p = blockIdx.x;
    const int e0 = eoff[p], K = eoff[p + 1] - e0;
    const int w0 = e0 + r * s;                                   // first edge of the window
    // the window's sets come from the round buffers (written by the inflation
    // kernels) and the decisions taken so far from LDS: this workgroup's own
    // global writes of this kernel are never read back
    auto set = [&](int h, const float** Ah, const float** bh, int* F) {
        const int sl = p * s + (h - w0);
        const int sh = rst[sl];
        *Ah = rA + (size_t)sl * cap * dof;
        *bh = rb + (size_t)sl * cap;
        *F = min(max(rnf[sl], 0), cap);
        return kept[h - w0] != 0 && (sh == 0 || sh == 1);
    };
    for (int i = 0; i < s && r * s + i < K; ++i) {
        const int slot = p * s + i, g = w0 + i;
        const float* v = verts + (size_t)(g + p) * dof;
        int h = 0x7fffffff;
        const bool inflated = covered_by[g] == -1;               // uniform over the workgroup
        if (inflated) h = first_containing_set(dof, v, w0, g, set, &best);
        if (threadIdx.x == 0) kept[i] = inflated && h == 0x7fffffff;
        if (inflated && h != 0x7fffffff) {
            if (threadIdx.x == 0) {
                covered_by[g] = h;
                n_faces[g] = 0;
                status[g] = 4;                                   // EZO_EDGE_CONTAINED
            }
        } else {
            const int F = min(max(rnf[slot], 0), cap);
            const float* sA = rA + (size_t)slot * cap * dof;
            float* dA = A + (size_t)g * cap * dof;
            for (int t = threadIdx.x; t < F * dof; t += blockDim.x) dA[t] = sA[t];
            for (int f = threadIdx.x; f < F; f += blockDim.x) bvec[(size_t)g * cap + f] = rb[(size_t)slot * cap + f];
            if (threadIdx.x == 0) {
                n_faces[g] = rnf[slot];
                status[g] = rst[slot];
            }
        }
        __syncthreads();                                         // kept[i] visible to the next edge
    }
}

// ---------------------------------------------------------------------------
// Collision map of a dynamic roadmap (appendix, DRM construction).  Voxel
// (i, j, k) of a dims.x x dims.y x dims.z grid of side `side` from corner lo
// has index v = (k dims.y + j) dims.x + i and stands for its circumscribing
// sphere (centre lo + side (i + 1/2, j + 1/2, k + 1/2), radius sqrt(3)/2 side).
// Bit n of row v of the map is set iff node n's robot collides with it.
// ---------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Voxel index range [i0, i1] along one axis whose centres lie within R of x
// (a superset: the exact test decides), clamped to the grid; empty if i0 > i1.
__device__ __forceinline__ void voxel_range(float x, float R, float lo, float inv, int n, int* i0, int* i1) {
    const float a = (x - R - lo) * inv - 0.5f, b = (x + R - lo) * inv - 0.5f;
    *i0 = (int)fmaxf(floorf(a), 0.f);
    *i1 = (int)fminf(ceilf(b), (float)(n - 1));
}

// One workgroup per tile of T nodes: FK into LDS, then every (node, sphere)
// and (node, box) item tests the voxels within reach and sets the node's bit
// in each hit voxel's row.
template <int T, bool BOX>
__global__ void __launch_bounds__(256) k_collision_map(RobotView rb, ObsView ob, const float* __restrict__ q,
                                                       int64_t n, float3 lo, float side, int3 dims,
                                                       uint32_t* __restrict__ map, int64_t row_words) {
    extern __shared__ __align__(16) char smem[];
    const int64_t base = (int64_t)blockIdx.x * T;
    if (base >= n) return;
    const int nv = (int)((n - base) < T ? (n - base) : T);
    TileSmem t = carve_tile(smem, T, tile_slots(rb.n_spheres, rb.n_boxes), blockDim.x >> 6);
    for (int i = threadIdx.x; i < T * rb.dof; i += blockDim.x) {
        const int c = i % T, j = i / T;
        if (c < nv) t.q[c * kMaxDof + j] = q[(base + c) * rb.dof + j];
    }
    __syncthreads();
    tile_fk<BOX>(rb, ob, t, T, nv);
    const float rv = 0.866025403784438647f * side, inv = 1.f / side;
    const int S = rb.n_spheres;
    for (ItemWalk w(nv); w.k < S; w.next(nv)) {
        const int c = w.c;
        const float4 C = t.cen[w.k * T + c];
        if (!(isfinite(C.x) && isfinite(C.y) && isfinite(C.z))) continue;
        const float R = C.w + rv;
        int i0, i1, j0, j1, k0, k1;
        voxel_range(C.x, R, lo.x, inv, dims.x, &i0, &i1);
        voxel_range(C.y, R, lo.y, inv, dims.y, &j0, &j1);
        voxel_range(C.z, R, lo.z, inv, dims.z, &k0, &k1);
        const int64_t node = base + c;
        const uint32_t bit = 1u << (node & 31);
        for (int k = k0; k <= k1; ++k) {
            const float dz = C.z - fmaf(side, (float)k + 0.5f, lo.z);
            for (int j = j0; j <= j1; ++j) {
                const float dy = C.y - fmaf(side, (float)j + 0.5f, lo.y);
                const float dyz = fmaf(dy, dy, dz * dz);
                for (int i = i0; i <= i1; ++i) {
                    const float dx = C.x - fmaf(side, (float)i + 0.5f, lo.x);
                    if (fmaf(dx, dx, dyz) < R * R) {
                        const int64_t v = ((int64_t)k * dims.y + j) * dims.x + i;
                        atomicOr(map + v * row_words + (node >> 5), bit);
                    }
                }
            }
        }
    }
    if (BOX) {
        for (ItemWalk w(nv); w.k < rb.n_boxes; w.next(nv)) {
            const int c = w.c;
            const DBox X = tile_box(t, S, T, w.k, c);
            if (!(isfinite(X.c[0]) && isfinite(X.c[1]) && isfinite(X.c[2]))) continue;
            float e[3];                        // half widths of the box's world AABB
#pragma unroll
            for (int a = 0; a < 3; ++a)
                e[a] = fmaf(X.h[0], fabsf(X.R[3 * a]), fmaf(X.h[1], fabsf(X.R[3 * a + 1]), X.h[2] * fabsf(X.R[3 * a + 2])));
            int i0, i1, j0, j1, k0, k1;
            voxel_range(X.c[0], e[0] + rv, lo.x, inv, dims.x, &i0, &i1);
            voxel_range(X.c[1], e[1] + rv, lo.y, inv, dims.y, &j0, &j1);
            voxel_range(X.c[2], e[2] + rv, lo.z, inv, dims.z, &k0, &k1);
            const int64_t node = base + c;
            const uint32_t bit = 1u << (node & 31);
            for (int k = k0; k <= k1; ++k)
                for (int j = j0; j <= j1; ++j)
                    for (int i = i0; i <= i1; ++i) {
                        const float x = fmaf(side, (float)i + 0.5f, lo.x), y = fmaf(side, (float)j + 0.5f, lo.y),
                                    z = fmaf(side, (float)k + 0.5f, lo.z);
                        if (hit_sphere_box(X, x, y, z, rv)) {
                            const int64_t v = ((int64_t)k * dims.y + j) * dims.x + i;
                            atomicOr(map + v * row_words + (node >> 5), bit);
                        }
                    }
        }
    }
}

// Colliding nodes per voxel: popcount of each row.  One wave per row.
__global__ void __launch_bounds__(256) k_row_popcount(const uint32_t* __restrict__ map, int64_t rows,
                                                      int64_t row_words, int64_t* __restrict__ counts) {
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (row >= rows) return;
    int64_t c = 0;
    for (int64_t w = lane; w < row_words; w += 64) c += __popc(map[row * row_words + w]);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane == 0) counts[row] = c;
}

// Exclusive prefix sum of counts[0..n) into offsets[0..n] (offsets[n] = total).
// One workgroup of 1024 threads, each summing a contiguous chunk.
__global__ void __launch_bounds__(1024) k_scan_counts(const int64_t* __restrict__ counts, int64_t n,
                                                      int64_t* __restrict__ offsets) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t a = min(n, tid * chunk), b = min(n, a + chunk);
    int64_t sum = 0;
    for (int64_t i = a; i < b; ++i) sum += counts[i];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {             // inclusive scan (Hillis-Steele)
        const int64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - sum;
    for (int64_t i = a; i < b; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
    if (tid == 1023) offsets[n] = part[1023];
}

// Node ids of each row in increasing order at offsets[row]: one wave per row,
// each lane one word at a time, the wave's exclusive prefix of the popcounts
// placing the lanes' ids.
__global__ void __launch_bounds__(256) k_map_lists(const uint32_t* __restrict__ map, int64_t rows, int64_t row_words,
                                                   int64_t n_nodes, const int64_t* __restrict__ offsets,
                                                   int32_t* __restrict__ ids) {
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (row >= rows) return;
    int64_t pos = offsets[row];
    for (int64_t w0 = 0; w0 < row_words; w0 += 64) {
        const int64_t w = w0 + lane;
        uint32_t bits = w < row_words ? map[row * row_words + w] : 0u;
        const int cnt = __popc(bits);
        int incl = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off);
            if (lane >= off) incl += v;
        }
        int64_t p = pos + incl - cnt;
        while (bits) {
            const int b = __builtin_ctz(bits);
            bits &= bits - 1u;
            const int64_t node = w * 32 + b;
            if (node < n_nodes) ids[p] = (int32_t)node;
            ++p;
        }
        pos += __shfl(incl, 63);
    }
}

// ---------------------------------------------------------------------------
// Recovery from collisions found on a trajectory (Sec. V-B)
// ---------------------------------------------------------------------------

// Pieces of segment i of a path through waypoints w [K][dof]:
// m_i = max(1, ceil(max_j |w_{i+1,j} - w_{i,j}| / step)), in FP64 from the
// FP32 waypoints (capped at 2^30).
__global__ void k_path_pieces(int dof, const float* __restrict__ w, int K, double step, int* __restrict__ m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K - 1) return;
    double mx = 0.0;
    for (int j = 0; j < dof; ++j)
        mx = fmax(mx, fabs((double)w[(size_t)(i + 1) * dof + j] - (double)w[(size_t)i * dof + j]));
    const double q = ceil(mx / step);
    m[i] = q < 1.0 ? 1 : (q > 1073741824.0 ? 1073741824 : (int)q);
}

// Points of the discretised path, row-major [n][dof]: segment i = blockIdx.x
// writes points j = 1..m_i (and j = 0 for i = 0), w_i + (j / m_i)(w_{i+1} -
// w_i) in FP32, from row off[i].
__global__ void __launch_bounds__(256) k_path_points(int dof, const float* __restrict__ w, const int* __restrict__ m,
                                                     const int64_t* __restrict__ off, float* __restrict__ pts) {
    const int i = blockIdx.x;
    const int mi = m[i];
    const int j0 = i == 0 ? 0 : 1;
    const float* a = w + (size_t)i * dof;
    const float* c = w + (size_t)(i + 1) * dof;
    for (int jj = threadIdx.x; jj <= mi - j0; jj += blockDim.x) {
        const int j = j0 + jj;
        const float t = (float)j / (float)mi;
        float* out = pts + (size_t)(off[i] + jj) * dof;
        for (int k = 0; k < dof; ++k) out[k] = fmaf(t, c[k] - a[k], a[k]);
    }
}

// out[r] = rows[idx[r]] for r < *n (rows of dof floats).
__global__ void k_gather_rows(int dof, const float* __restrict__ rows, const int* __restrict__ idx,
                              const int* __restrict__ n, int cap, float* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= cap || r >= *n) return;
    for (int k = 0; k < dof; ++k) out[(size_t)r * dof + k] = rows[(size_t)idx[r] * dof + k];
}

// Row-major [n][dof] -> coordinate-major [dof][n].
__global__ void k_rows_to_coords(int dof, const float* __restrict__ rows, int64_t n, float* __restrict__ coords) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < dof; ++k) coords[(size_t)k * n + i] = rows[(size_t)i * dof + k];
}

// flags[e][i] = 1 iff point i (coordinate-major pts [dof][n]) satisfies every
// row of polytope e and edge e's status is CERTIFIED or MAX_ITERS (a set
// that can be edited); blockIdx.y = e.
__global__ void __launch_bounds__(256) k_points_in_sets(int dof, const float* __restrict__ A,
                                                        const float* __restrict__ bvec,
                                                        const int* __restrict__ n_faces, int cap,
                                                        const int* __restrict__ status, const float* __restrict__ pts,
                                                        int64_t n, uint8_t* __restrict__ flags) {
    const int e = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool inside = status[e] == 0 || status[e] == 1;
    const int F = min(max(n_faces[e], 0), cap);
    float x[kMaxDof];
#pragma unroll
    for (int k = 0; k < kMaxDof; ++k) x[k] = k < dof ? pts[(size_t)k * n + i] : 0.f;
    const float* Ae = A + (size_t)e * cap * dof;
    for (int f = 0; f < F && inside; ++f) {
        float ax = 0.f;
        for (int k = 0; k < dof; ++k) ax = fmaf(Ae[(size_t)f * dof + k], x[k], ax);
        inside = ax <= bvec[(size_t)e * cap + f];
    }
    flags[(size_t)e * n + i] = inside ? 1 : 0;
}

// Edges with candidates run the placement (status -1), the rest are skipped.
__global__ void k_recover_begin(int n_edges, const int* __restrict__ n_cands, int* __restrict__ run,
                                int* __restrict__ n_placed) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_edges) return;
    run[e] = n_cands[e] > 0 ? -1 : 0;
    n_placed[e] = 0;
}

// A candidate within t_col of L or a colliding projection puts the edge in
// collision; planes_added[e] = planes placed.
__global__ void k_recover_end(int n_edges, const int* __restrict__ run, const int* __restrict__ n_placed,
                              int* __restrict__ status, int* __restrict__ planes_added) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_edges) return;
    if (run[e] == 2) status[e] = 2;   // EZO_EDGE_IN_COLLISION
    if (planes_added) planes_added[e] = n_placed[e];
}

// covered[k] = smallest set index whose polytope contains both ends of
// segment k (A v <= b + tol), -1 if none; blockIdx.x = k.
__global__ void __launch_bounds__(256) k_segments_contained(int dof, const float* __restrict__ A,
                                                            const float* __restrict__ bvec,
                                                            const int* __restrict__ n_faces, int cap, int n_sets,
                                                            const float* __restrict__ segs, float tol,
                                                            int* __restrict__ covered) {
    __shared__ int best;
    const int k = blockIdx.x;
    if (threadIdx.x == 0) best = 0x7fffffff;
    __syncthreads();
    const float* v = segs + (size_t)k * 2 * dof;
    for (int e = threadIdx.x; e < n_sets; e += blockDim.x) {
        const int F = min(max(n_faces[e], 0), cap);
        if (F == 0) continue;                    // an edge that holds no set
        const float* Ae = A + (size_t)e * cap * dof;
        bool in = true;
        for (int f = 0; f < F && in; ++f) {
            float a1 = 0.f, a2 = 0.f;
            for (int j = 0; j < dof; ++j) {
                const float a = Ae[(size_t)f * dof + j];
                a1 = fmaf(a, v[j], a1);
                a2 = fmaf(a, v[dof + j], a2);
            }
            const float bb = bvec[(size_t)e * cap + f] + tol;
            in = a1 <= bb && a2 <= bb;
        }
        if (in) atomicMin(&best, e);
    }
    __syncthreads();
    if (threadIdx.x == 0) covered[k] = best == 0x7fffffff ? -1 : best;
}

}  // namespace ezo
