// ezo_device.hpp -- device-side building blocks of the EI-ZO hot path on
// gfx950: Philox4x32-10, DH forward kinematics into LDS, and the workgroup
// "tile check" that decides collision for a tile of configurations.
//
// Tile check layout (one workgroup = W waves of 64 lanes):
//   * a tile holds T configurations (T in {8,16,32,64}); lane l of every
//     wave works on configuration (l % T) and on the sphere subset
//     (l / T) of that configuration, so one wave covers all T
//     configurations with 64/T lanes each;
//   * the W waves split the obstacle list into W contiguous slices.  The
//     obstacle index is wave-uniform, so obstacle records are read with
//     scalar loads and enter the pair arithmetic as SGPR operands;
//   * sphere centres of the tile live in LDS as [sphere][config] float4
//     (x, y, z, r), written once by the FK phase and read by every wave.
// Collision test per robot/obstacle pair, in a frame whose origin is the
// centre of the obstacle cloud (keeps |c|^2 and |o|^2 small):
//   v = (|c|^2 - r_c^2) + (|o|^2 - r_o^2) - 2 c.o - 2 r_c r_o = |c-o|^2 - (r_c+r_o)^2
// so a pair collides iff v < 0 (5 VALU ops + a running min).  The
// signed-distance mode evaluates |c - o| - r_o directly (difference form).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ezo {

// LDS (address space 3) views of generic pointers that point into the
// workgroup's LDS.  Through a generic pointer -- one that may also point to
// global memory, or any volatile access, which the compiler's address-space
// inference leaves alone -- every access is a flat instruction followed by a
// wait on both memory counters; through these it is a ds_* instruction.
template <class T>
using lds_ptr = __attribute__((address_space(3))) T*;
template <class T>
__device__ __forceinline__ lds_ptr<T> to_lds(T* p) { return (lds_ptr<T>)p; }

// Element i of an LDS array of int4 / int2 / float4, read as the compiler's
// native vectors (HIP's vector classes cannot be copied out of another
// address space).
typedef int lds_i4_t __attribute__((ext_vector_type(4)));
typedef int lds_i2_t __attribute__((ext_vector_type(2)));
typedef float lds_f4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int4 lds_load(lds_ptr<const int4> p, int i) {
    const lds_i4_t v = ((lds_ptr<const lds_i4_t>)p)[i];
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int2 lds_load(lds_ptr<const int2> p, int i) {
    const lds_i2_t v = ((lds_ptr<const lds_i2_t>)p)[i];
    return make_int2(v.x, v.y);
}
__device__ __forceinline__ float4 lds_load(lds_ptr<const float4> p, int i) {
    const lds_f4_t v = ((lds_ptr<const lds_f4_t>)p)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

constexpr int kMaxDof = 8;
constexpr float kHuge = 3.0e38f;

// ---------------------------------------------------------------------------
// Robot and obstacles as seen by kernels
// ---------------------------------------------------------------------------
struct RobotView {
    int dof;
    unsigned prismatic;        // bit j: joint j is prismatic (theta = 0, offset d_j + q_j)
    int n_spheres;
    int n_self;
    int n_blocks;
    const float4* dh;          // [dof] (a, d, cos alpha, sin alpha)
    const int* link_begin;     // [dof + 1] spheres of link i: [link_begin[i], link_begin[i+1])
    const float4* sph;         // [S] local (x, y, z), r -- sorted by link
    const int2* pairs;         // [P] self pairs, indices into the sorted order, grouped by block
    const float4* lbound;      // [kPartsPerLink dof] bounding sphere of each part of a link (part
                               // p of link l = index kPartsPerLink l + p, a consecutive run of the
                               // link's spheres): centre in the link frame, radius
    const int4* blocks;        // [n_blocks] per part pair: (part a, part b, first pair, pair count)
    // boxes on links, sorted by link: box k = four float4 in the link frame,
    // (centre, h_x), (rotation row 0, h_y), (row 1, h_z), (row 2, bounding
    // radius |h|); the rotation's columns are the box axes
    int n_boxes;
    int n_box_pairs;
    const float4* box;         // [B][4]
    const int* box_begin;      // [dof + 1] boxes of link i: [box_begin[i], box_begin[i+1])
    const int2* box_pairs;     // [Q] box self pairs (sorted indices)
    int staged;                // set by stage_robot: bit 0 blocks, bit 1 pairs in LDS (else 0)
};

// LDS rows of a tile's pose array: one per sphere, four per box.
__host__ __device__ inline int tile_slots(int n_spheres, int n_boxes) { return n_spheres + 4 * n_boxes; }

// Self-pair broad phase: each link's spheres split into kPartsPerLink parts
// (consecutive runs of its sphere list), each with its own bounding sphere;
// a work item (configuration, part pair) is taken by kItemLanes lanes.
constexpr int kPartsPerLink = 2;
constexpr int kItemLanes = 16;
constexpr int kMaxParts = kPartsPerLink * kMaxDof;
constexpr int kMaxPartPairs = kMaxParts * (kMaxParts + 1) / 2;   // part pairs, same-part pairs included
static_assert(kMaxPartPairs < 1024, "work items hold (part pair << 6) | configuration in 16 bits");

// Robot tables that a workgroup running many dependent tile checks (the
// bisection) copies into LDS once: DH rows, part bounding spheres, link
// sphere ranges, spheres, self-pair blocks and, up to kStagePairs of them,
// the self pairs; their reads in FK and in the self-pair sweep then cost an
// LDS access instead of a cache access.  At most this many bytes (slots >=
// spheres, n_self = self pairs, n_blocks = self-pair blocks).
constexpr int kStagePairs = 2048;

__host__ __device__ inline int robot_staged_pairs(int n_self) { return n_self <= kStagePairs ? n_self : 0; }

__host__ __device__ inline size_t robot_stage_bytes(int slots, int n_self, int n_blocks) {
    return 16 * (size_t)(kMaxDof + kMaxParts + (slots > 0 ? slots : 1) + (n_blocks > 0 ? n_blocks : 1)) +
           16 * ((kMaxDof + 4) / 4) + 16 * (((size_t)robot_staged_pairs(n_self) + 1) / 2);
}

// Copies the tables into LDS at `base` (16-byte aligned, robot_stage_bytes
// long) and returns a view whose table pointers address the copies (box
// tables, and self pairs beyond kStagePairs, stay in global memory).  The
// caller places a barrier before the first use.
__device__ inline RobotView stage_robot(const RobotView& rb, char* base) {
    float4* dh = reinterpret_cast<float4*>(base);
    float4* lb = dh + kMaxDof;
    float4* sph = lb + kMaxParts;
    int* lbeg = reinterpret_cast<int*>(sph + (rb.n_spheres > 0 ? rb.n_spheres : 1));
    int4* blk = reinterpret_cast<int4*>(lbeg + 4 * ((kMaxDof + 4) / 4));
    int2* prs = reinterpret_cast<int2*>(blk + (rb.n_blocks > 0 ? rb.n_blocks : 1));
    const int np = robot_staged_pairs(rb.n_self);
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < rb.dof; i += nt) dh[i] = rb.dh[i];
    for (int i = tid; i < kPartsPerLink * rb.dof; i += nt) lb[i] = rb.lbound[i];
    for (int i = tid; i <= rb.dof; i += nt) lbeg[i] = rb.link_begin[i];
    for (int i = tid; i < rb.n_blocks; i += nt) blk[i] = rb.blocks[i];
    for (int i = tid; i < rb.n_spheres; i += nt) sph[i] = rb.sph[i];
    for (int i = tid; i < np; i += nt) prs[i] = rb.pairs[i];
    RobotView v = rb;
    v.dh = dh;
    v.lbound = lb;
    v.blocks = blk;
    v.sph = sph;
    v.link_begin = lbeg;
    if (np > 0) v.pairs = prs;
    v.staged = 1 | (np > 0 ? 2 : 0);
    return v;
}

// Uniform grid over the obstacle cloud (shifted frame).  Cell k lists every
// obstacle that a robot sphere centred anywhere in cell k could touch: the
// distance from o to the cell's box is below r_o + r_sphere_max + slack (a
// sphere centre c in the box has |c - o| >= that distance).  A sphere centre
// outside the grid box is farther than r_sphere_max + r_o_max from every
// obstacle.  count[k] > cap marks an overflowing cell (scan all).
struct GridGeom {
    float ox, oy, oz;          // origin (min corner)
    float hx, hy, hz;          // cell size
    float ihx, ihy, ihz;       // 1 / cell size
    float reach;               // r_sphere_max + slack
};

struct GridView {
    int G;                     // cells per axis
    int cap;                   // list capacity per cell
    const GridGeom* geom;
    const int* count;          // [G^3]
    const unsigned short* list;  // [G^3][cap] obstacle indices
    unsigned long long* tests;   // optional [kTestSlots] counters of sphere-sphere tests performed
};

// Read-only global memory viewed through the constant address space: loads
// with a wave-uniform address then become scalar (s_load) loads.
typedef __attribute__((address_space(4))) const float cfloat;

__device__ __forceinline__ float4 cload4(const cfloat* p) { return make_float4(p[0], p[1], p[2], p[3]); }

struct ObsView {
    int n;
    int lds_n;                 // > 0: the workgroup stages the n records (x, y, z, r) in LDS
    const float4* rec;         // [n] (ox, oy, oz, ro), shifted frame
    const float4* centre;      // [1] shift applied to world coordinates (x' = x - centre)
    int n_ebox;                // obstacle boxes (world frame, packed like robot boxes)
    const float4* ebox;        // [n_ebox][4]
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11)
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit multiply (v_mad_u64_u32) gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        U4 n;
        n.x = hi1 ^ c.y ^ k0;
        n.y = lo1;
        n.z = hi0 ^ c.w ^ k1;
        n.w = lo0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// word -> (0, 1): ((x >> 9) + 1/2) * 2^-23, exact in FP32
__device__ __forceinline__ float u01(uint32_t x) {
    return ((float)(x >> 9) + 0.5f) * (1.0f / 8388608.0f);
}

__device__ __forceinline__ uint32_t word_of(const U4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// ---------------------------------------------------------------------------
// Forward kinematics: compose T <- T * A_l with the standard DH matrix
//   A = [[ct, -st ca,  st sa, a ct],
//        [st,  ct ca, -ct sa, a st],
//        [0,   sa,     ca,    d   ]]
// R is row-major 3x3, p the translation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dh_compose(float R[9], float p[3], float ct, float st, float4 dh) {
    const float a = dh.x, d = dh.y, ca = dh.z, sa = dh.w;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float r0 = R[3 * r + 0], r1 = R[3 * r + 1], r2 = R[3 * r + 2];
        const float u = fmaf(r0, ct, r1 * st);        // new column 0
        const float w = fmaf(r1, ct, -r0 * st);       // R * (-st, ct, 0)
        R[3 * r + 0] = u;
        R[3 * r + 1] = fmaf(w, ca, r2 * sa);
        R[3 * r + 2] = fmaf(r2, ca, -w * sa);
        p[r] = fmaf(a, u, fmaf(d, r2, p[r]));
    }
}

// ---------------------------------------------------------------------------
// Tile shared-memory carve-up (dynamic LDS)
// ---------------------------------------------------------------------------
struct TileSmem {
    float* q;          // [T][kMaxDof] configurations of the tile
    float2* trig;      // [kMaxDof][T] (cos, sin) of each joint
    float4* cen;       // [S + 4B][T] sphere centres (shifted frame) and radius, then each
                       // box's world pose as four rows (packed like RobotView::box)
    float4* lb;        // [kMaxParts][T] part bounding spheres (shifted frame)
    int* hit;          // [T] collision flag (flags mode) / validity
    int* scr;          // [T] 1 = the learned screen cleared this configuration's self pairs
    float* red;        // [2][W][T] partial minima (signed-distance mode)
    unsigned short* wl;  // [T][kMaxPartPairs] work list: (part pair << 6) | configuration, bounds overlapping
    int* wl_n;         // [1] work list length
    float4* obs;       // [lds_n] staged obstacle records (x, y, z, r), or NULL
};

__host__ __device__ inline size_t tile_smem_bytes(int T, int S, int W) {
    size_t b = 0;
    b += sizeof(float) * (size_t)T * kMaxDof;
    b += sizeof(float2) * (size_t)kMaxDof * T;
    b += sizeof(float4) * (size_t)(S > 0 ? S : 1) * T;
    b += sizeof(float4) * (size_t)kMaxParts * T;
    b += sizeof(int) * 2 * (size_t)T;
    b += sizeof(float) * 2 * (size_t)W * T;
    b += sizeof(unsigned short) * (size_t)T * kMaxPartPairs + sizeof(int);
    return (b + 15) & ~(size_t)15;
}

// Obstacle staging follows the tile region: tile_smem_bytes(T, S, W) + 16 lds_n.
__device__ inline TileSmem carve_tile(char* base, int T, int S, int W, int lds_n = 0) {
    TileSmem t;
    t.obs = lds_n > 0 ? reinterpret_cast<float4*>(base + tile_smem_bytes(T, S, W)) : nullptr;
    char* p = base;
    t.cen = reinterpret_cast<float4*>(p);   p += sizeof(float4) * (size_t)(S > 0 ? S : 1) * T;
    t.lb = reinterpret_cast<float4*>(p);    p += sizeof(float4) * (size_t)kMaxParts * T;
    t.trig = reinterpret_cast<float2*>(p);  p += sizeof(float2) * (size_t)kMaxDof * T;
    t.q = reinterpret_cast<float*>(p);      p += sizeof(float) * (size_t)T * kMaxDof;
    t.red = reinterpret_cast<float*>(p);    p += sizeof(float) * 2 * (size_t)W * T;
    t.hit = reinterpret_cast<int*>(p);      p += sizeof(int) * (size_t)T;
    t.scr = reinterpret_cast<int*>(p);      p += sizeof(int) * (size_t)T;
    t.wl = reinterpret_cast<unsigned short*>(p);  p += sizeof(unsigned short) * (size_t)T * kMaxPartPairs;
    t.wl_n = reinterpret_cast<int*>(p);
    return t;
}

// Work items (c, k), c < n, k < K, item index k n + c, spread over the
// workgroup's threads: one division per loop instead of one per item.
struct ItemWalk {
    int c, k, dc, dk;
    __device__ ItemWalk(int n) {
        const int nt = blockDim.x, tid = threadIdx.x;
        if ((n & (n - 1)) == 0) {                  // a power of two: shifts
            const int sh = __builtin_ctz(n);
            k = tid >> sh;
            dk = nt >> sh;
        } else {
            k = tid / n;
            dk = nt / n;
        }
        c = tid - k * n;
        dc = nt - dk * n;
    }
    __device__ void next(int n) {
        c += dc;
        k += dk;
        if (c >= n) {
            c -= n;
            ++k;
        }
    }
};

// FK phase: t.q[c][j] (c < n_valid) -> t.cen[s][c].  Ends with a barrier.
// Only the n_valid >= 1 configurations of the tile are computed.
// BOX = false compiles the sphere-only path (no box code, fewer registers);
// BOX = true adds the boxes of RobotView and ObsView.
template <bool BOX>
__device__ inline void tile_fk(const RobotView& rb, const ObsView& ob, const TileSmem& t, int T, int n_valid) {
    const int dof = rb.dof;
    for (ItemWalk w(n_valid); w.k < dof; w.next(n_valid)) {
        const int c = w.c, j = w.k;
        float s = 0.f, co = 1.f;
        if (!((rb.prismatic >> j) & 1u)) {
            // v_sin_f32 / v_cos_f32 take revolutions: q / (2 pi), rounded once
            const float rev = t.q[c * kMaxDof + j] * 0.15915494309189535f;
            s = __builtin_amdgcn_sinf(rev);
            co = __builtin_amdgcn_cosf(rev);
        }
        t.trig[j * T + c] = make_float2(co, s);
    }
    __syncthreads();
    const float4 sh = ob.centre[0];
    // P lanes per (configuration, link), P the largest power of two (<= 16)
    // with n_valid dof P items in one pass of the workgroup: each composes the
    // link's frame and places every P-th sphere (and box) of the link, so a
    // long link is spread over idle lanes instead of being placed by one
    int lp = 0;
    while (lp < 4 && n_valid * dof * (2 << lp) <= (int)blockDim.x) ++lp;
    const int P = 1 << lp;
    for (ItemWalk w(n_valid); w.k < dof * P; w.next(n_valid)) {
        const int c = w.c, link = w.k >> lp, part = w.k & (P - 1);
        float R[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
        float p[3] = {-sh.x, -sh.y, -sh.z};
        for (int l = 0; l <= link; ++l) {
            const float2 cs = t.trig[l * T + c];
            float4 dh = rb.dh[l];
            if ((rb.prismatic >> l) & 1u) dh.y += t.q[c * kMaxDof + l];
            dh_compose(R, p, cs.x, cs.y, dh);
        }
        if (part < kPartsPerLink) {       // the link's part bounds, spread over its P lanes
            for (int pp = part; pp < kPartsPerLink; pp += P) {
                const float4 lc = rb.lbound[kPartsPerLink * link + pp];
                float4 o;
                o.x = fmaf(R[0], lc.x, fmaf(R[1], lc.y, fmaf(R[2], lc.z, p[0])));
                o.y = fmaf(R[3], lc.x, fmaf(R[4], lc.y, fmaf(R[5], lc.z, p[1])));
                o.z = fmaf(R[6], lc.x, fmaf(R[7], lc.y, fmaf(R[8], lc.z, p[2])));
                o.w = lc.w;
                t.lb[(kPartsPerLink * link + pp) * T + c] = o;
            }
        }
        const int s1 = rb.link_begin[link + 1];
        for (int s = rb.link_begin[link] + part; s < s1; s += P) {
            const float4 ps = rb.sph[s];
            float4 o;
            o.x = fmaf(R[0], ps.x, fmaf(R[1], ps.y, fmaf(R[2], ps.z, p[0])));
            o.y = fmaf(R[3], ps.x, fmaf(R[4], ps.y, fmaf(R[5], ps.z, p[1])));
            o.z = fmaf(R[6], ps.x, fmaf(R[7], ps.y, fmaf(R[8], ps.z, p[2])));
            o.w = ps.w;
            t.cen[s * T + c] = o;
        }
        if (BOX && rb.n_boxes > 0) {
            const int S = rb.n_spheres;
            const int k1 = rb.box_begin[link + 1];
            for (int k = rb.box_begin[link] + part; k < k1; k += P) {
                const float4 b0 = rb.box[4 * k], b1 = rb.box[4 * k + 1], b2 = rb.box[4 * k + 2], b3 = rb.box[4 * k + 3];
                const float L[9] = {b1.x, b1.y, b1.z, b2.x, b2.y, b2.z, b3.x, b3.y, b3.z};
                float4* dst = t.cen + (size_t)(S + 4 * k) * T + c;
                float W[9];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        W[3 * i + j] = fmaf(R[3 * i], L[j], fmaf(R[3 * i + 1], L[3 + j], R[3 * i + 2] * L[6 + j]));
                dst[0] = make_float4(fmaf(R[0], b0.x, fmaf(R[1], b0.y, fmaf(R[2], b0.z, p[0]))),
                                     fmaf(R[3], b0.x, fmaf(R[4], b0.y, fmaf(R[5], b0.z, p[1]))),
                                     fmaf(R[6], b0.x, fmaf(R[7], b0.y, fmaf(R[8], b0.z, p[2]))), b0.w);
                dst[T] = make_float4(W[0], W[1], W[2], b1.w);
                dst[2 * T] = make_float4(W[3], W[4], W[5], b2.w);
                dst[3 * T] = make_float4(W[6], W[7], W[8], b3.w);
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Box geometry (FP32).  A box: centre c, rotation R (row-major, columns = the
// box axes), half extents h, bounding radius |h|.
// ---------------------------------------------------------------------------
struct DBox {
    float c[3];
    float R[9];
    float h[3];
    float rb;
};

// Row i of a box's four packed float4 (c, h_x), (R row 0, h_y), (R row 1, h_z),
// (R row 2, bounding radius); the centre shifted by -sh.
__device__ __forceinline__ DBox unpack_box(float4 b0, float4 b1, float4 b2, float4 b3, float3 sh) {
    DBox x;
    x.c[0] = b0.x - sh.x;
    x.c[1] = b0.y - sh.y;
    x.c[2] = b0.z - sh.z;
    x.R[0] = b1.x; x.R[1] = b1.y; x.R[2] = b1.z;
    x.R[3] = b2.x; x.R[4] = b2.y; x.R[5] = b2.z;
    x.R[6] = b3.x; x.R[7] = b3.y; x.R[8] = b3.z;
    x.h[0] = b0.w;
    x.h[1] = b1.w;
    x.h[2] = b2.w;
    x.rb = b3.w;
    return x;
}

__device__ __forceinline__ DBox tile_box(const TileSmem& t, int S, int T, int k, int c) {
    const float4* p = t.cen + (size_t)(S + 4 * k) * T + c;
    return unpack_box(p[0], p[T], p[2 * T], p[3 * T], make_float3(0.f, 0.f, 0.f));
}

// Per-axis excess of a point over the box, e_k = |p_k| - h_k with p the
// point in box coordinates; returns max_k e_k and sum_k max(e_k, 0)^2.
__device__ __forceinline__ void box_excess(const DBox& B, float x, float y, float z, float* emax, float* out2) {
    const float dx = x - B.c[0], dy = y - B.c[1], dz = z - B.c[2];
    float m = -INFINITY, o = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float pk = fmaf(B.R[k], dx, fmaf(B.R[3 + k], dy, B.R[6 + k] * dz));
        const float e = fabsf(pk) - B.h[k];
        m = fmaxf(m, e);
        const float ep = fmaxf(e, 0.f);
        o = fmaf(ep, ep, o);
    }
    *emax = m;
    *out2 = o;
}

// Signed distance sphere (x, r) - box: outside sqrt(sum max(e,0)^2) - r, inside
// max_k e_k - r (minus the distance to the nearest face, minus r).
__device__ __forceinline__ float sd_sphere_box(const DBox& B, float x, float y, float z, float r) {
    float m, o;
    box_excess(B, x, y, z, &m, &o);
    return (m <= 0.f ? m : sqrtf(o)) - r;
}

// Collision test of the same pair: signed distance < 0.
__device__ __forceinline__ bool hit_sphere_box(const DBox& B, float x, float y, float z, float r) {
    float m, o;
    box_excess(B, x, y, z, &m, &o);
    return m <= 0.f ? (m < r) : (o < r * r);
}

// Separating-axis value of two boxes: with C_ij = A_i . B_j and t_i = A_i . t
// (t = c_B - c_A, A_i and B_j the box axes), the face axes give
// |t_i| - h_Ai - sum_j h_Bj |C_ij| and |sum_i C_ij t_i| - sum_i h_Ai |C_ij| - h_Bj.
// A cross axis n = A_i x B_j is taken in A's frame, where it is
// (n_i, n_i1, n_i2) = (0, -C_i2,j, C_i1,j) (i1 = i+1, i2 = i+2 mod 3): its
// length is sqrt(C_i1,j^2 + C_i2,j^2) (a sum of squares, so nearly parallel
// edges keep their length to full relative precision; skipped below 1e-6),
// and every term of the unnormalised value
//   |t . n| - sum_k h_Ak |n_k| - sum_k h_Bk |B_k . n|,
//   B_k . n = C_i1,j C_i2,k - C_i2,j C_i1,k   (a cofactor of C; 0 for k = j)
// is a product of n's components, so its rounding error scales with |n| and
// the normalised value is as accurate as that of a well separated axis.
// Returns the largest value (exact: all axes).  With early = true it returns
// as soon as an axis has a value >= 0 (the boxes do not collide) and the
// result is then only that value.
template <bool EARLY>
__device__ inline float sat_value(const DBox& A, const DBox& B) {
    const float tx = B.c[0] - A.c[0], ty = B.c[1] - A.c[1], tz = B.c[2] - A.c[2];
    float C[3][3], aC[3][3], t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        t[i] = fmaf(A.R[i], tx, fmaf(A.R[3 + i], ty, A.R[6 + i] * tz));
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C[i][j] = fmaf(A.R[i], B.R[j], fmaf(A.R[3 + i], B.R[3 + j], A.R[6 + i] * B.R[6 + j]));
            aC[i][j] = fabsf(C[i][j]);
        }
    }
    float best = -INFINITY;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float v = fabsf(t[i]) - A.h[i] - fmaf(B.h[0], aC[i][0], fmaf(B.h[1], aC[i][1], B.h[2] * aC[i][2]));
        best = fmaxf(best, v);
        if (EARLY && v >= 0.f) return v;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float tb = fmaf(C[0][j], t[0], fmaf(C[1][j], t[1], C[2][j] * t[2]));
        const float v = fabsf(tb) - fmaf(A.h[0], aC[0][j], fmaf(A.h[1], aC[1][j], A.h[2] * aC[2][j])) - B.h[j];
        best = fmaxf(best, v);
        if (EARLY && v >= 0.f) return v;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            const float n2 = fmaf(C[i1][j], C[i1][j], C[i2][j] * C[i2][j]);
            if (n2 < 1e-12f) continue;
            const float bj1 = fmaf(C[i1][j], C[i2][j1], -C[i2][j] * C[i1][j1]);
            const float bj2 = fmaf(C[i1][j], C[i2][j2], -C[i2][j] * C[i1][j2]);
            const float u = fabsf(fmaf(t[i2], C[i1][j], -t[i1] * C[i2][j])) -
                            fmaf(A.h[i1], aC[i2][j], fmaf(A.h[i2], aC[i1][j],
                                 fmaf(B.h[j1], fabsf(bj1), B.h[j2] * fabsf(bj2))));
            const float v = u * rsqrtf(n2);
            best = fmaxf(best, v);
            if (EARLY && u >= 0.f) return v;
        }
    }
    return best;
}

// Copy the obstacle records (x, y, z, r) into the workgroup's LDS copy.
// Ends with a barrier.
__device__ inline void stage_obstacles(const ObsView& ob, const TileSmem& t) {
    if (t.obs)
        for (int o = threadIdx.x; o < ob.lds_n; o += blockDim.x) t.obs[o] = ob.rec[o];
    __syncthreads();
}

__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ bool wave_all(bool p) {
    return __ballot(p) == __ballot(true);
}

// Signed-distance pair sweep.  Results: t.red[0][0][c] = overall minimum,
// t.red[1][0][c] = self minimum; t.hit[c] = (overall < 0).  Barrier at exit.
// Distances by v_sqrt_f32 (one instruction, within about 1 ulp; the
// correctly rounded sqrtf takes several more per pair).
template <bool BOX>
__device__ inline void tile_pairs_sd(const RobotView& rb, const ObsView& ob, const TileSmem& t, int T,
                                     int n_valid) {
    const int tid = threadIdx.x;
    const int W = blockDim.x >> 6;
    const int w = wave_id();
    const int lane = tid & 63;
    const int c = lane % T;
    const int nsub = 64 / T;
    const int j = lane / T;
    const int S = rb.n_spheres;
    float env = INFINITY, self = INFINITY;
    {
        const int P = rb.n_self;
        for (int p = w * nsub + j; p < P; p += W * nsub) {
            const int2 pr = rb.pairs[p];
            const float4 a = t.cen[pr.x * T + c];
            const float4 b = t.cen[pr.y * T + c];
            const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
            const float d = __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
            self = fminf(self, d - a.w - b.w);
        }
    }
    const int o0 = (int)(((long)ob.n * w) / W);
    const int o1 = (int)(((long)ob.n * (w + 1)) / W);
    if (o1 > o0) {
        for (int s0 = 0; s0 < S; s0 += 2 * nsub) {
            const int sa = s0 + j, sb = s0 + nsub + j;
            const float4 A = sa < S ? t.cen[sa * T + c] : make_float4(kHuge, kHuge, kHuge, 0.f);
            const float4 B = sb < S ? t.cen[sb * T + c] : make_float4(kHuge, kHuge, kHuge, 0.f);
            float bestA = INFINITY, bestB = INFINITY;
            const cfloat* rec = (const cfloat*)ob.rec;
#pragma unroll 4
            for (int o = o0; o < o1; ++o) {
                const float4 P0 = cload4(rec + 4 * o);
                const float ax = A.x - P0.x, ay = A.y - P0.y, az = A.z - P0.z;
                const float bx = B.x - P0.x, by = B.y - P0.y, bz = B.z - P0.z;
                const float dA = __builtin_amdgcn_sqrtf(fmaf(ax, ax, fmaf(ay, ay, az * az)));
                const float dB = __builtin_amdgcn_sqrtf(fmaf(bx, bx, fmaf(by, by, bz * bz)));
                bestA = fminf(bestA, dA - P0.w);
                bestB = fminf(bestB, dB - P0.w);
            }
            if (sa < S) env = fminf(env, bestA - A.w);
            if (sb < S) env = fminf(env, bestB - B.w);
        }
    }
    if (BOX && (rb.n_boxes > 0 || ob.n_ebox > 0)) {
        const float4 shv = ob.centre[0];
        const float3 sh = make_float3(shv.x, shv.y, shv.z);
        const int B = rb.n_boxes;
        const bool ok = c < n_valid;
        for (int p = w * nsub + j; ok && p < rb.n_box_pairs; p += W * nsub) {
            const int2 pr = rb.box_pairs[p];
            self = fminf(self, sat_value<false>(tile_box(t, S, T, pr.x, c), tile_box(t, S, T, pr.y, c)));
        }
        for (int k = w * nsub + j; ok && k < B; k += W * nsub) {
            const DBox X = tile_box(t, S, T, k, c);
            for (int o = 0; o < ob.n; ++o) {
                const float4 O = ob.rec[o];
                env = fminf(env, sd_sphere_box(X, O.x, O.y, O.z, O.w));
            }
            for (int e = 0; e < ob.n_ebox; ++e)
                env = fminf(env, sat_value<false>(X, unpack_box(ob.ebox[4 * e], ob.ebox[4 * e + 1], ob.ebox[4 * e + 2],
                                                                ob.ebox[4 * e + 3], sh)));
        }
        for (int s2 = w * nsub + j; ok && ob.n_ebox > 0 && s2 < S; s2 += W * nsub) {
            const float4 C = t.cen[s2 * T + c];
            for (int e = 0; e < ob.n_ebox; ++e)
                env = fminf(env, sd_sphere_box(unpack_box(ob.ebox[4 * e], ob.ebox[4 * e + 1], ob.ebox[4 * e + 2],
                                                          ob.ebox[4 * e + 3], sh), C.x, C.y, C.z, C.w));
        }
    }
    // reduce over the lanes of one configuration, then over waves
    for (int off = T; off < 64; off <<= 1) {
        env = fminf(env, __shfl_xor(env, off));
        self = fminf(self, __shfl_xor(self, off));
    }
    if (j == 0) {
        t.red[(0 * W + w) * T + c] = fminf(env, self);
        t.red[(1 * W + w) * T + c] = self;
    }
    __syncthreads();
    if (tid < T) {
        float m = INFINITY, s = INFINITY;
        for (int k = 0; k < W; ++k) {
            m = fminf(m, t.red[(0 * W + k) * T + tid]);
            s = fminf(s, t.red[(1 * W + k) * T + tid]);
        }
        t.red[tid] = m;
        t.red[W * T + tid] = s;
        t.hit[tid] = (m < 0.f) ? 1 : 0;
    }
    __syncthreads();
}

// Flags-mode sweep with broad phase.  Self pairs: the bounding spheres of
// the two links of every (configuration, link pair) are tested first; the
// overlapping ones go to an LDS work list, and each wave then takes a work
// item and tests its link pair's sphere pairs one per lane (coalesced pair
// loads, no divergence).  Obstacles: a work item (configuration, sphere)
// tests only the obstacles listed in the sphere's grid cell.  Every skipped
// pair is provably separated, so the flag equals that of the all-pairs
// test.  The pair test is |c - o|^2 < (r_c + r_o)^2 (difference form).
// Needs *t.wl_n == 0 on entry.  Barrier at exit.
// Returns the number of sphere-sphere tests this thread performed (bound
// tests included).
// Box pairs of a tile, flags mode (after the sphere passes; configurations
// already hit are skipped): the box self pairs, every robot box against every
// obstacle sphere and obstacle box, every robot sphere against every obstacle
// box.  Each pair is first bounded by the two bounding spheres (a pair they
// prove apart cannot collide), then tested exactly.
__device__ inline void tile_boxes_flags(const RobotView& rb, const ObsView& ob, const TileSmem& t, int T,
                                        int n_valid) {
    const lds_ptr<volatile int> hit = to_lds((volatile int*)t.hit);
    const int S = rb.n_spheres, B = rb.n_boxes;
    const float4 shv = ob.centre[0];
    const float3 sh = make_float3(shv.x, shv.y, shv.z);
    for (ItemWalk w(n_valid); w.k < rb.n_box_pairs; w.next(n_valid)) {
        const int c = w.c;
        if (hit[c]) continue;
        const int2 pr = rb.box_pairs[w.k];
        const DBox X = tile_box(t, S, T, pr.x, c), Y = tile_box(t, S, T, pr.y, c);
        const float dx = X.c[0] - Y.c[0], dy = X.c[1] - Y.c[1], dz = X.c[2] - Y.c[2];
        const float Rr = X.rb + Y.rb;
        if (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) >= Rr * Rr) continue;
        if (sat_value<true>(X, Y) < 0.f) hit[c] = 1;
    }
    for (ItemWalk w(n_valid); w.k < B; w.next(n_valid)) {
        const int c = w.c;
        if (hit[c]) continue;
        const DBox X = tile_box(t, S, T, w.k, c);
        bool found = false;
        for (int o = 0; o < ob.n && !found; ++o) {
            const float4 O = t.obs ? t.obs[o] : ob.rec[o];
            const float dx = O.x - X.c[0], dy = O.y - X.c[1], dz = O.z - X.c[2];
            const float Rr = X.rb + O.w;
            if (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < Rr * Rr && hit_sphere_box(X, O.x, O.y, O.z, O.w)) found = true;
        }
        for (int e = 0; e < ob.n_ebox && !found; ++e) {
            const DBox E = unpack_box(ob.ebox[4 * e], ob.ebox[4 * e + 1], ob.ebox[4 * e + 2], ob.ebox[4 * e + 3], sh);
            const float dx = E.c[0] - X.c[0], dy = E.c[1] - X.c[1], dz = E.c[2] - X.c[2];
            const float Rr = X.rb + E.rb;
            if (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < Rr * Rr && sat_value<true>(X, E) < 0.f) found = true;
        }
        if (found) hit[c] = 1;
    }
    if (ob.n_ebox > 0) {
        for (ItemWalk w(n_valid); w.k < S; w.next(n_valid)) {
            const int c = w.c;
            if (hit[c]) continue;
            const float4 C = t.cen[w.k * T + c];
            bool found = false;
            for (int e = 0; e < ob.n_ebox && !found; ++e) {
                const DBox E = unpack_box(ob.ebox[4 * e], ob.ebox[4 * e + 1], ob.ebox[4 * e + 2], ob.ebox[4 * e + 3], sh);
                const float dx = E.c[0] - C.x, dy = E.c[1] - C.y, dz = E.c[2] - C.z;
                const float Rr = E.rb + C.w;
                if (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < Rr * Rr && hit_sphere_box(E, C.x, C.y, C.z, C.w)) found = true;
            }
            if (found) hit[c] = 1;
        }
    }
}

// Self-pair items of the work list (kItemLanes lanes each; blocks and pairs
// from LDS when the robot tables are staged, else from global memory).
template <class BlkF, class PairF>
__device__ __forceinline__ void tile_self_items(BlkF block, PairF pair, const TileSmem& t, int T,
                                                lds_ptr<volatile int> hit, unsigned& ntest) {
    // 64 / kItemLanes work items per wave, kItemLanes lanes each (a part
    // pair holds a fraction of its link pair's sphere pairs)
    constexpr int IPW = 64 / kItemLanes;
    const int n_items = *t.wl_n;
    const int lane = threadIdx.x & 63, sub = lane / kItemLanes, li = lane % kItemLanes;
    const int nw = blockDim.x >> 6;
    for (int it0 = IPW * wave_id(); it0 < n_items; it0 += IPW * nw) {
        const int it = it0 + sub;
        if (it >= n_items) continue;
        const int item = t.wl[it];
        const int c = item & 63;
        if (hit[c]) continue;                          // uniform in the lane group
        const int4 blk = block(item >> 6);
        bool found = false;
        for (int p = li; p < blk.w; p += kItemLanes) {
            const int2 pr = pair(blk.z + p);
            const float4 a = t.cen[pr.x * T + c];
            const float4 b = t.cen[pr.y * T + c];
            const float ex = a.x - b.x, ey = a.y - b.y, ez = a.z - b.z;
            const float Rr = a.w + b.w;
            ++ntest;
            found |= fmaf(ex, ex, fmaf(ey, ey, ez * ez)) < Rr * Rr;
        }
        if (found) hit[c] = 1;
    }
}

// Obstacle sweep: a (configuration, sphere) item tests the obstacles listed in
// its grid cell (records from LDS when staged, else from global memory); the
// four records of a list load are fetched together and tested branch-free.
template <class RecF>
__device__ __forceinline__ void tile_obstacle_items(RecF rec, const ObsView& ob, const GridView& gv, const TileSmem& t,
                                                    int T, int n_valid, int S, lds_ptr<volatile int> hit,
                                                    unsigned& ntest) {
    const GridGeom g = *gv.geom;
    const int G = gv.G;
    for (ItemWalk w(n_valid); w.k < S; w.next(n_valid)) {
        const int c = w.c, s = w.k;
        if (hit[c]) continue;
        const float4 C = t.cen[s * T + c];
        const float fx = (C.x - g.ox) * g.ihx, fy = (C.y - g.oy) * g.ihy, fz = (C.z - g.oz) * g.ihz;
        if (!(fx >= 0.f && fy >= 0.f && fz >= 0.f && fx < (float)G && fy < (float)G && fz < (float)G)) continue;
        const int cx = min((int)fx, G - 1), cy = min((int)fy, G - 1), cz = min((int)fz, G - 1);
        const int cell = (cz * G + cy) * G + cx;
        const int cnt = gv.count[cell];
        const bool full = cnt > gv.cap;
        const int n = full ? ob.n : cnt;
        // list entries four at a time (cell lists are 8-byte aligned)
        const ushort4* lst4 = reinterpret_cast<const ushort4*>(gv.list + (size_t)cell * gv.cap);
        bool found = false;
        for (int k0 = 0; k0 < n && !found; k0 += 4) {
            int oi[4];
            if (full) {
                oi[0] = k0; oi[1] = k0 + 1; oi[2] = k0 + 2; oi[3] = k0 + 3;
            } else {
                const ushort4 v = lst4[k0 >> 2];
                oi[0] = v.x; oi[1] = v.y; oi[2] = v.z; oi[3] = v.w;
            }
            float4 O[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) O[e] = rec((k0 + e < n) ? oi[e] : oi[0]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool ok = k0 + e < n;
                ntest += ok ? 1u : 0u;
                const float ex = C.x - O[e].x, ey = C.y - O[e].y, ez = C.z - O[e].z;
                const float Rr = C.w + O[e].w;
                found |= ok && fmaf(ex, ex, fmaf(ey, ey, ez * ez)) < Rr * Rr;
            }
        }
        if (found) hit[c] = 1;
    }
}

template <bool BOX>
__device__ inline unsigned tile_pairs_grid(const RobotView& rb, const ObsView& ob, const GridView& gv,
                                           const TileSmem& t, int T, int n_valid) {
    const lds_ptr<volatile int> hit = to_lds((volatile int*)t.hit);
    unsigned int ntest = 0;
    if (rb.n_blocks > 0) {
        const bool lblk = (rb.staged & 1) != 0, lprs = (rb.staged & 2) != 0;
        const lds_ptr<const int4> blocks_l = to_lds(rb.blocks);
        const lds_ptr<const int2> pairs_l = to_lds(rb.pairs);
        for (ItemWalk w(n_valid); w.k < rb.n_blocks; w.next(n_valid)) {
            const int c = w.c, bk = w.k;
            if (hit[c] || t.scr[c]) continue;
            const int4 blk = lblk ? lds_load(blocks_l, bk) : rb.blocks[bk];
            const float4 A = t.lb[blk.x * T + c], B = t.lb[blk.y * T + c];
            const float dx = A.x - B.x, dy = A.y - B.y, dz = A.z - B.z;
            const float R = A.w + B.w;
            ++ntest;
            if (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < R * R)
                t.wl[atomicAdd(t.wl_n, 1)] = (unsigned short)((bk << 6) | c);
        }
        __syncthreads();
        if (lblk && lprs)
            tile_self_items([=](int i) { return lds_load(blocks_l, i); }, [=](int i) { return lds_load(pairs_l, i); },
                            t, T, hit, ntest);
        else
            tile_self_items([=](int i) { return rb.blocks[i]; }, [=](int i) { return rb.pairs[i]; }, t, T, hit, ntest);
    }
    if (ob.n > 0) {
        if (t.obs) {
            const lds_ptr<const float4> rl = to_lds((const float4*)t.obs);
            tile_obstacle_items([=](int o) { return lds_load(rl, o); }, ob, gv, t, T, n_valid, rb.n_spheres, hit,
                                ntest);
        } else {
            const float4* rg = ob.rec;
            tile_obstacle_items([=](int o) { return rg[o]; }, ob, gv, t, T, n_valid, rb.n_spheres, hit, ntest);
        }
    }
    if (BOX && (rb.n_boxes > 0 || ob.n_ebox > 0)) tile_boxes_flags(rb, ob, t, T, n_valid);
    __syncthreads();
    return ntest;
}

// Adds the wave's test counts to one of kTestSlots counters (spread by
// workgroup, so that the atomics of many small workgroups do not queue on
// one address).  Every lane of the wave must call it.
constexpr int kTestSlots = 256;

__device__ inline void flush_tests(unsigned long long* tests, unsigned n) {
    unsigned long long v = n;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(tests + (blockIdx.x + 97u * blockIdx.y) % kTestSlots, v);
}

// Whole tile check on t.q[0..n_valid).  Flags mode fills t.hit; signed-
// distance mode also fills t.red[c] (overall) and t.red[W*T + c] (self).
// Returns the thread's count of pair tests (flags mode; 0 otherwise).
template <bool SD, bool BOX>
__device__ inline unsigned tile_check(const RobotView& rb, const ObsView& ob, const GridView& gv, const TileSmem& t,
                                      int T, int n_valid) {
    // cleared here, published by FK's barriers (every reader of the previous
    // check's flags and work list is behind a barrier the caller placed)
    if (threadIdx.x < (unsigned)T) t.hit[threadIdx.x] = (threadIdx.x < (unsigned)n_valid) ? 0 : 1;
    if (threadIdx.x == 0) *t.wl_n = 0;
    tile_fk<BOX>(rb, ob, t, T, n_valid);
    if (SD) {
        tile_pairs_sd<BOX>(rb, ob, t, T, n_valid);
        return 0;
    }
    return tile_pairs_grid<BOX>(rb, ob, gv, t, T, n_valid);
}

}  // namespace ezo
