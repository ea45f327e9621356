// ezo_api.hip -- host runtime and C ABI of the EI-ZO hot path (declared in
// include/ezo.h).  Contexts own a growable device workspace and one internal
// stream; robots are uploaded once and rounded to FP32; the fused inflation
// captures one iteration of kernels into a hipGraph and replays it, polling a
// 4-byte active-edge counter after each replay.
#include "ezo_internal.hpp"
#include "ezo_kernels.hpp"

using namespace ezo;

std::string g_create_err;

ezo_status ezo_fail(ezo_ctx* c, ezo_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_err = buf;
    return code;
}

ezo_status ezo_ws_get(ezo_ctx* c, int slot, size_t bytes, void** out) {
    DevBuf& b = c->ws[slot];
    if (bytes == 0) bytes = 16;
    if (b.bytes < bytes) {
        if (b.p) {
            hipError_t e = hipFree(b.p);
            (void)e;
            b.p = nullptr;
            b.bytes = 0;
        }
        size_t nb = bytes + bytes / 4 + 256;
        const hipError_t me = hipMalloc(&b.p, nb);
        if (me != hipSuccess) {
            b.p = nullptr;
            return ezo_fail(c, EZO_E_NOMEM, "device allocation of %zu bytes failed: %s", nb, hipGetErrorString(me));
        }
        b.bytes = nb;
    }
    *out = b.p;
    return EZO_OK;
}

namespace {


// Tile size for a tile check: largest T whose LDS fits and that still gives
// at least ~4 workgroups per CU; W waves split the obstacles.
constexpr size_t kObsStageBytes = 32768;   // obstacle records staged in LDS up to this size

int pick_T(const ezo_ctx* c, int64_t items, int S, int W, size_t extra = 0) {
    const int cand[4] = {64, 32, 16, 8};
    int fit = 0;
    for (int T : cand) {
        if (tile_smem_bytes(T, S, W) + extra > c->lds_cap) continue;
        if (!fit) fit = T;
        if (items / T >= 4 * kNumCU) return T;
    }
    if (!fit) {
        for (int T : {4, 2, 1})
            if (tile_smem_bytes(T, S, W) + extra <= c->lds_cap) return T;
        return 0;
    }
    // few items: smallest fitting tile gives the most workgroups
    int best = fit;
    for (int T : cand)
        if (tile_smem_bytes(T, S, W) + extra <= c->lds_cap) best = T;
    return best;
}

// Obstacle records go to LDS when they fit beside a tile of T (and `extra`
// bytes more: the bisection's staged robot tables).
bool stage_fits(const ezo_ctx* c, int T, int S, int W, int n_obs, size_t extra = 0) {
    const size_t b = 16 * (size_t)n_obs;
    return T > 0 && n_obs > 0 && b <= kObsStageBytes && tile_smem_bytes(T, S, W) + b + extra <= c->lds_cap;
}

int pick_W(int n_obs) {
    if (n_obs >= 1024) return 8;
    if (n_obs >= 128) return 8;
    if (n_obs >= 16) return 4;
    return 2;
}

constexpr int kGridCap = 128;
static_assert(kGridCap % 8 == 0, "the sweep loads cell lists eight entries (16 bytes) at a time");

int grid_dim(int n_obs) { return n_obs >= 256 ? 32 : (n_obs >= 32 ? 16 : 8); }

// Obstacle records, the frame shift and the broad-phase grid for one call,
// written to the given device buffers (every byte the kernels read later is
// rewritten here: nothing needs to start at zero).
ezo_status prep_obstacles_into(ezo_ctx* c, const ezo_robot* r, const float* obs, int n_obs, hipStream_t st,
                               void* rec, void* centre, void* geom, void* count, void* list, ObsView* ov,
                               GridView* gv, const EdgeInit* ei = nullptr) {
    const int G = grid_dim(n_obs);
    // indices above 65535 do not fit the list type: then every cell scans all
    const bool lists = n_obs <= 65535;
    // the cell counts are cleared by extra workgroups (2048 cells each), and
    // the fused loop's edge start rides along as further workgroups (ei)
    const int clear_wg = (G * G * G + 2047) / 2048;
    const int init_wg = (ei && ei->n_edges > 0) ? (ei->n_edges + 255) / 256 : 0;
    hipLaunchKernelGGL(k_prep_obstacles, dim3(1 + clear_wg + init_wg), dim3(256), 0, st, obs, n_obs, (float4*)rec,
                       (float4*)centre, (GridGeom*)geom, G, r ? r->r_max : 0.f, (int*)count, lists ? 0 : kGridCap + 1,
                       clear_wg, init_wg ? *ei : EdgeInit{});
    if (lists && n_obs > 0)
        hipLaunchKernelGGL(k_grid_scatter, dim3((unsigned)(((int64_t)n_obs * 64 + 255) / 256)), dim3(256), 0, st,
                           (const float4*)rec, n_obs, (const GridGeom*)geom, G, kGridCap, (int*)count,
                           (unsigned short*)list);
    HIP_TRY(c, hipGetLastError());
    ov->n = n_obs;
    ov->lds_n = 0;
    ov->rec = (const float4*)rec;
    ov->centre = (const float4*)centre;
    ov->n_ebox = c->n_ebox;
    ov->ebox = c->ebox;
    gv->G = G;
    gv->cap = kGridCap;
    gv->geom = (const GridGeom*)geom;
    gv->count = (const int*)count;
    gv->list = (const unsigned short*)list;
    gv->tests = nullptr;
    return EZO_OK;
}

// The same in the context's workspace.
ezo_status prep_obstacles(ezo_ctx* c, const ezo_robot* r, const float* obs, int n_obs, hipStream_t st,
                          ObsView* ov, GridView* gv, const EdgeInit* ei = nullptr) {
    ezo_status s;
    void *rec, *centre, *geom, *count, *list;
    const size_t cells = (size_t)grid_dim(n_obs) * grid_dim(n_obs) * grid_dim(n_obs);
    if ((s = ezo_ws_get(c, W_OBS_REC, sizeof(float4) * (size_t)std::max(n_obs, 1), &rec)) != EZO_OK) return s;
    if ((s = ezo_ws_get(c, W_OBS_CENTRE, sizeof(float4), &centre)) != EZO_OK) return s;
    if ((s = ezo_ws_get(c, W_GRID_GEOM, sizeof(GridGeom), &geom)) != EZO_OK) return s;
    if ((s = ezo_ws_get(c, W_GRID_COUNT, sizeof(int) * cells, &count)) != EZO_OK) return s;
    if ((s = ezo_ws_get(c, W_GRID_LIST, sizeof(unsigned short) * cells * kGridCap, &list)) != EZO_OK) return s;
    return prep_obstacles_into(c, r, obs, n_obs, st, rec, centre, geom, count, list, ov, gv, ei);
}

// ---------------------------------------------------------------------------
// Fixed scratch of ezo_check_collisions_noalloc: the obstacle records, frame
// shift, grid geometry, grid cell counts and cell lists of one call with up to
// EZO_NOALLOC_MAX_OBSTACLES obstacles (grid of 32^3 cells).  A file-scope
// device array: every device the library runs on holds one copy until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host that name is only a stand-in); it uses the device address taken with
// hipGetSymbolAddress at context creation.
// ---------------------------------------------------------------------------
constexpr size_t kScrRec = 0;
constexpr size_t kScrCentre = kScrRec + 16 * (size_t)EZO_NOALLOC_MAX_OBSTACLES;
constexpr size_t kScrGeom = kScrCentre + 256;
constexpr size_t kScrCount = kScrGeom + 256;
constexpr size_t kScrCells = 32 * 32 * 32;
constexpr size_t kScrList = kScrCount + sizeof(int) * kScrCells;
constexpr size_t kScrBytes = kScrList + sizeof(unsigned short) * kScrCells * kGridCap;
static_assert(sizeof(GridGeom) <= 256, "grid geometry slot");
static_assert(kScrList % 256 == 0, "list slot alignment");

static __device__ __align__(256) unsigned char scratch[kScrBytes];

// Device address of this device's `scratch`; the device must be current.
// Returns nullptr (and leaves no HIP error behind) when it cannot be taken.
unsigned char* scratch_address() {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return static_cast<unsigned char*>(ptr);
}

bool pow2_tile(int T) { return T == 1 || T == 2 || T == 4 || T == 8 || T == 16 || T == 32 || T == 64; }

// Configurations per tile check: T for a check; T candidates x (2^depth - 1)
// bisection points for the bisection.
int tile_configs(const TileCfg& g, bool bisect) { return bisect ? g.T * ((1 << g.depth) - 1) : g.T; }

// Bisection shapes that have a kernel instance.
bool bisect_shape_built(const TileCfg& g) {
    return (g.depth == 1 && g.T >= 2 && g.T <= 64) || (g.depth == 2 && g.T <= 16) || (g.depth == 3 && g.T <= 8);
}

// A shape is usable when its LDS fits and staging is possible where asked.
bool cfg_valid(const ezo_ctx* c, const TileCfg& g, int S, int P, int NB, int n_obs, bool sd, bool bisect = false) {
    if (!pow2_tile(g.T) || g.W < 1 || g.W > 16 || g.depth < 1 || g.depth > 3) return false;
    if (bisect ? !bisect_shape_built(g) : g.depth != 1) return false;
    const int T = tile_configs(g, bisect);
    const size_t rs = bisect ? robot_stage_bytes(S, P, NB) : 0;
    if (g.stage && (sd || !stage_fits(c, T, S, g.W, n_obs, rs))) return false;
    return tile_smem_bytes(T, S, g.W) + (g.stage ? 16 * (size_t)n_obs : 0) + rs <= c->lds_cap;
}

TuneKey tune_key(const ezo_ctx* c, const ezo_robot* r, TuneKind kind, int n_obs, int64_t items) {
    TuneKey k;
    k.arch = c->arch;
    k.kind = kind;
    k.dof = r->dof;
    k.S = r->S;
    k.P = r->P;
    k.B = r->B;
    k.n_obs = n_obs;
    k.bucket = ezo_tune_bucket(items);
    return k;
}

// Heuristic shapes, used when tuning is off and nothing is cached.
TileCfg heuristic_check(const ezo_ctx* c, const ezo_robot* r, int n_obs, int64_t items, bool sd) {
    TileCfg g;
    g.W = sd ? pick_W(n_obs) : 4;
    g.T = pick_T(c, items, r->slots, g.W);
    g.stage = (!sd && stage_fits(c, g.T, r->slots, g.W, n_obs)) ? 1 : 0;
    return g;
}

// items = candidate slots; one bisection level per round.
TileCfg heuristic_bisect(const ezo_ctx* c, const ezo_robot* r, int n_obs, int64_t items) {
    TileCfg g;
    g.W = 4;
    g.depth = 1;
    const size_t rs = robot_stage_bytes(r->slots, r->P, r->view.n_blocks);
    g.T = std::max(std::min(pick_T(c, items, r->slots, g.W, rs), 64), 2);
    g.stage = stage_fits(c, g.T, r->slots, g.W, n_obs, rs) ? 1 : 0;
    return g;
}

TileCfg resolve_cfg(const ezo_ctx* c, const TuneKey& k, const TileCfg& fallback, int S, int P, int NB, int n_obs, bool sd,
                    bool bisect = false) {
    TileCfg g;
    if (ezo_tune_lookup(k, &g) && cfg_valid(c, g, S, P, NB, n_obs, sd, bisect)) return g;
    return fallback;
}

// Candidate shapes: every fitting T x W x staging (x bisection depth 1..2);
// T = configurations (check, 4..64) or candidates (bisection, 1..64) per
// workgroup; items = configurations or candidate slots.
std::vector<TileCfg> tile_candidates(const ezo_ctx* c, int S, int P, int NB, int n_obs, bool sd, std::initializer_list<int> Ws,
                                     int64_t items, bool bisect = false) {
    std::vector<TileCfg> v;
    // (bisection: one or two levels per round; three, seven points per
    // candidate and round, never came near the fastest and only lengthened
    // the first call's search, so the kernel's depth-3 instances are reached
    // only through a shape given explicitly)
    for (int dp = 1; dp <= (bisect ? 2 : 1); ++dp)
        for (int T : {64, 32, 16, 8, 4, 2, 1}) {
            if ((!bisect && T < 4) || (T > 4 && items < 4LL * T)) continue;   // a handful of items: small tiles
            for (int W : Ws)
                for (int st = 0; st <= (sd ? 0 : 1); ++st) {
                    TileCfg g{T, W, st, dp};
                    if (cfg_valid(c, g, S, P, NB, n_obs, sd, bisect)) v.push_back(g);
                }
        }
    return v;
}

template <bool SD>
ezo_status launch_check(ezo_ctx* c, const ezo_robot* r, const ObsView& ov, const GridView& gv, const float* q, int64_t n,
                        int64_t sn, int64_t sd, int64_t q_batch, uint8_t* flags, float* min_sd,
                        float* min_sd_self, int64_t out_batch, int n_batch, const int* status,
                        const IterArgs& it, hipStream_t st, const float* pred = nullptr, float margin = 0.f,
                        EdgeStatsDev* stats = nullptr, const TileCfg* shape = nullptr) {
    TileCfg g;
    if (shape) {
        g = *shape;
    } else {
        const int64_t items = n * n_batch;
        g = resolve_cfg(c, tune_key(c, r, SD ? TUNE_CHECK_SD : TUNE_CHECK_FLAGS, ov.n, items),
                        heuristic_check(c, r, ov.n, items, SD), r->slots, r->P, r->view.n_blocks, ov.n, SD);
    }
    const int T = g.T, W = g.W;
    if (T == 0) return ezo_fail(c, EZO_E_UNSUPPORTED, "robot too large for one tile");
    ObsView ovs = ov;
    ovs.lds_n = g.stage ? ov.n : 0;
    const size_t lds = tile_smem_bytes(T, r->slots, W) + 16 * (size_t)ovs.lds_n;
    const int64_t tiles = (n + T - 1) / T;
    if (tiles <= 0) return EZO_OK;
    dim3 grid((unsigned)tiles, (unsigned)n_batch), block(64 * W);
    const bool box = r->B > 0 || ov.n_ebox > 0;
#define EZO_LAUNCH_CHECK(TT)                                                                                   \
    do {                                                                                                       \
        if (box)                                                                                               \
            EZO_KLAUNCH(c, (k_check<TT, SD, true>), grid, block, lds, st, r->view, ovs, gv, q, n, sn, sd, q_batch, \
                        flags, min_sd, min_sd_self, out_batch, status, it, pred, margin, stats);               \
        else                                                                                                   \
            EZO_KLAUNCH(c, (k_check<TT, SD, false>), grid, block, lds, st, r->view, ovs, gv, q, n, sn, sd,      \
                        q_batch, flags, min_sd, min_sd_self, out_batch, status, it, pred, margin, stats);      \
    } while (0)
    switch (T) {
        case 64: EZO_LAUNCH_CHECK(64); break;
        case 32: EZO_LAUNCH_CHECK(32); break;
        case 16: EZO_LAUNCH_CHECK(16); break;
        case 8: EZO_LAUNCH_CHECK(8); break;
        case 4: EZO_LAUNCH_CHECK(4); break;
        case 2: EZO_LAUNCH_CHECK(2); break;
        default: EZO_LAUNCH_CHECK(1); break;
    }
#undef EZO_LAUNCH_CHECK
    HIP_TRY(c, hipGetLastError());
    return EZO_OK;
}

TuneKey sample_key(const ezo_ctx* c, int dof, int64_t walks) {
    TuneKey k;
    k.arch = c->arch;
    k.kind = TUNE_SAMPLE;
    k.dof = dof;
    k.bucket = ezo_tune_bucket(walks);
    return k;
}

// Lanes per walk: 8 when walks are few (fill the chip), else 4.
TileCfg heuristic_sample(int64_t walks) {
    TileCfg g;
    g.T = (walks * 8 <= 64LL * 4 * 4 * kNumCU * 64) ? 8 : 4;
    g.W = 4;
    return g;
}

bool sample_cfg_valid(const TileCfg& g) {
    return (g.T == 1 || g.T == 2 || g.T == 4 || g.T == 8 || g.T == 16) && g.W == 4;
}

// Walks of all running edges up to which the fused loop's sampler splits a
// walk over 16 / 4 lanes (above: one lane per walk).  Measured on MI355X for
// the 7-DOF sampler at 14-144 rows: 16 lanes win at 10 k walks (up to 9x
// over one lane), 4 lanes at 160 k (by up to 1.4x), one lane at 960 k rows
// <= 74 (by 5-25 %).
constexpr int64_t kSampleWalks16 = 40000;
constexpr int64_t kSampleWalks4 = 400000;

// `active` (device, may be NULL): number of running edges; when given, the
// adaptive kernel chooses the lanes per walk on the device each launch.
ezo_status launch_sample(ezo_ctx* c, int dof, const float* A, const float* b, const int* n_faces, int cap,
                         const float* edges, int E, int max_samples, int n_mix, uint64_t seed, int64_t eid0,
                         float* S, int64_t stride, const int* status, const IterArgs& it, hipStream_t st,
                         const TileCfg* shape = nullptr, const int* active = nullptr,
                         const int* edge_ids = nullptr) {
    const int D = dof <= 4 ? 4 : 8;
    if (sample_smem_bytes(D, 16, cap, 256) > c->lds_cap)
        return ezo_fail(c, EZO_E_UNSUPPORTED, "face capacity %d too large for the sampler", cap);
    if (max_samples <= 0 || E <= 0) return EZO_OK;
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    if (active) {
        const size_t lds = sample_smem_bytes(D, 16, cap, 256);
        dim3 grid((unsigned)(((int64_t)max_samples * 16 + 255) / 256), (unsigned)E), block(256);
        // a 7-DOF arm walks in exactly seven coordinates (the eighth of the
        // padded width only adds zero terms: the samples are the same bits)
        if (D == 4)
            EZO_KLAUNCH(c, k_sample_auto<4>, grid, block, lds, st, dof, A, b, n_faces, cap, edges, key0, key1, eid0,
                        n_mix, S, stride, status, it, active, kSampleWalks16, kSampleWalks4, edge_ids);
        else if (dof == 7)
            EZO_KLAUNCH(c, k_sample_auto<7>, grid, block, sample_smem_bytes(7, 16, cap, 256), st, dof, A, b, n_faces,
                        cap, edges, key0, key1, eid0, n_mix, S, stride, status, it, active, kSampleWalks16,
                        kSampleWalks4, edge_ids);
        else
            EZO_KLAUNCH(c, k_sample_auto<8>, grid, block, lds, st, dof, A, b, n_faces, cap, edges, key0, key1, eid0,
                        n_mix, S, stride, status, it, active, kSampleWalks16, kSampleWalks4, edge_ids);
        HIP_TRY(c, hipGetLastError());
        return EZO_OK;
    }
    const int64_t walks = (int64_t)max_samples * E;
    TileCfg g;
    if (shape) {
        g = *shape;
    } else {
        const TileCfg h = heuristic_sample(walks);
        g = (ezo_tune_lookup(sample_key(c, dof, walks), &g) && sample_cfg_valid(g)) ? g : h;
    }
    if (!sample_cfg_valid(g)) return ezo_fail(c, EZO_E_INVALID, "sampler shape T=%d W=%d", g.T, g.W);
    const int L = g.T;
    const size_t lds = sample_smem_bytes(D, L, cap, 256);
    const int64_t threads = (int64_t)max_samples * L;
    dim3 grid((unsigned)((threads + 255) / 256), (unsigned)E), block(256);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#define EZO_LAUNCH_SAMPLE(DD, LL)                                                                                 \
    EZO_KLAUNCH(c, (k_sample<DD, LL>), grid, block, lds, st, dof, A, b, n_faces, cap, edges, k0, k1, eid0, n_mix, \
                       S, stride, status, it)
    if (D == 4) {
        switch (L) {
            case 1: EZO_LAUNCH_SAMPLE(4, 1); break;
            case 2: EZO_LAUNCH_SAMPLE(4, 2); break;
            case 4: EZO_LAUNCH_SAMPLE(4, 4); break;
            case 8: EZO_LAUNCH_SAMPLE(4, 8); break;
            default: EZO_LAUNCH_SAMPLE(4, 16); break;
        }
    } else {
        switch (L) {
            case 1: EZO_LAUNCH_SAMPLE(8, 1); break;
            case 2: EZO_LAUNCH_SAMPLE(8, 2); break;
            case 4: EZO_LAUNCH_SAMPLE(8, 4); break;
            case 8: EZO_LAUNCH_SAMPLE(8, 8); break;
            default: EZO_LAUNCH_SAMPLE(8, 16); break;
        }
    }
#undef EZO_LAUNCH_SAMPLE
    HIP_TRY(c, hipGetLastError());
    return EZO_OK;
}

ezo_status launch_project_bisect(ezo_ctx* c, const ezo_robot* r, const ObsView& ov, const GridView& gv,
                                 const float* edges, int E,
                                 const float* S, int64_t stride, const int* cand_idx, const int* n_cands,
                                 int cand_cap, int n_b, float* c_star, float* a_dir, float* t_star,
                                 uint8_t* pcol, uint8_t* pany, const int* status, hipStream_t st,
                                 const TileCfg* shape = nullptr, int64_t s_edge = -1, const MlpView* screen = nullptr,
                                 EdgeStatsDev* stats = nullptr) {
    if (s_edge < 0) s_edge = (int64_t)r->dof * stride;   // samples [E][dof][stride]
    TileCfg g;
    if (shape) {
        g = *shape;
    } else {
        const int64_t items = (int64_t)cand_cap * E;
        g = resolve_cfg(c, tune_key(c, r, TUNE_BISECT, ov.n, items), heuristic_bisect(c, r, ov.n, items), r->slots, r->P, r->view.n_blocks,
                        ov.n, false, true);
    }
    const bool box = r->B > 0 || ov.n_ebox > 0;
    // the screened form (sphere robots): one bisection level per round, at
    // most 16 points per tile, at least four waves (the network's layers)
    const bool scr = screen && screen->P && !box;
    if (scr) {
        g.depth = 1;
        g.T = std::min(std::max(g.T, 2), 16);
        g.W = std::max(g.W, 4);
    }
    const int TC = g.T, W = g.W, dp = g.depth;
    if (!bisect_shape_built(g) || W < 1 || W > 16)
        return ezo_fail(c, EZO_E_INVALID, "bisection shape T=%d W=%d depth=%d", TC, W, dp);
    ObsView ovs = ov;
    ovs.lds_n = g.stage ? ov.n : 0;
    size_t lds = tile_smem_bytes(tile_configs(g, true), r->slots, W) + 16 * (size_t)ovs.lds_n +
                 robot_stage_bytes(r->slots, r->P, r->view.n_blocks);
    if (scr) {
        lds += mlp_tile_smem_bytes(1) + 16 * sizeof(float);
        if (lds > c->lds_cap && ovs.lds_n > 0) {        // drop the obstacle staging first
            lds -= 16 * (size_t)ovs.lds_n;
            ovs.lds_n = 0;
        }
    }
    if (lds > c->lds_cap) return ezo_fail(c, EZO_E_UNSUPPORTED, "robot too large for one tile");
    dim3 grid((unsigned)((cand_cap + TC - 1) / TC), (unsigned)E), block(64 * W);
    const MlpView mv = scr ? *screen : MlpView{0, 0, nullptr, nullptr, nullptr, 0.f};
    if (scr) {
        switch (TC) {
            case 16: EZO_KLAUNCH(c, (k_project_bisect<16, 1, false, true>), grid, block, lds, st, r->view, ovs, gv,
                                 edges, S, stride, s_edge, cand_idx, n_cands, cand_cap, n_b, c_star, a_dir, t_star,
                                 pcol, pany, status, mv, stats); break;
            case 8: EZO_KLAUNCH(c, (k_project_bisect<8, 1, false, true>), grid, block, lds, st, r->view, ovs, gv,
                                edges, S, stride, s_edge, cand_idx, n_cands, cand_cap, n_b, c_star, a_dir, t_star,
                                pcol, pany, status, mv, stats); break;
            case 4: EZO_KLAUNCH(c, (k_project_bisect<4, 1, false, true>), grid, block, lds, st, r->view, ovs, gv,
                                edges, S, stride, s_edge, cand_idx, n_cands, cand_cap, n_b, c_star, a_dir, t_star,
                                pcol, pany, status, mv, stats); break;
            default: EZO_KLAUNCH(c, (k_project_bisect<2, 1, false, true>), grid, block, lds, st, r->view, ovs, gv,
                                 edges, S, stride, s_edge, cand_idx, n_cands, cand_cap, n_b, c_star, a_dir, t_star,
                                 pcol, pany, status, mv, stats); break;
        }
        HIP_TRY(c, hipGetLastError());
        return EZO_OK;
    }
#define EZO_LAUNCH_PB(TT, DD)                                                                                       \
    do {                                                                                                            \
        if (box)                                                                                                    \
            EZO_KLAUNCH(c, (k_project_bisect<TT, DD, true>), grid, block, lds, st, r->view, ovs, gv, edges, S, stride, \
                        s_edge, cand_idx, n_cands, cand_cap, n_b, c_star, a_dir, t_star, pcol, pany, status, mv,     \
                        stats);                                                                                     \
        else                                                                                                        \
            EZO_KLAUNCH(c, (k_project_bisect<TT, DD, false>), grid, block, lds, st, r->view, ovs, gv, edges, S,       \
                        stride, s_edge, cand_idx, n_cands, cand_cap, n_b, c_star, a_dir, t_star, pcol, pany, status, \
                        mv, stats);                                                                                 \
    } while (0)
    if (dp == 1) {
        switch (TC) {
            case 64: EZO_LAUNCH_PB(64, 1); break;
            case 32: EZO_LAUNCH_PB(32, 1); break;
            case 16: EZO_LAUNCH_PB(16, 1); break;
            case 8: EZO_LAUNCH_PB(8, 1); break;
            case 4: EZO_LAUNCH_PB(4, 1); break;
            default: EZO_LAUNCH_PB(2, 1); break;
        }
    } else if (dp == 2) {
        switch (TC) {
            case 16: EZO_LAUNCH_PB(16, 2); break;
            case 8: EZO_LAUNCH_PB(8, 2); break;
            case 4: EZO_LAUNCH_PB(4, 2); break;
            case 2: EZO_LAUNCH_PB(2, 2); break;
            default: EZO_LAUNCH_PB(1, 2); break;
        }
    } else {
        switch (TC) {
            case 8: EZO_LAUNCH_PB(8, 3); break;
            case 4: EZO_LAUNCH_PB(4, 3); break;
            case 2: EZO_LAUNCH_PB(2, 3); break;
            default: EZO_LAUNCH_PB(1, 3); break;
        }
    }
#undef EZO_LAUNCH_PB
    HIP_TRY(c, hipGetLastError());
    return EZO_OK;
}

// ---------------------------------------------------------------------------
// Autotuning (first use of a key, when enabled)
// ---------------------------------------------------------------------------

// Raw checker: time the candidate shapes on a prefix of the call's own
// configurations (the kernel only writes outputs, so repeated launches are
// harmless).  The prefix keeps one timing launch to a few milliseconds
// while leaving far more workgroups than CUs.
template <bool SD>
ezo_status tune_check_inplace(ezo_ctx* c, const ezo_robot* r, const ObsView& ov, const GridView& gv, const float* q,
                              int64_t n, int64_t sn, int64_t sd, uint8_t* flags, float* min_sd, float* min_sd_self,
                              hipStream_t st) {
    const TuneKey k = tune_key(c, r, SD ? TUNE_CHECK_SD : TUNE_CHECK_FLAGS, ov.n, n);
    TileCfg g;
    if (!c->autotune || ezo_tune_lookup(k, &g)) return EZO_OK;
    const int64_t n_t = SD ? std::min<int64_t>(n, std::max<int64_t>(65536, (1LL << 28) / std::max(ov.n, 256)))
                           : std::min<int64_t>(n, 1LL << 19);
    const auto cands = SD ? tile_candidates(c, r->slots, r->P, r->view.n_blocks, ov.n, true, {1, 2, 4, 8, 16}, n_t)
                          : tile_candidates(c, r->slots, r->P, r->view.n_blocks, ov.n, false, {1, 2, 4, 8}, n_t);
    if (cands.empty()) return EZO_OK;
    IterArgs it{nullptr, 0, 0, 0, 0};
    auto run = [&](const TileCfg& cfg) {
        return launch_check<SD>(c, r, ov, gv, q, n_t, sn, sd, 0, flags, min_sd, min_sd_self, 0, 1, nullptr, it, st,
                                nullptr, 0.f, nullptr, &cfg);
    };
    return ezo_tune_search(c, k, cands, st, run, &g);
}

// Driven projection + bisection: the call's own candidates (outputs only).
ezo_status tune_bisect_inplace(ezo_ctx* c, const ezo_robot* r, const ObsView& ov, const GridView& gv,
                               const float* edges, int E, const float* S, int64_t stride, const int* cand_idx,
                               const int* n_cands, int cand_cap, int n_b, float* c_star, float* a_dir, float* t_star,
                               uint8_t* pcol, hipStream_t st) {
    const TuneKey k = tune_key(c, r, TUNE_BISECT, ov.n, (int64_t)cand_cap * E);
    TileCfg g;
    if (!c->autotune || ezo_tune_lookup(k, &g)) return EZO_OK;
    const auto cands = tile_candidates(c, r->slots, r->P, r->view.n_blocks, ov.n, false, {1, 2, 4, 8, 16}, (int64_t)cand_cap * E, true);
    if (cands.empty()) return EZO_OK;
    auto run = [&](const TileCfg& cfg) {
        return launch_project_bisect(c, r, ov, gv, edges, E, S, stride, cand_idx, n_cands, cand_cap, n_b, c_star,
                                     a_dir, t_star, pcol, nullptr, nullptr, st, &cfg);
    };
    return ezo_tune_search(c, k, cands, st, run, &g);
}

// Fused inflation: the loop's workspace (and the caller's A, b, n_faces) are
// free until the edges are initialised, so the shapes of the loop's check
// and bisection launches are timed there on a stand-in for the loop's
// iterations (the loop's sampler picks its lanes per walk on the device):
// the joint box written as 2 dof + 2 n_f rows (box rows repeated), |S|
// hit-and-run samples per edge from it, and as candidates the first n_p of
// them in collision.  The box collides widely, so these candidates stand for
// a first iteration only; the loop goes on until about an eps fraction of
// the samples collide, so a bisection shape is timed on the full candidate
// lists once plus three times on their first max(16, 2 eps n_p) entries per
// edge (the lighter iterations after the first).
constexpr int kItersPerGraph = 4;        // iterations captured per replayed graph
// Candidate sample counts N_p of the sample-count tuner, largest first (its
// order of preference: more samples give more hyperplanes per iteration), the
// margin by which a smaller count must be faster to be picked, and the count
// used when tuning is off and nothing is cached.
constexpr int kSampleCounts[] = {10000, 5000, 2000, 1000};
constexpr double kSampleCountSlack = 0.05;
constexpr int kDefaultSampleCount = 10000;
// The sample-count tuner's inflations draw from key seed ^ kTuneSeedMix.
constexpr uint64_t kTuneSeedMix = 0x9E3779B97F4A7C15ull;
// Edges per round of ezo_inflate_paths (a path window of s = kPathBatch / paths edges).
constexpr int kPathBatch = 128;

ezo_status tune_inflation(ezo_ctx* c, const ezo_robot* r, const ObsView& ov, const GridView& gv, const float* edges,
                          int E, const ezo_params* p, int S_cap, int64_t stride, float* A, float* b, int* n_faces,
                          float* w_s, uint8_t* w_f, int* w_ci, int* w_nc, float* w_cs, float* w_ad, float* w_ts,
                          uint8_t* w_pc, const int* w_active, hipStream_t st, bool* launched) {
    if (!c->autotune) return EZO_OK;
    const int dof = r->dof, cap = p->face_capacity, cand_cap = p->n_p;
    const TuneKey kc = tune_key(c, r, TUNE_CHECK_FLAGS, ov.n, (int64_t)S_cap * E);
    const TuneKey kb = tune_key(c, r, TUNE_BISECT, ov.n, (int64_t)cand_cap * E);
    TileCfg g;
    const bool need_c = !ezo_tune_lookup(kc, &g), need_b = !ezo_tune_lookup(kb, &g);
    if (!need_c && !need_b) return EZO_OK;
    *launched = true;                         // the runs below overwrite A, b, n_faces and the loop's state
    const int n_run = E;                      // the sampler's running-edge count during tuning
    HIP_TRY(c, hipMemcpyAsync((void*)w_active, &n_run, sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    const int F = std::min(cap, 2 * dof + 2 * p->n_f);
    hipLaunchKernelGGL(k_tune_polytope, dim3((E + 63) / 64), dim3(64), 0, st, dof, r->q_lo, r->q_hi, E, cap, F, A, b,
                       n_faces);
    HIP_TRY(c, hipGetLastError());
    IterArgs its{nullptr, 1, 0, 0, S_cap};
    ezo_status s;
    if ((s = launch_sample(c, dof, A, b, n_faces, cap, edges, E, S_cap, p->n_mix, p->seed, p->edge_id_base, w_s,
                           stride, nullptr, its, st, nullptr, w_active)))
        return s;
    IterArgs it{nullptr, 0, 0, 0, 0};
    auto run_c = [&](const TileCfg& cfg) {
        return launch_check<false>(c, r, ov, gv, w_s, S_cap, 1, stride, (int64_t)dof * stride, w_f, nullptr, nullptr,
                                   stride, E, nullptr, it, st, nullptr, 0.f, nullptr, &cfg);
    };
    if (need_c) {
        const auto cands = tile_candidates(c, r->slots, r->P, r->view.n_blocks, ov.n, false, {1, 2, 4, 8}, (int64_t)S_cap * E);
        if (!cands.empty() && (s = ezo_tune_search(c, kc, cands, st, run_c, &g))) return s;
    }
    if (!need_b) return EZO_OK;
    if ((s = run_c(heuristic_check(c, r, ov.n, (int64_t)S_cap * E, false)))) return s;
    IterArgs sel{nullptr, 0, S_cap, -1, S_cap};     // T = -1: never accept, always select
    hipLaunchKernelGGL(k_test_select, dim3(E), dim3(1024), 0, st, w_f, stride, p->n_p, p->n_b, w_ci, cand_cap, w_nc,
                       nullptr, nullptr, nullptr, nullptr, sel);
    HIP_TRY(c, hipGetLastError());
    const auto cands = tile_candidates(c, r->slots, r->P, r->view.n_blocks, ov.n, false, {1, 2, 4, 8, 16}, (int64_t)cand_cap * E, true);
    if (cands.empty()) return EZO_OK;
    const int light = std::max(16, (int)std::ceil(2.0 * p->eps * cand_cap));
    int* w_nc_light = reinterpret_cast<int*>(w_f);      // the flags are free once selected (E <= stride E / 4)
    hipLaunchKernelGGL(k_cap_counts, dim3((E + 255) / 256), dim3(256), 0, st, (const int*)w_nc, w_nc_light, E, light);
    HIP_TRY(c, hipGetLastError());
    auto run_b = [&](const TileCfg& cfg) {
        ezo_status e = launch_project_bisect(c, r, ov, gv, edges, E, w_s, stride, w_ci, w_nc, cand_cap, p->n_b, w_cs,
                                             w_ad, w_ts, w_pc, nullptr, nullptr, st, &cfg);
        for (int i = 0; i < 3 && e == EZO_OK; ++i)
            e = launch_project_bisect(c, r, ov, gv, edges, E, w_s, stride, w_ci, w_nc_light, cand_cap, p->n_b, w_cs,
                                      w_ad, w_ts, w_pc, nullptr, nullptr, st, &cfg);
        return e;
    };
    c->bisect_key = kb;
    return ezo_tune_search(c, kb, cands, st, run_b, &g, kTuneSlack, c->shape_trial ? nullptr : &c->bisect_finalists);
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

ezo_status ezo_ctx_create(int32_t device, ezo_ctx** out) {
    if (!out) return ezo_fail(nullptr, EZO_E_INVALID, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return ezo_fail(nullptr, EZO_E_HIP, "no HIP device");
    if (device < 0 || device >= n) return ezo_fail(nullptr, EZO_E_INVALID, "device %d out of range", device);
    if (hipSetDevice(device) != hipSuccess) return ezo_fail(nullptr, EZO_E_HIP, "hipSetDevice failed");
    ezo_ctx* c = new ezo_ctx();
    c->device = device;
    c->ws.resize(W_NSLOTS);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->arch = prop.gcnArchName;
        const size_t colon = c->arch.find(':');
        if (colon != std::string::npos) c->arch.resize(colon);
    }
    if (c->arch.empty()) c->arch = "unknown";
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->lds_cap = std::min<size_t>((size_t)lds, 65536);
    // this device's copy of the no-allocation entry point's scratch (device
    // current); nullptr makes that entry point report an error
    c->scratch = scratch_address();
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&c->pinned, sizeof(int) * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostGetDevicePointer((void**)&c->pinned_dev, c->pinned, 0) != hipSuccess) {
        ezo_ctx_destroy(c);
        return ezo_fail(nullptr, EZO_E_HIP, "stream/event/pinned allocation failed");
    }
    *out = c;
    return EZO_OK;
}

void ezo_ctx_destroy(ezo_ctx* c) {
    if (!c) return;
    hipError_t e;
    e = hipSetDevice(c->device);
    if (c->stream) e = hipStreamSynchronize(c->stream);
    for (auto& b : c->ws)
        if (b.p) e = hipFree(b.p);
    if (c->pinned) e = hipHostFree(c->pinned);
    if (c->pinned_stats) e = hipHostFree(c->pinned_stats);
    if (c->ev_in) e = hipEventDestroy(c->ev_in);
    if (c->ev_out) e = hipEventDestroy(c->ev_out);
    for (auto& ev : c->tev)
        if (ev) e = hipEventDestroy(ev);
    for (auto& ev : c->tune_ev)
        if (ev) e = hipEventDestroy(ev);
    if (c->loop_exec) e = hipGraphExecDestroy(c->loop_exec);
    if (c->d_tests) e = hipFree(c->d_tests);
    if (c->ebox) e = hipFree(c->ebox);
    if (c->stream) e = hipStreamDestroy(c->stream);
    (void)e;
    (void)hipGetLastError();
    delete c;
}

const char* ezo_last_error(const ezo_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

ezo_status ezo_set_obstacle_boxes(ezo_ctx* c, const float* boxes, int32_t n) {
    if (!c) return EZO_E_INVALID;
    if (n < 0 || (n > 0 && !boxes)) return ezo_fail(c, EZO_E_INVALID, "bad argument");
    if (n > EZO_MAX_OBSTACLE_BOXES)
        return ezo_fail(c, EZO_E_UNSUPPORTED, "%d obstacle boxes (at most %d)", n, EZO_MAX_OBSTACLE_BOXES);
    std::vector<float4> pk(4 * (size_t)std::max(n, 1));
    for (int e = 0; e < n; ++e) {
        const float* x = boxes + 15 * (size_t)e;
        for (int i = 0; i < 15; ++i)
            if (!std::isfinite(x[i])) return ezo_fail(c, EZO_E_INVALID, "obstacle box %d not finite", e);
        if (x[12] < 0.f || x[13] < 0.f || x[14] < 0.f)
            return ezo_fail(c, EZO_E_INVALID, "obstacle box %d has a negative half extent", e);
        const double rad = std::sqrt((double)x[12] * x[12] + (double)x[13] * x[13] + (double)x[14] * x[14]);
        pk[4 * e] = make_float4(x[0], x[1], x[2], x[12]);
        pk[4 * e + 1] = make_float4(x[3], x[4], x[5], x[13]);
        pk[4 * e + 2] = make_float4(x[6], x[7], x[8], x[14]);
        pk[4 * e + 3] = make_float4(x[9], x[10], x[11], (float)(rad * (1.0 + 1e-5) + 1e-5));
    }
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));        // no call in flight still reads the old boxes
    if (!c->ebox) {
        // allocated once at the maximum size, so the address never changes
        if (hipMalloc((void**)&c->ebox, sizeof(float4) * 4 * EZO_MAX_OBSTACLE_BOXES) != hipSuccess) {
            c->ebox = nullptr;
            return ezo_fail(c, EZO_E_NOMEM, "obstacle box allocation failed");
        }
    }
    if (n > 0) HIP_TRY(c, hipMemcpy(c->ebox, pk.data(), sizeof(float4) * 4 * (size_t)n, hipMemcpyHostToDevice));
    c->n_ebox = n;
    return EZO_OK;
}

ezo_status ezo_robot_create(ezo_ctx* c, const ezo_robot_desc* d, ezo_robot** out) {
    if (!c || !d || !out) return ezo_fail(c, EZO_E_INVALID, "NULL argument");
    *out = nullptr;
    if (d->dof < 1 || d->dof > EZO_MAX_DOF) return ezo_fail(c, EZO_E_UNSUPPORTED, "dof %d not in [1, %d]", d->dof, EZO_MAX_DOF);
    if (d->n_spheres < 0 || d->n_spheres > EZO_MAX_SPHERES)
        return ezo_fail(c, EZO_E_UNSUPPORTED, "n_spheres %d not in [0, %d]", d->n_spheres, EZO_MAX_SPHERES);
    if (d->n_self_pairs < 0) return ezo_fail(c, EZO_E_INVALID, "n_self_pairs < 0");
    if (!d->dh_a || !d->dh_alpha || !d->dh_d || !d->q_lo || !d->q_hi)
        return ezo_fail(c, EZO_E_INVALID, "NULL DH or limit array");
    if (d->n_spheres > 0 && (!d->sphere_link || !d->sphere_xyz || !d->sphere_r))
        return ezo_fail(c, EZO_E_INVALID, "NULL sphere array");
    if (d->n_self_pairs > 0 && !d->self_pairs) return ezo_fail(c, EZO_E_INVALID, "NULL self_pairs");
    const int dof = d->dof, S = d->n_spheres, P = d->n_self_pairs;
    for (int j = 0; j < dof; ++j)
        if (!(d->q_lo[j] <= d->q_hi[j])) return ezo_fail(c, EZO_E_INVALID, "q_lo[%d] > q_hi[%d]", j, j);
    for (int s = 0; s < S; ++s) {
        if (d->sphere_link[s] < 0 || d->sphere_link[s] >= dof)
            return ezo_fail(c, EZO_E_INVALID, "sphere %d has link %d", s, d->sphere_link[s]);
        if (!(d->sphere_r[s] >= 0.0)) return ezo_fail(c, EZO_E_INVALID, "sphere %d has a negative radius", s);
    }
    for (int p = 0; p < 2 * P; ++p)
        if (d->self_pairs[p] < 0 || d->self_pairs[p] >= S)
            return ezo_fail(c, EZO_E_INVALID, "self pair entry %d = %d out of range", p, d->self_pairs[p]);
    unsigned prismatic = 0;
    if (d->joint_type)
        for (int j = 0; j < dof; ++j) {
            if (d->joint_type[j] != 0 && d->joint_type[j] != 1)
                return ezo_fail(c, EZO_E_INVALID, "joint %d has type %d (0 revolute, 1 prismatic)", j, d->joint_type[j]);
            if (d->joint_type[j] == 1) prismatic |= 1u << j;
        }
    if (d->n_boxes < 0 || d->n_boxes > EZO_MAX_BOXES)
        return ezo_fail(c, EZO_E_UNSUPPORTED, "n_boxes %d not in [0, %d]", d->n_boxes, EZO_MAX_BOXES);
    if (d->n_box_pairs < 0) return ezo_fail(c, EZO_E_INVALID, "n_box_pairs < 0");
    if (d->n_boxes > 0 && (!d->box_link || !d->box_pose || !d->box_half))
        return ezo_fail(c, EZO_E_INVALID, "NULL box array");
    if (d->n_box_pairs > 0 && !d->box_pairs) return ezo_fail(c, EZO_E_INVALID, "NULL box_pairs");
    for (int k = 0; k < d->n_boxes; ++k) {
        if (d->box_link[k] < 0 || d->box_link[k] >= dof)
            return ezo_fail(c, EZO_E_INVALID, "box %d has link %d", k, d->box_link[k]);
        for (int i = 0; i < 12; ++i)
            if (!std::isfinite(d->box_pose[12 * k + i])) return ezo_fail(c, EZO_E_INVALID, "box %d pose not finite", k);
        for (int i = 0; i < 3; ++i)
            if (!(d->box_half[3 * k + i] >= 0.0) || !std::isfinite(d->box_half[3 * k + i]))
                return ezo_fail(c, EZO_E_INVALID, "box %d has a bad half extent", k);
    }
    for (int p = 0; p < 2 * d->n_box_pairs; ++p)
        if (d->box_pairs[p] < 0 || d->box_pairs[p] >= d->n_boxes)
            return ezo_fail(c, EZO_E_INVALID, "box pair entry %d = %d out of range", p, d->box_pairs[p]);
    // sort spheres by link (stable), remember the original order
    std::vector<int> order(S);
    for (int s = 0; s < S; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d->sphere_link[a] < d->sphere_link[b]; });
    std::vector<int> orig_to_sorted(S);
    for (int s = 0; s < S; ++s) orig_to_sorted[order[s]] = s;
    std::vector<float4> dh(dof), sph(std::max(S, 1));
    std::vector<int> link_begin(dof + 1, 0), s2o(std::max(S, 1));
    std::vector<int2> pairs(std::max(P, 1));
    std::vector<float> lim(2 * dof);
    for (int j = 0; j < dof; ++j) {
        dh[j] = make_float4((float)d->dh_a[j], (float)d->dh_d[j], (float)std::cos((double)(float)d->dh_alpha[j]),
                            (float)std::sin((double)(float)d->dh_alpha[j]));
        lim[j] = (float)d->q_lo[j];
        lim[dof + j] = (float)d->q_hi[j];
    }
    for (int s = 0; s < S; ++s) {
        const int o = order[s];
        sph[s] = make_float4((float)d->sphere_xyz[3 * o], (float)d->sphere_xyz[3 * o + 1], (float)d->sphere_xyz[3 * o + 2],
                             (float)d->sphere_r[o]);
        s2o[s] = o;
        link_begin[d->sphere_link[o] + 1]++;
    }
    for (int j = 0; j < dof; ++j) link_begin[j + 1] += link_begin[j];
    // parts: kPartsPerLink consecutive runs of each link's (sorted) spheres,
    // part p of link l = kPartsPerLink l + p covering local indices
    // [p n / K, (p + 1) n / K); self pairs grouped into blocks by (lower
    // part, higher part)
    constexpr int K = kPartsPerLink;
    auto part_of = [&](int sorted) {
        int l = 0;
        while (sorted >= link_begin[l + 1]) ++l;
        const int n = link_begin[l + 1] - link_begin[l], i = sorted - link_begin[l];
        int p = 0;
        while (p + 1 < K && i >= (p + 1) * n / K) ++p;
        return K * l + p;
    };
    std::vector<std::pair<std::pair<int, int>, int2>> keyed(P);
    for (int p = 0; p < P; ++p) {
        const int a = orig_to_sorted[d->self_pairs[2 * p]], bb = orig_to_sorted[d->self_pairs[2 * p + 1]];
        const int pa = part_of(a), pb = part_of(bb);
        keyed[p] = {{std::min(pa, pb), std::max(pa, pb)}, make_int2(a, bb)};
    }
    std::stable_sort(keyed.begin(), keyed.end(),
                     [](const auto& x, const auto& y) { return x.first < y.first; });
    std::vector<int4> blocks;
    for (int p = 0; p < P; ++p) {
        pairs[p] = keyed[p].second;
        if (p == 0 || keyed[p].first != keyed[p - 1].first)
            blocks.push_back(make_int4(keyed[p].first.first, keyed[p].first.second, p, 0));
        blocks.back().w++;
    }
    if (blocks.empty()) blocks.push_back(make_int4(0, 0, 0, 0));
    const int NB = P > 0 ? (int)blocks.size() : 0;
    // bounding sphere of each part's spheres (link frame): centre of the
    // centres' box, radius = max distance + sphere radius
    std::vector<float4> lbound((size_t)K * dof, make_float4(0.f, 0.f, 0.f, 0.f));
    float r_max = 0.f;
    for (int j = 0; j < K * dof; ++j) {
        const int l = j / K, p = j % K, n = link_begin[l + 1] - link_begin[l];
        const int s0 = link_begin[l] + p * n / K, s1 = link_begin[l] + (p + 1) * n / K;
        if (s1 <= s0) continue;
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int s2 = s0; s2 < s1; ++s2) {
            const double v[3] = {sph[s2].x, sph[s2].y, sph[s2].z};
            for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], v[k]); hi[k] = std::max(hi[k], v[k]); }
        }
        const double cc[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
        double R = 0.0;
        for (int s2 = s0; s2 < s1; ++s2) {
            const double dx = sph[s2].x - cc[0], dy = sph[s2].y - cc[1], dz = sph[s2].z - cc[2];
            R = std::max(R, std::sqrt(dx * dx + dy * dy + dz * dz) + (double)sph[s2].w);
        }
        // small relative + absolute pad covers FP32 rounding of the transformed centres
        lbound[j] = make_float4((float)cc[0], (float)cc[1], (float)cc[2], (float)(R * (1.0 + 1e-5) + 1e-5));
    }
    for (int s2 = 0; s2 < S; ++s2) r_max = std::max(r_max, sph[s2].w);
    // boxes sorted by link (stable); four float4 each: (centre, h_x), (rotation
    // row 0, h_y), (row 1, h_z), (row 2, bounding radius |h| padded for FP32)
    const int B = d->n_boxes, Q = d->n_box_pairs;
    std::vector<int> border(B);
    for (int k = 0; k < B; ++k) border[k] = k;
    std::stable_sort(border.begin(), border.end(), [&](int x, int y) { return d->box_link[x] < d->box_link[y]; });
    std::vector<int> box_o2s(std::max(B, 1));
    std::vector<float4> boxv(4 * (size_t)std::max(B, 1), make_float4(0.f, 0.f, 0.f, 0.f));
    std::vector<int> box_begin(dof + 1, 0);
    std::vector<int2> bpairs(std::max(Q, 1), make_int2(0, 0));
    for (int k = 0; k < B; ++k) {
        const int o = border[k];
        box_o2s[o] = k;
        const double* ps = d->box_pose + 12 * (size_t)o;
        const double* h = d->box_half + 3 * (size_t)o;
        const double rad = std::sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
        boxv[4 * k] = make_float4((float)ps[0], (float)ps[1], (float)ps[2], (float)h[0]);
        boxv[4 * k + 1] = make_float4((float)ps[3], (float)ps[4], (float)ps[5], (float)h[1]);
        boxv[4 * k + 2] = make_float4((float)ps[6], (float)ps[7], (float)ps[8], (float)h[2]);
        boxv[4 * k + 3] = make_float4((float)ps[9], (float)ps[10], (float)ps[11], (float)(rad * (1.0 + 1e-5) + 1e-5));
        box_begin[d->box_link[o] + 1]++;
    }
    for (int j = 0; j < dof; ++j) box_begin[j + 1] += box_begin[j];
    for (int p = 0; p < Q; ++p) bpairs[p] = make_int2(box_o2s[d->box_pairs[2 * p]], box_o2s[d->box_pairs[2 * p + 1]]);
    // one allocation: [dh][sph][pairs][lbound][blocks][link_begin][s2o][limits][boxes][box_begin][box pairs]
    size_t off_dh = 0;
    size_t off_sph = off_dh + sizeof(float4) * dof;
    size_t off_pairs = off_sph + sizeof(float4) * sph.size();
    size_t off_lbd = off_pairs + sizeof(int2) * pairs.size();
    size_t off_blk = off_lbd + sizeof(float4) * lbound.size();
    size_t off_lb = off_blk + sizeof(int4) * blocks.size();
    size_t off_s2o = off_lb + sizeof(int) * link_begin.size();
    size_t off_lim = off_s2o + sizeof(int) * s2o.size();
    size_t off_box = (off_lim + sizeof(float) * lim.size() + 15) & ~(size_t)15;
    size_t off_bb = off_box + sizeof(float4) * boxv.size();
    size_t off_bp = off_bb + sizeof(int) * box_begin.size();
    size_t total = off_bp + sizeof(int2) * bpairs.size();
    std::vector<char> host(total);
    memcpy(host.data() + off_dh, dh.data(), sizeof(float4) * dof);
    memcpy(host.data() + off_sph, sph.data(), sizeof(float4) * sph.size());
    memcpy(host.data() + off_pairs, pairs.data(), sizeof(int2) * pairs.size());
    memcpy(host.data() + off_lbd, lbound.data(), sizeof(float4) * lbound.size());
    memcpy(host.data() + off_blk, blocks.data(), sizeof(int4) * blocks.size());
    memcpy(host.data() + off_lb, link_begin.data(), sizeof(int) * link_begin.size());
    memcpy(host.data() + off_s2o, s2o.data(), sizeof(int) * s2o.size());
    memcpy(host.data() + off_lim, lim.data(), sizeof(float) * lim.size());
    memcpy(host.data() + off_box, boxv.data(), sizeof(float4) * boxv.size());
    memcpy(host.data() + off_bb, box_begin.data(), sizeof(int) * box_begin.size());
    memcpy(host.data() + off_bp, bpairs.data(), sizeof(int2) * bpairs.size());
    HIP_TRY(c, hipSetDevice(c->device));
    void* buf = nullptr;
    if (hipMalloc(&buf, total) != hipSuccess) return ezo_fail(c, EZO_E_NOMEM, "robot allocation failed");
    if (hipMemcpy(buf, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
        hipError_t e = hipFree(buf);
        (void)e;
        return ezo_fail(c, EZO_E_HIP, "robot upload failed");
    }
    ezo_robot* r = new ezo_robot();
    r->ctx = c;
    r->device = c->device;
    r->dof = dof;
    r->S = S;
    r->P = P;
    r->B = B;
    r->Q = Q;
    r->slots = tile_slots(S, B);
    r->buf = buf;
    char* b = reinterpret_cast<char*>(buf);
    r->r_max = r_max;
    r->view.dof = dof;
    r->view.prismatic = prismatic;
    r->view.n_spheres = S;
    r->view.n_self = P;
    r->view.n_blocks = NB;
    r->view.lbound = reinterpret_cast<const float4*>(b + off_lbd);
    r->view.blocks = reinterpret_cast<const int4*>(b + off_blk);
    r->view.dh = reinterpret_cast<const float4*>(b + off_dh);
    r->view.sph = reinterpret_cast<const float4*>(b + off_sph);
    r->view.pairs = reinterpret_cast<const int2*>(b + off_pairs);
    r->view.link_begin = reinterpret_cast<const int*>(b + off_lb);
    r->view.n_boxes = B;
    r->view.n_box_pairs = Q;
    r->view.box = reinterpret_cast<const float4*>(b + off_box);
    r->view.box_begin = reinterpret_cast<const int*>(b + off_bb);
    r->view.box_pairs = reinterpret_cast<const int2*>(b + off_bp);
    r->sorted_to_orig = reinterpret_cast<const int*>(b + off_s2o);
    r->q_lo = reinterpret_cast<const float*>(b + off_lim);
    r->q_hi = r->q_lo + dof;
    *out = r;
    return EZO_OK;
}

void ezo_robot_destroy(ezo_robot* r) {
    if (!r) return;
    hipError_t e = hipSetDevice(r->device);
    if (r->buf) e = hipFree(r->buf);
    (void)e;
    (void)hipGetLastError();                 // leave no error behind for the caller's next check
    delete r;
}

ezo_status ezo_test_constants(double eps, double delta, double tau, int32_t k, int64_t* M, int64_t* T) {
    if (!M || !T || !(eps > 0 && eps < 1) || !(delta > 0 && delta < 1) || !(tau > 0 && tau < 1) || k < 1)
        return EZO_E_INVALID;
    const double pi = 3.14159265358979323846;
    const double dk = 6.0 * delta / (pi * pi * (double)k * (double)k);
    const double m = std::ceil(2.0 * std::log(1.0 / dk) / (eps * tau * tau));
    *M = (int64_t)m;
    *T = (int64_t)std::floor(m * (1.0 - tau) * eps + 1e-9);
    return EZO_OK;
}

ezo_status ezo_check_collisions(ezo_ctx* c, const ezo_robot* r, const float* obs, int32_t n_obs, const float* q,
                                int64_t n, int64_t stride_n, int64_t stride_d, uint8_t* flags, float* min_sd,
                                float* min_sd_self, void* stream) {
    if (!c) return EZO_E_INVALID;
    if (!r) return ezo_fail(c, EZO_E_INVALID, "robot is NULL");
    if (n < 0 || n_obs < 0) return ezo_fail(c, EZO_E_INVALID, "negative size");
    if (n == 0) return EZO_OK;
    if (!q || !flags || (n_obs > 0 && !obs)) return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = as_stream(stream);
    ObsView ov;
    GridView gv;
    ezo_status s = prep_obstacles(c, r, obs, n_obs, st, &ov, &gv);
    if (s) return s;
    IterArgs it{nullptr, 0, 0, 0, 0};
    if (min_sd || min_sd_self) {
        if ((s = tune_check_inplace<true>(c, r, ov, gv, q, n, stride_n, stride_d, flags, min_sd, min_sd_self, st)))
            return s;
        return launch_check<true>(c, r, ov, gv, q, n, stride_n, stride_d, 0, flags, min_sd, min_sd_self, 0, 1,
                                  nullptr, it, st);
    }
    if ((s = tune_check_inplace<false>(c, r, ov, gv, q, n, stride_n, stride_d, flags, nullptr, nullptr, st))) return s;
    return launch_check<false>(c, r, ov, gv, q, n, stride_n, stride_d, 0, flags, nullptr, nullptr, 0, 1, nullptr, it,
                               st);
}

ezo_status ezo_check_collisions_noalloc(ezo_ctx* c, const ezo_robot* r, const float* obs, int32_t n_obs,
                                        const float* q, int64_t n, int64_t stride_n, int64_t stride_d, uint8_t* flags,
                                        float* min_sd, float* min_sd_self, void* stream) {
    if (!c) return EZO_E_INVALID;
    if (!r) return ezo_fail(c, EZO_E_INVALID, "robot is NULL");
    if (n < 0 || n_obs < 0) return ezo_fail(c, EZO_E_INVALID, "negative size");
    if (n_obs > EZO_NOALLOC_MAX_OBSTACLES)
        return ezo_fail(c, EZO_E_CAPACITY, "%d obstacles exceed the fixed scratch of %d", n_obs,
                        EZO_NOALLOC_MAX_OBSTACLES);
    if (n == 0) return EZO_OK;
    if (!q || !flags || (n_obs > 0 && !obs)) return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    if (!c->scratch) return ezo_fail(c, EZO_E_HIP, "the fixed scratch's device address is not available");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = as_stream(stream);
    ObsView ov;
    GridView gv;
    unsigned char* p = c->scratch;
    ezo_status s = prep_obstacles_into(c, r, obs, n_obs, st, p + kScrRec, p + kScrCentre, p + kScrGeom,
                                       p + kScrCount, p + kScrList, &ov, &gv);
    if (s) return s;
    // launch shapes: the tuning cache or the size heuristic (never a timing
    // search, which would write the outputs repeatedly)
    IterArgs it{nullptr, 0, 0, 0, 0};
    if (min_sd || min_sd_self)
        return launch_check<true>(c, r, ov, gv, q, n, stride_n, stride_d, 0, flags, min_sd, min_sd_self, 0, 1,
                                  nullptr, it, st);
    return launch_check<false>(c, r, ov, gv, q, n, stride_n, stride_d, 0, flags, nullptr, nullptr, 0, 1, nullptr, it,
                               st);
}

ezo_status ezo_sphere_centres(ezo_ctx* c, const ezo_robot* r, const float* q, int64_t n, int64_t stride_n,
                              int64_t stride_d, float* centres, void* stream) {
    if (!c) return EZO_E_INVALID;
    if (!r || n < 0) return ezo_fail(c, EZO_E_INVALID, "bad argument");
    if (n == 0 || r->S == 0) return EZO_OK;
    if (!q || !centres) return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = as_stream(stream);
    ObsView ov;
    GridView gv;
    ezo_status s = prep_obstacles(c, r, nullptr, 0, st, &ov, &gv);   // zero shift
    if (s) return s;
    int T = 16;
    while (T > 1 && tile_smem_bytes(T, r->slots, 4) > c->lds_cap) T >>= 1;
    const size_t lds = tile_smem_bytes(T, r->slots, 4);
    dim3 grid((unsigned)((n + T - 1) / T)), block(256);
    switch (T) {
        case 16: hipLaunchKernelGGL(k_centres<16>, grid, block, lds, st, r->view, ov, r->sorted_to_orig, q, n, stride_n, stride_d, centres); break;
        case 8: hipLaunchKernelGGL(k_centres<8>, grid, block, lds, st, r->view, ov, r->sorted_to_orig, q, n, stride_n, stride_d, centres); break;
        case 4: hipLaunchKernelGGL(k_centres<4>, grid, block, lds, st, r->view, ov, r->sorted_to_orig, q, n, stride_n, stride_d, centres); break;
        case 2: hipLaunchKernelGGL(k_centres<2>, grid, block, lds, st, r->view, ov, r->sorted_to_orig, q, n, stride_n, stride_d, centres); break;
        default: hipLaunchKernelGGL(k_centres<1>, grid, block, lds, st, r->view, ov, r->sorted_to_orig, q, n, stride_n, stride_d, centres); break;
    }
    HIP_TRY(c, hipGetLastError());
    return EZO_OK;
}

ezo_status ezo_sample_polytopes(ezo_ctx* c, int32_t dof, const float* A, const float* b, const int32_t* n_faces,
                                int32_t face_capacity, const float* edges, int32_t n_edges, int32_t n_samples,
                                int32_t n_mix, uint64_t seed, int64_t edge_id_base, int32_t iteration,
                                float* samples, int64_t sample_stride, void* stream) {
    if (!c) return EZO_E_INVALID;
    if (dof < 1 || dof > EZO_MAX_DOF || n_edges < 0 || n_samples < 0 || n_mix < 0 || iteration < 0 ||
        face_capacity < 1 || sample_stride < n_samples)
        return ezo_fail(c, EZO_E_INVALID, "bad sizes");
    if (n_edges == 0 || n_samples == 0) return EZO_OK;
    if (!A || !b || !n_faces || !edges || !samples) return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    HIP_TRY(c, hipSetDevice(c->device));
    IterArgs it{nullptr, iteration, 0, 0, n_samples};
    hipStream_t st = as_stream(stream);
    const TuneKey k = sample_key(c, dof, (int64_t)n_samples * n_edges);
    TileCfg g;
    if (c->autotune && !ezo_tune_lookup(k, &g)) {       // time the lane counts on this call (writes samples only)
        const std::vector<TileCfg> cands = {{1, 4, 0}, {2, 4, 0}, {4, 4, 0}, {8, 4, 0}, {16, 4, 0}};
        auto run = [&](const TileCfg& cfg) {
            return launch_sample(c, dof, A, b, n_faces, face_capacity, edges, n_edges, n_samples, n_mix, seed,
                                 edge_id_base, samples, sample_stride, nullptr, it, st, &cfg);
        };
        ezo_status s = ezo_tune_search(c, k, cands, st, run, &g);
        if (s) return s;
    }
    return launch_sample(c, dof, A, b, n_faces, face_capacity, edges, n_edges, n_samples, n_mix, seed, edge_id_base,
                         samples, sample_stride, nullptr, it, st);
}

ezo_status ezo_test_and_select(ezo_ctx* c, const uint8_t* flags, int32_t n_edges, int64_t sample_stride,
                               int32_t n_samples, int64_t M, int64_t T, int32_t n_p, int32_t* cand_idx,
                               int32_t* n_cands, int32_t cand_capacity, uint8_t* accept, int32_t* test_count,
                               void* stream) {
    if (!c) return EZO_E_INVALID;
    if (n_edges < 0 || n_samples < 0 || M < 0 || M > n_samples || n_p < 1 || n_p > cand_capacity ||
        sample_stride < n_samples || M > 0x7fffffff)
        return ezo_fail(c, EZO_E_INVALID, "bad sizes");
    if (n_edges == 0) return EZO_OK;
    if (!flags || !cand_idx || !n_cands) return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    HIP_TRY(c, hipSetDevice(c->device));
    IterArgs it{nullptr, 0, (int)M, (int)std::min<int64_t>(T, 0x7fffffff), n_samples};
    hipLaunchKernelGGL(k_test_select, dim3(n_edges), dim3(1024), 0, as_stream(stream), flags, sample_stride, n_p, 0,
                       cand_idx, cand_capacity, n_cands, accept, test_count, nullptr, nullptr, it);
    HIP_TRY(c, hipGetLastError());
    return EZO_OK;
}

ezo_status ezo_project_bisect(ezo_ctx* c, const ezo_robot* r, const float* obs, int32_t n_obs, const float* edges,
                              int32_t n_edges, const float* samples, int64_t sample_stride, const int32_t* cand_idx,
                              const int32_t* n_cands, int32_t cand_capacity, int32_t n_b, float* c_star,
                              float* a_dir, float* t_star, uint8_t* proj_collides, void* stream) {
    if (!c) return EZO_E_INVALID;
    if (!r || n_edges < 0 || n_obs < 0 || cand_capacity < 0 || n_b < 0) return ezo_fail(c, EZO_E_INVALID, "bad argument");
    if (n_edges == 0 || cand_capacity == 0) return EZO_OK;
    if (!edges || !samples || !cand_idx || !n_cands || !c_star || !a_dir || !t_star || !proj_collides ||
        (n_obs > 0 && !obs))
        return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = as_stream(stream);
    ObsView ov;
    GridView gv;
    ezo_status s = prep_obstacles(c, r, obs, n_obs, st, &ov, &gv);
    if (s) return s;
    if ((s = tune_bisect_inplace(c, r, ov, gv, edges, n_edges, samples, sample_stride, cand_idx, n_cands,
                                 cand_capacity, n_b, c_star, a_dir, t_star, proj_collides, st)))
        return s;
    return launch_project_bisect(c, r, ov, gv, edges, n_edges, samples, sample_stride, cand_idx, n_cands, cand_capacity,
                                 n_b, c_star, a_dir, t_star, proj_collides, nullptr, nullptr, st);
}

ezo_status ezo_place_hyperplanes(ezo_ctx* c, int32_t dof, const float* edges, int32_t n_edges, const float* c_star,
                                 const float* a_dir, const float* t_star, const int32_t* n_cands,
                                 int32_t cand_capacity, int32_t n_f, double step_back_max, double t_col, float* A,
                                 float* b, int32_t* n_faces, int32_t face_capacity, int32_t* edge_status,
                                 int32_t* placed_idx, int32_t* n_placed, void* stream) {
    if (!c) return EZO_E_INVALID;
    if (dof < 1 || dof > EZO_MAX_DOF || n_edges < 0 || cand_capacity < 0 || n_f < 0 || face_capacity < 1 ||
        !finite_pos(step_back_max) || !std::isfinite(t_col))
        return ezo_fail(c, EZO_E_INVALID, "bad argument");
    if (n_edges == 0) return EZO_OK;
    if (!edges || !c_star || !a_dir || !t_star || !n_cands || !A || !b || !n_faces || !edge_status)
        return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    if ((size_t)cand_capacity > c->lds_cap - kPlaceStaticLds) return ezo_fail(c, EZO_E_UNSUPPORTED, "cand_capacity too large");
    HIP_TRY(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_place, dim3(n_edges), dim3(1024), (size_t)std::max(cand_capacity, 16), as_stream(stream), dof,
                       edges, c_star, a_dir, t_star, n_cands, cand_capacity, n_f, (float)step_back_max, (float)t_col, A,
                       b, n_faces, face_capacity, edge_status, placed_idx, n_placed, nullptr, nullptr, nullptr,
                       IterEnd{});
    HIP_TRY(c, hipGetLastError());
    return EZO_OK;
}

}  // extern "C"

// The fused inflation of E edges.  edge_ids (device, optional): edge e draws
// the random stream of edge id edge_id_base + edge_ids[e] instead of
// edge_id_base + e.  skip (device, optional): edges with skip[e] != 0 are not
// inflated (status CONTAINED, no rows).
static ezo_status inflate_core(ezo_ctx* c, const ezo_robot* r, const float* obs, int32_t n_obs, const float* edges,
                               int32_t n_edges, const ezo_params* p, float* A, float* b, int32_t* n_faces,
                               int32_t* edge_status, ezo_edge_stats* stats, void* stream, const int* edge_ids,
                               const uint8_t* skip) {
    if (!c) return EZO_E_INVALID;
    if (!r || !p) return ezo_fail(c, EZO_E_INVALID, "NULL robot or params");
    if (n_edges < 0 || n_obs < 0) return ezo_fail(c, EZO_E_INVALID, "negative size");
    if (!(p->eps > 0 && p->eps < 1) || !(p->delta > 0 && p->delta < 1) || !(p->tau > 0 && p->tau < 1) ||
        !finite_pos(p->step_back_max) || !std::isfinite(p->t_col) || p->n_p < 0 || p->n_f < 1 || p->n_b < 0 ||
        p->n_mix < 0 || p->max_iters < 1)
        return ezo_fail(c, EZO_E_INVALID, "parameter out of range");
    const int dof = r->dof;
    if ((int64_t)p->face_capacity < 2LL * dof + (int64_t)p->n_f * p->max_iters)
        return ezo_fail(c, EZO_E_CAPACITY, "face_capacity %d < 2 dof + n_f max_iters = %lld", p->face_capacity,
                    (long long)(2LL * dof + (int64_t)p->n_f * p->max_iters));
    if (n_edges == 0) return EZO_OK;
    if (!edges || !A || !b || !n_faces || !edge_status || (n_obs > 0 && !obs))
        return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    if (p->n_p == 0) {
        // N_p chosen by measurement: whole inflations of this call's edges
        // with each candidate count, drawn from an independent random stream
        // (key seed ^ kTuneSeedMix) and thrown away (they use the call's
        // outputs as scratch; the inflation below overwrites them).  Kept per
        // key is the largest count within kSampleCountSlack of the fastest.
        // The choice thus never depends on the draws of the returned sets: a
        // run whose test happened to accept early finishes sooner, and picking
        // by time on the returned stream would favour it.  Certification does
        // not depend on N_p: the test always uses the first M_k samples.
        const TuneKey k = tune_key(c, r, TUNE_SAMPLE_COUNT, n_obs, n_edges);
        TileCfg g;
        if (!ezo_tune_lookup(k, &g)) {
            if (!c->autotune) {
                g.T = kDefaultSampleCount;
            } else {
                HIP_TRY(c, hipEventRecord(c->ev_in, as_stream(stream)));
                HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_in, 0));
                std::vector<TileCfg> cands;
                for (int np : kSampleCounts) {
                    TileCfg t;
                    t.T = np;
                    t.W = 1;
                    cands.push_back(t);
                }
                const uint64_t tune_seed = p->seed ^ kTuneSeedMix;
                struct Search {
                    ezo_ctx* c;
                    ~Search() { c->np_search = false; }
                } search{c};
                c->np_search = true;
                auto run = [&](const TileCfg& t) -> ezo_status {
                    ezo_params q = *p;
                    q.n_p = t.T;
                    q.seed = tune_seed;
                    q.row_points = nullptr;
                    return inflate_core(c, r, obs, n_obs, edges, n_edges, &q, A, b, n_faces, edge_status, nullptr,
                                        c->stream, edge_ids, skip);
                };
                ezo_status ts = ezo_tune_search(c, k, cands, c->stream, run, &g, kSampleCountSlack);
                if (ts) return ts;
                ezo_tune_note_seed(k, tune_seed);
            }
        }
        ezo_params q = *p;
        q.n_p = g.T;
        return inflate_core(c, r, obs, n_obs, edges, n_edges, &q, A, b, n_faces, edge_status, stats, stream, edge_ids,
                            skip);
    }
    const int cap = p->face_capacity;
    if (sample_smem_bytes(dof <= 4 ? 4 : 8, 16, cap, 256) > c->lds_cap)
        return ezo_fail(c, EZO_E_UNSUPPORTED, "face_capacity %d too large", cap);
    if ((size_t)p->n_p > c->lds_cap - kPlaceStaticLds) return ezo_fail(c, EZO_E_UNSUPPORTED, "n_p %d too large", p->n_p);
    // per-iteration constants, FP64 on the host
    std::vector<int4> table(p->max_iters + 2, make_int4(0, 0, 0, 0));
    int S_cap = 0;
    for (int k = 1; k <= p->max_iters; ++k) {
        int64_t M, T;
        ezo_test_constants(p->eps, p->delta, p->tau, k, &M, &T);
        if (M > (1 << 28)) return ezo_fail(c, EZO_E_UNSUPPORTED, "M_%d = %lld samples is too many", k, (long long)M);
        const int nS = (int)std::max<int64_t>(p->n_p, M);
        table[k] = make_int4((int)M, (int)std::min<int64_t>(T, 1 << 30), nS, k);
        S_cap = std::max(S_cap, nS);
    }
    table[p->max_iters + 1] = table[p->max_iters];
    table[p->max_iters + 1].w = p->max_iters + 1;
    HIP_TRY(c, hipSetDevice(c->device));
    const int E = n_edges;
    const int64_t stride = ((int64_t)S_cap + 63) / 64 * 64;
    const int cand_cap = p->n_p;
    void *w_s, *w_f, *w_ci, *w_nc, *w_cs, *w_ad, *w_ts, *w_pc, *w_pa, *w_st, *w_tb, *w_k, *w_ac, *w_pred = nullptr;
    ezo_status s;
    if ((s = ezo_ws_get(c, W_SAMPLES, sizeof(float) * (size_t)E * dof * stride, &w_s)) ||
        (s = ezo_ws_get(c, W_FLAGS, (size_t)E * stride, &w_f)) ||
        (s = ezo_ws_get(c, W_CAND, sizeof(int) * (size_t)E * cand_cap, &w_ci)) ||
        (s = ezo_ws_get(c, W_NCAND, sizeof(int) * (size_t)E, &w_nc)) ||
        (s = ezo_ws_get(c, W_CSTAR, sizeof(float) * (size_t)E * dof * cand_cap, &w_cs)) ||
        (s = ezo_ws_get(c, W_ADIR, sizeof(float) * (size_t)E * dof * cand_cap, &w_ad)) ||
        (s = ezo_ws_get(c, W_TSTAR, sizeof(float) * (size_t)E * cand_cap, &w_ts)) ||
        (s = ezo_ws_get(c, W_PCOL, (size_t)E * cand_cap, &w_pc)) || (s = ezo_ws_get(c, W_PANY, (size_t)E, &w_pa)) ||
        (s = ezo_ws_get(c, W_STATS, sizeof(EdgeStatsDev) * (size_t)E, &w_st)) ||
        (s = ezo_ws_get(c, W_TABLE, sizeof(int4) * table.size(), &w_tb)) || (s = ezo_ws_get(c, W_KDEV, sizeof(int4), &w_k)) ||
        (s = ezo_ws_get(c, W_ACTIVE, sizeof(int), &w_ac)))
        return s;
    if (p->surrogate) {
        if (p->surrogate->D != dof) return ezo_fail(c, EZO_E_INVALID, "screen dof %d != robot dof %d", p->surrogate->D, dof);
        if ((s = ezo_ws_get(c, W_PRED, sizeof(float) * (size_t)E * stride, &w_pred))) return s;
        // the screen's activation buffers must exist before the graph capture
        if ((s = ezo_surrogate_reserve(c, p->surrogate, (int64_t)E * stride))) return s;
    }
    hipStream_t st = c->stream;
    HIP_TRY(c, hipEventRecord(c->ev_in, as_stream(stream)));
    HIP_TRY(c, hipStreamWaitEvent(st, c->ev_in, 0));
    // the per-iteration table is copied only when it differs from the one the
    // slot already holds
    if (c->table_dev != w_tb || c->table_host.size() != table.size() ||
        std::memcmp(c->table_host.data(), table.data(), sizeof(int4) * table.size()) != 0) {
        HIP_TRY(c, hipMemcpyAsync(w_tb, table.data(), sizeof(int4) * table.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(c, hipStreamSynchronize(st));       // the host vector is reused below
        c->table_host = table;
        c->table_dev = w_tb;
    }
    ObsView ov;
    GridView gv;
    // the edges' start (P = D, statuses, statistics, the loop's row and
    // count) is launched with the obstacle preparation; a tuning run in
    // between overwrites it, and then it is launched again below
    const EdgeInit ei{dof, r->q_lo, r->q_hi, edges, E, A, b, n_faces, cap, edge_status, (EdgeStatsDev*)w_st,
                      (uint8_t*)w_pa, (int4*)w_k, (const int4*)w_tb, (int*)w_ac, skip};
    if ((s = prep_obstacles(c, r, obs, n_obs, st, &ov, &gv, &ei))) return s;
    bool tuned = false;
    if ((s = tune_inflation(c, r, ov, gv, edges, E, p, S_cap, stride, A, b, n_faces, (float*)w_s, (uint8_t*)w_f,
                            (int*)w_ci, (int*)w_nc, (float*)w_cs, (float*)w_ad, (float*)w_ts, (uint8_t*)w_pc,
                            (const int*)w_ac, st, &tuned)))
        return s;
    if (c->bisect_finalists.size() > 1 && !c->shape_trial) {
        tuned = true;
        // The stand-in's bisection finalists, timed on whole inflations of
        // this call's edges: the loop's later iterations have fewer
        // candidates than any stand-in, which favours larger tiles.  The runs
        // draw from an independent random stream (seed ^ kTuneSeedMix) and
        // use this call's outputs and workspace as scratch (same sizes, so the
        // same buffers; the obstacles are prepared again identically); the
        // inflation below overwrites them.  The timing, like every shape
        // choice, changes no result.
        std::vector<TileCfg> fin;
        fin.swap(c->bisect_finalists);
        const TuneKey kb = c->bisect_key;
        struct Trial {
            ezo_ctx* c;
            ~Trial() { c->shape_trial = false; }
        } trial{c};
        c->shape_trial = true;
        auto run = [&](const TileCfg& g) -> ezo_status {
            ezo_tune_store(kb, g);
            ezo_params q = *p;
            q.seed = p->seed ^ kTuneSeedMix;
            q.row_points = nullptr;
            return inflate_core(c, r, obs, n_obs, edges, n_edges, &q, A, b, n_faces, edge_status, nullptr, st,
                                edge_ids, skip);
        };
        TileCfg g;
        if ((s = ezo_tune_search(c, kb, fin, st, run, &g))) return s;
    }
    c->bisect_finalists.clear();
    if (tuned) hipLaunchKernelGGL(k_init_edges, dim3((E + 63) / 64), dim3(64), 0, st, ei);
    HIP_TRY(c, hipGetLastError());
    IterArgs it{(const int4*)w_k, 0, 0, 0, 0};
    // the learned screen inside the loop: the fused forward pass for widths
    // up to kMlpMaxH (a multiple of 16), else the layer-by-layer kernels
    // (samples only)
    const ezo_surrogate* sur = p->surrogate;
    const bool fused_screen = sur && sur->H <= kMlpMaxH && sur->H % 16 == 0;
    const bool screen_samples = sur && (sur->scope & EZO_SCREEN_SAMPLES);
    const bool screen_mid = fused_screen && (sur->scope & EZO_SCREEN_MIDPOINTS);
    const MlpView screen_view = sur ? MlpView{sur->D, sur->H, sur->P, sur->W2b, sur->W3b, sur->margin}
                                    : MlpView{0, 0, nullptr, nullptr, nullptr, 0.f};
    const uint32_t k0 = (uint32_t)p->seed, k1 = (uint32_t)(p->seed >> 32);
    (void)k0;
    (void)k1;
    // ---- one iteration: six kernels on the internal stream ----
    // Normal mode: captured once into a hipGraph and replayed.  Timing mode:
    // launched directly with hipEvents recorded between the phases (event
    // records inside a captured graph do not time the kernels).
    // Every k_advance writes the running-edge count and, when asked for, the
    // edges' statistics straight into pinned host memory, so that a replay
    // ends in one stream synchronisation and no copies; the last replay's
    // values are the final ones.
    const size_t stats_bytes = stats ? sizeof(EdgeStatsDev) * (size_t)E : 0;
    if (stats_bytes > c->pinned_stats_bytes) {
        if (c->pinned_stats) HIP_TRY(c, hipHostFree(c->pinned_stats));
        c->pinned_stats = c->pinned_stats_dev = nullptr;
        c->pinned_stats_bytes = 0;
        if (hipHostMalloc(&c->pinned_stats, stats_bytes, hipHostMallocDefault) != hipSuccess ||
            hipHostGetDevicePointer(&c->pinned_stats_dev, c->pinned_stats, 0) != hipSuccess) {
            (void)hipGetLastError();
            if (c->pinned_stats) (void)hipHostFree(c->pinned_stats);
            c->pinned_stats = c->pinned_stats_dev = nullptr;
            return ezo_fail(c, EZO_E_NOMEM, "pinned statistics buffer");
        }
        c->pinned_stats_bytes = stats_bytes;
    }
    EdgeStatsDev* host_stats = stats ? static_cast<EdgeStatsDev*>(c->pinned_stats_dev) : nullptr;
    auto launch_iteration = [&](bool marks) -> ezo_status {
        ezo_status ls = EZO_OK;
        auto mark = [&](int i) {          // the next launch belongs to phase i
            if (marks && i < EZO_NUM_PHASES) {
                c->ev_a = c->tev[2 * i];
                c->ev_b = c->tev[2 * i + 1];
            } else {
                c->ev_a = c->ev_b = nullptr;
            }
        };
        mark(EZO_PHASE_SAMPLE);
        if ((ls = launch_sample(c, dof, A, b, n_faces, cap, edges, E, S_cap, p->n_mix, p->seed, p->edge_id_base,
                                (float*)w_s, stride, edge_status, it, st, nullptr, (const int*)w_ac, edge_ids))) {
            mark(EZO_NUM_PHASES);
            return ls;
        }
        if (screen_samples && fused_screen) {
            // predictions for the rows the screen may skip, [M_k, |S|) of
            // every running edge, one fused forward pass per 64 rows
            EZO_KLAUNCH(c, k_screen_samples, dim3((unsigned)((S_cap + kScreenRows - 1) / kScreenRows), (unsigned)E),
                        dim3(256), 0, st, screen_view, (const float*)w_s, stride, dof, (float*)w_pred, edge_status,
                        it);
        } else if (screen_samples) {
            RowSource src{};
            src.q = (const float*)w_s;
            src.sn = 1;
            src.sd = stride;
            src.rows_per_batch = stride;
            src.qb = (int64_t)dof * stride;
            src.rows = (int64_t)E * stride;
            if ((ls = ezo_surrogate_forward_rows(c, p->surrogate, src, (float*)w_pred, edge_status, st))) {
                mark(EZO_NUM_PHASES);
                return ls;
            }
        }
        mark(EZO_PHASE_CHECK);
        GridView gvc = gv, gvb = gv;
        if (marks && c->d_tests) {
            gvc.tests = c->d_tests + (size_t)EZO_PHASE_CHECK * kTestSlots;
            gvb.tests = c->d_tests + (size_t)EZO_PHASE_BISECT * kTestSlots;
        }
        if ((ls = launch_check<false>(c, r, ov, gvc, (const float*)w_s, S_cap, 1, stride, (int64_t)dof * stride,
                                      (uint8_t*)w_f, nullptr, nullptr, stride, E, edge_status, it, st,
                                      screen_samples ? (const float*)w_pred : nullptr,
                                      screen_samples ? p->surrogate->margin : 0.f, (EdgeStatsDev*)w_st))) {
            mark(EZO_NUM_PHASES);
            return ls;
        }
        mark(EZO_PHASE_TEST);
        EZO_KLAUNCH(c, k_test_select, dim3(E), dim3(1024), 0, st, (const uint8_t*)w_f, stride, p->n_p, p->n_b,
                           (int*)w_ci, cand_cap, (int*)w_nc, nullptr, nullptr, edge_status, (EdgeStatsDev*)w_st, it);
        mark(EZO_PHASE_BISECT);
        if ((ls = launch_project_bisect(c, r, ov, gvb, edges, E, (const float*)w_s, stride, (const int*)w_ci,
                                        (const int*)w_nc, cand_cap, p->n_b, (float*)w_cs, (float*)w_ad,
                                        (float*)w_ts, (uint8_t*)w_pc, (uint8_t*)w_pa, edge_status, st, nullptr, -1,
                                        screen_mid ? &screen_view : nullptr, (EdgeStatsDev*)w_st))) {
            mark(EZO_NUM_PHASES);
            return ls;
        }
        mark(EZO_PHASE_PLACE);
        // one edge: the placement's single workgroup ends the iteration itself
        // (no k_advance launch; its phase then times nothing)
        const IterEnd ie = E == 1 ? IterEnd{(int4*)w_k, (const int4*)w_tb, p->max_iters, (int*)w_ac, c->pinned_dev,
                                            host_stats}
                                  : IterEnd{};
        EZO_KLAUNCH(c, k_place, dim3(E), dim3(1024), (size_t)std::max(cand_cap, 16), st, dof, edges,
                           (const float*)w_cs, (const float*)w_ad, (const float*)w_ts, (const int*)w_nc, cand_cap,
                           p->n_f, (float)p->step_back_max, (float)p->t_col, A, b, n_faces, cap, edge_status,
                           nullptr, nullptr, (const uint8_t*)w_pa, (EdgeStatsDev*)w_st, p->row_points, ie);
        mark(EZO_PHASE_ADVANCE);
        if (E != 1)
            EZO_KLAUNCH(c, k_advance, dim3(1), dim3(256), 0, st, (int4*)w_k, (const int4*)w_tb, p->max_iters,
                        edge_status, E, (int*)w_ac, c->pinned_dev, (const EdgeStatsDev*)w_st, host_stats);
        mark(EZO_NUM_PHASES);
        if (ls == EZO_OK) {
            hipError_t le = hipGetLastError();
            if (le != hipSuccess) ls = ezo_fail(c, EZO_E_HIP, "kernel launch failed: %s", hipGetErrorString(le));
        }
        return ls;
    };
    // Normal mode: kItersPerGraph iterations per graph (extra iterations after
    // every edge is final are no-ops: each kernel skips final edges), one
    // 4-byte poll per replay.  The executable graph is kept by the context and
    // updated in place with the next call's capture (same topology, new
    // arguments); instantiation happens only when the topology changes.
    hipGraphExec_t exec = nullptr;
    int per = 1;
    // Tuning runs (the sample-count search and the bisection shape trials)
    // launch their iterations directly, kItersPerGraph per poll: each would
    // otherwise capture and instantiate a graph of its own (its seed or shape
    // differs from the kept graph's), which costs more than the run.
    const bool direct = c->timing || c->shape_trial || c->np_search;
    // Everything the captured launches depend on: when a call repeats the
    // previous one's key, the kept executable graph is replayed as it is.
    std::vector<uintptr_t> key;
    if (!direct) {
        auto push = [&](const void* ptr) { key.push_back(reinterpret_cast<uintptr_t>(ptr)); };
        push(r);
        push(r->buf);
        push(obs);
        push(edges);
        push(A);
        push(b);
        push(n_faces);
        push(edge_status);
        push(st);
        push(edge_ids);
        push(skip);
        push(c->ebox);
        push(c->pinned_dev);
        push(host_stats);
        key.push_back((uintptr_t)(uint32_t)c->n_ebox);
        key.push_back((uintptr_t)(uint32_t)n_obs);
        key.push_back((uintptr_t)(uint32_t)E);
        key.push_back((uintptr_t)S_cap);
        key.push_back((uintptr_t)stride);
        const unsigned char* pb = reinterpret_cast<const unsigned char*>(p);
        for (size_t i = 0; i < sizeof(ezo_params); i += sizeof(uint32_t)) {
            uint32_t wv = 0;
            std::memcpy(&wv, pb + i, std::min(sizeof(uint32_t), sizeof(ezo_params) - i));
            key.push_back(wv);
        }
        if (p->surrogate) {
            uint32_t mb;
            std::memcpy(&mb, &p->surrogate->margin, sizeof(mb));
            key.push_back(mb);
            push(p->surrogate->P);
            push(p->surrogate->W2b);
            push(p->surrogate->W3b);
            key.push_back((uintptr_t)p->surrogate->D);
            key.push_back((uintptr_t)p->surrogate->H);
            key.push_back((uintptr_t)p->surrogate->scope);
        }
        for (const DevBuf& wb : c->ws) push(wb.p);
        const TileCfg gc = resolve_cfg(c, tune_key(c, r, TUNE_CHECK_FLAGS, ov.n, (int64_t)S_cap * E),
                                       heuristic_check(c, r, ov.n, (int64_t)S_cap * E, false), r->slots, r->P, r->view.n_blocks, ov.n, false);
        const TileCfg gb = resolve_cfg(c, tune_key(c, r, TUNE_BISECT, ov.n, (int64_t)cand_cap * E),
                                       heuristic_bisect(c, r, ov.n, (int64_t)cand_cap * E), r->slots, r->P, r->view.n_blocks, ov.n, false, true);
        for (const TileCfg& g : {gc, gb}) {
            key.push_back((uintptr_t)g.T);
            key.push_back((uintptr_t)g.W);
            key.push_back((uintptr_t)g.stage);
            key.push_back((uintptr_t)g.depth);
        }
    }
    if (direct) {
        per = c->timing ? 1 : kItersPerGraph;
    } else if (c->loop_exec && key == c->loop_key) {
        per = kItersPerGraph;
        exec = c->loop_exec;
    } else {
        per = kItersPerGraph;
        hipGraph_t graph = nullptr;
        HIP_TRY(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        ezo_status cs = EZO_OK;
        for (int i = 0; i < per && cs == EZO_OK; ++i) cs = launch_iteration(false);
        hipError_t ce = hipStreamEndCapture(st, &graph);
        if (cs) {
            if (graph) (void)hipGraphDestroy(graph);
            return cs;
        }
        if (ce != hipSuccess) return ezo_fail(c, EZO_E_HIP, "graph capture failed: %s", hipGetErrorString(ce));
        if (c->loop_exec) {
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult ur = hipGraphExecUpdateError;
            if (hipGraphExecUpdate(c->loop_exec, graph, &bad, &ur) != hipSuccess || ur != hipGraphExecUpdateSuccess) {
                (void)hipGetLastError();
                (void)hipGraphExecDestroy(c->loop_exec);
                c->loop_exec = nullptr;
            }
        }
        if (!c->loop_exec && hipGraphInstantiate(&c->loop_exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            c->loop_exec = nullptr;
            (void)hipGraphDestroy(graph);
            return ezo_fail(c, EZO_E_HIP, "graph instantiation failed");
        }
        (void)hipGraphDestroy(graph);
        exec = c->loop_exec;
        c->loop_key = key;
    }
    ezo_status result = EZO_OK;
    for (int k = 1; k <= p->max_iters; k += per) {
        hipError_t e1 = hipSuccess;
        if (exec) {
            e1 = hipGraphLaunch(exec, st);
        } else {
            for (int i = 0; i < per && result == EZO_OK; ++i) result = launch_iteration(c->timing);
            if (result) break;
        }
        const hipError_t e2 = hipStreamSynchronize(st);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            result = ezo_fail(c, EZO_E_HIP, "iteration %d failed: %s", k,
                              hipGetErrorString(e1 != hipSuccess ? e1 : e2));
            break;
        }
        if (c->timing) {
            for (int ph = 0; ph < EZO_NUM_PHASES; ++ph) {
                if (ph == EZO_PHASE_ADVANCE && E == 1) continue;   // done inside the placement
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, c->tev[2 * ph], c->tev[2 * ph + 1]) == hipSuccess)
                    c->phase_ms[ph] += ms;
                else
                    (void)hipGetLastError();               // leave no error for the next check
            }
            c->timed_iters++;
        }
        if (c->pinned[0] == 0) break;
    }
    if (result) return result;
    if (stats) {
        const EdgeStatsDev* hs = static_cast<const EdgeStatsDev*>(c->pinned_stats);
        for (int e = 0; e < E; ++e) {
            stats[e].iterations = (int32_t)hs[e].iterations;
            stats[e].planes = (int32_t)hs[e].planes;
            stats[e].final_m = hs[e].final_m;
            stats[e].test_collisions = hs[e].test_collisions;
            stats[e].samples = hs[e].samples;
            stats[e].exact_checks = hs[e].exact_checks;
            stats[e].screened_checks = hs[e].screened;
        }
    }
    // (no event for the caller's stream: the host has already waited for
    // every launch of this call, so later work on any stream follows it)
    return EZO_OK;
}

extern "C" {

ezo_status ezo_inflate_edges(ezo_ctx* c, const ezo_robot* r, const float* obs, int32_t n_obs, const float* edges,
                             int32_t n_edges, const ezo_params* p, float* A, float* b, int32_t* n_faces,
                             int32_t* edge_status, ezo_edge_stats* stats, void* stream) {
    return inflate_core(c, r, obs, n_obs, edges, n_edges, p, A, b, n_faces, edge_status, stats, stream, nullptr,
                        nullptr);
}

// ---------------------------------------------------------------------------
// Sequential inflation of paths with the containment skip (Sec. V-A)
// ---------------------------------------------------------------------------

ezo_status ezo_inflate_paths(ezo_ctx* c, const ezo_robot* r, const float* obs, int32_t n_obs, const float* vertices,
                             const int32_t* path_vertices, int32_t n_paths, const ezo_params* p, float* A, float* b,
                             int32_t* n_faces, int32_t* edge_status, int32_t* covered_by, ezo_edge_stats* stats,
                             void* stream) {
    if (!c) return EZO_E_INVALID;
    if (!r || !p) return ezo_fail(c, EZO_E_INVALID, "NULL robot or params");
    if (n_paths < 0 || n_obs < 0) return ezo_fail(c, EZO_E_INVALID, "negative size");
    if (n_paths == 0) return EZO_OK;
    if (!path_vertices) return ezo_fail(c, EZO_E_INVALID, "NULL path_vertices");
    std::vector<int> eoff(n_paths + 1, 0);
    int max_k = 0;
    for (int q = 0; q < n_paths; ++q) {
        const int nv = path_vertices[q];
        if (nv < 2) return ezo_fail(c, EZO_E_INVALID, "path %d has %d vertices (at least 2)", q, nv);
        if ((int64_t)eoff[q] + nv - 1 > INT32_MAX / 2) return ezo_fail(c, EZO_E_INVALID, "too many edges");
        eoff[q + 1] = eoff[q] + nv - 1;
        max_k = std::max(max_k, nv - 1);
    }
    if (!vertices || !A || !b || !n_faces || !edge_status || !covered_by || (n_obs > 0 && !obs))
        return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    const int dof = r->dof, P = n_paths, cap = p->face_capacity;
    if (cap < 1) return ezo_fail(c, EZO_E_CAPACITY, "face_capacity %d", cap);
    // window of s edges per path and round: enough edges per round to keep
    // the chip busy (kPathBatch), at most the longest path (one round)
    const int s_win = std::max(1, std::min({max_k, (kPathBatch + P - 1) / P, kPathWindowMax}));
    const int slots = P * s_win, rounds = (max_k + s_win - 1) / s_win;
    HIP_TRY(c, hipSetDevice(c->device));
    void *w_eo, *w_re, *w_ri, *w_rs, *w_ra, *w_rb, *w_rn, *w_rt;
    ezo_status s;
    if ((s = ezo_ws_get(c, W_PATH_EOFF, sizeof(int) * (size_t)(P + 1), &w_eo)) ||
        (s = ezo_ws_get(c, W_ROUND_EDGES, sizeof(float) * (size_t)slots * 2 * dof, &w_re)) ||
        (s = ezo_ws_get(c, W_ROUND_IDS, sizeof(int) * (size_t)slots, &w_ri)) ||
        (s = ezo_ws_get(c, W_ROUND_SKIP, (size_t)slots, &w_rs)) ||
        (s = ezo_ws_get(c, W_ROUND_A, sizeof(float) * (size_t)slots * cap * dof, &w_ra)) ||
        (s = ezo_ws_get(c, W_ROUND_B, sizeof(float) * (size_t)slots * cap, &w_rb)) ||
        (s = ezo_ws_get(c, W_ROUND_NF, sizeof(int) * (size_t)slots, &w_rn)) ||
        (s = ezo_ws_get(c, W_ROUND_ST, sizeof(int) * (size_t)slots, &w_rt)))
        return s;
    hipStream_t st = c->stream;
    HIP_TRY(c, hipEventRecord(c->ev_in, as_stream(stream)));
    HIP_TRY(c, hipStreamWaitEvent(st, c->ev_in, 0));
    HIP_TRY(c, hipMemcpyAsync(w_eo, eoff.data(), sizeof(int) * (P + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(c, hipStreamSynchronize(st));            // eoff is a host vector
    std::vector<ezo_edge_stats> rstats(slots);
    ezo_params pr = *p;
    pr.row_points = nullptr;           // the round buffers are indexed by window slot
    for (int rr = 0; rr < rounds; ++rr) {
        EZO_KLAUNCH(c, k_path_round, dim3(P), dim3(256), 0, st, dof, vertices, (const int*)w_eo, rr, s_win, A, b,
                    n_faces, edge_status, cap, covered_by, (float*)w_re, (int*)w_ri, (uint8_t*)w_rs);
        HIP_TRY(c, hipGetLastError());
        if ((s = inflate_core(c, r, obs, n_obs, (const float*)w_re, slots, &pr, (float*)w_ra, (float*)w_rb,
                              (int*)w_rn, (int*)w_rt, stats ? rstats.data() : nullptr, st, (const int*)w_ri,
                              (const uint8_t*)w_rs)))
            return s;
        EZO_KLAUNCH(c, k_path_resolve, dim3(P), dim3(256), 0, st, dof, vertices, (const int*)w_eo, rr, s_win,
                    (const float*)w_ra, (const float*)w_rb, (const int*)w_rn, (const int*)w_rt, cap, A, b, n_faces,
                    edge_status, covered_by);
        HIP_TRY(c, hipGetLastError());
        if (stats)
            for (int q = 0; q < P; ++q)
                for (int i = 0; i < s_win; ++i)
                    if (rr * s_win + i < eoff[q + 1] - eoff[q]) stats[eoff[q] + rr * s_win + i] = rstats[q * s_win + i];
    }
    if (stats) {
        // an edge inflated in its window but then found inside an earlier
        // edge's set of the same window holds no set: no statistics
        std::vector<int32_t> cov(eoff[P]);
        HIP_TRY(c, hipMemcpyAsync(cov.data(), covered_by, sizeof(int32_t) * cov.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        for (size_t g = 0; g < cov.size(); ++g)
            if (cov[g] >= 0) stats[g] = ezo_edge_stats{};
    }
    HIP_TRY(c, hipEventRecord(c->ev_out, st));
    HIP_TRY(c, hipStreamWaitEvent(as_stream(stream), c->ev_out, 0));
    return EZO_OK;
}

// ---------------------------------------------------------------------------
// Collision map of a dynamic roadmap (appendix, DRM construction)
// ---------------------------------------------------------------------------

ezo_status ezo_collision_map(ezo_ctx* c, const ezo_robot* r, const float* q, int64_t n_nodes, const float* lo,
                             float side, const int32_t* dims, uint32_t* map, int64_t row_words, void* stream) {
    if (!c) return EZO_E_INVALID;
    if (!r || n_nodes < 0 || !lo || !dims || !(side > 0.f) || !std::isfinite(side))
        return ezo_fail(c, EZO_E_INVALID, "bad argument");
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || !std::isfinite(lo[a])) return ezo_fail(c, EZO_E_INVALID, "bad voxel grid");
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2];
    if (row_words < (n_nodes + 31) / 32) return ezo_fail(c, EZO_E_INVALID, "row_words < ceil(n_nodes / 32)");
    if (n_nodes > 0 && (!q || !map)) return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    if (V > ((int64_t)1 << 40) / std::max<int64_t>(row_words, 1)) return ezo_fail(c, EZO_E_UNSUPPORTED, "map too large");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = as_stream(stream);
    if (map && row_words > 0) {
        const int64_t words = V * row_words;
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 65535)), dim3(256), 0,
                           st, map, words, 0u);
        HIP_TRY(c, hipGetLastError());
    }
    if (n_nodes == 0) return EZO_OK;
    ObsView ov;
    GridView gv;
    ezo_status s = prep_obstacles(c, r, nullptr, 0, st, &ov, &gv);   // zero shift: world frame
    if (s) return s;
    ov.n_ebox = 0;                                                    // the map holds the robot only
    int T = 16;
    while (T > 1 && tile_smem_bytes(T, r->slots, 4) > c->lds_cap) T >>= 1;
    const size_t lds = tile_smem_bytes(T, r->slots, 4);
    dim3 grid((unsigned)((n_nodes + T - 1) / T)), block(256);
    const float3 lo3 = make_float3(lo[0], lo[1], lo[2]);
    const int3 d3 = make_int3(dims[0], dims[1], dims[2]);
#define EZO_LAUNCH_MAP(TT)                                                                                    \
    do {                                                                                                      \
        if (r->B > 0)                                                                                         \
            hipLaunchKernelGGL((k_collision_map<TT, true>), grid, block, lds, st, r->view, ov, q, n_nodes, lo3, \
                               side, d3, map, row_words);                                                     \
        else                                                                                                  \
            hipLaunchKernelGGL((k_collision_map<TT, false>), grid, block, lds, st, r->view, ov, q, n_nodes,     \
                               lo3, side, d3, map, row_words);                                                \
    } while (0)
    switch (T) {
        case 16: EZO_LAUNCH_MAP(16); break;
        case 8: EZO_LAUNCH_MAP(8); break;
        case 4: EZO_LAUNCH_MAP(4); break;
        case 2: EZO_LAUNCH_MAP(2); break;
        default: EZO_LAUNCH_MAP(1); break;
    }
#undef EZO_LAUNCH_MAP
    HIP_TRY(c, hipGetLastError());
    return EZO_OK;
}

ezo_status ezo_collision_map_lists(ezo_ctx* c, const uint32_t* map, int64_t n_rows, int64_t row_words,
                                   int64_t n_nodes, int64_t* offsets, int32_t* ids, int64_t capacity, int64_t* total,
                                   void* stream) {
    if (!c) return EZO_E_INVALID;
    if (n_rows < 0 || n_nodes < 0 || capacity < 0 || row_words < (n_nodes + 31) / 32)
        return ezo_fail(c, EZO_E_INVALID, "bad sizes");
    if (!offsets || (n_rows > 0 && row_words > 0 && !map) || (capacity > 0 && !ids))
        return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = as_stream(stream);
    void* w_cnt;
    ezo_status s;
    if ((s = ezo_ws_get(c, W_MAP_COUNTS, sizeof(int64_t) * (size_t)std::max<int64_t>(n_rows, 1), &w_cnt))) return s;
    if (n_rows > 0) {
        hipLaunchKernelGGL(k_row_popcount, dim3((unsigned)((n_rows * 64 + 255) / 256)), dim3(256), 0, st, map, n_rows,
                           row_words, (int64_t*)w_cnt);
        HIP_TRY(c, hipGetLastError());
    }
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, (const int64_t*)w_cnt, n_rows, offsets);
    HIP_TRY(c, hipGetLastError());
    int64_t tot = 0;
    HIP_TRY(c, hipMemcpyAsync(&tot, offsets + n_rows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (total) *total = tot;
    if (tot > capacity) return ezo_fail(c, EZO_E_CAPACITY, "%lld ids > capacity %lld", (long long)tot, (long long)capacity);
    if (n_rows > 0 && tot > 0) {
        hipLaunchKernelGGL(k_map_lists, dim3((unsigned)((n_rows * 64 + 255) / 256)), dim3(256), 0, st, map, n_rows,
                           row_words, n_nodes, (const int64_t*)offsets, ids);
        HIP_TRY(c, hipGetLastError());
    }
    return EZO_OK;
}

// ---------------------------------------------------------------------------
// Recovery from collisions found on a trajectory (Sec. V-B)
// ---------------------------------------------------------------------------

ezo_status ezo_check_path(ezo_ctx* c, const ezo_robot* r, const float* obs, int32_t n_obs, const float* waypoints,
                          int32_t n_waypoints, double max_step, float* points_out, int32_t point_capacity,
                          int64_t* n_points, int64_t* n_colliding, void* stream) {
    if (!c) return EZO_E_INVALID;
    if (!r || n_waypoints < 1 || n_obs < 0 || point_capacity < 0 || !(max_step > 0.0) || !std::isfinite(max_step))
        return ezo_fail(c, EZO_E_INVALID, "bad argument");
    if (!waypoints || (n_obs > 0 && !obs) || (point_capacity > 0 && !points_out))
        return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = as_stream(stream);
    const int dof = r->dof, K = n_waypoints, nseg = std::max(K - 1, 1);
    ezo_status s;
    void *wm, *woff, *wpts, *widx, *wcnt, *wflags;
    if ((s = ezo_ws_get(c, W_PATH_M, sizeof(int) * nseg, &wm)) ||
        (s = ezo_ws_get(c, W_PATH_OFF, sizeof(int64_t) * nseg, &woff)))
        return s;
    // pieces per segment (device, FP64), offsets on the host
    std::vector<int> m(nseg, 0);
    std::vector<int64_t> off(nseg, 0);
    int64_t N = 1;
    if (K > 1) {
        hipLaunchKernelGGL(k_path_pieces, dim3((K - 1 + 255) / 256), dim3(256), 0, st, dof, waypoints, K, max_step,
                           (int*)wm);
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipMemcpyAsync(m.data(), wm, sizeof(int) * (K - 1), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        N = 0;
        for (int i = 0; i < K - 1; ++i) {
            off[i] = N;
            N += (int64_t)m[i] + (i == 0 ? 1 : 0);
        }
    }
    if (N > (1LL << 28)) return ezo_fail(c, EZO_E_UNSUPPORTED, "%lld path points: step too fine", (long long)N);
    if ((s = ezo_ws_get(c, W_PATH_PTS, sizeof(float) * (size_t)N * dof, &wpts)) ||
        (s = ezo_ws_get(c, W_PATH_IDX, sizeof(int) * (size_t)std::max(point_capacity, 1), &widx)) ||
        (s = ezo_ws_get(c, W_PATH_CNT, sizeof(int) * 2, &wcnt)) ||
        (s = ezo_ws_get(c, W_FLAGS, (size_t)N, &wflags)))
        return s;
    if (K > 1) {
        HIP_TRY(c, hipMemcpyAsync(woff, off.data(), sizeof(int64_t) * (K - 1), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_path_points, dim3(K - 1), dim3(256), 0, st, dof, waypoints, (const int*)wm,
                           (const int64_t*)woff, (float*)wpts);
    } else {
        HIP_TRY(c, hipMemcpyAsync(wpts, waypoints, sizeof(float) * dof, hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(c, hipGetLastError());
    ObsView ov;
    GridView gv;
    if ((s = prep_obstacles(c, r, obs, n_obs, st, &ov, &gv))) return s;
    IterArgs it{nullptr, 0, 0, 0, 0};
    if ((s = launch_check<false>(c, r, ov, gv, (const float*)wpts, N, dof, 1, 0, (uint8_t*)wflags, nullptr, nullptr,
                                 0, 1, nullptr, it, st)))
        return s;
    // colliding points in path order: the first point_capacity of them, and their count
    IterArgs sel{nullptr, 0, (int)std::min<int64_t>(N, 0x7fffffff), -1, (int)N};
    int* cnt = (int*)wcnt;
    hipLaunchKernelGGL(k_test_select, dim3(1), dim3(1024), 0, st, (const uint8_t*)wflags, N,
                       std::max(point_capacity, 1), 0, (int*)widx, std::max(point_capacity, 1), cnt, nullptr, cnt + 1,
                       nullptr, nullptr, sel);
    if (point_capacity > 0)
        hipLaunchKernelGGL(k_gather_rows, dim3((point_capacity + 255) / 256), dim3(256), 0, st, dof,
                           (const float*)wpts, (const int*)widx, (const int*)cnt, point_capacity, points_out);
    HIP_TRY(c, hipGetLastError());
    int h[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (n_points) *n_points = N;
    if (n_colliding) *n_colliding = h[1];
    return EZO_OK;
}

ezo_status ezo_update_polytopes(ezo_ctx* c, const ezo_robot* r, const float* obs, int32_t n_obs, const float* edges,
                                int32_t n_edges, const float* points, int32_t n_points, int32_t n_b, int32_t n_f,
                                double step_back_max, double t_col, float* A, float* b, int32_t* n_faces,
                                int32_t face_capacity, int32_t* edge_status, int32_t* planes_added, void* stream) {
    if (!c) return EZO_E_INVALID;
    if (!r || n_edges < 0 || n_points < 0 || n_obs < 0 || n_b < 0 || n_f < 0 || face_capacity < 1 ||
        !finite_pos(step_back_max) || !std::isfinite(t_col))
        return ezo_fail(c, EZO_E_INVALID, "bad argument");
    if (n_edges == 0 || n_points == 0) return EZO_OK;
    if (!edges || !points || !A || !b || !n_faces || !edge_status || (n_obs > 0 && !obs))
        return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    if ((size_t)n_points > c->lds_cap - kPlaceStaticLds)
        return ezo_fail(c, EZO_E_UNSUPPORTED, "%d points: at most %zu per call", n_points, c->lds_cap - kPlaceStaticLds);
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = as_stream(stream);
    const int dof = r->dof, E = n_edges, N = n_points;
    ezo_status s;
    void *w_s, *w_f, *w_ci, *w_nc, *w_cs, *w_ad, *w_ts, *w_pc, *w_pa, *w_run, *w_np;
    if ((s = ezo_ws_get(c, W_SAMPLES, sizeof(float) * (size_t)dof * N, &w_s)) ||
        (s = ezo_ws_get(c, W_FLAGS, (size_t)E * N, &w_f)) ||
        (s = ezo_ws_get(c, W_CAND, sizeof(int) * (size_t)E * N, &w_ci)) ||
        (s = ezo_ws_get(c, W_NCAND, sizeof(int) * (size_t)E, &w_nc)) ||
        (s = ezo_ws_get(c, W_CSTAR, sizeof(float) * (size_t)E * dof * N, &w_cs)) ||
        (s = ezo_ws_get(c, W_ADIR, sizeof(float) * (size_t)E * dof * N, &w_ad)) ||
        (s = ezo_ws_get(c, W_TSTAR, sizeof(float) * (size_t)E * N, &w_ts)) ||
        (s = ezo_ws_get(c, W_PCOL, (size_t)E * N, &w_pc)) || (s = ezo_ws_get(c, W_PANY, (size_t)E, &w_pa)) ||
        (s = ezo_ws_get(c, W_RUN, sizeof(int) * (size_t)E, &w_run)) ||
        (s = ezo_ws_get(c, W_NPLACED, sizeof(int) * (size_t)E, &w_np)))
        return s;
    // found collisions inside each editable set, in point order, become the candidates
    hipLaunchKernelGGL(k_rows_to_coords, dim3((N + 255) / 256), dim3(256), 0, st, dof, points, (int64_t)N,
                       (float*)w_s);
    hipLaunchKernelGGL(k_points_in_sets, dim3((N + 255) / 256, E), dim3(256), 0, st, dof, A, b, n_faces,
                       face_capacity, edge_status, (const float*)w_s, (int64_t)N, (uint8_t*)w_f);
    IterArgs sel{nullptr, 0, 0, -1, N};
    hipLaunchKernelGGL(k_test_select, dim3(E), dim3(1024), 0, st, (const uint8_t*)w_f, (int64_t)N, N, n_b,
                       (int*)w_ci, N, (int*)w_nc, nullptr, nullptr, nullptr, nullptr, sel);
    hipLaunchKernelGGL(k_recover_begin, dim3((E + 255) / 256), dim3(256), 0, st, E, (const int*)w_nc, (int*)w_run,
                       (int*)w_np);
    HIP_TRY(c, hipMemsetAsync(w_pa, 0, (size_t)E, st));
    HIP_TRY(c, hipGetLastError());
    ObsView ov;
    GridView gv;
    if ((s = prep_obstacles(c, r, obs, n_obs, st, &ov, &gv))) return s;
    // the last three steps of Alg. 1 on those candidates
    if ((s = launch_project_bisect(c, r, ov, gv, edges, E, (const float*)w_s, N, (const int*)w_ci, (const int*)w_nc,
                                   N, n_b, (float*)w_cs, (float*)w_ad, (float*)w_ts, (uint8_t*)w_pc,
                                   (uint8_t*)w_pa, (const int*)w_run, st, nullptr, 0)))
        return s;
    hipLaunchKernelGGL(k_place, dim3(E), dim3(1024), (size_t)std::max(N, 16), st, dof, edges, (const float*)w_cs,
                       (const float*)w_ad, (const float*)w_ts, (const int*)w_nc, N, n_f, (float)step_back_max,
                       (float)t_col, A, b, n_faces, face_capacity, (int*)w_run, nullptr, (int*)w_np,
                       (const uint8_t*)w_pa, nullptr, nullptr, IterEnd{});
    hipLaunchKernelGGL(k_recover_end, dim3((E + 255) / 256), dim3(256), 0, st, E, (const int*)w_run,
                       (const int*)w_np, edge_status, planes_added);
    HIP_TRY(c, hipGetLastError());
    return EZO_OK;
}

ezo_status ezo_segments_contained(ezo_ctx* c, int32_t dof, const float* A, const float* b, const int32_t* n_faces,
                                  int32_t face_capacity, int32_t n_sets, const float* segments, int32_t n_segments,
                                  double tol, int32_t* covered, void* stream) {
    if (!c) return EZO_E_INVALID;
    if (dof < 1 || dof > EZO_MAX_DOF || face_capacity < 1 || n_sets < 0 || n_segments < 0 || !std::isfinite(tol))
        return ezo_fail(c, EZO_E_INVALID, "bad argument");
    if (n_segments == 0) return EZO_OK;
    if (!segments || !covered || (n_sets > 0 && (!A || !b || !n_faces))) return ezo_fail(c, EZO_E_INVALID, "NULL buffer");
    HIP_TRY(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_segments_contained, dim3(n_segments), dim3(256), 0, as_stream(stream), dof, A, b, n_faces,
                       face_capacity, n_sets, segments, (float)tol, covered);
    HIP_TRY(c, hipGetLastError());
    return EZO_OK;
}

ezo_status ezo_set_phase_timing(ezo_ctx* c, int32_t enable) {
    if (!c) return EZO_E_INVALID;
    HIP_TRY(c, hipSetDevice(c->device));
    if (enable) {
        for (auto& ev : c->tev)
            if (!ev) HIP_TRY(c, hipEventCreate(&ev));
        const size_t tb = sizeof(unsigned long long) * EZO_NUM_PHASES * kTestSlots;
        if (!c->d_tests) HIP_TRY(c, hipMalloc((void**)&c->d_tests, tb));
        HIP_TRY(c, hipMemsetAsync(c->d_tests, 0, tb, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    c->timing = enable != 0;
    for (double& m : c->phase_ms) m = 0.0;
    c->timed_iters = 0;
    return EZO_OK;
}

ezo_status ezo_get_phase_timing(ezo_ctx* c, double* ms_out, int64_t* iterations_out, int64_t* tests_out) {
    if (!c || !ms_out) return EZO_E_INVALID;
    for (int i = 0; i < EZO_NUM_PHASES; ++i) ms_out[i] = c->phase_ms[i];
    if (iterations_out) *iterations_out = c->timed_iters;
    if (tests_out) {
        std::vector<unsigned long long> h((size_t)EZO_NUM_PHASES * kTestSlots, 0ull);
        if (c->d_tests) {
            HIP_TRY(c, hipSetDevice(c->device));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            HIP_TRY(c, hipMemcpy(h.data(), c->d_tests, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost));
        }
        for (int i = 0; i < EZO_NUM_PHASES; ++i) {
            unsigned long long t = 0;
            for (int k = 0; k < kTestSlots; ++k) t += h[(size_t)i * kTestSlots + k];
            tests_out[i] = (int64_t)t;
        }
    }
    return EZO_OK;
}

}  // extern "C"
