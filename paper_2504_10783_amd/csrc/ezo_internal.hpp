// ezo_internal.hpp -- host-side definitions shared by the library's
// translation units (ezo_api.hip: collision checking and inflation;
// ezo_surrogate.hip: the learned self-collision screen).  Not installed.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "ezo.h"
#include "ezo_device.hpp"

constexpr int kNumCU = 256;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Workspace slots of a context (grown on demand, reused across calls).
enum Slot {
    W_OBS_REC, W_OBS_CENTRE, W_GRID_GEOM, W_GRID_COUNT, W_GRID_LIST, W_SAMPLES, W_FLAGS, W_CAND, W_NCAND, W_CSTAR,
    W_ADIR, W_TSTAR, W_PCOL, W_PANY, W_STATS, W_TABLE, W_KDEV, W_ACTIVE, W_PRED, W_SCREENED, W_MLP_H1, W_MLP_H2,
    W_MLP_CNT, W_PATH_M, W_PATH_OFF, W_PATH_PTS, W_PATH_IDX, W_PATH_CNT, W_RUN, W_NPLACED, W_PATH_EOFF,
    W_ROUND_EDGES, W_ROUND_IDS, W_ROUND_SKIP, W_ROUND_A, W_ROUND_B, W_ROUND_NF, W_ROUND_ST, W_MAP_COUNTS, W_NSLOTS
};

// ---------------------------------------------------------------------------
// Launch shapes of the tile kernels and their tuning cache
// ---------------------------------------------------------------------------
// T configurations per workgroup, W waves per workgroup, obstacle records
// staged in LDS (stage = 1) or read from global memory; for the bisection,
// depth = bisection levels per round (T >> depth candidates per workgroup).
// T = 0: not chosen.
struct TileCfg {
    int T = 0, W = 0, stage = 0, depth = 1;
};

// For the sampler, T = lanes per walk and W = waves per workgroup.
// TUNE_SAMPLE_COUNT: T = the inflation's N_p (samples per iteration).
enum TuneKind { TUNE_CHECK_FLAGS = 0, TUNE_CHECK_SD = 1, TUNE_BISECT = 2, TUNE_SAMPLE = 3, TUNE_SAMPLE_COUNT = 4,
                TUNE_NKINDS };

// A tuned shape applies to calls with the same device architecture, kernel,
// robot size (dof, spheres, self pairs), obstacle count and work size
// (bucket = floor(log2(items))).  Sampler keys hold the dof and the walk
// count only (spheres = self pairs = obstacles = 0).
struct TuneKey {
    std::string arch;
    int kind = 0, dof = 0, S = 0, P = 0, n_obs = 0, bucket = 0, B = 0;
    bool operator<(const TuneKey& o) const;
};

struct ezo_ctx {
    int device = 0;
    hipStream_t stream = nullptr;      // internal stream (default priority)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    size_t lds_cap = 65536;
    std::string err;
    std::vector<DevBuf> ws;            // named workspace slots
    int* pinned = nullptr;             // host-pinned poll word, written by the device
    int* pinned_dev = nullptr;         // its device address
    void* pinned_stats = nullptr;      // host-pinned copy of the edges' statistics (grown on demand)
    void* pinned_stats_dev = nullptr;  // its device address
    size_t pinned_stats_bytes = 0;
    bool timing = false;               // per-phase timing of the fused loop
    hipEvent_t tev[2 * EZO_NUM_PHASES] = {};   // (start, stop) of each phase's kernel
    hipEvent_t ev_a = nullptr, ev_b = nullptr;   // events for the next kernel launch (timing mode)
    double phase_ms[EZO_NUM_PHASES] = {};
    int64_t timed_iters = 0;
    unsigned long long* d_tests = nullptr;   // [EZO_NUM_PHASES] sphere-sphere tests per phase
    std::string arch;                  // device architecture name (tuning cache key)
    bool autotune = true;              // time launch shapes on first use of a tuning key
    hipEvent_t tune_ev[2] = {};
    hipGraphExec_t loop_exec = nullptr;   // the inflation loop's graph, updated in place by later calls
    std::vector<uintptr_t> loop_key;      // everything the captured loop's launches depend on
    std::vector<int4> table_host;         // per-iteration table last copied to table_dev
    const void* table_dev = nullptr;
    float4* ebox = nullptr;               // obstacle boxes [n_ebox][4] (packed like robot boxes), world frame
    int n_ebox = 0;
    unsigned char* scratch = nullptr;     // device address of this device's fixed scratch (no-allocation calls)
    // bisection shapes that the stand-in timing left as finalists, to be timed
    // on whole inflations by the call that tuned them (see inflate_core)
    std::vector<TileCfg> bisect_finalists;
    TuneKey bisect_key;
    bool shape_trial = false;             // inside such a timing run
    bool np_search = false;               // inside the sample-count search's runs
};

struct ezo_robot {
    ezo_ctx* ctx = nullptr;
    int device = 0;                    // the context's device (destroy does not read the context)
    int dof = 0, S = 0, P = 0;
    int B = 0, Q = 0;                  // boxes, box self pairs
    int slots = 0;                     // LDS pose rows per configuration: S + 4 B
    float r_max = 0.f;                 // largest sphere radius
    void* buf = nullptr;               // one device allocation holding everything below
    ezo::RobotView view{};
    const int* sorted_to_orig = nullptr;
    const float* q_lo = nullptr;
    const float* q_hi = nullptr;
};

// Rows of the screen's input.  Row r (after adding rbase) reads configuration
// idx ? idx[r] : r, coordinate j at q[cfg * sn + j * sd]; with
// rows_per_batch > 0, row r belongs to batch r / rows_per_batch whose
// configurations start at q + batch * qb.
struct RowSource {
    const float* q;
    int64_t sn, sd;
    const int* idx;
    int64_t rows_per_batch;
    int64_t qb;
    int64_t rbase;
    int64_t rows;               // valid rows (after rbase)
};

struct ezo_surrogate {
    ezo_ctx* ctx = nullptr;
    int device = 0;                     // the context's device (destroy does not read the context)
    int D = 0, H = 0;
    int64_t n_params = 0;
    float margin = INFINITY;            // screen threshold (calibrated); +inf screens nothing
    int scope = EZO_SCREEN_SAMPLES | EZO_SCREEN_MIDPOINTS;   // what an inflation screens
    float* P = nullptr;                 // FP32 master parameters
    float* G = nullptr;                 // gradient
    float* m = nullptr;                 // Adam moments
    float* v = nullptr;
    __bf16* W2b = nullptr;              // BF16 copies for the MFMA layers
    __bf16* W3b = nullptr;
    int64_t adam_steps = 0;
    // training batch buffers
    int batch = 0;
    void* tb = nullptr;
};

int ezo_tune_bucket(int64_t items);
bool ezo_tune_lookup(const TuneKey& k, TileCfg* out);
// Times every candidate once, then the fastest few over several launches
// (launches of `run` on stream st, host-synchronising), and caches the
// pick under k: the first candidate in `cands` order whose time is within
// (1 + slack) of the fastest.  The default slack (3 %, about the spread of
// repeated timings) lets repeated tunings of near-equal shapes agree.
// Candidates whose launch fails are skipped.  Needs at least one candidate.
constexpr double kTuneSlack = 0.03;
// `finalists` (optional) receives the shapes timed over several launches,
// fastest first.
ezo_status ezo_tune_search(ezo_ctx* c, const TuneKey& k, const std::vector<TileCfg>& cands, hipStream_t st,
                           const std::function<ezo_status(const TileCfg&)>& run, TileCfg* best,
                           double slack = kTuneSlack, std::vector<TileCfg>* finalists = nullptr);
// Sets the cached shape of k (a shape on trial).
void ezo_tune_store(const TuneKey& k, const TileCfg& g);

// Records, for a cached entry, the Philox key that the timed runs drew from
// (the sample-count tuner's own stream; exported as "tune_seed").
void ezo_tune_note_seed(const TuneKey& k, uint64_t seed);

extern std::string g_create_err;
ezo_status ezo_fail(ezo_ctx* c, ezo_status code, const char* fmt, ...);
ezo_status ezo_ws_get(ezo_ctx* c, int slot, size_t bytes, void** out);
inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Screen predictions for `src.rows` rows into pred[0..rows) (chunked MLP
// forward).  Rows of batches whose status is final (status != NULL) are
// skipped.  Launches only; no synchronisation.
ezo_status ezo_surrogate_forward_rows(ezo_ctx* c, const ezo_surrogate* s, const RowSource& src, float* pred,
                                      const int* status, hipStream_t st);
// Grows the forward pass's workspace for `rows` rows (no allocation happens
// in ezo_surrogate_forward_rows afterwards for at most that many rows).
ezo_status ezo_surrogate_reserve(ezo_ctx* c, const ezo_surrogate* s, int64_t rows);

#define HIP_TRY(ctx, call)                                                                                 \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess) return ezo_fail(ctx, EZO_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Kernel launch; in timing mode the dispatch itself records c->ev_a / c->ev_b
// at its start and end (hipExtLaunchKernelGGL), so elapsed time is the
// kernel's own duration.
#define EZO_KLAUNCH(c, K, grid, block, lds, st, ...)                                              \
    do {                                                                                          \
        if ((c)->ev_a)                                                                            \
            hipExtLaunchKernelGGL(K, grid, block, lds, st, (c)->ev_a, (c)->ev_b, 0, __VA_ARGS__); \
        else                                                                                      \
            hipLaunchKernelGGL(K, grid, block, lds, st, __VA_ARGS__);                              \
    } while (0)
