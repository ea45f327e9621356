// ezo_tune.hip -- launch-shape autotuner of the tile kernels (collision check
// in both modes, projection + bisection) and of the sampler.
//
// The shape of a tile kernel (configurations per workgroup T, waves W,
// obstacle records in LDS or not) never changes its results: every
// configuration's flag and signed distance, and every candidate's bisection,
// are computed from the same pair tests whatever the split.  The sampler's
// lanes per walk split the polytope's rows, whose chord bounds are combined
// by exact min/max.  So the shape is chosen by time alone.  The first call with a new key times each candidate
// shape on the call's own (or representative) input and keeps the fastest in
// a process-wide cache; later calls with that key use it without timing.
// The cache can be exported as text and imported in another process.
#include <algorithm>
#include <map>
#include <mutex>
#include <sstream>

#include "ezo_internal.hpp"

namespace {

constexpr int kTuneReps = 3;
constexpr int kTuneFinalists = 4;

const char* kKindNames[TUNE_NKINDS] = {"check_flags", "check_sd", "bisect", "sample", "samples"};

struct Entry {
    TileCfg cfg;
    double us = 0.0;
    bool has_seed = false;      // the timed runs drew from Philox key `seed`
    uint64_t seed = 0;
};

std::mutex g_mu;
std::map<TuneKey, Entry> g_cache;

// Position just after `"key"` and the ':' that follows it (blanks allowed
// around the colon), or npos.
size_t value_pos(const std::string& line, const char* key) {
    const std::string pat = std::string("\"") + key + "\"";
    size_t p = line.find(pat);
    if (p == std::string::npos) return p;
    p += pat.size();
    while (p < line.size() && (line[p] == ' ' || line[p] == '\t')) ++p;
    if (p >= line.size() || line[p] != ':') return std::string::npos;
    ++p;
    while (p < line.size() && (line[p] == ' ' || line[p] == '\t')) ++p;
    return p;
}

bool find_num(const std::string& line, const char* key, double* out) {
    const size_t p = value_pos(line, key);
    if (p == std::string::npos) return false;
    char* end = nullptr;
    const char* s = line.c_str() + p;
    const double v = std::strtod(s, &end);
    if (end == s) return false;
    *out = v;
    return true;
}

bool find_str(const std::string& line, const char* key, std::string* out) {
    const size_t p = value_pos(line, key);
    if (p == std::string::npos || line[p] != '"') return false;
    const size_t q = line.find('"', p + 1);
    if (q == std::string::npos) return false;
    *out = line.substr(p + 1, q - p - 1);
    return true;
}

}  // namespace

bool TuneKey::operator<(const TuneKey& o) const {
    if (arch != o.arch) return arch < o.arch;
    const int a[7] = {kind, dof, S, P, n_obs, bucket, B};
    const int b[7] = {o.kind, o.dof, o.S, o.P, o.n_obs, o.bucket, o.B};
    for (int i = 0; i < 7; ++i)
        if (a[i] != b[i]) return a[i] < b[i];
    return false;
}

int ezo_tune_bucket(int64_t items) {
    int b = 0;
    while (items > 1) {
        items >>= 1;
        ++b;
    }
    return b;
}

bool ezo_tune_lookup(const TuneKey& k, TileCfg* out) {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_cache.find(k);
    if (it == g_cache.end()) return false;
    *out = it->second.cfg;
    return true;
}

// Mean time of `reps` launches of one shape (ms), +inf if a launch fails.
static ezo_status time_shape(ezo_ctx* c, hipStream_t st, const std::function<ezo_status(const TileCfg&)>& run,
                             const TileCfg& cfg, int reps, double* ms_out) {
    *ms_out = INFINITY;
    HIP_TRY(c, hipEventRecord(c->tune_ev[0], st));
    ezo_status s = EZO_OK;
    for (int r = 0; r < reps && s == EZO_OK; ++r) s = run(cfg);
    HIP_TRY(c, hipEventRecord(c->tune_ev[1], st));
    HIP_TRY(c, hipEventSynchronize(c->tune_ev[1]));
    if (s != EZO_OK) {                   // e.g. a shape the device cannot launch
        (void)hipGetLastError();
        return EZO_OK;
    }
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->tune_ev[0], c->tune_ev[1]));
    *ms_out = ms / reps;
    return EZO_OK;
}

ezo_status ezo_tune_search(ezo_ctx* c, const TuneKey& k, const std::vector<TileCfg>& cands, hipStream_t st,
                           const std::function<ezo_status(const TileCfg&)>& run, TileCfg* best, double slack,
                           std::vector<TileCfg>* finalists) {
    if (cands.empty()) return ezo_fail(c, EZO_E_INVALID, "no launch shape to tune");
    for (auto& ev : c->tune_ev)
        if (!ev) HIP_TRY(c, hipEventCreate(&ev));
    // screening: one launch of every shape (after one warm-up launch of the
    // first), then the kTuneFinalists fastest again with kTuneReps launches
    ezo_status s;
    if (run(cands[0]) != EZO_OK) (void)hipGetLastError();
    std::vector<std::pair<double, int>> order;
    for (int i = 0; i < (int)cands.size(); ++i) {
        double ms;
        if ((s = time_shape(c, st, run, cands[i], 1, &ms))) return s;
        if (std::isfinite(ms)) order.push_back({ms, i});
    }
    if (order.empty()) return ezo_fail(c, EZO_E_HIP, "no launch shape ran during tuning");
    std::sort(order.begin(), order.end());
    double best_ms = INFINITY;
    std::vector<std::pair<double, int>> fin;      // (ms, candidate index) of the finalists
    for (int f = 0; f < std::min<int>(kTuneFinalists, (int)order.size()); ++f) {
        double ms;
        if ((s = time_shape(c, st, run, cands[order[f].second], kTuneReps, &ms))) return s;
        fin.push_back({ms, order[f].second});
        best_ms = std::min(best_ms, ms);
    }
    if (!std::isfinite(best_ms)) return ezo_fail(c, EZO_E_HIP, "no launch shape ran during tuning");
    if (finalists) {
        std::vector<std::pair<double, int>> f = fin;
        std::sort(f.begin(), f.end());
        finalists->clear();
        for (const auto& e : f)
            if (std::isfinite(e.first)) finalists->push_back(cands[e.second]);
    }
    // the earliest candidate (in the caller's order of preference) within
    // (1 + slack) of the fastest
    int pick_i = -1;
    double pick_ms = best_ms;
    for (const auto& f : fin)
        if (f.first <= best_ms * (1.0 + slack) && (pick_i < 0 || f.second < pick_i)) {
            pick_i = f.second;
            pick_ms = f.first;
        }
    const TileCfg pick = cands[pick_i];
    best_ms = pick_ms;
    c->err.clear();
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_cache[k] = Entry{pick, 1e3 * best_ms};
    }
    *best = pick;
    return EZO_OK;
}

void ezo_tune_store(const TuneKey& k, const TileCfg& g) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache[k] = Entry{g, 0.0};
}

void ezo_tune_note_seed(const TuneKey& k, uint64_t seed) {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_cache.find(k);
    if (it == g_cache.end()) return;
    it->second.has_seed = true;
    it->second.seed = seed;
}

extern "C" {

ezo_status ezo_set_autotune(ezo_ctx* c, int32_t enable) {
    if (!c) return EZO_E_INVALID;
    c->autotune = enable != 0;
    return EZO_OK;
}

ezo_status ezo_tune_cache_export(char* buf, int64_t capacity, int64_t* length) {
    std::ostringstream os;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        for (const auto& kv : g_cache) {
            const TuneKey& k = kv.first;
            const Entry& e = kv.second;
            char line[512], seed[64] = "";
            if (e.has_seed) std::snprintf(seed, sizeof(seed), ",\"tune_seed\":%llu", (unsigned long long)e.seed);
            std::snprintf(line, sizeof(line),
                          "{\"arch\":\"%s\",\"kernel\":\"%s\",\"dof\":%d,\"spheres\":%d,\"self_pairs\":%d,"
                          "\"boxes\":%d,\"obstacles\":%d,\"log2_items\":%d,\"T\":%d,\"W\":%d,\"stage\":%d,"
                          "\"depth\":%d,\"us\":%.3f%s}\n",
                          k.arch.c_str(), kKindNames[k.kind], k.dof, k.S, k.P, k.B, k.n_obs, k.bucket, e.cfg.T,
                          e.cfg.W, e.cfg.stage, e.cfg.depth, e.us, seed);
            os << line;
        }
    }
    const std::string text = os.str();
    if (length) *length = (int64_t)text.size();
    if (buf && capacity > 0) {
        const size_t n = std::min<size_t>(text.size(), (size_t)capacity - 1);
        std::memcpy(buf, text.data(), n);
        buf[n] = '\0';
        if (text.size() + 1 > (size_t)capacity) return EZO_E_CAPACITY;
    }
    return EZO_OK;
}

ezo_status ezo_tune_cache_import(const char* text, int32_t* n_imported) {
    if (!text) return EZO_E_INVALID;
    std::istringstream is(text);
    std::string line;
    int n = 0;
    std::map<TuneKey, Entry> add;
    while (std::getline(is, line)) {
        if (line.find('{') == std::string::npos) continue;
        TuneKey k;
        std::string kern;
        double v[9];
        const char* keys[9] = {"dof", "spheres", "self_pairs", "obstacles", "log2_items", "T", "W", "stage", "us"};
        bool ok = find_str(line, "arch", &k.arch) && find_str(line, "kernel", &kern);
        for (int i = 0; i < 9 && ok; ++i) ok = find_num(line, keys[i], &v[i]);
        int kind = -1;
        for (int i = 0; i < TUNE_NKINDS && ok; ++i)
            if (kern == kKindNames[i]) kind = i;
        const int T = ok ? (int)v[5] : 0, W = ok ? (int)v[6] : 0;
        double depth = 1.0;                          // optional key (bisection only)
        if (ok) find_num(line, "depth", &depth);
        double boxes = 0.0;                          // optional key (robots with boxes)
        if (ok) find_num(line, "boxes", &boxes);
        const bool count = kind == TUNE_SAMPLE_COUNT;   // T is a sample count, not a tile size
        const bool shape_ok = (count ? (T >= 1 && T <= (1 << 24))
                                     : (T == 1 || T == 2 || T == 4 || T == 8 || T == 16 || T == 32 || T == 64)) &&
                              W >= 1 && W <= 16 && (v[7] == 0 || v[7] == 1) && (depth == 1 || depth == 2 || depth == 3);
        if (!ok || kind < 0 || !shape_ok) return EZO_E_INVALID;
        k.kind = kind;
        k.dof = (int)v[0];
        k.S = (int)v[1];
        k.P = (int)v[2];
        k.n_obs = (int)v[3];
        k.bucket = (int)v[4];
        k.B = (int)boxes;
        Entry e;
        e.cfg.T = T;
        e.cfg.W = W;
        e.cfg.stage = (int)v[7];
        e.cfg.depth = (int)depth;
        e.us = v[8];
        add[k] = e;
        ++n;
    }
    {
        std::lock_guard<std::mutex> lock(g_mu);
        for (const auto& kv : add) g_cache[kv.first] = kv.second;
    }
    if (n_imported) *n_imported = n;
    return EZO_OK;
}

void ezo_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache.clear();
}

}  // extern "C"
