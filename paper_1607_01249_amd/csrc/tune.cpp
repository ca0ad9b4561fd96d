// Autotuner and tune table (Sec. 2.1 stages 2-6; Sec. 2.3).
//
// The paper's TTC generates C++/CUDA source for each ranked candidate,
// compiles it and times it, then stores the fastest ("solution") in an SQL
// database consulted before any new search.  Here the candidates are
// run-time configurations of pre-instantiated kernels (tile shape from the
// menu, loop order, XCD swizzle, streaming stores), so stage 4 (compile)
// disappears and stage 5 times each candidate directly on the GPU.  The
// database is an in-process table keyed by the merged problem, with a
// one-line-per-entry text format for saving and loading.  A table file can
// also be attached as a database shared across processes: its entries are
// merged in (lowest time per key) and every new tuning result is appended
// to it under an exclusive file lock (TTX_TUNE_DB names one at start-up).
#include <sys/file.h>
#include <unistd.h>

#include <atomic>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <vector>

#include "ttx_internal.h"

namespace ttx {

struct TableEntry {
    ttx_config cfg;
    double usec;
};

static std::mutex g_table_mu;
static std::map<std::string, TableEntry> g_table;
static std::atomic<uint64_t> g_table_gen{1};
static std::string g_db_path;   // attached database file ("" when none); under g_table_mu
static const char* const kTableHeader =
    "# ttx tune table v3: key | family tile_a tile_b threads flags group_a group_b n_order order... "
    "[c<tile_c>] [l<lds_pad>] | usec\n";

static ttx_status attach_db(const char* path);
static ttx_status merge_file(const char* path);

// Before the table is first used: the table named by TTX_TUNE_TABLE is
// loaded (read only; e.g. the shipped per-architecture table) and the
// database named by TTX_TUNE_DB attached.
static void attach_env_db() {
    static std::once_flag once;
    std::call_once(once, [] {
        const char* table = std::getenv("TTX_TUNE_TABLE");
        if (table && *table) (void)merge_file(table);
        const char* path = std::getenv("TTX_TUNE_DB");
        if (path && *path) (void)attach_db(path);
    });
}

uint64_t table_generation() {
    attach_env_db();
    return g_table_gen.load();
}

// Key: dtype, beta == 0, and the merged problem (extents, permutation and
// both stride vectors), so that every call that plans to the same merged
// problem shares a solution (Sec. 2.1: lookup happens after merging).
// Entries for size-specialised execution carry the prefix "j:" (their best
// configuration can differ from the generic kernels').
static std::string table_key(const Problem& p, bool beta0, bool specialised = false) {
    std::ostringstream os;
    if (specialised) os << "j:";
    os << "d" << p.code << ":b" << (beta0 ? 1 : 0) << ":n" << p.n << ":s";
    for (int i = 0; i < p.n; ++i) os << (i ? "," : "") << p.dim[i].size;
    os << ":p";
    for (int i = 0; i < p.n; ++i) os << (i ? "," : "") << p.perm[i];
    os << ":a";
    for (int i = 0; i < p.n; ++i) os << (i ? "," : "") << p.dim[i].sa;
    os << ":o";
    for (int i = 0; i < p.n; ++i) os << (i ? "," : "") << p.dim[i].sb;
    return os.str();
}

bool table_lookup(const Problem& p, bool beta0, ttx_config* out, bool specialised) {
    attach_env_db();
    std::lock_guard<std::mutex> lock(g_table_mu);
    auto it = g_table.find(table_key(p, beta0, specialised));
    if (it == g_table.end() || !config_valid(p, it->second.cfg, nullptr)) return false;
    *out = it->second.cfg;
    return true;
}

static std::string config_text(const ttx_config& c);

// Appends one entry to the attached database under an exclusive lock, so
// that processes sharing the file never interleave partial lines.
static void db_append(const std::string& path, const std::string& line) {
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;
    if (flock(fileno(f), LOCK_EX) == 0) {
        std::fputs(line.c_str(), f);
        std::fflush(f);
        (void)flock(fileno(f), LOCK_UN);
    }
    std::fclose(f);
}

void table_store(const Problem& p, bool beta0, const ttx_config& c, double usec, bool specialised) {
    attach_env_db();
    const std::string key = table_key(p, beta0, specialised);
    std::string db;
    {
        std::lock_guard<std::mutex> lock(g_table_mu);
        g_table[key] = TableEntry{c, usec};
        g_table_gen.fetch_add(1);
        db = g_db_path;
    }
    if (!db.empty()) {
        std::ostringstream os;
        os << key << " | " << config_text(c) << " | " << usec << "\n";
        db_append(db, os.str());
    }
}

static std::string config_text(const ttx_config& c) {
    std::ostringstream os;
    os << c.family << " " << c.tile_a << " " << c.tile_b << " " << c.threads << " " << c.flags << " "
       << c.group_a << " " << c.group_b << " " << c.n_order;
    for (int i = 0; i < c.n_order; ++i) os << " " << c.order[i];
    if (c.tile_c > 1) os << " c" << c.tile_c;
    if (c.lds_pad != 1) os << " l" << c.lds_pad;
    return os.str();
}

static bool parse_config(std::istringstream& is, ttx_config* c) {
    std::memset(c, 0, sizeof(*c));
    if (!(is >> c->family >> c->tile_a >> c->tile_b >> c->threads >> c->flags >> c->group_a >> c->group_b >>
          c->n_order))
        return false;
    if (c->n_order < 0 || c->n_order > kMaxDims) return false;
    for (int i = 0; i < c->n_order; ++i)
        if (!(is >> c->order[i])) return false;
    // optional "c<planes>" (dense tiles) and "l<padding>" (LDS rows; 1 when absent)
    c->lds_pad = 1;
    std::string extra;
    while (is >> extra) {
        if (extra.size() < 2 || (extra[0] != 'c' && extra[0] != 'l')) return false;
        char* end = nullptr;
        const long v = std::strtol(extra.c_str() + 1, &end, 10);
        if (*end != '\0') return false;
        if (extra[0] == 'c') {
            if (v < 1) return false;
            c->tile_c = int(v);
        } else {
            if (v < 0 || v > TTX_MAX_LDS_PAD) return false;
            c->lds_pad = int(v);
        }
    }
    return true;
}

// A scratch area that evicts L2 and the 256 MiB Infinity Cache between timed
// runs ("the caches are cleared before each run", Sec. 3).
static constexpr size_t kFlushBytes = size_t(1) << 30;

// One flush area per device, allocated on first use and kept for the life of
// the process (tuning many small shapes would otherwise allocate 1 GiB each).
static void* flush_area() {
    static std::mutex mu;
    static void* area[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!area[dev] && hipMalloc(&area[dev], kFlushBytes) != hipSuccess) area[dev] = nullptr;
    return area[dev];
}

struct TuneScratch {
    void* A = nullptr;
    void* B = nullptr;
    void* flush = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneScratch() {
        if (A) (void)hipFree(A);
        if (B) (void)hipFree(B);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

ttx_status time_candidates(const Problem& p, bool beta0, int count, int reps,
                           const std::function<hipError_t(int, const void*, void*, hipStream_t)>& launch,
                           int* best_i, double* best_us, double* all_us) {
    if (reps <= 0) reps = 3;
    TuneScratch s;
    s.flush = flush_area();
    if (!s.flush || hipMalloc(&s.A, size_t(p.extent_a) + 16) != hipSuccess ||
        hipMalloc(&s.B, size_t(p.extent_b) + 16) != hipSuccess)
        return fail(TTX_ENOMEM, "tuner scratch allocation failed");
    if (hipStreamCreate(&s.stream) != hipSuccess || hipEventCreate(&s.e0) != hipSuccess ||
        hipEventCreate(&s.e1) != hipSuccess)
        return fail(TTX_EHIP, "tuner stream/event creation failed");
    if (hipMemsetAsync(s.A, 0, size_t(p.extent_a), s.stream) != hipSuccess ||
        hipMemsetAsync(s.B, 0, size_t(p.extent_b), s.stream) != hipSuccess)
        return fail(TTX_EHIP, "tuner scratch initialisation failed");
    (void)beta0;
    *best_i = -1;
    *best_us = 1e300;
    for (int i = 0; i < count; ++i) {
        hipError_t e = launch(i, s.A, s.B, s.stream);
        if (e != hipSuccess) return fail(TTX_EHIP, std::string("tuner launch: ") + hipGetErrorString(e));
        double t_min = 1e300;
        for (int r = 0; r < reps; ++r) {
            if (hipMemsetAsync(s.flush, r & 0xff, kFlushBytes, s.stream) != hipSuccess ||
                hipEventRecord(s.e0, s.stream) != hipSuccess)
                return fail(TTX_EHIP, "tuner timing failed");
            e = launch(i, s.A, s.B, s.stream);
            if (e != hipSuccess || hipEventRecord(s.e1, s.stream) != hipSuccess ||
                hipEventSynchronize(s.e1) != hipSuccess)
                return fail(TTX_EHIP, "tuner timing failed");
            float ms = 0;
            (void)hipEventElapsedTime(&ms, s.e0, s.e1);
            if (ms * 1e3 < t_min) t_min = ms * 1e3;
        }
        if (all_us) all_us[i] = t_min;
        if (t_min < *best_us) {   // ties keep the earlier (better-ranked) candidate
            *best_us = t_min;
            *best_i = i;
        }
    }
    if (hipStreamSynchronize(s.stream) != hipSuccess) return fail(TTX_EHIP, "tuner sync failed");
    return TTX_OK;
}

// Second search stage: the workgroup variants (threads per workgroup x LDS
// row padding) of the TTX_TUNE_VARIANT_BASES fastest distinct candidates of
// the first stage (times in us[]), each compiled as a size-specialised
// kernel before it is timed (a variant whose compilation fails is skipped;
// the pre-compiled configurations among them run their generic kernels
// unless `specialised`).  *best and *best_us are replaced by a faster
// variant; *timed grows by the variants timed.
static ttx_status tune_variants(const Problem& p, bool beta0, const std::vector<ttx_config>& cands,
                                const std::vector<double>& us, int reps, bool specialised, ttx_config* best,
                                double* best_us, int* timed) {
    if (p.family != TTX_FAMILY_MOVED && p.family != TTX_FAMILY_PRESERVED) return TTX_OK;
    std::vector<int> order(cands.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = int(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return us[x] < us[y]; });
    const Scalar alpha(1.25), beta(beta0 ? 0.0 : 0.75);
    std::vector<ttx_config> vars;
    std::vector<const JitKernel*> ks;
    ttx_config buf[2 * 4 * (TTX_MAX_LDS_PAD + 1)];
    for (int b = 0, taken = 0; b < int(order.size()) && taken < TTX_TUNE_VARIANT_BASES; ++b) {
        const int nv = workgroup_variants(p, cands[order[b]], buf, int(sizeof(buf) / sizeof(buf[0])));
        ++taken;
        for (int v = 1; v < nv; ++v) {   // buf[0] is the base, timed in the first stage
            bool dup = false;
            for (const ttx_config& c : vars) dup |= std::memcmp(&c, &buf[v], sizeof(c)) == 0;
            if (dup) continue;
            const JitKernel* k = nullptr;
            if (specialised || config_needs_jit(p, buf[v])) {
                TiledLaunch L;
                void* a = reinterpret_cast<void*>(uintptr_t(1) << 20);
                void* bb = reinterpret_cast<void*>(uintptr_t(3) << 20);
                if (!prepare_tiled(p, buf[v], beta0, a, beta0 ? nullptr : bb, bb, alpha, beta, &L)) continue;
                const std::string saved = ttx_last_error();
                if (jit_kernel(L, &k) != TTX_OK) {   // no kernel for this variant: leave it out
                    fail(TTX_OK, saved);
                    continue;
                }
            }
            vars.push_back(buf[v]);
            ks.push_back(k);
        }
    }
    if (vars.empty()) return TTX_OK;
    int vi = -1;
    double vus = 0;
    ttx_status st = time_candidates(
        p, beta0, int(vars.size()), reps,
        [&](int i, const void* A, void* B, hipStream_t s) {
            const void* Bsrc = beta0 ? nullptr : B;
            if (ks[i]) {
                TiledLaunch L;
                if (!prepare_tiled(p, vars[i], beta0, A, Bsrc, B, alpha, beta, &L)) return hipErrorInvalidValue;
                if (jit_matches(*ks[i], L)) return jit_launch(*ks[i], L, s);
            }
            return launch_tiles(p, vars[i], beta0, A, Bsrc, B, alpha, beta, s);
        },
        &vi, &vus);
    if (st != TTX_OK) return st;
    *timed += int(vars.size());
    if (vi >= 0 && vus < *best_us) {
        *best = vars[vi];
        *best_us = vus;
    }
    return TTX_OK;
}

// Ranks the candidates of p, times the best max_candidates of them and
// stores the fastest in the tune table (ttx_tune for a built problem).
ttx_status tune_problem(const Problem& p, bool beta0, int max_candidates, int reps, ttx_config* best,
                        int* n_timed) {
    if (n_timed) *n_timed = 0;
    if (p.family == TTX_FAMILY_EMPTY) {
        *best = default_config(p);
        return TTX_OK;
    }
    const int keep = max_candidates == 0 ? 200 : max_candidates;
    std::vector<ttx_config> cands(keep < 0 ? 1 << 17 : keep);
    int nc = rank_candidates(p, max_candidates, cands.data(), nullptr, int(cands.size()));
    if (nc <= 0) return fail(TTX_EUNSUPPORTED, "no candidate for this problem");
    cands.resize(nc);
    int best_i = -1;
    double best_us = 0;
    std::vector<double> us(nc, 0.0);
    ttx_status st = time_candidates(
        p, beta0, int(cands.size()), reps,
        [&](int i, const void* A, void* B, hipStream_t s) {
            return launch_tiles(p, cands[i], beta0, A, B, B, 1.0, beta0 ? 0.0 : 1.0, s);
        },
        &best_i, &best_us, us.data());
    if (st != TTX_OK) return st;
    *best = cands[best_i];
    int timed = nc;
    st = tune_variants(p, beta0, cands, us, reps, false, best, &best_us, &timed);
    if (st != TTX_OK) return st;
    if (n_timed) *n_timed = timed;
    table_store(p, beta0, *best, best_us);
    return TTX_OK;
}

// Stages 4 and 5 of Sec. 2.1 as the paper's compiler runs them: every kept
// candidate is compiled (here at run time, as a size-specialised kernel) and
// timed, and the fastest goes into the table.  Problems without tiles take
// the generic search.
ttx_status tune_problem_specialised(const Problem& p, bool beta0, int max_candidates, int reps, ttx_config* best,
                                    int* n_timed) {
    if (n_timed) *n_timed = 0;
    if (p.family != TTX_FAMILY_MOVED && p.family != TTX_FAMILY_PRESERVED)
        return tune_problem(p, beta0, max_candidates, reps, best, n_timed);
    const int keep = max_candidates == 0 ? 24 : max_candidates;
    std::vector<ttx_config> cands(keep < 0 ? 1 << 17 : keep);
    int nc = rank_candidates(p, keep, cands.data(), nullptr, int(cands.size()));
    if (nc <= 0) return fail(TTX_EUNSUPPORTED, "no candidate for this problem");
    cands.resize(nc);
    // compile every candidate for aligned tensors (the tuner's scratch
    // tensors are hipMalloc'd, so each launch finds its specialised kernel)
    const Scalar alpha(1.25), beta(beta0 ? 0.0 : 0.75);
    std::vector<const JitKernel*> ks(nc, nullptr);
    for (int i = 0; i < nc; ++i) {
        TiledLaunch L;
        void* a = reinterpret_cast<void*>(uintptr_t(1) << 20);
        void* b = reinterpret_cast<void*>(uintptr_t(3) << 20);
        if (!prepare_tiled(p, cands[i], beta0, a, beta0 ? nullptr : b, b, alpha, beta, &L))
            return fail(TTX_EUNSUPPORTED, "candidate without a tile kernel");
        ttx_status st = jit_kernel(L, &ks[i]);
        if (st != TTX_OK) return st;
    }
    int best_i = -1;
    double best_us = 0;
    std::vector<double> us(nc, 0.0);
    ttx_status st = time_candidates(
        p, beta0, nc, reps,
        [&](int i, const void* A, void* B, hipStream_t s) {
            const void* Bsrc = beta0 ? nullptr : B;
            TiledLaunch L;
            if (!prepare_tiled(p, cands[i], beta0, A, Bsrc, B, alpha, beta, &L)) return hipErrorInvalidValue;
            if (jit_matches(*ks[i], L)) return jit_launch(*ks[i], L, s);
            return launch_tiles(p, cands[i], beta0, A, Bsrc, B, alpha, beta, s);
        },
        &best_i, &best_us, us.data());
    if (st != TTX_OK) return st;
    *best = cands[best_i];
    int timed = nc;
    st = tune_variants(p, beta0, cands, us, reps, true, best, &best_us, &timed);
    if (st != TTX_OK) return st;
    if (n_timed) *n_timed = timed;
    table_store(p, beta0, *best, best_us, true);
    return TTX_OK;
}

// Reads a table file; a key listed more than once keeps its lowest time
// (a database file collects appended results).
static ttx_status read_table(const char* path, std::map<std::string, TableEntry>* out) {
    std::ifstream f(path);
    if (!f) return fail(TTX_ENOTFOUND, "cannot open tune table");
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        size_t a = line.find(" | "), b = line.rfind(" | ");
        if (a == std::string::npos || b == a) return fail(TTX_EINVAL, "malformed tune table line");
        TableEntry e;
        std::istringstream cs(line.substr(a + 3, b - a - 3));
        if (!parse_config(cs, &e.cfg)) return fail(TTX_EINVAL, "malformed config in tune table");
        e.usec = std::atof(line.substr(b + 3).c_str());
        const std::string key = line.substr(0, a);
        auto it = out->find(key);
        if (it == out->end() || e.usec < it->second.usec) (*out)[key] = e;
    }
    return TTX_OK;
}

// Merges a table file into the table, keeping the lowest time per key.
static ttx_status merge_file(const char* path) {
    std::map<std::string, TableEntry> loaded;
    ttx_status st = read_table(path, &loaded);
    if (st != TTX_OK) return st;
    std::lock_guard<std::mutex> lock(g_table_mu);
    for (auto& kv : loaded) {
        auto it = g_table.find(kv.first);
        if (it == g_table.end() || kv.second.usec < it->second.usec) g_table[kv.first] = kv.second;
    }
    g_table_gen.fetch_add(1);
    return TTX_OK;
}

static ttx_status attach_db(const char* path) {
    std::map<std::string, TableEntry> loaded;
    ttx_status st = read_table(path, &loaded);
    if (st == TTX_ENOTFOUND) {   // a new database: create it with the header line
        FILE* f = std::fopen(path, "a");
        if (!f) return fail(TTX_EINVAL, "cannot create the tune database");
        if (flock(fileno(f), LOCK_EX) == 0) {
            if (std::ftell(f) == 0) std::fputs(kTableHeader, f);
            (void)flock(fileno(f), LOCK_UN);
        }
        std::fclose(f);
        st = TTX_OK;
    }
    if (st != TTX_OK) return st;
    std::lock_guard<std::mutex> lock(g_table_mu);
    for (auto& kv : loaded) {
        auto it = g_table.find(kv.first);
        if (it == g_table.end() || kv.second.usec < it->second.usec) g_table[kv.first] = kv.second;
    }
    g_db_path = path;
    g_table_gen.fetch_add(1);
    return TTX_OK;
}

}  // namespace ttx

using namespace ttx;

extern "C" {

ttx_status ttx_tune_candidates(ttx_dtype dtype, int n, const int* perm, const int64_t* size,
                               const int64_t* outer_a, const int64_t* outer_b, int max_candidates,
                               ttx_config* out, double* cost, int cap, int* count) {
    if (!out || !count || cap < 0) return fail(TTX_EINVAL, "NULL output or negative cap");
    Problem p;
    ttx_status st = make_problem(dtype, n, perm, size, outer_a, outer_b, &p);
    if (st != TTX_OK) return st;
    *count = rank_candidates(p, max_candidates, out, cost, cap);
    return TTX_OK;
}

ttx_status ttx_tune_variants(ttx_dtype dtype, int n, const int* perm, const int64_t* size,
                             const int64_t* outer_a, const int64_t* outer_b, const ttx_config* base,
                             ttx_config* out, int cap, int* count) {
    if (!base || !out || !count || cap < 0) return fail(TTX_EINVAL, "NULL argument or negative cap");
    Problem p;
    ttx_status st = make_problem(dtype, n, perm, size, outer_a, outer_b, &p);
    if (st != TTX_OK) return st;
    std::string why;
    if (!config_valid(p, *base, &why)) return fail(TTX_EINVAL, why);
    *count = workgroup_variants(p, *base, out, cap);
    return TTX_OK;
}

ttx_status ttx_tile_shapes(ttx_dtype dtype, int family, int run_time_only, int* tile_a, int* tile_b, int cap,
                           int* count) {
    if (!count || cap < 0 || (cap > 0 && (!tile_a || !tile_b))) return fail(TTX_EINVAL, "NULL argument or negative cap");
    if (!dtype_valid(dtype)) return fail(TTX_EINVAL, "unknown dtype");
    if (family != TTX_FAMILY_MOVED && family != TTX_FAMILY_PRESERVED)
        return fail(TTX_EINVAL, "tile shapes exist for the moved and preserved families");
    const TileShape* s = nullptr;
    int n = 0;
    if (!run_time_only)
        n = tile_menu(dtype_b_of(dtype), family, &s);
    else if (family == TTX_FAMILY_MOVED)
        n = large_tile_menu(dtype_b_of(dtype), &s);
    for (int i = 0; i < n && i < cap; ++i) {
        tile_a[i] = s[i].ta;
        tile_b[i] = s[i].tb;
    }
    *count = n;
    return TTX_OK;
}

ttx_status ttx_tune(ttx_dtype dtype, int n, const int* perm, const int64_t* size,
                    const int64_t* outer_a, const int64_t* outer_b, int beta_is_zero,
                    int max_candidates, int reps, ttx_config* best, int* n_timed) {
    if (!best) return fail(TTX_EINVAL, "best must not be NULL");
    Problem p;
    ttx_status st = make_problem(dtype, n, perm, size, outer_a, outer_b, &p);
    if (st != TTX_OK) return st;
    return tune_problem(p, beta_is_zero != 0, max_candidates, reps, best, n_timed);
}
ttx_status ttx_tune_specialised(ttx_dtype dtype, int n, const int* perm, const int64_t* size,
                                const int64_t* outer_a, const int64_t* outer_b, int beta_is_zero,
                                int max_candidates, int reps, ttx_config* best, int* n_timed) {
    if (!best) return fail(TTX_EINVAL, "best must not be NULL");
    Problem p;
    ttx_status st = make_problem(dtype, n, perm, size, outer_a, outer_b, &p);
    if (st != TTX_OK) return st;
    return tune_problem_specialised(p, beta_is_zero != 0, max_candidates, reps, best, n_timed);
}
ttx_status ttx_tune_table_save(const char* path) {
    if (!path) return fail(TTX_EINVAL, "NULL path");
    std::ofstream f(path);
    if (!f) return fail(TTX_EINVAL, "cannot open tune table for writing");
    attach_env_db();
    std::lock_guard<std::mutex> lock(g_table_mu);
    f << kTableHeader;
    for (const auto& kv : g_table)
        f << kv.first << " | " << config_text(kv.second.cfg) << " | " << kv.second.usec << "\n";
    return f ? TTX_OK : fail(TTX_EINVAL, "write failed");
}

ttx_status ttx_tune_table_load(const char* path) {
    if (!path) return fail(TTX_EINVAL, "NULL path");
    attach_env_db();
    std::map<std::string, TableEntry> loaded;
    ttx_status st = read_table(path, &loaded);
    if (st != TTX_OK) return st;
    std::lock_guard<std::mutex> lock(g_table_mu);
    for (auto& kv : loaded) g_table[kv.first] = kv.second;
    g_table_gen.fetch_add(1);
    return TTX_OK;
}

ttx_status ttx_tune_db_attach(const char* path) {
    if (!path || !*path) return fail(TTX_EINVAL, "NULL or empty path");
    attach_env_db();
    return attach_db(path);
}

ttx_status ttx_tune_db_detach(void) {
    std::lock_guard<std::mutex> lock(g_table_mu);
    g_db_path.clear();
    return TTX_OK;
}

ttx_status ttx_tune_table_clear(void) {
    attach_env_db();
    std::lock_guard<std::mutex> lock(g_table_mu);
    g_table.clear();
    g_table_gen.fetch_add(1);
    return TTX_OK;
}

int ttx_tune_table_size(void) {
    attach_env_db();
    std::lock_guard<std::mutex> lock(g_table_mu);
    return int(g_table.size());
}

}  // extern "C"
