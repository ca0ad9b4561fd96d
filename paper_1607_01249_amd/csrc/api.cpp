// C ABI: errors, plans, the per-call entry point and the ceiling kernels.
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>

#include "ttx_internal.h"

// What a plan runs for one beta class: the configuration and, when one is
// attached, the size-specialised kernel compiled for it.  Published as one
// immutable object, so that an execution running concurrently with
// ttx_plan_specialise or ttx_plan_set_config sees either the old pair or the
// new one, never a mix.
struct PlanExec {
    ttx_config cfg;
    int from_table;
    const ttx::JitKernel* jit;   // owned by the JIT cache (lives until the process ends)
};

struct ttx_plan {
    ttx::Problem prob;
    std::shared_ptr<const PlanExec> exec[2];   // [beta_is_zero]; read and replaced with std::atomic_load/store
    std::mutex mu;                             // serialises the writers
    bool user_set[2] = {false, false};
    uint64_t table_gen = 0;
    uint32_t calls[2] = {0, 0};                // per-call entry points: calls so far (automatic specialisation)
    bool jit_tried[2] = {false, false};        // automatic specialisation attempted

    std::shared_ptr<const PlanExec> load(int z) const { return std::atomic_load(&exec[z]); }
    void publish(int z, const ttx_config& cfg, int from_table, const ttx::JitKernel* jit) {
        std::atomic_store(&exec[z], std::shared_ptr<const PlanExec>(new PlanExec{cfg, from_table, jit}));
    }
};

namespace ttx {

static thread_local std::string g_last_error;

ttx_status fail(ttx_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

void clear_error() { g_last_error.clear(); }

static void resolve_configs(ttx_plan* plan) {
    plan->table_gen = table_generation();
    for (int z = 0; z < 2; ++z) {
        if (plan->user_set[z]) continue;
        ttx_config c;
        if (table_lookup(plan->prob, z == 1, &c))
            plan->publish(z, c, 1, nullptr);
        else
            plan->publish(z, default_config(plan->prob), 0, nullptr);
    }
}

static ttx_status new_plan(ttx_plan** out, int dtype, int n, const int* perm, const int64_t* size,
                           const int64_t* outer_a, const int64_t* outer_b) {
    Problem p;
    ttx_status st = make_problem(dtype, n, perm, size, outer_a, outer_b, &p);
    if (st != TTX_OK) return st;
    ttx_plan* plan = new (std::nothrow) ttx_plan();
    if (!plan) return fail(TTX_ENOMEM, "out of host memory");
    plan->prob = p;
    resolve_configs(plan);
    *out = plan;
    return TTX_OK;
}

static bool ranges_overlap(const void* x, int64_t xlen, const void* y, int64_t ylen) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(x), b = reinterpret_cast<uintptr_t>(y);
    return a < b + uint64_t(ylen) && b < a + uint64_t(xlen);
}

bool beta_is_zero(int dtype, const Scalar& beta) {
    if (dtype == TTX_F32 || dtype == TTX_C32) return float(beta.re) == 0.0f && float(beta.im) == 0.0f;
    return beta.re == 0.0 && beta.im == 0.0;
}

ttx_status check_pointers(const Problem& p, const void* A, const void* Bin, const void* Bout,
                          bool beta0) {
    if (p.family == TTX_FAMILY_EMPTY) return TTX_OK;
    if (!A || !Bout || (!beta0 && !Bin)) return fail(TTX_EINVAL, "NULL tensor pointer");
    const uintptr_t esa = uintptr_t(elem_bytes(p.dtype_a)), esz = uintptr_t(elem_bytes(p.dtype));
    if (reinterpret_cast<uintptr_t>(A) % esa || reinterpret_cast<uintptr_t>(Bout) % esz ||
        (!beta0 && reinterpret_cast<uintptr_t>(Bin) % esz))
        return fail(TTX_EINVAL, "tensor pointer not aligned to the element size");
    if (ranges_overlap(A, p.extent_a, Bout, p.extent_b))
        return fail(TTX_EOVERLAP, "A and B overlap (the operation is out-of-place)");
    if (!beta0 && Bin != Bout && ranges_overlap(Bin, p.extent_b, Bout, p.extent_b))
        return fail(TTX_EOVERLAP, "B_in and B_out overlap without being equal");
    return TTX_OK;
}

static ttx_status execute(const ttx_plan* plan, const Scalar& alpha, const void* A, const Scalar& beta,
                          const void* Bin, void* Bout, hipStream_t stream) {
    const Problem& p = plan->prob;
    if (!dtype_complex(p.dtype) && (alpha.im != 0.0 || beta.im != 0.0))
        return fail(TTX_EINVAL, "complex alpha or beta for a real element type");
    if (p.family == TTX_FAMILY_EMPTY) return TTX_OK;
    const bool beta0 = beta_is_zero(p.dtype, beta);
    ttx_status st = check_pointers(p, A, Bin, Bout, beta0);
    if (st != TTX_OK) return st;
    const std::shared_ptr<const PlanExec> x = plan->load(beta0 ? 1 : 0);
    if (x->jit) {
        TiledLaunch L;
        if (prepare_tiled(p, x->cfg, beta0, A, Bin, Bout, alpha, beta, &L) && jit_matches(*x->jit, L)) {
            const hipError_t e = jit_launch(*x->jit, L, stream);
            if (e != hipSuccess) return fail(TTX_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
            return TTX_OK;
        }
    }
    hipError_t e = launch_tiles(p, x->cfg, beta0, A, beta0 ? nullptr : Bin, Bout, alpha, beta, stream);
    if (e != hipSuccess) return fail(TTX_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return TTX_OK;
}

// Plan cache for ttx_transpose, keyed by the raw arguments.
static std::mutex g_cache_mu;
static std::unordered_map<std::string, std::shared_ptr<ttx_plan>> g_cache;
static constexpr size_t kCacheCap = 4096;

static std::string cache_key(int dtype, int n, const int* perm, const int64_t* size,
                             const int64_t* outer_a, const int64_t* outer_b) {
    std::string k;
    k.reserve(16 + n * 28);
    auto put = [&](const void* src, size_t len) { k.append(static_cast<const char*>(src), len); };
    put(&dtype, sizeof(dtype));
    put(&n, sizeof(n));
    put(perm, sizeof(int) * n);
    put(size, sizeof(int64_t) * n);
    const char na = outer_a ? 1 : 0, nb = outer_b ? 1 : 0;
    put(&na, 1);
    if (outer_a) put(outer_a, sizeof(int64_t) * n);
    put(&nb, 1);
    if (outer_b) put(outer_b, sizeof(int64_t) * n);
    return k;
}

// Automatic specialisation of the per-call entry points' plans: a shape's
// size-specialised kernel is compiled at its n-th call in a beta class
// (0: never).  The default comes from TTX_AUTO_SPECIALISE.
static std::mutex g_auto_mu;
static std::atomic<int> g_auto_calls{-1};
static int g_auto_specialised = 0;

static int auto_calls() {
    int n = g_auto_calls.load(std::memory_order_relaxed);
    if (n >= 0) return n;
    const char* env = std::getenv("TTX_AUTO_SPECIALISE");
    const int v = env ? std::atoi(env) : 0;
    int expected = -1;
    g_auto_calls.compare_exchange_strong(expected, v < 0 ? 0 : v);
    return g_auto_calls.load(std::memory_order_relaxed);
}

static void maybe_specialise(ttx_plan* plan, const Scalar& beta, int hot) {
    const int z = beta_is_zero(plan->prob.dtype, beta) ? 1 : 0;
    {
        std::lock_guard<std::mutex> lock(g_auto_mu);
        if (plan->jit_tried[z] || ++plan->calls[z] < uint32_t(hot)) return;
        plan->jit_tried[z] = true;
    }
    if (plan->prob.family != TTX_FAMILY_MOVED && plan->prob.family != TTX_FAMILY_PRESERVED) return;
    const std::string saved = g_last_error;
    int kept = 0;
    if (ttx_plan_specialise(plan, z, 0, &kept) != TTX_OK) {
        g_last_error = saved;   // the shape keeps its generic kernel
    } else if (kept) {
        std::lock_guard<std::mutex> lock(g_auto_mu);
        ++g_auto_specialised;
    }
}

ttx_status transpose_cached(int dtype, int n, const int* perm, const int64_t* size,
                            const int64_t* outer_a, const int64_t* outer_b, const Scalar& alpha,
                            const void* A, const Scalar& beta, const void* Bin, void* Bout,
                            hipStream_t stream) {
    if (n < 1 || n > kMaxDims || !perm || !size) {
        Problem p;
        return make_problem(dtype, n, perm, size, outer_a, outer_b, &p);
    }
    const std::string key = cache_key(dtype, n, perm, size, outer_a, outer_b);
    std::shared_ptr<ttx_plan> plan;
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) plan = it->second;
    }
    if (!plan || plan->table_gen != table_generation()) {
        ttx_plan* raw = nullptr;
        ttx_status st = new_plan(&raw, dtype, n, perm, size, outer_a, outer_b);
        if (st != TTX_OK) return st;
        plan.reset(raw);
        std::lock_guard<std::mutex> lock(g_cache_mu);
        if (g_cache.size() >= kCacheCap) g_cache.clear();
        g_cache[key] = plan;
    }
    const int hot = auto_calls();
    if (hot > 0) maybe_specialise(plan.get(), beta, hot);
    return execute(plan.get(), alpha, A, beta, Bin, Bout, stream);
}

static void cache_info(int* plans, int* specialised) {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    int s = 0;
    for (const auto& kv : g_cache) s += (kv.second->load(0)->jit || kv.second->load(1)->jit) ? 1 : 0;
    if (plans) *plans = int(g_cache.size());
    if (specialised) *specialised = s;
}

}  // namespace ttx

using namespace ttx;

extern "C" {

const char* ttx_status_string(ttx_status s) {
    switch (s) {
        case TTX_OK: return "ok";
        case TTX_EINVAL: return "invalid argument";
        case TTX_EPERM: return "perm is not a permutation";
        case TTX_EOVERLAP: return "A and B overlap";
        case TTX_EUNSUPPORTED: return "unsupported";
        case TTX_ENOMEM: return "out of memory";
        case TTX_EHIP: return "HIP error";
        case TTX_EBUSY: return "busy: request not admitted";
        case TTX_ENOTFOUND: return "not found";
    }
    return "unknown status";
}

const char* ttx_last_error(void) { return g_last_error.c_str(); }

const char* ttx_version(void) { return "ttx 0.1 gfx950"; }

ttx_status ttx_plan_create(ttx_plan** plan, ttx_dtype dtype, int n, const int* perm,
                           const int64_t* size, const int64_t* outer_a, const int64_t* outer_b) {
    if (!plan) return fail(TTX_EINVAL, "plan must not be NULL");
    return new_plan(plan, dtype, n, perm, size, outer_a, outer_b);
}

ttx_status ttx_plan_execute(const ttx_plan* plan, double alpha, const void* A, double beta, void* B,
                            hipStream_t stream) {
    if (!plan) return fail(TTX_EINVAL, "plan must not be NULL");
    return execute(plan, alpha, A, beta, B, B, stream);
}

ttx_status ttx_plan_execute_split(const ttx_plan* plan, double alpha, const void* A, double beta,
                                  const void* B_in, void* B_out, hipStream_t stream) {
    if (!plan) return fail(TTX_EINVAL, "plan must not be NULL");
    return execute(plan, alpha, A, beta, B_in, B_out, stream);
}

ttx_status ttx_plan_execute_c(const ttx_plan* plan, const double* alpha, const void* A,
                              const double* beta, const void* B_in, void* B_out, hipStream_t stream) {
    if (!plan || !alpha || !beta) return fail(TTX_EINVAL, "NULL argument");
    return execute(plan, Scalar(alpha[0], alpha[1]), A, Scalar(beta[0], beta[1]), B_in, B_out, stream);
}

ttx_status ttx_plan_describe(const ttx_plan* plan, ttx_plan_info* info) {
    if (!plan || !info) return fail(TTX_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    const Problem& p = plan->prob;
    info->dtype = p.code;
    info->family = p.family;
    info->n = p.n;
    for (int d = 0; d < p.n; ++d) {
        info->perm[d] = p.perm[d];
        info->size[d] = p.dim[d].size;
        info->stride_a[d] = p.dim[d].sa;
        info->stride_b[d] = p.dim[d].sb;
    }
    info->elements = p.elements;
    info->extent_a_bytes = p.extent_a;
    info->extent_b_bytes = p.extent_b;
    for (int z = 0; z < 2; ++z) {
        const std::shared_ptr<const PlanExec> x = plan->load(z);
        info->config[z] = x->cfg;
        info->config_from_table[z] = x->from_table;
        info->specialised[z] = x->jit != nullptr;
    }
    return TTX_OK;
}

ttx_status ttx_plan_set_config(ttx_plan* plan, int beta_is_zero, const ttx_config* config) {
    if (!plan || !config) return fail(TTX_EINVAL, "NULL argument");
    std::string why;
    if (!config_valid(plan->prob, *config, &why)) return fail(TTX_EINVAL, why);
    const int z = beta_is_zero ? 1 : 0;
    std::lock_guard<std::mutex> lock(plan->mu);
    plan->user_set[z] = true;
    plan->publish(z, *config, 0, nullptr);
    return TTX_OK;
}

// Stand-in pointers for specialisation: aligned for every vector path (the
// kernel flags depend only on alignment), never dereferenced.
static void* fake_ptr(uintptr_t at) { return reinterpret_cast<void*>(at); }

static ttx_status specialised_launch(const Problem& p, const ttx_config& cfg, int beta_is_zero, TiledLaunch* L) {
    const bool beta0 = beta_is_zero != 0;
    if (!prepare_tiled(p, cfg, beta0, fake_ptr(1u << 20), beta0 ? nullptr : fake_ptr(2u << 20),
                       fake_ptr(3u << 20), Scalar(1.0), Scalar(beta0 ? 0.0 : 1.0), L))
        return fail(TTX_EINVAL, "nothing to specialise (empty or single-index problem)");
    return TTX_OK;
}

// A specialised kernel is kept by a timed specialisation only when it beats
// the generic one by more than this fraction (timing noise).
static constexpr double kSpecialiseMargin = 0.01;

ttx_status ttx_plan_specialise(ttx_plan* plan, int beta_is_zero, int reps, int* kept) {
    if (kept) *kept = 0;
    if (!plan) return fail(TTX_EINVAL, "NULL argument");
    const int z = beta_is_zero ? 1 : 0;
    std::lock_guard<std::mutex> lock(plan->mu);
    const std::shared_ptr<const PlanExec> prev = plan->load(z);
    // the generic configuration: the one in effect without a specialised kernel
    ttx_config generic = prev->cfg;
    int generic_from_table = prev->from_table;
    if (prev->jit && !plan->user_set[z]) {   // a specialised configuration may be in effect: look again
        ttx_config c;
        generic_from_table = table_lookup(plan->prob, z == 1, &c) ? 1 : 0;
        generic = generic_from_table ? c : default_config(plan->prob);
    }
    plan->publish(z, generic, generic_from_table, nullptr);
    if (plan->prob.family != TTX_FAMILY_MOVED && plan->prob.family != TTX_FAMILY_PRESERVED) return TTX_OK;
    // a configuration tuned for specialised execution, when the table has one
    // and the caller has not set the config
    ttx_config cfg = generic;
    int from_table = generic_from_table;
    ttx_config cs;
    if (!plan->user_set[z] && table_lookup(plan->prob, z == 1, &cs, true)) {
        cfg = cs;
        from_table = 1;
    }
    TiledLaunch L;
    ttx_status st = specialised_launch(plan->prob, cfg, z, &L);
    if (st != TTX_OK) return st;
    const JitKernel* k = nullptr;
    st = jit_kernel(L, &k);
    if (st != TTX_OK) return st;
    if (reps > 0) {
        // candidate 0: the generic kernel with its own configuration, 1: the
        // specialised one, on the tuner's scratch tensors (hipMalloc'd, so in
        // the compiled alignment class)
        const Problem& p = plan->prob;
        const bool beta0 = z == 1;
        const Scalar alpha(1.25), beta(beta0 ? 0.0 : 0.75);
        auto launch = [&](int i, const void* A, void* B, hipStream_t stream) -> hipError_t {
            const void* Bsrc = beta0 ? nullptr : B;
            if (i == 0) return launch_tiles(p, generic, beta0, A, Bsrc, B, alpha, beta, stream);
            TiledLaunch T;
            if (!prepare_tiled(p, cfg, beta0, A, Bsrc, B, alpha, beta, &T) || !jit_matches(*k, T))
                return hipErrorInvalidValue;
            return jit_launch(*k, T, stream);
        };
        int best = 0;
        double best_us = 0, us[2] = {0, 0};
        st = time_candidates(p, beta0, 2, reps, launch, &best, &best_us, us);
        if (st != TTX_OK) return st;
        // not faster: the plan keeps its generic kernel and configuration
        if (!(us[1] < us[0] * (1.0 - kSpecialiseMargin))) return TTX_OK;
    }
    plan->publish(z, cfg, from_table, k);
    if (kept) *kept = 1;
    return TTX_OK;
}

ttx_status ttx_plan_specialised_source(const ttx_plan* plan, int beta_is_zero, char* buf, int len) {
    if (!plan || !buf || len <= 0) return fail(TTX_EINVAL, "NULL argument");
    TiledLaunch L;
    ttx_status st = specialised_launch(plan->prob, plan->load(beta_is_zero ? 1 : 0)->cfg, beta_is_zero, &L);
    if (st != TTX_OK) return st;
    const std::string src = jit_source(L);
    if (int64_t(src.size()) >= int64_t(len)) return fail(TTX_EINVAL, "buffer too small");
    std::memcpy(buf, src.c_str(), src.size() + 1);
    return TTX_OK;
}

ttx_status ttx_plan_kernel_name(const ttx_plan* plan, double beta, const void* A, const void* B,
                                char* buf, int len) {
    if (!plan || !buf || len <= 0) return fail(TTX_EINVAL, "NULL argument");
    const Problem& p = plan->prob;
    const bool beta0 = beta_is_zero(p.dtype, beta);
    const std::shared_ptr<const PlanExec> x = plan->load(beta0 ? 1 : 0);
    std::string name;
    TiledLaunch L;
    if (x->jit && prepare_tiled(p, x->cfg, beta0, A, B, const_cast<void*>(B), Scalar(1.0), Scalar(beta), &L) &&
        jit_matches(*x->jit, L))
        name = jit_name(*x->jit);
    else
        name = kernel_name(p, x->cfg, beta0, A, B, B);
    if (int(name.size()) >= len) return fail(TTX_EINVAL, "buffer too small");
    std::memcpy(buf, name.c_str(), name.size() + 1);
    return TTX_OK;
}

ttx_status ttx_plan_destroy(ttx_plan* plan) {
    delete plan;
    return TTX_OK;
}

ttx_status ttx_transpose(ttx_dtype dtype, int n, const int* perm, const int64_t* size,
                         const int64_t* outer_a, const int64_t* outer_b, double alpha,
                         const void* A, double beta, void* B, hipStream_t stream) {
    return transpose_cached(dtype, n, perm, size, outer_a, outer_b, alpha, A, beta, B, B, stream);
}

ttx_status ttx_transpose_c(ttx_dtype dtype, int n, const int* perm, const int64_t* size,
                           const int64_t* outer_a, const int64_t* outer_b, const double* alpha,
                           const void* A, const double* beta, void* B, hipStream_t stream) {
    if (!alpha || !beta) return fail(TTX_EINVAL, "alpha and beta must not be NULL");
    return transpose_cached(dtype, n, perm, size, outer_a, outer_b, Scalar(alpha[0], alpha[1]), A,
                            Scalar(beta[0], beta[1]), B, B, stream);
}

ttx_status ttx_set_auto_specialise(int calls) {
    if (calls < 0) return fail(TTX_EINVAL, "calls must be >= 0");
    g_auto_calls.store(calls, std::memory_order_relaxed);
    return TTX_OK;
}

ttx_status ttx_transpose_cache_info(int* plans, int* specialised) {
    cache_info(plans, specialised);
    return TTX_OK;
}

ttx_status ttx_copy_kernel(const void* src, void* dst, int64_t bytes, hipStream_t stream) {
    if (!src || !dst || bytes < 0 || bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 ||
        reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(TTX_EINVAL, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
    if (bytes == 0) return TTX_OK;
    hipError_t e = launch_copy16(src, dst, bytes, stream);
    return e == hipSuccess ? TTX_OK : fail(TTX_EHIP, hipGetErrorString(e));
}

ttx_status ttx_axpby_kernel(ttx_dtype dtype, int64_t n, double alpha, const void* x, double beta,
                            void* y, hipStream_t stream) {
    if ((dtype != TTX_F32 && dtype != TTX_F64) || n < 0 || !x || !y ||
        reinterpret_cast<uintptr_t>(x) % 16 || reinterpret_cast<uintptr_t>(y) % 16)
        return fail(TTX_EINVAL, "axpby needs a valid dtype and 16-byte aligned pointers");
    if (n == 0) return TTX_OK;
    hipError_t e = launch_axpby(dtype, n, alpha, x, beta, y, stream);
    return e == hipSuccess ? TTX_OK : fail(TTX_EHIP, hipGetErrorString(e));
}

}  // extern "C"
