// Size-specialised kernels, compiled at run time with hipRTC.
//
// TTC generates a solution per transposition, with the sizes as template
// parameters so that trip counts are known at compile time (Sec. 2.1, the
// size-generic solution).  The pre-instantiated kernels here take every
// extent, stride, tile count and index divisor as run-time arguments; a
// specialised kernel is the same tile code compiled with the problem's
// TileArgsHost as a compile-time constant (run_specialised), so that the
// index arithmetic folds into immediates and loops over the merged indices
// unroll.  It computes exactly what the generic kernel computes (same tile,
// same operation order).
//
// The tile headers are embedded in the library at build time and handed to
// hipRTC as named headers.  Compiled kernels are cached for the process
// (per device) and, when TTX_JIT_CACHE names a directory, as code objects
// on disk keyed by a hash of the source, the options and the headers.
#include <hip/hiprtc.h>

#include <cerrno>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <sys/stat.h>
#include <unistd.h>

#include "ttx_internal.h"
#include "ttx_jit_headers.inc"   // kJitHeaderNames, kJitHeaderSources, kJitHeaderCount (generated)

namespace ttx {

struct JitKernel {
    int device;
    std::string key;
    std::string name;
    hipModule_t module;
    hipFunction_t fn;
    uint32_t dense_grid;   // dense tiles and pipelined grids: workgroups that fill the device with this kernel
};

static const char* const kJitOptions[] = {"-O3", "-std=c++17", "-ffp-contract=off", "-Xclang", "-target-feature",
                                          "-Xclang", "-packed-fp32-ops"};
static constexpr int kJitOptionCount = int(sizeof(kJitOptions) / sizeof(kJitOptions[0]));

static uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

// What a specialised kernel is compiled for: the tile kind and template
// parameters, the element types, the beta class, the kernel flags and the
// bytes of the problem-dependent arguments.
static std::string jit_key(const TiledLaunch& L) {
    const int head[] = {L.p.code,   L.kind,     L.va,        L.vb,           L.n0,
                        L.cap,      L.flags,    L.beta0 ? 1 : 0, L.c.tile_a, L.c.tile_b,
                        L.c.threads, config_pad(L.c), L.c.flags & (TTX_CFG_ALIGN_A | TTX_CFG_PIPELINED)};
    std::string k(reinterpret_cast<const char*>(head), sizeof(head));
    k.append(reinterpret_cast<const char*>(L.args), sizeof(TileArgsHost));
    return k;
}

// The kernel's name: kind, element types, beta class, tile shape, the
// workgroup size and LDS padding when they differ from the pre-compiled
// kernels' (256, 1), and a hash of the problem, so that profiles tell
// specialised kernels apart.
std::string jit_entry_name(const TiledLaunch& L) {
    static const char* const kKind[] = {"moved", "preserved", "staged", "dense"};
    auto type = [](int dtype) {
        std::string t = element_type_name(dtype);
        return t.rfind("ttx::", 0) == 0 ? t.substr(5) : t;
    };
    std::string n = std::string("ttx_jit_") + kKind[L.kind] + "_" + type(L.p.dtype);
    if (L.p.dtype_a != L.p.dtype) n += "_" + type(L.p.dtype_a);
    n += L.beta0 ? "_b0_" : "_b_";
    n += std::to_string(L.c.tile_a) + "x" + std::to_string(L.c.tile_b);
    if (L.c.threads != kThreads) n += "_t" + std::to_string(L.c.threads);
    if (config_pad(L.c) != 1) n += "_p" + std::to_string(config_pad(L.c));
    if (L.c.flags & TTX_CFG_ALIGN_A) n += "_al";
    if (L.c.flags & TTX_CFG_PIPELINED) n += "_pl";
    const std::string key = jit_key(L);
    char h[16];
    std::snprintf(h, sizeof(h), "_%08x", unsigned(fnv1a(key.data(), key.size()) & 0xffffffffu));
    return n + h;
}

std::string jit_source(const TiledLaunch& L) {
    const std::string T = element_type_name(L.p.dtype), S = element_type_name(L.p.dtype_a);
    const char* b0 = L.beta0 ? "true" : "false";
    char tile[224];
    int lds = 0, waves = 0;
    bool pipe = false;
    const int nt = L.c.threads, pad = config_pad(L.c);
    // the tiles, shared memory and occupancy hints of the generic kernels,
    // with the config's workgroup size and LDS row padding (store kind -1:
    // taken from the constant kernel flags)
    switch (L.kind) {
        case kTileMoved:
            std::snprintf(tile, sizeof(tile), "ttx::MovedTile<%s, %s, %d, %d, %d, %d, %s, -1, %d, %d, %d>", T.c_str(),
                          b0, L.c.tile_a, L.c.tile_b, L.va, L.vb, S.c_str(), nt, pad,
                          config_align_elems(L.c, elem_bytes(L.p.dtype_a)));
            lds = L.c.tile_b * (L.c.tile_a + pad);
            waves = (L.va == 1 || L.vb == 1) ? 4 : 1;
            break;
        case kTilePreserved:
            std::snprintf(tile, sizeof(tile), "ttx::PreservedTile<%s, %s, %d, %d, %d, %s, -1, %d>", T.c_str(), b0,
                          L.c.tile_a, L.c.tile_b, L.va, S.c_str(), nt);
            waves = L.va == 1 ? 4 : 1;
            break;
        case kTileStaged:
            std::snprintf(tile, sizeof(tile), "ttx::StagedTile<%s, %s, %d, %d, %d, %s, -1, %d, %d>", T.c_str(), b0,
                          L.n0, L.c.tile_a, L.c.tile_b, S.c_str(), nt, pad);
            lds = L.c.tile_b * (L.c.tile_a * L.n0 + pad);
            waves = 4;
            break;
        default:
            std::snprintf(tile, sizeof(tile), "ttx::DenseTile<%s, %s, %d, %s, -1, %d>", T.c_str(), b0, L.cap,
                          S.c_str(), nt);
            lds = 2 * L.cap;
            pipe = true;
    }
    if (L.c.flags & TTX_CFG_PIPELINED) pipe = true;   // a persistent grid: tiles overlap
    std::string s;
    s.reserve(8192);
    s += "// size-specialised transposition kernel\n#include \"tile_kernels.h\"\n\n";
    s += "namespace {\n// the bytes of the problem's ttx::TileArgsHost\nstruct Image {\n    unsigned char b[";
    s += std::to_string(sizeof(TileArgsHost)) + "];\n};\nconstexpr Image kImage = {{";
    char num[8];
    for (size_t i = 0; i < sizeof(TileArgsHost); ++i) {
        if (i % 24 == 0) s += "\n   ";
        std::snprintf(num, sizeof(num), " %u,", unsigned(L.args[i]));
        s += num;
    }
    s += "\n}};\nstatic_assert(sizeof(Image) == sizeof(ttx::TileArgsHost), \"argument layout\");\n";
    s += "constexpr ttx::TileArgsHost kHost = __builtin_bit_cast(ttx::TileArgsHost, kImage);\n}  // namespace\n\n";
    s += "extern \"C\" __global__ __launch_bounds__(" + std::to_string(nt) + ")";
    if (waves) s += " __attribute__((amdgpu_waves_per_eu(" + std::to_string(waves) + ")))";
    s += "\nvoid " + jit_entry_name(L) + "(ttx::TileArgs<" + T + ", " + S + "> a) {\n";
    if (lds)
        s += "    __shared__ " + T + " lds[" + std::to_string(lds) + "];\n";
    else
        s += "    " + T + "* const lds = nullptr;\n";
    s += "    ttx::run_specialised<" + std::string(tile) + ", " + (pipe ? "true" : "false") + ", kHost, " +
         std::to_string(L.flags) + ">(lds, a);\n}\n";
    return s;
}


static std::string device_arch(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

static std::string cache_file(const std::string& arch, const std::string& src) {
    const char* dir = std::getenv("TTX_JIT_CACHE");
    if (!dir || !*dir) return "";
    uint64_t h = fnv1a(arch.data(), arch.size());
    for (int i = 0; i < kJitOptionCount; ++i) h = fnv1a(kJitOptions[i], std::strlen(kJitOptions[i]) + 1, h);
    for (int i = 0; i < kJitHeaderCount; ++i) h = fnv1a(kJitHeaderSources[i], std::strlen(kJitHeaderSources[i]), h);
    h = fnv1a(src.data(), src.size(), h);
    char name[64];
    std::snprintf(name, sizeof(name), "/ttx-%016llx.co", static_cast<unsigned long long>(h));
    return std::string(dir) + name;
}

static bool read_file(const std::string& path, std::string* out) {
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    std::string data;
    char buf[65536];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) data.append(buf, n);
    const bool ok = !std::ferror(f);
    std::fclose(f);
    if (ok) *out = std::move(data);
    return ok && !out->empty();
}

static void write_file_atomic(const std::string& path, const std::string& data) {
    const std::string tmp = path + ".tmp." + std::to_string(getpid());
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;   // the disk cache is best effort
    const bool ok = std::fwrite(data.data(), 1, data.size(), f) == data.size();
    if (std::fclose(f) == 0 && ok && std::rename(tmp.c_str(), path.c_str()) == 0) return;
    std::remove(tmp.c_str());
}

// Compiles src for arch with hipRTC; *code receives the code object.
static ttx_status compile(const std::string& src, const std::string& arch, std::string* code) {
    hiprtcProgram prog;
    hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), "ttx_jit.hip", kJitHeaderCount,
                                         kJitHeaderSources, kJitHeaderNames);
    if (r != HIPRTC_SUCCESS) return fail(TTX_EHIP, std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r));
    std::vector<const char*> opts(kJitOptions, kJitOptions + kJitOptionCount);
    const std::string arch_opt = "--offload-arch=" + arch;
    opts.push_back(arch_opt.c_str());
    r = hiprtcCompileProgram(prog, int(opts.size()), opts.data());
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        std::string log;
        if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
            log.resize(n);
            if (hiprtcGetProgramLog(prog, &log[0]) != HIPRTC_SUCCESS) log.clear();
        }
        hiprtcDestroyProgram(&prog);
        if (log.size() > 2000) log.resize(2000);
        return fail(TTX_EHIP, std::string("hipRTC compilation failed: ") + log);
    }
    size_t n = 0;
    r = hiprtcGetCodeSize(prog, &n);
    if (r == HIPRTC_SUCCESS && n > 0) {
        code->resize(n);
        r = hiprtcGetCode(prog, &(*code)[0]);
    }
    hiprtcDestroyProgram(&prog);
    if (r != HIPRTC_SUCCESS || n == 0) return fail(TTX_EHIP, "hipRTC returned no code object");
    return TTX_OK;
}

static std::mutex g_jit_mu;
// Kernels live until the process ends (plans hold plain pointers to them).
static std::map<std::pair<int, std::string>, std::unique_ptr<JitKernel>> g_jit;

ttx_status jit_kernel(const TiledLaunch& L, const JitKernel** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(TTX_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    const std::string key = jit_key(L);
    std::lock_guard<std::mutex> lock(g_jit_mu);
    auto it = g_jit.find({dev, key});
    if (it != g_jit.end()) {
        *out = it->second.get();
        return TTX_OK;
    }
    const std::string arch = device_arch(dev);
    if (arch.empty()) return fail(TTX_EHIP, "cannot read the device architecture");
    const std::string src = jit_source(L);
    const std::string path = cache_file(arch, src);
    std::string code;
    const bool from_disk = !path.empty() && read_file(path, &code);
    if (!from_disk) {
        ttx_status st = compile(src, arch, &code);
        if (st != TTX_OK) return st;
        if (!path.empty()) {
            const char* dir = std::getenv("TTX_JIT_CACHE");
            if (mkdir(dir, 0777) == 0 || errno == EEXIST) write_file_atomic(path, code);
        }
    }
    std::unique_ptr<JitKernel> k(new JitKernel());
    k->device = dev;
    k->key = key;
    k->name = jit_entry_name(L);
    e = hipModuleLoadData(&k->module, code.data());
    if (e != hipSuccess && from_disk) {   // a damaged cache file: compile again
        ttx_status st = compile(src, arch, &code);
        if (st != TTX_OK) return st;
        write_file_atomic(path, code);
        e = hipModuleLoadData(&k->module, code.data());
    }
    if (e != hipSuccess) return fail(TTX_EHIP, std::string("hipModuleLoadData: ") + hipGetErrorString(e));
    e = hipModuleGetFunction(&k->fn, k->module, k->name.c_str());
    if (e != hipSuccess) {
        hipModuleUnload(k->module);
        return fail(TTX_EHIP, std::string("hipModuleGetFunction: ") + hipGetErrorString(e));
    }
    k->dense_grid = 0;
    if (L.kind == kTileDense || (L.c.flags & TTX_CFG_PIPELINED)) {
        int nb = 0, cus = 0;
        if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k->fn, L.c.threads, 0) != hipSuccess || nb <= 0)
            nb = 4;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        k->dense_grid = uint32_t(nb) * uint32_t(cus);
    }
    *out = k.get();
    g_jit[{dev, key}] = std::move(k);
    return TTX_OK;
}

const std::string& jit_name(const JitKernel& k) { return k.name; }

bool jit_matches(const JitKernel& k, const TiledLaunch& L) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != k.device) return false;
    return jit_key(L) == k.key;
}

hipError_t jit_launch(const JitKernel& k, const TiledLaunch& L, hipStream_t stream) {
    uint32_t grid = L.grid;
    if (L.kind == kTileDense || (L.c.flags & TTX_CFG_PIPELINED))
        grid = L.ntiles < k.dense_grid ? L.ntiles : k.dense_grid;
    void* params[] = {const_cast<unsigned char*>(L.args)};
    return hipModuleLaunchKernel(k.fn, grid, 1, 1, uint32_t(L.c.threads), 1, 1, 0, stream, params, nullptr);
}

}  // namespace ttx
