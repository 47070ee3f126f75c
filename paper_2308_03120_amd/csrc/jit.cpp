// Run-time compilation of generated kernels with hipRTC for gfx950, with an
// in-memory table and an on-disk code-object cache.  The paper's library
// compiles its kernels at start-up for the device it finds and caches them in
// ~/.bandicoot (Section 3); here kernels are compiled per expression on first
// use and cached the same way, keyed by the full source and compile options.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "jit.h"

namespace coot {

static const char* kOpts[] = {
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
};

JitStats g_jit_stats;

static std::mutex g_mu;
static std::unordered_map<std::string, Kernel> g_mem;  // key: module name
static std::string g_cache_dir;

static std::string default_cache_dir()
{
    const char* e = getenv("COOT_CACHE_DIR");
    if (e && *e) return e;
    const char* x = getenv("XDG_CACHE_HOME");
    if (x && *x) return std::string(x) + "/coot_mi355x";
    const char* h = getenv("HOME");
    if (h && *h) return std::string(h) + "/.cache/coot_mi355x";
    return "/tmp/coot_mi355x";
}

static void mkdirs(const std::string& d)
{
    std::string cur;
    std::stringstream ss(d);
    std::string part;
    if (!d.empty() && d[0] == '/') cur = "/";
    while (std::getline(ss, part, '/')) {
        if (part.empty()) continue;
        cur += part + "/";
        mkdir(cur.c_str(), 0755);
    }
}

const std::string& cache_dir()
{
    if (g_cache_dir.empty()) {
        g_cache_dir = default_cache_dir();
        mkdirs(g_cache_dir);
    }
    return g_cache_dir;
}

static uint64_t options_hash()
{
    static uint64_t h = 0;
    if (!h) {
        std::string s = prelude_source();
        for (const char* o : kOpts) s += o;
        int maj = 0, mnr = 0;
        hiprtcVersion(&maj, &mnr);
        s += std::to_string(maj) + "." + std::to_string(mnr);
        h = fnv1a(s);
    }
    return h;
}

static std::string path_of(const std::string& name) { return cache_dir() + "/" + name + "_" + hex64(options_hash()) + ".co"; }

static bool read_file(const std::string& p, std::vector<char>* out)
{
    std::ifstream f(p, std::ios::binary);
    if (!f) return false;
    f.seekg(0, std::ios::end);
    std::streamsize n = f.tellg();
    if (n <= 16) return false;
    f.seekg(0);
    out->resize((size_t)n);
    f.read(out->data(), n);
    // an ELF code object starts with 0x7f 'E' 'L' 'F'; anything else is corrupt
    return f.good() && (*out)[0] == 0x7f && (*out)[1] == 'E' && (*out)[2] == 'L' && (*out)[3] == 'F';
}

static void write_file_atomic(const std::string& p, const std::vector<char>& data)
{
    std::string tmp = p + ".tmp" + std::to_string(getpid());
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f) return;
        f.write(data.data(), (std::streamsize)data.size());
    }
    rename(tmp.c_str(), p.c_str());
}

// compile `src` (prelude + body) to a code object
static std::vector<char> compile(const std::string& name, const std::string& body)
{
    if (getenv("COOT_FAULT") && std::string(getenv("COOT_FAULT")) == "jit")
        fail(COOT_ERR_JIT, "kernel compilation disabled by COOT_FAULT=jit");
    auto t0 = std::chrono::steady_clock::now();
    std::string src = prelude_source() + "\n" + body;
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), (name + ".hip").c_str(), 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        fail(COOT_ERR_JIT, "hiprtcCreateProgram failed");
    hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof kOpts / sizeof kOpts[0]), kOpts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        fail(COOT_ERR_JIT, "compilation of " + name + " failed:\n" + log.substr(0, 4000));
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    std::vector<char> code(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    g_jit_stats.compiles++;
    g_jit_stats.seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return code;
}

// ---- grouped compilation: many kernels in one code object ------------------
// Each kernel body is wrapped in a namespace of its own (its helper functions
// have the same names in every body); the entry points keep their C names.  A
// small index file per kernel names the module file that holds it.
static bool g_collect = false;
static std::vector<std::pair<std::string, std::string>> g_pending;
static std::unordered_map<std::string, hipModule_t> g_modules;  // module path -> loaded module

static std::string index_of(const std::string& name) { return cache_dir() + "/" + name + "_" + hex64(options_hash()) + ".idx"; }

static bool cached(const std::string& name)
{
    std::ifstream a(path_of(name)), b(index_of(name));
    return (bool)a || (bool)b;
}

int precompile_kernel(const std::string& name, const std::string& body)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (cached(name)) return 0;
    if (g_collect) {
        for (auto& kv : g_pending)
            if (kv.first == name) return 0;
        g_pending.emplace_back(name, body);
        return 1;
    }
    std::vector<char> code = compile(name, body);
    write_file_atomic(path_of(name), code);
    return 1;
}

void precompile_begin()
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_collect = true;
    g_pending.clear();
}

int precompile_end(int per_module)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_collect = false;
    if (per_module < 1) per_module = 1;
    int done = 0;
    for (size_t s = 0; s < g_pending.size(); s += (size_t)per_module) {
        size_t e = std::min(g_pending.size(), s + (size_t)per_module);
        std::string body, names;
        for (size_t i = s; i < e; ++i) {
            body += "namespace k" + std::to_string(i - s) + " {\n" + g_pending[i].second + "\n}\n";
            names += g_pending[i].first + ";";
        }
        std::string mod = "coot_mod_" + hex64(fnv1a(names));
        std::vector<char> code = compile(mod, body);
        std::string mpath = path_of(mod);
        write_file_atomic(mpath, code);
        for (size_t i = s; i < e; ++i) {
            std::string idx = mpath.substr(mpath.find_last_of('/') + 1);
            write_file_atomic(index_of(g_pending[i].first), std::vector<char>(idx.begin(), idx.end()));
            ++done;
        }
    }
    g_pending.clear();
    return done;
}

Kernel get_kernel(const std::string& name, const std::string& body, bool has_comb)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_mem.find(name);
    if (it != g_mem.end()) {
        g_jit_stats.mem_hits++;
        return it->second;
    }
    std::vector<char> code;
    std::string p = path_of(name);
    // a kernel compiled together with others lives in a shared module
    {
        std::ifstream ix(index_of(name));
        std::string mfile;
        if (ix && std::getline(ix, mfile) && !mfile.empty() && mfile.find('/') == std::string::npos) {
            std::string mpath = cache_dir() + "/" + mfile;
            hipModule_t m = nullptr;
            auto mi = g_modules.find(mpath);
            if (mi != g_modules.end()) {
                m = mi->second;
            } else if (read_file(mpath, &code) && hipModuleLoadData(&m, code.data()) == hipSuccess) {
                g_modules[mpath] = m;
            } else {
                (void)hipGetLastError();
                m = nullptr;
            }
            Kernel k;
            if (m && hipModuleGetFunction(&k.fn, m, name.c_str()) == hipSuccess) {
                k.mod = m;
                k.fn2 = nullptr;
                if (!has_comb || hipModuleGetFunction(&k.fn2, m, (name + "_comb").c_str()) == hipSuccess) {
                    g_jit_stats.disk_hits++;
                    g_mem[name] = k;
                    return k;
                }
            }
            (void)hipGetLastError();
            code.clear();
        }
    }
    if (read_file(p, &code)) {
        g_jit_stats.disk_hits++;
    } else {
        code = compile(name, body);
        write_file_atomic(p, code);
    }
    Kernel k;
    if (hipModuleLoadData(&k.mod, code.data()) != hipSuccess) {
        // a stale or damaged cache file: rebuild once from source
        (void)hipGetLastError();
        code = compile(name, body);
        write_file_atomic(p, code);
        hipError_t e = hipModuleLoadData(&k.mod, code.data());
        if (e != hipSuccess) fail(COOT_ERR_HIP, std::string("hipModuleLoadData: ") + hipGetErrorString(e));
    }
    hipError_t e = hipModuleGetFunction(&k.fn, k.mod, name.c_str());
    if (e != hipSuccess) fail(COOT_ERR_HIP, std::string("hipModuleGetFunction: ") + hipGetErrorString(e));
    k.fn2 = nullptr;
    if (has_comb) {
        e = hipModuleGetFunction(&k.fn2, k.mod, (name + "_comb").c_str());
        if (e != hipSuccess) fail(COOT_ERR_HIP, std::string("hipModuleGetFunction(comb): ") + hipGetErrorString(e));
    }
    g_mem[name] = k;
    return k;
}

bool find_loaded_kernel(const std::string& name, bool has_comb, Kernel* k)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_mem.find(name);
    if (it == g_mem.end() || (has_comb && !it->second.fn2)) return false;
    *k = it->second;
    return true;
}

void jit_unload_all()
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_mem) {
        bool shared = false;
        for (auto& m : g_modules) shared = shared || m.second == kv.second.mod;
        if (!shared) (void)hipModuleUnload(kv.second.mod);
    }
    for (auto& m : g_modules) (void)hipModuleUnload(m.second);
    g_mem.clear();
    g_modules.clear();
}

}  // namespace coot
