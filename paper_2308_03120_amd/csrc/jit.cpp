// Run-time compilation of generated kernels with hipRTC for gfx950, with an
// in-memory table and an on-disk code-object cache.  The paper's library
// compiles its kernels at start-up for the device it finds and caches them in
// ~/.bandicoot (Section 3); here kernels are compiled per expression on first
// use and cached the same way, keyed by the full source and compile options.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

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

int precompile_kernel(const std::string& name, const std::string& body)
{
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<char> code;
    std::string p = path_of(name);
    if (read_file(p, &code)) return 0;
    code = compile(name, body);
    write_file_atomic(p, code);
    return 1;
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

void jit_unload_all()
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_mem) (void)hipModuleUnload(kv.second.mod);
    g_mem.clear();
}

}  // namespace coot
