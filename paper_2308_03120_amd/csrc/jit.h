// Run-time kernel compilation (hipRTC) and code-object cache.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

namespace coot {

struct Kernel {
    hipModule_t mod;
    hipFunction_t fn;
    hipFunction_t fn2;  // second entry point ("<name>_comb") when the kind has one
};

struct JitStats {
    long long compiles = 0;
    long long disk_hits = 0;
    long long mem_hits = 0;
    double seconds = 0.0;
};
extern JitStats g_jit_stats;

const std::string& cache_dir();

// Load (compiling on a cache miss) the module of `body` and its entry point(s).
Kernel get_kernel(const std::string& name, const std::string& body, bool has_comb);

// The kernel only if its module is already loaded (no compilation, no load).
bool find_loaded_kernel(const std::string& name, bool has_comb, Kernel* k);

// Compile into the disk cache only (no device needed).  1 = compiled, 0 = cached.
int precompile_kernel(const std::string& name, const std::string& body);

// Grouped compilation: between begin and end, precompile_kernel only collects;
// end compiles the collected kernels, per_module to a code object.
void precompile_begin();
int precompile_end(int per_module);

void jit_unload_all();

}  // namespace coot
