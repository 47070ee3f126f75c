// Device state shared by the entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace coot {

struct Scratch {
    void* part = nullptr;
    size_t part_bytes = 0;
    void* res = nullptr;
    size_t res_bytes = 0;
};

struct State {
    bool init = false;
    int device = -1;
    int cus = 256;
    int xcds = 8;         // L2 domains: consecutive block indices go to them in turn
    std::string name, arch;
    size_t hbm = 0;
    int clock_khz = 0;
    std::mutex mu;
    std::unordered_map<hipStream_t, Scratch> scratch;
    long long launches = 0;
    // launch-configuration choice
    int tune_mode = COOT_TUNE_DEFAULT;
    std::unordered_map<std::string, int> tuned;  // tune_key -> config index
    bool model_ok = false;
    std::vector<float> model_params, feat_mean, feat_std;
};

extern State g_state;

void hipchk(hipError_t e, const char* what);
void ensure_init();
Scratch& scratch_for(hipStream_t st, size_t part_bytes, size_t res_bytes);
int64_t grid_cap(const LaunchCfg& c);
void launch(hipFunction_t f, int64_t grid, int block, coot_kargs& a, hipStream_t st);
// device memory that stands in for the per-stream partials (allocation-free calls)
struct FixedScratch {
    void* ptr;
    size_t bytes;
};
void run_plan(const Plan& p, const LaunchCfg& cfg, const coot_operand* ops, const coot_operand* out, hipStream_t st,
              const FixedScratch* fixed = nullptr);
LaunchCfg choose_config(const Plan& p, const coot_config& user);
LaunchCfg choose_config_noalloc(const Plan& p, const coot_config& user);

// allocation-free entry point (noalloc.hip): look up the static scratch
// array's address on `device` (current)
void noalloc_setup(int device);
std::string tune_key(const Plan& p);
uint64_t kernel_stamp();  // host only: identity of the kernels and geometries of the 64 configurations

// cost model (tune.cpp)
int model_pick(const Plan& p);
int model_cached_pick(const Plan& p);  // an earlier prediction for p's size class, else -1

// batched plans (batched.cpp)
void batch_destroy_all();

}  // namespace coot
