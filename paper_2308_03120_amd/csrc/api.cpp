// C ABI entry points: device state, scratch memory, launches.
//
// The paper's runtime layer is a singleton (coot_rt_t) of static functions on
// raw device memory that hides the backend (Section 7).  This file plays that
// role for one HIP backend: it turns a validated plan into a kernel launch on
// the caller's stream, owns per-stream scratch memory for the reductions, and
// implements the two baselines the fused form is measured against (one kernel
// per node with temporaries; a reduction of a materialised value).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "jit.h"
#include "runtime.h"

namespace coot {

static thread_local std::string t_err;

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }
void set_error(int, const std::string& msg) { t_err = msg; }

State g_state;

template <class F>
static int guard(F&& f)
{
    try {
        return f();
    } catch (const Error& e) {
        t_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        t_err = "out of host memory";
        return COOT_ERR_NOMEM;
    } catch (const std::exception& e) {
        t_err = e.what();
        return COOT_ERR_ARG;
    }
}

void hipchk(hipError_t e, const char* what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? COOT_ERR_NOMEM : COOT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}

static void init_device(int device, unsigned flags)
{
    std::lock_guard<std::mutex> lk(g_state.mu);
    if (g_state.init && g_state.device == device) return;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
        (void)hipGetLastError();
        fail(COOT_ERR_HIP, "no HIP device available");
    }
    if (device < 0 || device >= n) fail(COOT_ERR_ARG, "device index out of range");
    hipchk(hipSetDevice(device), "hipSetDevice");
    noalloc_setup(device);
    hipDeviceProp_t prop;
    hipchk(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    g_state.device = device;
    g_state.cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    g_state.name = prop.name;
    g_state.arch = prop.gcnArchName;
    // gfx950 (MI355X): 8 XCDs of 32 CUs, each with its own L2; the dispatcher
    // hands consecutive workgroups to the XCDs in turn
    g_state.xcds = g_state.arch.compare(0, 6, "gfx950") == 0 ? 8 : 1;
    g_state.hbm = prop.totalGlobalMem;
    g_state.clock_khz = prop.clockRate;
    // temporaries of the unfused and materialising paths come from the
    // stream-ordered pool; keep freed blocks in it instead of unmapping them
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    g_state.init = true;
    if (flags & COOT_PRINT_INFO) {
        printf("coot: device %d: %s (%s), %d CUs, %.0f MHz, %.1f GiB HBM, kernel cache %s\n", device, prop.name,
               prop.gcnArchName, g_state.cus, prop.clockRate / 1000.0, prop.totalGlobalMem / 1073741824.0,
               cache_dir().c_str());
        fflush(stdout);
    }
}

void ensure_init()
{
    if (g_state.init) return;
    int d = 0;
    hipchk(hipGetDevice(&d), "hipGetDevice");
    init_device(d, 0);
}

Scratch& scratch_for(hipStream_t st, size_t part_bytes, size_t res_bytes)
{
    std::lock_guard<std::mutex> lk(g_state.mu);
    Scratch& s = g_state.scratch[st];
    if (s.part_bytes < part_bytes) {
        if (s.part) {
            hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
            (void)hipFree(s.part);
            s.part = nullptr;
        }
        size_t want = std::max<size_t>(part_bytes, 1 << 20);
        hipchk(hipMalloc(&s.part, want), "hipMalloc(scratch)");
        s.part_bytes = want;
    }
    if (s.res_bytes < res_bytes) {
        if (s.res) {
            hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
            (void)hipFree(s.res);
            s.res = nullptr;
        }
        size_t want = std::max<size_t>(res_bytes, 4096);
        hipchk(hipMalloc(&s.res, want), "hipMalloc(result)");
        s.res_bytes = want;
    }
    return s;
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// split 1, 2, 4: split * (1024 / block) blocks per CU (a persistent, grid-stride
// launch); split 8: one pass, as many blocks as the work needs.
int64_t grid_cap(const LaunchCfg& c)
{
    if (c.split >= 8) return INT64_C(1) << 40;
    return (int64_t)g_state.cus * c.split * std::max(1, 1024 / c.block);
}

void launch(hipFunction_t f, int64_t grid, int block, coot_kargs& a, hipStream_t st)
{
    if (grid < 1) grid = 1;
    if (grid > 0x7fffffff) fail(COOT_ERR_ARG, "grid too large");
    void* params[] = {&a};
    hipchk(hipModuleLaunchKernel(f, (unsigned)grid, 1, 1, (unsigned)block, 1, 1, 0, st, params, nullptr),
           "hipModuleLaunchKernel");
    g_state.launches++;
}

// Size class of a call for the tuned and model caches: kernel signature,
// floor(log2) of the element count and of the row count (the shape decides
// the grid of the per-dimension kinds).
std::string tune_key(const Plan& p)
{
    auto lg2 = [](int64_t v) {
        int lg = 0;
        while (lg < 62 && (int64_t(1) << (lg + 1)) <= v) ++lg;
        return lg;
    };
    return std::to_string(p.kind) + "|" + std::to_string(p.ve) + "|" + std::to_string(p.red_op) + "|" +
           std::to_string(p.pairwise) + "|" + std::to_string(p.dim) + "|" + std::to_string(p.tile_lr) + "," +
           std::to_string(p.tile_lc) + "|t" + std::to_string(p.thin_k) + (p.thin_rows ? "r" : "c") + "|" +
           std::to_string(p.out_dtype) + "|" +
           p.body_sig + "|n" + std::to_string(lg2(p.n)) + "|r" + std::to_string(lg2(p.rows));
}

LaunchCfg choose_config(const Plan& p, const coot_config& user)
{
    if (user.ept) return LaunchCfg{user.ept, user.block, user.split};
    if (g_state.tune_mode != COOT_TUNE_DEFAULT) {
        std::lock_guard<std::mutex> lk(g_state.mu);
        auto it = g_state.tuned.find(tune_key(p));
        if (it != g_state.tuned.end()) return config_of(it->second);
    }
    if (g_state.tune_mode == COOT_TUNE_MODEL && g_state.model_ok) {
        int idx = model_pick(p);
        if (idx >= 0) return config_of(idx);
    }
    return default_config(p);
}

// choose_config without running the learned model (no kernel launch, no
// synchronisation): the caller's, a tuned or an already-predicted
// configuration, else the default
LaunchCfg choose_config_noalloc(const Plan& p, const coot_config& user)
{
    if (user.ept) return LaunchCfg{user.ept, user.block, user.split};
    if (g_state.tune_mode != COOT_TUNE_DEFAULT) {
        std::lock_guard<std::mutex> lk(g_state.mu);
        auto it = g_state.tuned.find(tune_key(p));
        if (it != g_state.tuned.end()) return config_of(it->second);
    }
    if (g_state.tune_mode == COOT_TUNE_MODEL && g_state.model_ok) {
        int idx = model_cached_pick(p);
        if (idx >= 0) return config_of(idx);
    }
    return default_config(p);
}

// grid, block and second-launch details for a plan
struct Geometry {
    int64_t grid;
    int block;
    int64_t splits;
    int64_t comb_grid;
    size_t part_bytes;
    int64_t aux;
};

static Geometry geometry(const Plan& p, const LaunchCfg& c)
{
    Geometry G{1, c.block, 1, 0, 0, 0};
    const int64_t cap = grid_cap(c);
    switch (p.kind) {
    case K_EW_FLAT:
    case K_RED_FLAT: {
        int64_t nv = p.n / p.ve;
        G.grid = std::max<int64_t>(1, std::min(ceil_div(nv, (int64_t)c.block * c.ept), cap));
        if (p.kind == K_RED_FLAT) G.grid = std::min<int64_t>(G.grid, 16384);
        break;
    }
    case K_EW_TILED:
    case K_RED_TILED: {
        if (p.thin_k) {
            // groups of thin_v long-side positions, 8 / K groups per thread in flight
            const int64_t ng = (p.thin_rows ? p.cols : p.rows) / p.thin_v;
            const int64_t need = std::max<int64_t>(1, ceil_div(ng, 256 * std::max(1, 8 / p.thin_k)));
            G.block = 256;
            G.grid = std::min(need, c.split >= 8 ? need : (int64_t)g_state.cus * c.split * 2);
            break;
        }
        int64_t nt = ceil_div(p.rows, int64_t(1) << p.tile_lr) * ceil_div(p.cols, int64_t(1) << p.tile_lc);
        G.block = 256;
        G.grid = std::max<int64_t>(1, std::min(nt, c.split >= 8 ? nt : (int64_t)g_state.cus * c.split * 2));
        break;
    }
    case K_RED_COL: {
        // enough waves to stream: cut few long columns into row segments
        const int64_t target = (int64_t)g_state.cus * 16;
        int64_t S = 1;
        if (p.cols < target) {
            S = ceil_div(target, std::max<int64_t>(1, p.cols));
            S = std::min<int64_t>(S, std::max<int64_t>(1, p.rows / (64 * p.ve * 4)));
            S = std::min<int64_t>(S, 4096);
        }
        int64_t seg = ceil_div(p.rows, S);
        seg = ceil_div(seg, p.ve) * p.ve;  // segments start on a vector boundary
        S = std::max<int64_t>(1, ceil_div(p.rows, seg));
        G.splits = S;
        G.aux = seg;
        G.grid = std::max<int64_t>(1, std::min(ceil_div(p.cols * S * 64, c.block), cap));
        if (S > 1) {
            G.comb_grid = std::min<int64_t>(p.cols, (int64_t)g_state.cus * 16);
            G.part_bytes = (size_t)(p.cols * S) * red_partial_bytes(p.red_op);
        }
        break;
    }
    case K_RED_COLT:
        G.grid = std::max<int64_t>(1, std::min(ceil_div(p.cols, c.block), cap));
        break;
    case K_RED_ROW: {
        // work units along the rows: vector groups of ve rows plus the leftover rows
        const int64_t units = p.rows / p.ve + p.rows % p.ve;
        int64_t target = (int64_t)g_state.cus * 1024;
        int64_t q = std::max<int64_t>(1, ceil_div(target, std::max<int64_t>(1, units)));
        // every split walks at least 64 columns (partials stay a small
        // fraction of the data)
        q = std::min<int64_t>(q, std::min<int64_t>(std::max<int64_t>(1, p.cols / 64), 65536));
        G.splits = q;
        G.grid = std::max<int64_t>(1, std::min(ceil_div(units * q, c.block), cap));
        if (q > 1) {
            // the combine kernel takes a block per row from 256 splits on, a
            // block per 64 rows from 16, else a thread per row
            const int64_t per_block = q >= 256 ? 1 : (q >= 16 ? 64 : 256);
            G.comb_grid = std::max<int64_t>(1, std::min<int64_t>(ceil_div(p.rows, per_block), (int64_t)g_state.cus * 16));
            G.part_bytes = (size_t)(p.rows * q) * red_partial_bytes(p.red_op);
        }
        break;
    }
    }
    if (p.kind == K_RED_FLAT || p.kind == K_RED_TILED) G.part_bytes = (size_t)G.grid * red_partial_bytes(p.red_op);
    return G;
}

// Identity of what the 64 launch configurations run: FNV-1a over the device
// prelude and, for a fixed set of calls covering every kernel kind, each
// configuration's generated source and launch geometry.  A cost model timed
// on other kernels (or another geometry) gets another stamp.
uint64_t kernel_stamp()
{
    const uintptr_t G = uintptr_t(1) << 40;
    auto op = [&](int k, int64_t r, int64_t c, int dt) {
        return coot_operand{(void*)(G * (uintptr_t)k), r, c, std::max<int64_t>(1, r), dt, 0, {0.0, 0.0}};
    };
    // x, y leaves; z = sqrt(abs(x)) % y - x / (1 + abs(y)); trans(x) + 0.5 y; x % y
    const coot_node z_tree[] = {{COOT_LEAF, 0, -1, 0, 0.0},       {COOT_ABS, 0, -1, 0, 0.0},
                                {COOT_SQRT, 1, -1, 0, 0.0},       {COOT_LEAF, 1, -1, 0, 0.0},
                                {COOT_SCHUR, 2, 3, 0, 0.0},       {COOT_ABS, 3, -1, 0, 0.0},
                                {COOT_SCAL_PLUS, 5, -1, 0, 1.0},  {COOT_DIV, 0, 6, 0, 0.0},
                                {COOT_MINUS, 4, 7, 0, 0.0}};
    const coot_node t_tree[] = {{COOT_LEAF, 0, -1, 0, 0.0},
                                {COOT_TRANS, 0, -1, 0, 0.0},
                                {COOT_LEAF, 1, -1, 0, 0.0},
                                {COOT_SCAL_TIMES, 2, -1, 0, 0.5},
                                {COOT_PLUS, 1, 3, 0, 0.0}};
    const coot_node p_tree[] = {{COOT_LEAF, 0, -1, 0, 0.0}, {COOT_LEAF, 1, -1, 0, 0.0}, {COOT_SCHUR, 0, 1, 0, 0.0}};
    struct Call {
        int red, dim;
        const coot_node* nodes;
        int nn;
        int64_t r, c;
        int dt;
        bool trans;
    };
    const Call calls[] = {
        {-1, -1, z_tree, 9, 1 << 24, 1, COOT_F32, false},  {-1, -1, z_tree, 9, 1 << 24, 1, COOT_F64, false},
        {-1, -1, z_tree, 9, 1 << 24, 1, COOT_BF16, false}, {COOT_RED_DOT, -1, p_tree, 3, 1 << 24, 1, COOT_F32, false},
        {COOT_RED_ACCU, -1, p_tree, 3, 1 << 24, 1, COOT_F16, false},
        {-1, -1, t_tree, 5, 4096, 4096, COOT_F32, true},  {-1, -1, t_tree, 5, 2, 1 << 22, COOT_F32, true},
        {COOT_RED_ACCU, -1, t_tree, 5, 4096, 4096, COOT_F32, true},
        {COOT_RED_SUM, 0, p_tree, 3, 4096, 4096, COOT_F32, false}, {COOT_RED_SUM, 0, p_tree, 3, 8, 1 << 16, COOT_F32, false},
        {COOT_RED_SUM, 1, p_tree, 3, 4096, 4096, COOT_F32, false}, {COOT_RED_SUM, 1, p_tree, 3, 1 << 20, 3, COOT_F64, false},
    };
    uint64_t h = fnv1a(prelude_source());
    auto mix = [&](const std::string& t) { h = fnv1a(hex64(h) + t); };
    for (const Call& k : calls) {
        coot_operand ops[2] = {k.trans ? op(1, k.c, k.r, k.dt) : op(1, k.r, k.c, k.dt), op(2, k.r, k.c, k.dt)};
        const int64_t orows = k.red < 0 ? k.r : (k.dim == 0 ? 1 : (k.dim == 1 ? k.r : 1));
        const int64_t ocols = k.red < 0 ? k.c : (k.dim == 0 ? k.c : 1);
        const int odt = k.red < 0 ? k.dt : (k.dt == COOT_F64 ? COOT_F64 : COOT_F32);
        coot_operand out = op(3, orows, ocols, odt);
        out.ld = std::max<int64_t>(1, orows);
        coot_expr e{k.nodes, k.nn, 0, {0, 0, 0, 0}};
        Plan p = make_plan(k.red, k.dim, &e, ops, 2, &out);
        // the generated text depends on the configuration only through ept
        std::unordered_map<int, uint64_t> src_hash;
        for (int i = 0; i < COOT_N_CONFIGS; ++i) {
            LaunchCfg c = normalise_config(p, config_of(i));
            auto it = src_hash.find(c.ept);
            if (it == src_hash.end()) it = src_hash.emplace(c.ept, fnv1a(kernel_source(p, c, nullptr, nullptr))).first;
            Geometry g = geometry(p, c);
            mix(hex64(it->second) + "|" + std::to_string(g.grid) + "," + std::to_string(g.block) +
                "," + std::to_string(g.splits) + "," + std::to_string(g.comb_grid) + "," + std::to_string(g.aux) +
                "," + std::to_string(i == config_index(default_config(p))));
        }
    }
    return h;
}

static void fill_reads(const Plan& p, const coot_operand* ops, coot_kargs& a)
{
    for (size_t j = 0; j < p.reads.size(); ++j) {
        a.leaf[j] = ops[p.reads[j].slot].ptr;
        a.ld[j] = p.reads[j].ld;
    }
}

// Rows by which the 64 x 64 tile grid starts above the value, so that column
// segments begin on 128-byte lines: a segment of a column that starts e
// elements into a line spans whole lines when the tiles start at rows
// 64k - e, instead of sharing its first and last line with the neighbouring
// tiles.  The output decides (a line written by two tiles costs far more
// than a line read by two: a 16383^2 FP32 view scaled into a view one
// element off its lines took 800 us, against 506 us with the read side
// misaligned and 410 us with neither); a reduction follows the majority of
// its reads in the value's order.  Operands whose column stride is not a
// multiple of 128 bytes have no common phase and do not vote.

// One fused launch (two for split per-row reductions) of a plan.
// kernels by plan signature: a repeated call skips source generation
static std::mutex g_sig_mu;
static std::unordered_map<std::string, Kernel> g_sig_kernels;

static std::string sig_key(const Plan& p, const LaunchCfg& c)
{
    return std::to_string(p.kind) + "|" + std::to_string(p.ve) + "|" + std::to_string(c.ept) + "|" +
           std::to_string(p.out_dtype) + "|" + std::to_string(p.red_op) + "|" + std::to_string(p.pairwise) + "|" +
           std::to_string(p.alias_out) + "|" + std::to_string(p.tile_gen) + std::to_string(p.tile_off32) + std::to_string(p.tile_tall) + std::to_string(p.tile_v4) + "c" + std::to_string(p.tile_cached) +
           std::to_string(p.tile_lr) + "," + std::to_string(p.tile_lc) + "|t" + std::to_string(p.thin_k) +
           (p.thin_rows ? "r" : "c") + std::to_string(p.thin_v) + "v" + std::to_string(p.thin_vec) + "|" + p.body_sig;
}

// loaded_only: never compile or load a module (the allocation-free entry
// point); a kernel not yet resident fails with COOT_ERR_NOT_READY
static Kernel kernel_for(const Plan& p, const LaunchCfg& c, bool loaded_only = false)
{
    std::string key = sig_key(p, c);
    {
        std::lock_guard<std::mutex> lk(g_sig_mu);
        auto it = g_sig_kernels.find(key);
        if (it != g_sig_kernels.end()) return it->second;
    }
    std::string name;
    std::string src = kernel_source(p, c, &name, nullptr);
    const bool comb = p.kind == K_RED_ROW || p.kind == K_RED_COL || p.kind == K_RED_FLAT || p.kind == K_RED_TILED;
    Kernel k;
    if (loaded_only) {
        if (!find_loaded_kernel(name, comb, &k))
            fail(COOT_ERR_NOT_READY, "the kernel of this call (" + name +
                                         ") is not loaded yet: make the same call once through coot_reduce first");
    } else {
        k = get_kernel(name, src, comb);
    }
    std::lock_guard<std::mutex> lk(g_sig_mu);
    g_sig_kernels[key] = k;
    return k;
}

void forget_kernels()
{
    std::lock_guard<std::mutex> lk(g_sig_mu);
    g_sig_kernels.clear();
}

void run_plan(const Plan& p, const LaunchCfg& cfg_in, const coot_operand* ops, const coot_operand* out,
              hipStream_t st, const FixedScratch* fixed)
{
    LaunchCfg c = normalise_config(p, cfg_in);
    Kernel k = kernel_for(p, c, fixed != nullptr);
    Geometry G = geometry(p, c);
    coot_kargs a;
    std::memset(&a, 0, sizeof a);
    fill_reads(p, ops, a);
    a.rows = p.rows;
    a.cols = p.cols;
    a.n = p.n;
    a.splits = G.splits;
    a.aux = G.aux;
    if ((p.kind == K_EW_TILED || p.kind == K_RED_TILED) && !p.thin_k) {
        if (!p.tile_gen || p.tile_tall) a.aux = p.tile_sh;
    }
    if (p.red_op < 0) {
        a.out = out->ptr;
        a.ld_out = out->ld;
        launch(k.fn, G.grid, G.block, a, st);
        return;
    }
    const int64_t n_out = p.dim < 0 ? 1 : (p.dim == 0 ? p.cols : p.rows);
    const bool host = (out->flags & COOT_OPERAND_HOST) != 0;
    const size_t res_bytes = (size_t)n_out * 8;
    if (fixed) {
        if (host) fail(COOT_ERR_ARG, "the allocation-free entry point needs a device output");
        if (G.part_bytes > fixed->bytes)
            fail(COOT_ERR_ARG, "the call needs " + std::to_string(G.part_bytes) + " bytes of partials, more than the " +
                                   std::to_string(fixed->bytes) + " bytes of the static scratch array");
        a.part = fixed->ptr;
        a.res = out->ptr;
    } else {
        Scratch& s = scratch_for(st, G.part_bytes, host ? res_bytes : 0);
        a.part = s.part;
        a.res = host ? s.res : out->ptr;
    }
    if (p.kind == K_RED_FLAT || p.kind == K_RED_TILED) {
        // pass 1 leaves one partial per block; pass 2 (one block) combines them
        a.splits = G.grid;
        launch(k.fn, G.grid, G.block, a, st);
        launch(k.fn2, 1, 256, a, st);
    } else {
        launch(k.fn, G.grid, G.block, a, st);
        if ((p.kind == K_RED_ROW || p.kind == K_RED_COL) && G.splits > 1) launch(k.fn2, G.comb_grid, 256, a, st);
    }
    if (host) {
        hipchk(hipMemcpyAsync(out->ptr, a.res, res_bytes / 8 * (size_t)itemsize(out->dtype), hipMemcpyDeviceToHost, st),
               "hipMemcpyAsync");
        hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
    }
}

// device temporaries for the unfused and materialising paths
struct Temp {
    void* p = nullptr;
    hipStream_t st = nullptr;
    Temp() = default;
    Temp(const Temp&) = delete;
    ~Temp()
    {
        if (p) (void)hipFreeAsync(p, st);
    }
    void alloc(size_t bytes, hipStream_t s)
    {
        st = s;
        hipchk(hipMallocAsync(&p, std::max<size_t>(bytes, 16), s), "hipMallocAsync(temporary)");
    }
};

static int do_eval(const coot_expr* expr, const coot_operand* ops, int n_ops, const coot_operand* out, hipStream_t st);
static int do_reduce(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                     const coot_operand* out, hipStream_t st);

// The paper's evaluation order: every node's apply() runs its own kernel and
// writes a temporary (Section 7).  Used as the unfused baseline.
static int run_unfused(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                       const coot_operand* out, hipStream_t st)
{
    const int nn = expr->n_nodes;
    std::vector<coot_operand> val(nn);
    std::vector<Temp> tmp(nn);
    // shapes and precisions of the user's nodes
    std::vector<int64_t> R(nn), C(nn);
    std::vector<int> prec(nn);
    for (int i = 0; i < nn; ++i) {
        const coot_node& N = expr->nodes[i];
        if (N.op == COOT_LEAF) {
            val[i] = ops[N.a];
            R[i] = ops[N.a].n_rows;
            C[i] = ops[N.a].n_cols;
            prec[i] = dtype_prec(ops[N.a].dtype);
            continue;
        }
        R[i] = N.op == COOT_TRANS ? C[N.a] : R[N.a];
        C[i] = N.op == COOT_TRANS ? R[N.a] : C[N.a];
        prec[i] = N.op == COOT_CONV ? dtype_prec(N.b) : prec[N.a];
        bool last = i == nn - 1;
        coot_node mini[3];
        int m = 0, nops = 0;
        coot_operand mops[2];
        mini[m++] = coot_node{COOT_LEAF, 0, -1, 0, 0.0};
        mops[nops++] = val[N.a];
        int bidx = -1;
        if (op_is_binary(N.op)) {
            mini[m++] = coot_node{COOT_LEAF, 1, -1, 0, 0.0};
            mops[nops++] = val[N.b];
            bidx = 1;
        }
        mini[m] = coot_node{N.op, 0, N.op == COOT_CONV ? N.b : bidx, 0, N.k};
        m++;
        coot_expr me{mini, m, 0, expr->cfg};
        if (last && red_op < 0) return do_eval(&me, mops, nops, out, st);
        int dt = prec[i] == 64 ? COOT_F64 : COOT_F32;
        if (N.op == COOT_CONV && (N.b == COOT_F16 || N.b == COOT_BF16)) dt = N.b;
        tmp[i].alloc((size_t)(R[i] * C[i]) * itemsize(dt), st);
        val[i] = coot_operand{tmp[i].p, R[i], C[i], std::max<int64_t>(1, R[i]), dt, 0};
        int rc = do_eval(&me, mops, nops, &val[i], st);
        if (rc) return rc;
    }
    if (red_op < 0) {  // the root is a leaf: plain copy through a one-node kernel
        coot_node one{COOT_LEAF, 0, -1, 0, 0.0};
        coot_expr me{&one, 1, 0, expr->cfg};
        return do_eval(&me, &val[nn - 1], 1, out, st);
    }
    int base = red_op & 0xff;
    int flags = red_op & COOT_RED_PAIRWISE;
    if (base == COOT_RED_DOT) base = COOT_RED_ACCU;
    coot_node one{COOT_LEAF, 0, -1, 0, 0.0};
    coot_expr me{&one, 1, 0, expr->cfg};
    return do_reduce(base | flags, dim, &me, &val[nn - 1], 1, out, st);
}

static int do_eval(const coot_expr* expr, const coot_operand* ops, int n_ops, const coot_operand* out, hipStream_t st)
{
    Plan p = make_plan_cached(-1, -1, expr, ops, n_ops, out);
    ensure_init();
    if (expr->flags & COOT_EXPR_UNFUSED) return run_unfused(-1, -1, expr, ops, n_ops, out, st);
    if (p.n == 0) return COOT_OK;
    run_plan(p, choose_config(p, expr->cfg), ops, out, st);
    return COOT_OK;
}

static int do_reduce(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                     const coot_operand* out, hipStream_t st)
{
    Plan p = make_plan_cached(red_op, dim, expr, ops, n_ops, out);
    ensure_init();
    if (expr->flags & COOT_EXPR_UNFUSED) return run_unfused(red_op, dim, expr, ops, n_ops, out, st);
    const int64_t n_out = p.dim < 0 ? 1 : (p.dim == 0 ? p.cols : p.rows);
    if (n_out == 0) return COOT_OK;
    if (p.temp_needed) {
        // per-dimension reduction of a tree that reads an operand transposed:
        // materialise the value once, then reduce it
        Temp t;
        int dt = p.root_prec == 64 ? COOT_F64 : COOT_F32;
        t.alloc((size_t)p.n * itemsize(dt), st);
        coot_operand tv{t.p, p.rows, p.cols, std::max<int64_t>(1, p.rows), dt, 0};
        coot_expr e2 = *expr;
        e2.flags = 0;
        int rc = do_eval(&e2, ops, n_ops, &tv, st);
        if (rc) return rc;
        coot_node one{COOT_LEAF, 0, -1, 0, 0.0};
        coot_expr me{&one, 1, 0, expr->cfg};
        return do_reduce(red_op == COOT_RED_DOT ? COOT_RED_ACCU : red_op, dim, &me, &tv, 1, out, st);
    }
    run_plan(p, choose_config(p, expr->cfg), ops, out, st);
    return COOT_OK;
}

}  // namespace coot

using namespace coot;

extern "C" {

int coot_init(int device, unsigned flags)
{
    return guard([&] {
        init_device(device, flags);
        return COOT_OK;
    });
}

int coot_finalize(void)
{
    return guard([&] {
        if (!g_state.init) return COOT_OK;
        (void)hipDeviceSynchronize();
        {
            std::lock_guard<std::mutex> lk(g_state.mu);
            for (auto& kv : g_state.scratch) {
                if (kv.second.part) (void)hipFree(kv.second.part);
                if (kv.second.res) (void)hipFree(kv.second.res);
            }
            g_state.scratch.clear();
        }
        batch_destroy_all();
        forget_kernels();
        jit_unload_all();
        g_state.init = false;
        return COOT_OK;
    });
}

int coot_eval(const coot_expr* expr, const coot_operand* ops, int n_ops, const coot_operand* out, void* stream)
{
    return guard([&] { return do_eval(expr, ops, n_ops, out, (hipStream_t)stream); });
}

int coot_reduce(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                const coot_operand* out, void* stream)
{
    return guard([&] {
        if (red_op < 0) fail(COOT_ERR_ARG, "red_op must be a COOT_RED_* value");
        return do_reduce(red_op, dim, expr, ops, n_ops, out, (hipStream_t)stream);
    });
}

int coot_synchronise(void* stream)
{
    return guard([&] {
        hipchk(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
        return COOT_OK;
    });
}

const char* coot_last_error(void) { return t_err.c_str(); }

int coot_validate(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                  const coot_operand* out)
{
    return guard([&] {
        make_plan(red_op, dim, expr, ops, n_ops, out);
        return COOT_OK;
    });
}

int64_t coot_kernel_source(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                           const coot_operand* out, char* buf, int64_t cap)
{
    int64_t result = 0;
    int rc = guard([&] {
        Plan p = make_plan(red_op, dim, expr, ops, n_ops, out);
        LaunchCfg c = expr->cfg.ept ? LaunchCfg{expr->cfg.ept, expr->cfg.block, expr->cfg.split} : default_config(p);
        std::string src = prelude_source() + "\n" + kernel_source(p, normalise_config(p, c), nullptr, nullptr);
        if (buf && cap > 0) {
            int64_t m = std::min<int64_t>(cap - 1, (int64_t)src.size());
            std::memcpy(buf, src.data(), (size_t)m);
            buf[m] = '\0';
        }
        result = (int64_t)src.size();
        return COOT_OK;
    });
    return rc ? rc : result;
}

// every fused kernel a call launches (two for a per-dimension reduction of a
// tree that reads an operand transposed: the tree into a temporary, then the
// reduction of the temporary)
static int precompile_call(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                           const coot_operand* out)
{
    Plan p = make_plan(red_op, dim, expr, ops, n_ops, out);
    LaunchCfg c = expr->cfg.ept ? LaunchCfg{expr->cfg.ept, expr->cfg.block, expr->cfg.split} : default_config(p);
    if (p.temp_needed) {
        int dt = p.root_prec == 64 ? COOT_F64 : COOT_F32;
        // a stand-in address far from every operand (only alignment matters here)
        coot_operand tv{(void*)(uintptr_t(1) << 46), p.rows, p.cols, std::max<int64_t>(1, p.rows), dt, 0};
        coot_expr e2 = *expr;
        e2.flags = 0;
        int n = precompile_call(-1, -1, &e2, ops, n_ops, &tv);
        coot_node one{COOT_LEAF, 0, -1, 0, 0.0};
        coot_expr me{&one, 1, 0, expr->cfg};
        return n + precompile_call(red_op == COOT_RED_DOT ? COOT_RED_ACCU : red_op, dim, &me, &tv, 1, out);
    }
    std::string name;
    std::string src = kernel_source(p, normalise_config(p, c), &name, nullptr);
    return precompile_kernel(name, src);
}

int coot_precompile(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                    const coot_operand* out)
{
    return guard([&] { return precompile_call(red_op, dim, expr, ops, n_ops, out); });
}

int coot_default_config(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                        const coot_operand* out)
{
    return guard([&] {
        Plan p = make_plan(red_op, dim, expr, ops, n_ops, out);
        return config_index(default_config(p));
    });
}

int coot_precompile_begin(void)
{
    return guard([&] {
        precompile_begin();
        return COOT_OK;
    });
}

int coot_precompile_end(int kernels_per_module)
{
    return guard([&] { return precompile_end(kernels_per_module); });
}

int coot_get_stats(coot_stats* s)
{
    return guard([&] {
        if (!s) fail(COOT_ERR_ARG, "stats is NULL");
        s->launches = g_state.launches;
        s->jit_compiles = g_jit_stats.compiles;
        s->jit_disk_hits = g_jit_stats.disk_hits;
        s->jit_mem_hits = g_jit_stats.mem_hits;
        s->jit_seconds = g_jit_stats.seconds;
        return COOT_OK;
    });
}

int coot_config_of(int index, coot_config* cfg)
{
    return guard([&] {
        if (index < 0 || index >= COOT_N_CONFIGS || !cfg) fail(COOT_ERR_ARG, "config index out of range");
        LaunchCfg c = config_of(index);
        *cfg = coot_config{c.ept, c.block, c.split, 0};
        return COOT_OK;
    });
}

}  // extern "C"
