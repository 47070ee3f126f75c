// Launch-configuration choice: the exhaustive autotuner, the features of a
// call, and the learned cost model (a 32-64-64 MLP run by the library's own
// HIP kernels).  The paper does not tune launches; this is the learned part
// of the method built on top of its expression-tree evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <mutex>
#include <vector>

#include "internal.h"
#include "runtime.h"

extern "C" int coot_copy_launch(void* dst, const void* src, int64_t bytes, int cus, void* stream);
extern "C" int coot_probe_launch(int kind, int shape, void* dst, const void* src, int64_t bytes, void* stream);
extern "C" int coot_mlp_forward_launch(const float* P, const float* X, int B, float* Y, float* Z1, float* H,
                                       void* stream);
extern "C" int coot_mlp_backward_launch(const float* P, const float* X, const float* T, const float* M, int B,
                                        float* grad, float* loss, float* ws, void* stream);
extern "C" int coot_mlp_adam_launch(float* w, const float* g, float* m, float* v, int n, int t, float lr, float b1,
                                    float b2, float eps, void* stream);

namespace coot {

// ------------------------------------------------------------------ features
void plan_features(const Plan& p, float* f)
{
    std::fill(f, f + COOT_N_FEATURES, 0.0f);
    auto l2 = [](double x) { return (float)std::log2(x + 1.0); };
    // depth of every node
    std::vector<int> depth(p.nodes.size(), 1);
    int n_ops = 0;
    int cnt_add = 0, cnt_mul = 0, cnt_div = 0, cnt_scal = 0, cnt_exp = 0, cnt_log = 0, cnt_sqrt = 0, cnt_abs = 0,
        cnt_conv = 0;
    double flops = 0.0;
    for (size_t i = 0; i < p.nodes.size(); ++i) {
        const PNode& n = p.nodes[i];
        int d = 1;
        if (n.op != COOT_LEAF && n.op != PN_GEN) {
            ++n_ops;
            d = 1 + depth[n.a];
            if (n.b >= 0 && n.op != COOT_CONV) d = std::max(d, 1 + depth[n.b]);
        }
        depth[i] = d;
        const double w64 = n.prec == 64 ? 2.0 : 1.0;
        switch (n.op) {
        case COOT_PLUS:
        case COOT_MINUS: ++cnt_add; flops += w64; break;
        case COOT_SCHUR: ++cnt_mul; flops += w64; break;
        case COOT_DIV: ++cnt_div; flops += 10 * w64; break;
        case COOT_EXP: ++cnt_exp; flops += 20 * w64; break;
        case COOT_LOG: ++cnt_log; flops += 20 * w64; break;
        case COOT_SQRT: ++cnt_sqrt; flops += 8 * w64; break;
        case COOT_ABS: ++cnt_abs; flops += w64; break;
        case COOT_CONV: ++cnt_conv; flops += 2; break;
        case COOT_SQUARE: ++cnt_mul; flops += w64; break;
        case COOT_LOG10:
        case COOT_LOG2: ++cnt_log; flops += 20 * w64; break;
        case COOT_EXP2:
        case COOT_SCAL_POW:
        case COOT_COS:
        case COOT_SIN:
        case COOT_TAN:
        case COOT_ACOS:
        case COOT_ASIN:
        case COOT_ATAN:
        case COOT_COSH:
        case COOT_SINH:
        case COOT_TANH: ++cnt_exp; flops += 20 * w64; break;
        case COOT_FLOOR:
        case COOT_CEIL:
        case COOT_ROUND:
        case COOT_TRUNC:
        case COOT_SIGN: ++cnt_abs; flops += w64; break;
        case COOT_LEAF: break;
        default: ++cnt_scal; flops += (n.op == COOT_SCAL_DIV_POST || n.op == COOT_SCAL_DIV_PRE ? 10 : 1) * w64; break;
        }
    }
    int bytes_el = 0, ntrans = 0;
    int dt[4] = {0, 0, 0, 0};
    for (const Read& r : p.reads) {
        bytes_el += itemsize(r.dtype);
        if (r.trans) ++ntrans;
        if (r.dtype >= 0 && r.dtype < 4) dt[r.dtype]++;
    }
    const bool red = p.red_op >= 0;
    if (!red) bytes_el += itemsize(p.out_dtype);
    const float nr = (float)std::max<size_t>(1, p.reads.size());
    f[0] = l2((double)p.n);
    f[1] = l2((double)p.rows);
    f[2] = l2((double)p.cols);
    f[3] = (float)n_ops;
    f[4] = (float)depth[p.root];
    f[5] = (float)p.reads.size();
    f[6] = (float)ntrans;
    for (int k = 0; k < 4; ++k) f[7 + k] = dt[k] / nr;
    f[11] = red ? 0.0f : (float)itemsize(p.out_dtype);
    f[12] = (float)bytes_el;
    f[13] = l2((double)p.n * bytes_el);
    f[14] = (float)cnt_add;
    f[15] = (float)cnt_mul;
    f[16] = (float)cnt_div;
    f[17] = (float)cnt_scal;
    f[18] = (float)cnt_exp;
    f[19] = (float)cnt_log;
    f[20] = (float)cnt_sqrt;
    f[21] = (float)cnt_abs;
    f[22] = (float)cnt_conv;
    f[23] = red ? 1.0f : 0.0f;
    bool sum = red && (p.red_op == COOT_RED_ACCU || p.red_op == COOT_RED_SUM || p.red_op == COOT_RED_DOT ||
                       p.red_op == COOT_RED_NORM1 || p.red_op == COOT_RED_NORM2);
    f[24] = sum ? 1.0f : 0.0f;
    f[25] = (red && !sum) ? 1.0f : 0.0f;
    f[26] = (red && p.dim == 0) ? 1.0f : 0.0f;
    f[27] = (red && p.dim == 1) ? 1.0f : 0.0f;
    f[28] = (p.kind == K_EW_FLAT || p.kind == K_RED_FLAT) ? 1.0f : 0.0f;
    f[29] = (p.kind == K_EW_TILED || p.kind == K_RED_TILED || p.temp_needed) ? 1.0f : 0.0f;
    f[30] = (float)p.ve;
    f[31] = (float)(flops / std::max(1, bytes_el));
}

// --------------------------------------------------------------- cost model
static hipStream_t g_model_stream = nullptr;
static float* g_model_dev = nullptr;  // params, then X[32], then Y[64]
static std::unordered_map<std::string, int> g_model_cache;

static void model_upload()
{
    ensure_init();
    if (!g_model_stream) hipchk(hipStreamCreateWithFlags(&g_model_stream, hipStreamNonBlocking), "hipStreamCreate");
    if (!g_model_dev)
        hipchk(hipMalloc((void**)&g_model_dev, (COOT_MLP_N_PARAMS + 32 + 64) * sizeof(float)), "hipMalloc(model)");
    hipchk(hipMemcpy(g_model_dev, g_state.model_params.data(), COOT_MLP_N_PARAMS * sizeof(float), hipMemcpyHostToDevice),
           "hipMemcpy(model)");
    g_model_cache.clear();
}

// index of the configuration with the smallest predicted time (GPU inference)
int model_cached_pick(const Plan& p)
{
    auto it = g_model_cache.find(tune_key(p));
    return it == g_model_cache.end() ? -1 : it->second;
}

int model_pick(const Plan& p)
{
    std::string key = tune_key(p);
    {
        auto it = g_model_cache.find(key);
        if (it != g_model_cache.end()) return it->second;
    }
    float f[COOT_N_FEATURES];
    plan_features(p, f);
    for (int k = 0; k < COOT_N_FEATURES; ++k)
        f[k] = (f[k] - g_state.feat_mean[k]) / (g_state.feat_std[k] > 0 ? g_state.feat_std[k] : 1.0f);
    float* X = g_model_dev + COOT_MLP_N_PARAMS;
    float* Y = X + 32;
    hipchk(hipMemcpyAsync(X, f, sizeof f, hipMemcpyHostToDevice, g_model_stream), "hipMemcpyAsync(features)");
    if (coot_mlp_forward_launch(g_model_dev, X, 1, Y, nullptr, nullptr, g_model_stream)) fail(COOT_ERR_HIP, "mlp forward");
    float y[64];
    hipchk(hipMemcpyAsync(y, Y, sizeof y, hipMemcpyDeviceToHost, g_model_stream), "hipMemcpyAsync(prediction)");
    hipchk(hipStreamSynchronize(g_model_stream), "hipStreamSynchronize(model)");
    int best = 0;
    for (int k = 1; k < 64; ++k)
        if (y[k] < y[best]) best = k;
    g_model_cache[key] = best;
    return best;
}

}  // namespace coot

using namespace coot;

namespace {
template <class F>
int guard2(F&& f)
{
    try {
        return f();
    } catch (const Error& e) {
        set_error(e.code, e.msg);
        return e.code;
    } catch (const std::exception& e) {
        set_error(COOT_ERR_ARG, e.what());
        return COOT_ERR_ARG;
    }
}
}  // namespace

extern "C" {

// Cost-model file: the 8 bytes "COOTMLP2", the feature schema (u32), a zero
// u32, the kernel stamp (u64), then the FP32 parameters, feature means and
// feature standard deviations.
static const char MODEL_MAGIC[8] = {'C', 'O', 'O', 'T', 'M', 'L', 'P', '2'};

int coot_set_tuning(int mode, const char* model_path)
{
    return guard2([&] {
        if (mode < COOT_TUNE_DEFAULT || mode > COOT_TUNE_MODEL) fail(COOT_ERR_ARG, "unknown tuning mode");
        if (mode == COOT_TUNE_MODEL && model_path && *model_path) {
            // a file that does not fit the library leaves the tuned cache, then the default
            auto reject = [&](const std::string& why) {
                g_state.model_ok = false;
                g_state.tune_mode = COOT_TUNE_CACHE;
                fail(COOT_ERR_ARG, std::string("cost model ") + model_path + " rejected (" + why +
                                       "); tuning falls back to the tuned cache, then the default");
            };
            std::ifstream in(model_path, std::ios::binary);
            if (!in) fail(COOT_ERR_ARG, std::string("cannot open model file ") + model_path);
            char magic[8] = {0};
            uint32_t schema = 0, zero = 1;
            uint64_t stamp = 0;
            in.read(magic, 8);
            in.read((char*)&schema, 4);
            in.read((char*)&zero, 4);
            in.read((char*)&stamp, 8);
            if (!in || std::memcmp(magic, MODEL_MAGIC, 8) != 0 || zero != 0)
                reject("not a stamped cost-model file");
            if (schema != COOT_FEATURE_SCHEMA)
                reject("feature schema " + std::to_string(schema) + ", the library's is " +
                       std::to_string(COOT_FEATURE_SCHEMA));
            const uint64_t mine = kernel_stamp();
            if (stamp != mine)
                reject("trained on kernels " + hex64(stamp) + ", the library's are " + hex64(mine) +
                       ": retrain it on these kernels");
            std::vector<float> buf(COOT_MLP_N_PARAMS + 64);
            in.read((char*)buf.data(), (std::streamsize)(buf.size() * sizeof(float)));
            if (in.gcount() != (std::streamsize)(buf.size() * sizeof(float)) || in.peek() != EOF)
                reject("wrong size");
            g_state.model_params.assign(buf.begin(), buf.begin() + COOT_MLP_N_PARAMS);
            g_state.feat_mean.assign(buf.begin() + COOT_MLP_N_PARAMS, buf.begin() + COOT_MLP_N_PARAMS + 32);
            g_state.feat_std.assign(buf.begin() + COOT_MLP_N_PARAMS + 32, buf.end());
            g_state.model_ok = true;
            model_upload();
        }
        g_state.tune_mode = mode;
        return COOT_OK;
    });
}

int coot_kernel_stamp(uint64_t* stamp)
{
    return guard2([&] {
        if (!stamp) fail(COOT_ERR_ARG, "stamp is NULL");
        *stamp = kernel_stamp();
        return COOT_FEATURE_SCHEMA;
    });
}

int coot_model_set(const float* params, const float* mean, const float* sd)
{
    return guard2([&] {
        if (!params || !mean || !sd) fail(COOT_ERR_ARG, "NULL model array");
        g_state.model_params.assign(params, params + COOT_MLP_N_PARAMS);
        g_state.feat_mean.assign(mean, mean + 32);
        g_state.feat_std.assign(sd, sd + 32);
        g_state.model_ok = true;
        model_upload();
        return COOT_OK;
    });
}

int coot_model_choose(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                      const coot_operand* out)
{
    return guard2([&] {
        Plan p = make_plan(red_op, dim, expr, ops, n_ops, out);
        if (!g_state.model_ok) fail(COOT_ERR_ARG, "no cost model installed");
        return model_pick(p);
    });
}

int coot_features(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                  const coot_operand* out, float* features)
{
    return guard2([&] {
        if (!features) fail(COOT_ERR_ARG, "features is NULL");
        Plan p = make_plan(red_op, dim, expr, ops, n_ops, out);
        plan_features(p, features);
        return COOT_OK;
    });
}

int coot_autotune(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                  const coot_operand* out, int reps, float* times_ms, void* stream)
{
    return guard2([&] {
        if (!times_ms) fail(COOT_ERR_ARG, "times_ms is NULL");
        if (reps < 1 || reps > 1000) fail(COOT_ERR_ARG, "reps must be in [1, 1000]");
        Plan p = make_plan(red_op, dim, expr, ops, n_ops, out);
        if (expr->flags & COOT_EXPR_UNFUSED) fail(COOT_ERR_ARG, "autotune needs the fused form");
        if (out->flags & COOT_OPERAND_HOST) fail(COOT_ERR_ARG, "autotune needs a device output");
        ensure_init();
        hipStream_t st = (hipStream_t)stream;
        std::vector<hipEvent_t> ev(2 * reps);
        for (auto& e : ev) hipchk(hipEventCreate(&e), "hipEventCreate");
        int best = 0;
        // the per-dimension path of a transposed tree reduces a temporary
        std::function<void(const LaunchCfg&)> run = [&](const LaunchCfg& c) {
            coot_expr e2 = *expr;
            e2.cfg = coot_config{c.ept, c.block, c.split, 0};
            int rc = red_op >= 0 ? coot_reduce(red_op, dim, &e2, ops, n_ops, out, stream)
                                 : coot_eval(&e2, ops, n_ops, out, stream);
            if (rc) fail(rc, coot_last_error());
        };
        for (int idx = 0; idx < COOT_N_CONFIGS; ++idx) {
            LaunchCfg c = config_of(idx);
            run(c);  // compile + warm
            run(c);
            for (int r = 0; r < reps; ++r) {
                hipchk(hipEventRecord(ev[2 * r], st), "hipEventRecord");
                run(c);
                hipchk(hipEventRecord(ev[2 * r + 1], st), "hipEventRecord");
            }
            hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
            std::vector<float> t(reps);
            for (int r = 0; r < reps; ++r) hipchk(hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]), "hipEventElapsedTime");
            std::sort(t.begin(), t.end());
            times_ms[idx] = t[reps / 2];
            if (times_ms[idx] < times_ms[best]) best = idx;
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
        {
            std::lock_guard<std::mutex> lk(g_state.mu);
            g_state.tuned[tune_key(p)] = best;
        }
        return best;
    });
}

int coot_mlp_forward(const float* params, const float* X, int B, float* Y, float* ws, void* stream)
{
    return guard2([&] {
        if (!params || !X || !Y || B < 0) fail(COOT_ERR_ARG, "bad MLP arguments");
        ensure_init();
        float* Z1 = ws ? ws : nullptr;
        float* H = ws ? ws + (int64_t)B * 64 : nullptr;
        if (coot_mlp_forward_launch(params, X, B, Y, Z1, H, stream)) fail(COOT_ERR_HIP, "mlp forward launch");
        return COOT_OK;
    });
}

int coot_mlp_backward(const float* params, const float* X, const float* T, const float* M, int B, float* grad,
                      float* loss, float* ws, void* stream)
{
    return guard2([&] {
        if (!params || !X || !T || !M || !grad || !ws || B < 1) fail(COOT_ERR_ARG, "bad MLP arguments");
        ensure_init();
        if (coot_mlp_backward_launch(params, X, T, M, B, grad, loss, ws, stream)) fail(COOT_ERR_HIP, "mlp backward launch");
        return COOT_OK;
    });
}

int coot_mlp_adam(float* params, const float* grad, float* m, float* v, int n, int t, float lr, float beta1,
                  float beta2, float eps, void* stream)
{
    return guard2([&] {
        if (!params || !grad || !m || !v || n < 0 || t < 1) fail(COOT_ERR_ARG, "bad Adam arguments");
        ensure_init();
        if (coot_mlp_adam_launch(params, grad, m, v, n, t, lr, beta1, beta2, eps, stream)) fail(COOT_ERR_HIP, "adam launch");
        return COOT_OK;
    });
}

int coot_copy(void* dst, const void* src, int64_t bytes, void* stream)
{
    return guard2([&] {
        if (bytes < 0 || (bytes > 0 && (!dst || !src))) fail(COOT_ERR_ARG, "bad copy arguments");
        if (((uintptr_t)dst | (uintptr_t)src) & 15) fail(COOT_ERR_ARG, "copy needs 16-byte aligned pointers");
        ensure_init();
        if (bytes == 0) return COOT_OK;
        if (coot_copy_launch(dst, src, bytes, g_state.cus, stream)) fail(COOT_ERR_HIP, "copy launch");
        return COOT_OK;
    });
}

int coot_bandwidth_probe(int kind, void* dst, const void* src, int64_t bytes, void* stream)
{
    return guard2([&] {
        const int base = kind & 0xff, shape = kind >> 8;
        if (base < COOT_PROBE_COPY || base > COOT_PROBE_TILED_READ2_WRITE1) fail(COOT_ERR_ARG, "unknown probe kind");
        if (shape < 0 || shape > 3) fail(COOT_ERR_ARG, "unknown probe launch shape");
        if (bytes < 0 || bytes % 16) fail(COOT_ERR_ARG, "probe length must be a nonnegative multiple of 16 bytes");
        if (base >= COOT_PROBE_TILED_COPY && bytes % (INT64_C(4) << 20))
            fail(COOT_ERR_ARG, "a tiled probe's length must be a multiple of 4 MiB (64 columns of 16384 rows)");
        if (bytes > 0 && ((base != COOT_PROBE_WRITE && !src) || !dst)) fail(COOT_ERR_ARG, "NULL probe buffer");
        if (((uintptr_t)dst | (uintptr_t)src) & 15) fail(COOT_ERR_ARG, "probe needs 16-byte aligned pointers");
        ensure_init();
        if (bytes == 0) return COOT_OK;
        if (base == COOT_PROBE_COPY && shape == 0) {
            if (coot_copy_launch(dst, src, bytes, g_state.cus, stream)) fail(COOT_ERR_HIP, "copy launch");
        } else if (coot_probe_launch(base, shape, dst, src, bytes, stream)) {
            fail(COOT_ERR_HIP, "probe launch");
        }
        return COOT_OK;
    });
}

}  // extern "C"
