// Allocation-free reduction entry point.
//
// coot_reduce keeps its block partials in per-stream device memory that it
// allocates on first use.  Callers that cannot allocate (code under HIP graph
// capture, serving loops, harnesses that forbid hipMalloc) call
// coot_reduce_noalloc instead: the same plan, kernels and launches, with the
// partials in one static device array per GPU.  Host code never passes the
// array's name to a kernel: at set-up the array's device address is looked up
// once per device and kept, and only that address is used afterwards.
#include <hip/hip_runtime.h>

#include <new>
#include <string>

#include "internal.h"
#include "runtime.h"

namespace coot {

// partials of every coot_reduce_noalloc call on this GPU (kept until the
// process ends; calls that overlap on one GPU race on it)
static __device__ __align__(256) unsigned char scratch[COOT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices];          // device address of `scratch`, per device
std::string g_scratch_err[kMaxDevices];    // why the lookup failed, if it did
}  // namespace

// Called by the device set-up with `device` current.  A failure is kept and
// reported by the entry point (it does not fail coot_init).
void noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices || g_scratch_dev[device]) return;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        g_scratch_err[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return;
    }
    g_scratch_dev[device] = p;
}

}  // namespace coot

using namespace coot;

extern "C" int coot_reduce_noalloc(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                                   const coot_operand* out, void* stream)
{
    try {
        if (red_op < 0) fail(COOT_ERR_ARG, "red_op must be a COOT_RED_* value");
        if (!g_state.init) fail(COOT_ERR_NOT_INIT, "coot_init has not been called");
        int dev = -1;
        hipchk(hipGetDevice(&dev), "hipGetDevice");
        if (dev < 0 || dev >= kMaxDevices || !g_scratch_dev[dev]) {
            std::string why = (dev >= 0 && dev < kMaxDevices) ? g_scratch_err[dev] : std::string();
            fail(why.empty() ? COOT_ERR_NOT_INIT : COOT_ERR_HIP,
                 why.empty() ? "coot_init has not been called on device " + std::to_string(dev) : why);
        }
        if (expr && (expr->flags & COOT_EXPR_UNFUSED))
            fail(COOT_ERR_ARG, "the unfused form needs temporaries: not available without allocation");
        Plan p = make_plan_cached(red_op, dim, expr, ops, n_ops, out);
        if (out->flags & COOT_OPERAND_HOST) fail(COOT_ERR_ARG, "the allocation-free entry point needs a device output");
        const int64_t n_out = p.dim < 0 ? 1 : (p.dim == 0 ? p.cols : p.rows);
        if (n_out == 0) return COOT_OK;
        if (p.temp_needed)
            fail(COOT_ERR_ARG, "a per-dimension reduction of a tree that reads an operand transposed needs a "
                               "temporary: not available without allocation");
        const FixedScratch fx{g_scratch_dev[dev], (size_t)COOT_NOALLOC_SCRATCH_BYTES};
        run_plan(p, choose_config_noalloc(p, expr->cfg), ops, out, (hipStream_t)stream, &fx);
        return COOT_OK;
    } catch (const Error& e) {
        set_error(e.code, e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error(COOT_ERR_NOMEM, "out of host memory");
        return COOT_ERR_NOMEM;
    } catch (const std::exception& e) {
        set_error(COOT_ERR_ARG, e.what());
        return COOT_ERR_ARG;
    }
}
