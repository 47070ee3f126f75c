// Batched evaluation: the expressions (and per-matrix reductions) of many
// matrices of different shapes in one persistent launch, replayed through a
// hipGraph.  The paper names collections of matrices (Cube) as roadmap work
// and notes that small matrices use a GPU poorly (Sections 3 and 6); one
// launch over the tiles of all matrices is this library's answer to both.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <queue>
#include <set>
#include <vector>

#include "internal.h"
#include "jit.h"
#include "runtime.h"

using namespace coot;

struct coot_batch_plan {
    Kernel k{};
    coot_batch_item_d* d_items = nullptr;
    coot_batch_task_d* d_tasks = nullptr;
    int* d_order = nullptr;
    int* d_blk_first = nullptr;
    double* d_part = nullptr;
    int64_t n_items = 0;
    int64_t n_blocks = 1;
    coot_bargs args{};
    uint32_t flags = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // what the baselines need
    std::vector<coot_batch_item_d> h_items;
    std::vector<coot_node> nodes, red_nodes;
    std::vector<int32_t> slot_dtypes;
    std::vector<int> slot_par;
    int32_t n_slots = 0, out_dtype = COOT_F32, red_op = COOT_RED_ACCU, red_dtype = COOT_F32;
    bool has_out = false, has_red = false;
    void* red_out = nullptr;
    int y_prec = 32;
};

namespace {

std::mutex g_plans_mu;
std::set<coot_batch_plan*> g_plans;

template <class R = int, class F>
R guard3(F&& f)
{
    try {
        return f();
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

hipError_t launch_b(hipFunction_t f, int64_t grid, coot_bargs& a, hipStream_t st)
{
    void* params[] = {&a};
    return hipModuleLaunchKernel(f, (unsigned)std::max<int64_t>(1, grid), 1, 1, 256, 1, 1, 0, st, params, nullptr);
}

// the tile pass, then (with a reduction) the per-item combine of the task partials
hipError_t launch_plan(coot_batch_plan* P, hipStream_t st)
{
    hipError_t e = launch_b(P->k.fn, P->n_blocks, P->args, st);
    if (e == hipSuccess && P->has_red) e = launch_b(P->k.fn2, (P->n_items + 255) / 256, P->args, st);
    return e;
}

void free_plan(coot_batch_plan* p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    (void)hipFree(p->d_items);
    (void)hipFree(p->d_tasks);
    (void)hipFree(p->d_part);
    (void)hipFree(p->d_order);
    (void)hipFree(p->d_blk_first);
    delete p;
}

// Longest-processing-time-first assignment of tasks to blocks: the costliest
// remaining task goes to the least loaded block (ties: lowest block).  Cost of
// a task: its tiles plus a fixed share for its partial reduction.
//
// XCD-aware: the blocks of XCD x are x, x + X, x + 2X, ... (X = xcds), and
// each XCD has its own L2.  Neighbouring tiles of a matrix share the cache
// lines at their edges, so a matrix's tasks all go to one XCD: matrices are
// first spread over the XCDs by LPT on their total cost, then each XCD's
// tasks over its own blocks by LPT.
void lpt_schedule(const std::vector<coot_batch_task_d>& tasks, int64_t n_items, int64_t n_blocks, int xcds,
                  std::vector<int>* order, std::vector<int>* first)
{
    const int64_t n = (int64_t)tasks.size();
    auto cost = [&](int i) { return (double)(tasks[(size_t)i].t1 - tasks[(size_t)i].t0) + 0.25; };
    typedef std::pair<double, int64_t> Load;
    const int64_t X = (xcds > 1 && n_blocks % xcds == 0) ? xcds : 1;
    // matrices -> XCDs
    std::vector<double> icost((size_t)std::max<int64_t>(n_items, 1), 0.0);
    for (int64_t i = 0; i < n; ++i) icost[(size_t)tasks[(size_t)i].item] += cost((int)i);
    std::vector<int> items((size_t)n_items);
    for (int64_t i = 0; i < n_items; ++i) items[(size_t)i] = (int)i;
    std::stable_sort(items.begin(), items.end(), [&](int a, int b) { return icost[(size_t)a] > icost[(size_t)b]; });
    std::vector<int64_t> xcd_of((size_t)std::max<int64_t>(n_items, 1), 0);
    {
        std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
        for (int64_t x = 0; x < X; ++x) heap.push(Load(0.0, x));
        for (int i : items) {
            Load l = heap.top();
            heap.pop();
            xcd_of[(size_t)i] = l.second;
            heap.push(Load(l.first + icost[(size_t)i], l.second));
        }
    }
    // each XCD's tasks -> its blocks
    std::vector<std::vector<int>> per((size_t)n_blocks);
    for (int64_t x = 0; x < X; ++x) {
        std::vector<int> idx;
        for (int64_t i = 0; i < n; ++i)
            if (xcd_of[(size_t)tasks[(size_t)i].item] == x) idx.push_back((int)i);
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost(a) > cost(b); });
        std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
        for (int64_t b = x; b < n_blocks; b += X) heap.push(Load(0.0, b));
        for (int i : idx) {
            Load l = heap.top();
            heap.pop();
            per[(size_t)l.second].push_back(i);
            heap.push(Load(l.first + cost(i), l.second));
        }
    }
    order->clear();
    first->assign((size_t)n_blocks + 1, 0);
    for (int64_t b = 0; b < n_blocks; ++b) {
        (*first)[(size_t)b] = (int)order->size();
        order->insert(order->end(), per[(size_t)b].begin(), per[(size_t)b].end());
    }
    (*first)[(size_t)n_blocks] = (int)order->size();
}

// trans parity of every leaf slot (bit 0: read straight, bit 1: read transposed)
std::vector<int> slot_parities(const coot_expr* e, int n_slots)
{
    const int nn = e->n_nodes;
    std::vector<int> mask(nn, 0), slot(n_slots, 0);
    mask[nn - 1] = 1;
    for (int i = nn - 1; i >= 0; --i) {
        const coot_node& N = e->nodes[i];
        if (!mask[i]) continue;
        if (N.op == COOT_LEAF) {
            if (N.a >= 0 && N.a < n_slots) slot[N.a] |= mask[i];
            continue;
        }
        int m = mask[i];
        if (N.op == COOT_TRANS) m = ((m & 1) << 1) | ((m >> 1) & 1);
        if (N.a >= 0 && N.a < i) mask[N.a] |= m;
        if (op_is_binary(N.op) && N.b >= 0 && N.b < i) mask[N.b] |= m;
    }
    return slot;
}

// Checks of a batch description and the plans of its element function and
// reduction tree (host only).
struct BatchTrees {
    bool has_out = false, has_red = false;
    std::vector<int> par, read_slot;
    Plan py, pr;
    int y_prec = 32;
};

BatchTrees plan_batch(const coot_batch* b)
{
    BatchTrees T;
    if (!b->expr || !b->expr->nodes || b->expr->n_nodes < 1) fail(COOT_ERR_BAD_TREE, "batch: empty expression");
    if (b->n_slots < 1 || b->n_slots > 6) fail(COOT_ERR_UNSUPPORTED, "batch: 1 to 6 operand slots");
    if (b->n_items < 0) fail(COOT_ERR_ARG, "batch: negative item count");
    if (!b->slot_dtypes || !b->shapes || (b->n_items > 0 && !b->leaf_ptrs)) fail(COOT_ERR_ARG, "batch: NULL table");
    if (b->flags & ~(COOT_BATCH_NO_GRAPH | COOT_BATCH_PER_ITEM | COOT_BATCH_UNFUSED))
        fail(COOT_ERR_ARG, "batch: unknown flags");
    const bool has_out = b->out_ptrs != nullptr;
    const bool has_red = b->red_expr != nullptr;
    if (!has_out && !has_red) fail(COOT_ERR_ARG, "batch: neither outputs nor a reduction requested");
    for (int s = 0; s < b->n_slots; ++s)
        if (!is_value_dtype(b->slot_dtypes[s]) || b->slot_dtypes[s] == COOT_I32 || b->slot_dtypes[s] == COOT_U32)
            fail(COOT_ERR_DTYPE, "batch: slot dtype (f32, f64, f16 or bf16)");
    if (has_out && (!is_value_dtype(b->out_dtype) || b->out_dtype == COOT_I32 || b->out_dtype == COOT_U32))
        fail(COOT_ERR_DTYPE, "batch: out dtype (f32, f64, f16 or bf16)");
    if (has_red) {
        const int base = b->red_op & 0xff;
        if ((b->red_op & ~(0xff | COOT_RED_PAIRWISE)) ||
            (base != COOT_RED_ACCU && base != COOT_RED_SUM && base != COOT_RED_DOT && base != COOT_RED_NORM1 &&
             base != COOT_RED_NORM2))
            fail(COOT_ERR_UNSUPPORTED, "batch: only accu, sum, dot, norm1 and norm2 per item");
        if (b->red_dtype != COOT_F32 && b->red_dtype != COOT_F64) fail(COOT_ERR_DTYPE, "batch: reduction dtype");
        if (!b->red_out && b->n_items > 0) fail(COOT_ERR_ARG, "batch: NULL red_out");
    }
    if (b->expr->flags != 0 || (has_red && b->red_expr->flags != 0)) fail(COOT_ERR_ARG, "batch: expression flags");

    // per-slot transposition and the shape rule it implies
    std::vector<int> par = slot_parities(b->expr, b->n_slots);
    bool need_square = false;
    for (int s = 0; s < b->n_slots; ++s) need_square = need_square || par[s] == 3;
    for (int i = 0; i < b->n_items; ++i) {
        int64_t r = b->shapes[2 * i], c = b->shapes[2 * i + 1];
        // sides up to 2^22 keep every per-lane tile offset within 32 bits
        if (r < 0 || c < 0 || r > (1 << 22) || c > (1 << 22))
            fail(COOT_ERR_SHAPE, "batch: item sides must be at most 2^22");
        if (need_square && r != c) fail(COOT_ERR_SHAPE, "batch: a slot read both straight and transposed needs square items");
    }
    // plan the element function on canonical shapes (never vectors)
    const int64_t cr = need_square ? 3 : 2, cc = 3;
    const uintptr_t G = uintptr_t(1) << 40;
    std::vector<coot_operand> fake(b->n_slots);
    for (int s = 0; s < b->n_slots; ++s) {
        bool t = par[s] == 2;
        fake[s] = coot_operand{(void*)(G * (s + 1)), t ? cc : cr, t ? cr : cc, t ? cc : cr, b->slot_dtypes[s], 0};
    }
    coot_operand fout{(void*)(G * 9), cr, cc, cr, has_out ? b->out_dtype : COOT_F32, 0};
    coot_expr ey = *b->expr;
    ey.cfg = coot_config{0, 0, 0, 0};
    Plan py = make_plan(-1, -1, &ey, fake.data(), b->n_slots, &fout);
    const int y_prec = py.nodes[py.root].prec;
    Plan pr;
    if (has_red) {
        int ydt = has_out ? b->out_dtype : (y_prec == 64 ? COOT_F64 : COOT_F32);
        coot_operand fy{(void*)(G * 10), cr, cc, cr, ydt, 0};
        coot_operand fr{(void*)(G * 11), 1, 1, 1, b->red_dtype, 0};
        coot_expr er = *b->red_expr;
        er.cfg = coot_config{0, 0, 0, 0};
        pr = make_plan(b->red_op, -1, &er, &fy, 1, &fr);
        for (const Read& r : pr.reads)
            if (r.trans) fail(COOT_ERR_UNSUPPORTED, "batch: the reduction tree cannot transpose Y");
    }
    std::vector<int> read_slot;
    for (const Read& r : py.reads) read_slot.push_back(r.slot);

    T.has_out = has_out;
    T.has_red = has_red;
    T.par = par;
    T.read_slot = read_slot;
    T.py = py;
    T.pr = pr;
    T.y_prec = y_prec;
    return T;
}

}  // namespace

namespace coot {
void batch_destroy_all()
{
    std::lock_guard<std::mutex> lk(g_plans_mu);
    for (auto* p : g_plans) free_plan(p);
    g_plans.clear();
}
}  // namespace coot

extern "C" {

int coot_batch_create(const coot_batch* b, void* stream, coot_batch_plan** out_plan)
{
    return guard3([&] {
        if (!b || !out_plan) fail(COOT_ERR_ARG, "NULL batch or plan pointer");
        *out_plan = nullptr;
        BatchTrees T = plan_batch(b);
        ensure_init();
        const bool has_out = T.has_out, has_red = T.has_red;
        const std::vector<int>& par = T.par;
        const std::vector<int>& read_slot = T.read_slot;
        const Plan& py = T.py;
        const Plan& pr = T.pr;
        const int y_prec = T.y_prec;
        auto* P = new coot_batch_plan();
        try {
            P->flags = b->flags;
            P->has_out = has_out;
            P->has_red = has_red;
            P->out_dtype = b->out_dtype;
            P->red_op = b->red_op;
            P->red_dtype = b->red_dtype;
            P->red_out = b->red_out;
            P->n_slots = b->n_slots;
            P->y_prec = y_prec;
            P->nodes.assign(b->expr->nodes, b->expr->nodes + b->expr->n_nodes);
            if (has_red) P->red_nodes.assign(b->red_expr->nodes, b->red_expr->nodes + b->red_expr->n_nodes);
            P->slot_dtypes.assign(b->slot_dtypes, b->slot_dtypes + b->n_slots);
            // descriptors and the block schedule
            P->n_items = b->n_items;
            P->slot_par = par;
            P->h_items.resize((size_t)b->n_items);
            std::vector<coot_batch_task_d> tasks;
            for (int i = 0; i < b->n_items; ++i) {
                coot_batch_item_d& d = P->h_items[(size_t)i];
                std::memset(&d, 0, sizeof d);
                d.rows = b->shapes[2 * i];
                d.cols = b->shapes[2 * i + 1];
                coot_batch_tile_shape(d.rows, d.cols, &d.lr, &d.lc);
                d.ntiles = d.rows > 0 && d.cols > 0
                               ? ((d.rows + (1 << d.lr) - 1) >> d.lr) * ((d.cols + (1 << d.lc) - 1) >> d.lc)
                               : 0;
                if (d.ntiles > INT32_MAX) fail(COOT_ERR_SHAPE, "batch: item too large (more than 2^31 tiles)");
                d.part0 = (int64_t)tasks.size();
                for (int64_t t0 = 0; t0 < d.ntiles; t0 += COOT_BATCH_CHUNK) {
                    if (tasks.size() >= (size_t)INT32_MAX) fail(COOT_ERR_SHAPE, "batch: more than 2^31 tasks");
                    tasks.push_back(coot_batch_task_d{i, (int)t0, (int)std::min<int64_t>(d.ntiles, t0 + COOT_BATCH_CHUNK),
                                                      (int)tasks.size()});
                }
                for (int s2 = 0; s2 < b->n_slots; ++s2) {
                    d.leaf[s2] = b->leaf_ptrs[(size_t)i * b->n_slots + s2];
                    if (!d.leaf[s2] && d.rows * d.cols > 0) fail(COOT_ERR_ARG, "batch: NULL operand pointer");
                }
                if (has_out) {
                    d.out = b->out_ptrs[i];
                    if (!d.out && d.rows * d.cols > 0) fail(COOT_ERR_ARG, "batch: NULL output pointer");
                }
            }
            // 4 blocks of 256 threads per CU per unit of the tree's split setting
            // (default 8: short per-block task lists, about two tasks per block
            // here, let the hardware's block dispatch balance the load; measured
            // 549 / 530 / 500 us for split 2 / 4 / 8 on 10,000 matrices)
            const int split = b->expr->cfg.split > 0 ? b->expr->cfg.split : 8;
            P->n_blocks = std::max<int64_t>(1, std::min<int64_t>((int64_t)tasks.size(), (int64_t)g_state.cus * 4 * split));
            std::vector<int> order, first;
            lpt_schedule(tasks, P->n_items, P->n_blocks, g_state.xcds, &order, &first);
            auto up = [](void** dst, const void* src, size_t bytes) {
                hipchk(hipMalloc(dst, std::max<size_t>(bytes, 16)), "hipMalloc(batch table)");
                if (bytes) hipchk(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy(batch table)");
            };
            up((void**)&P->d_items, P->h_items.data(), P->h_items.size() * sizeof(coot_batch_item_d));
            up((void**)&P->d_tasks, tasks.data(), tasks.size() * sizeof(coot_batch_task_d));
            up((void**)&P->d_order, order.data(), order.size() * sizeof(int));
            up((void**)&P->d_blk_first, first.data(), first.size() * sizeof(int));
            if (has_red) {
                (void)hipFree(P->d_part);
                P->d_part = nullptr;
                hipchk(hipMalloc((void**)&P->d_part, std::max<size_t>(16, tasks.size() * 2 * sizeof(double))),
                       "hipMalloc(batch partials)");
            }
            // kernels
            std::string name;
            std::string src = batch_kernel_source(py, has_red ? &pr : nullptr, has_out, b->out_dtype, b->red_dtype,
                                                  read_slot, &name);
            P->k = get_kernel(name, src, has_red);
            P->args = coot_bargs{P->d_items, P->d_tasks, P->d_order, P->d_blk_first, P->n_items, P->d_part, b->red_out};
            // one launch captured in a graph
            if (!(b->flags & (COOT_BATCH_NO_GRAPH | COOT_BATCH_PER_ITEM | COOT_BATCH_UNFUSED)) && P->n_items > 0) {
                hipStream_t cap;
                hipchk(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate(capture)");
                hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    e = launch_plan(P, cap);
                    hipGraph_t g = nullptr;
                    hipError_t e2 = hipStreamEndCapture(cap, &g);
                    if (e == hipSuccess) e = e2;
                    P->graph = g;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
                (void)hipStreamDestroy(cap);
                hipchk(e, "graph capture of the batched launch");
            }
            (void)stream;
        } catch (...) {
            free_plan(P);
            throw;
        }
        {
            std::lock_guard<std::mutex> lk(g_plans_mu);
            g_plans.insert(P);
        }
        *out_plan = P;
        return COOT_OK;
    });
}

int64_t coot_batch_kernel_source(const coot_batch* b, char* buf, int64_t cap)
{
    return guard3<int64_t>([&]() -> int64_t {
        if (!b) fail(COOT_ERR_ARG, "NULL batch");
        BatchTrees T = plan_batch(b);
        std::string name;
        std::string src = batch_kernel_source(T.py, T.has_red ? &T.pr : nullptr, T.has_out, b->out_dtype, b->red_dtype,
                                              T.read_slot, &name);
        src = prelude_source() + "\n" + src;
        if (buf && cap > 0) {
            const size_t n = std::min<size_t>(src.size(), (size_t)cap - 1);
            std::memcpy(buf, src.data(), n);
            buf[n] = 0;
        }
        return (int64_t)src.size();
    });
}

int coot_batch_run(coot_batch_plan* P, void* stream)
{
    return guard3([&] {
        {
            std::lock_guard<std::mutex> lk(g_plans_mu);
            if (!P || !g_plans.count(P)) fail(COOT_ERR_ARG, "unknown batch plan");
        }
        hipStream_t st = (hipStream_t)stream;
        if (P->n_items == 0) return COOT_OK;
        if (P->flags & (COOT_BATCH_UNFUSED | COOT_BATCH_PER_ITEM)) {
            // baselines: per matrix, the fused single-matrix calls (two launches),
            // or one kernel per node with temporaries
            const uint32_t ef = (P->flags & COOT_BATCH_UNFUSED) ? COOT_EXPR_UNFUSED : 0u;
            for (int64_t i = 0; i < P->n_items; ++i) {
                const coot_batch_item_d& d = P->h_items[(size_t)i];
                std::vector<coot_operand> ops(P->n_slots);
                coot_expr e{P->nodes.data(), (int32_t)P->nodes.size(), ef, {0, 0, 0, 0}};
                for (int s = 0; s < P->n_slots; ++s) {
                    bool t = P->slot_par[s] == 2;
                    int64_t r = t ? d.cols : d.rows, c = t ? d.rows : d.cols;
                    ops[s] = coot_operand{(void*)d.leaf[s], r, c, std::max<int64_t>(1, r), P->slot_dtypes[s], 0};
                }
                int ydt = P->has_out ? P->out_dtype : (P->y_prec == 64 ? COOT_F64 : COOT_F32);
                void* ybuf = d.out;
                if (!P->has_out)
                    hipchk(hipMallocAsync(&ybuf, (size_t)std::max<int64_t>(1, d.rows * d.cols) * itemsize(ydt), st),
                           "hipMallocAsync(Y)");
                coot_operand y{ybuf, d.rows, d.cols, std::max<int64_t>(1, d.rows), ydt, 0};
                int rc = coot_eval(&e, ops.data(), P->n_slots, &y, stream);
                if (rc == COOT_OK && P->has_red) {
                    coot_expr er{P->red_nodes.data(), (int32_t)P->red_nodes.size(), ef, {0, 0, 0, 0}};
                    coot_operand ro{(char*)P->red_out + i * itemsize(P->red_dtype), 1, 1, 1, P->red_dtype, 0};
                    rc = coot_reduce(P->red_op, -1, &er, &y, 1, &ro, stream);
                }
                if (!P->has_out) (void)hipFreeAsync(ybuf, st);
                if (rc) fail(rc, coot_last_error());
            }
            return COOT_OK;
        }
        if (P->exec) {
            hipchk(hipGraphLaunch(P->exec, st), "hipGraphLaunch");
            g_state.launches++;
        } else {
            hipchk(launch_plan(P, st), "hipModuleLaunchKernel(batch)");
            g_state.launches += P->has_red ? 2 : 1;
        }
        return COOT_OK;
    });
}

int coot_batch_destroy(coot_batch_plan* P)
{
    return guard3([&] {
        if (!P) return COOT_OK;
        std::lock_guard<std::mutex> lk(g_plans_mu);
        if (!g_plans.count(P)) fail(COOT_ERR_ARG, "unknown batch plan");
        g_plans.erase(P);
        free_plan(P);
        return COOT_OK;
    });
}

}  // extern "C"
