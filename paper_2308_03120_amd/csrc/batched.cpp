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
#include <string>
#include <vector>

#include "internal.h"
#include "jit.h"
#include "runtime.h"

using namespace coot;

struct coot_batch_plan {
    Kernel k{};
    coot_batch_item_d* d_items = nullptr;
    coot_batch_unit_d* d_units = nullptr;
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
    (void)hipFree(p->d_units);
    (void)hipFree(p->d_part);
    (void)hipFree(p->d_blk_first);
    delete p;
}

// Units of item `item` (Y_i of R x Cn) for units of at most E elements, in
// order (their partial slots follow this order):
//  - an item of at most E/4 elements whose staged rows fit a quarter of the
//    LDS stage is one unit (a small unit: a wave can run it);
//  - short columns (R <= E/32): units of whole columns, k >= 32 of them, the
//    item split into equal parts (contiguous runs of Y_i);
//  - long columns: 64-column blocks of E/64 rows.
// Every unit fits the stage: rc * (k + 1) <= E + E/32.
bool item_units(int item, int64_t R, int64_t Cn, int64_t E, std::vector<coot_batch_unit_d>* out)
{
    const int64_t n = R * Cn;
    if (n == 0) return false;
    const int64_t cap = coot_batch_stage_cap(E);
    auto push = [&](int64_t p0, int64_t q0, int64_t rc, int64_t k) {
        out->push_back(coot_batch_unit_d{item, (int)p0, (int)q0, (int)rc, (int)k, 0});
    };
    if (n <= E / 4 && R * (Cn | 1) <= cap / 4) {
        push(0, 0, R, Cn);
        return true;
    }
    if (R <= E / 32) {
        const int64_t kmax = E / R;
        const int64_t nq = (Cn + kmax - 1) / kmax;
        const int64_t k = (Cn + nq - 1) / nq;
        for (int64_t q0 = 0; q0 < Cn; q0 += k) push(0, q0, R, std::min(k, Cn - q0));
        return false;
    }
    const int64_t rc = E / 64, kc = 64;
    for (int64_t q0 = 0; q0 < Cn; q0 += kc)
        for (int64_t p0 = 0; p0 < R; p0 += rc) push(p0, q0, std::min(rc, R - p0), std::min(kc, Cn - q0));
    return false;
}

// Block schedule.  XCD-aware: blocks x, x + X, x + 2X, ... (X = xcds) run on
// XCD x, whose L2 the XCD's blocks share, so all units of an item go to one
// XCD (items spread over the XCDs longest first, each to the least loaded);
// an XCD runs its large items' units first, largest item first, each unit a
// block of its own, then its small units four to a block.  Shorter XCD lists
// are padded with empty blocks.  Returns the units in block order and each
// block's first unit.
void schedule_units(const std::vector<std::vector<coot_batch_unit_d>>& per_item, const std::vector<bool>& small,
                    int xcds, std::vector<coot_batch_unit_d>* units, std::vector<int>* first)
{
    const int64_t n_items = (int64_t)per_item.size();
    const int64_t X = std::max(1, xcds);
    auto cost = [&](int64_t i) {
        double c = 0.0;
        for (const auto& u : per_item[(size_t)i]) c += (double)u.rc * u.k + 256.0;
        return c;
    };
    std::vector<int64_t> items;
    std::vector<double> icost((size_t)n_items);
    for (int64_t i = 0; i < n_items; ++i) {
        icost[(size_t)i] = cost(i);
        if (!per_item[(size_t)i].empty()) items.push_back(i);
    }
    std::stable_sort(items.begin(), items.end(), [&](int64_t a, int64_t b) { return icost[(size_t)a] > icost[(size_t)b]; });
    typedef std::pair<double, int64_t> Load;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int64_t x = 0; x < X; ++x) heap.push(Load(0.0, x));
    std::vector<std::vector<int64_t>> xi((size_t)X);
    for (int64_t i : items) {
        Load l = heap.top();
        heap.pop();
        xi[(size_t)l.second].push_back(i);
        heap.push(Load(l.first + icost[(size_t)i], l.second));
    }
    // per XCD: blocks as lists of units
    std::vector<std::vector<std::vector<coot_batch_unit_d>>> xb((size_t)X);
    size_t longest = 0;
    for (int64_t x = 0; x < X; ++x) {
        auto& bl = xb[(size_t)x];
        std::vector<coot_batch_unit_d> pack;
        for (int64_t i : xi[(size_t)x]) {
            if (small[(size_t)i]) continue;
            for (const auto& u : per_item[(size_t)i]) bl.push_back({u});
        }
        for (int64_t i : xi[(size_t)x]) {
            if (!small[(size_t)i]) continue;
            pack.push_back(per_item[(size_t)i][0]);
            if (pack.size() == 4) {
                bl.push_back(pack);
                pack.clear();
            }
        }
        if (!pack.empty()) bl.push_back(pack);
        longest = std::max(longest, bl.size());
    }
    units->clear();
    first->clear();
    for (size_t j = 0; j < longest; ++j)
        for (int64_t x = 0; x < X; ++x) {
            first->push_back((int)units->size());
            if (j < xb[(size_t)x].size())
                units->insert(units->end(), xb[(size_t)x][j].begin(), xb[(size_t)x][j].end());
        }
    first->push_back((int)units->size());
    if (first->size() < 2) first->push_back((int)units->size());  // no units: one empty block
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


// Every tile of every item may run at the same time as any other, so an
// output that overlaps memory the launch reads or writes elsewhere races.
// The one overlap allowed is the single-matrix in-place rule: item i's output
// is exactly its own operand slot s (same first byte, same size, same element
// type) and slot s is only read straight, so each element is read before it
// is written, by the same lane.  Anything else (another item's operand, a
// slot read through trans(), two outputs, the reduction results) fails.
void check_batch_aliasing(const coot_batch* b, const BatchTrees& T)
{
    struct Ext {
        uintptr_t lo, hi;
        int item, slot;  // slot -1: an output or the reduction results
    };
    std::vector<Ext> reads, writes;
    for (int i = 0; i < b->n_items; ++i) {
        const int64_t r = b->shapes[2 * i], c = b->shapes[2 * i + 1];
        if (r * c == 0) continue;
        for (int s = 0; s < b->n_slots; ++s) {
            const uintptr_t p = (uintptr_t)b->leaf_ptrs[(size_t)i * b->n_slots + s];
            if (p && T.par[(size_t)s]) reads.push_back(Ext{p, p + (uintptr_t)(r * c * itemsize(b->slot_dtypes[s])), i, s});
        }
        if (T.has_out && b->out_ptrs[i]) {
            const uintptr_t p = (uintptr_t)b->out_ptrs[i];
            writes.push_back(Ext{p, p + (uintptr_t)(r * c * itemsize(b->out_dtype)), i, -1});
        }
    }
    if (T.has_red && b->red_out && b->n_items > 0) {
        const uintptr_t p = (uintptr_t)b->red_out;
        writes.push_back(Ext{p, p + (uintptr_t)b->n_items * (uintptr_t)itemsize(b->red_dtype), -1, -1});
    }
    auto by_lo = [](const Ext& a, const Ext& c) { return a.lo < c.lo || (a.lo == c.lo && a.hi < c.hi); };
    std::sort(writes.begin(), writes.end(), by_lo);
    for (size_t k = 1; k < writes.size(); ++k)
        if (writes[k].lo < writes[k - 1].hi) fail(COOT_ERR_ALIAS, "batch: two outputs overlap");
    std::sort(reads.begin(), reads.end(), by_lo);
    uintptr_t longest = 0;
    for (const Ext& e : reads) longest = std::max(longest, e.hi - e.lo);
    for (const Ext& w : writes) {
        // reads that can overlap w start in (w.lo - longest, w.hi)
        const uintptr_t from = w.lo > longest ? w.lo - longest : 0;
        auto it = std::lower_bound(reads.begin(), reads.end(), Ext{from, 0, 0, 0}, by_lo);
        for (; it != reads.end() && it->lo < w.hi; ++it) {
            if (it->hi <= w.lo) continue;
            const bool in_place = w.item >= 0 && it->item == w.item && it->lo == w.lo && it->hi == w.hi &&
                                  T.par[(size_t)it->slot] == 1 && b->slot_dtypes[it->slot] == b->out_dtype;
            if (!in_place)
                fail(COOT_ERR_ALIAS, "batch: item " + std::to_string(w.item >= 0 ? w.item : it->item) +
                                         ": an output overlaps an operand (only an item's own slot read straight, "
                                         "with the same extent and element type, may be its output)");
        }
    }
}

// ---- one-call batched evaluation: plans cached by descriptor contents ----
// The descriptor is walked field by field (trees, dtypes, every pointer and
// shape, flags); a Sink either appends the bytes to a key or compares them
// with a stored key, so a lookup copies nothing.
template <class Sink>
void walk_batch(const coot_batch* b, Sink& k)
{
    auto expr = [&](const coot_expr* e) {
        const int32_t nn = e ? e->n_nodes : -1;
        k.put(&nn, sizeof nn);
        if (!e || nn <= 0 || !e->nodes) return;
        k.put(&e->flags, sizeof e->flags);
        k.put(&e->cfg, sizeof e->cfg);
        k.put(e->nodes, sizeof(coot_node) * (size_t)nn);
    };
    expr(b->expr);
    expr(b->red_expr);
    const int32_t head[6] = {b->n_slots, b->n_items, b->out_dtype, b->red_op, b->red_dtype, (int32_t)b->flags};
    k.put(head, sizeof head);
    if (b->n_slots <= 0 || b->n_items < 0) return;
    if (b->slot_dtypes) k.put(b->slot_dtypes, sizeof(int32_t) * (size_t)b->n_slots);
    const size_t n = (size_t)b->n_items;
    if (b->shapes) k.put(b->shapes, sizeof(int64_t) * 2 * n);
    if (b->leaf_ptrs) k.put(b->leaf_ptrs, sizeof(void*) * n * (size_t)b->n_slots);
    const int32_t has_out = b->out_ptrs != nullptr;
    k.put(&has_out, sizeof has_out);
    if (has_out) k.put(b->out_ptrs, sizeof(void*) * n);
    k.put(&b->red_out, sizeof b->red_out);
}

struct KeyWriter {
    std::string key;
    void put(const void* p, size_t n) { key.append((const char*)p, n); }
};

struct KeyMatcher {
    const std::string& key;
    size_t at = 0;
    bool same = true;
    void put(const void* p, size_t n)
    {
        if (!same) return;
        same = at + n <= key.size() && std::memcmp(key.data() + at, p, n) == 0;
        at += n;
    }
};

struct CachedPlan {
    std::string key;
    coot_batch_plan* plan;
};
constexpr size_t EVAL_CACHE_MAX = 16;
std::mutex g_eval_mu;
std::vector<CachedPlan> g_eval_cache;  // most recently used first
}  // namespace

namespace coot {
void batch_destroy_all()
{
    {
        std::lock_guard<std::mutex> lk(g_eval_mu);
        g_eval_cache.clear();
    }
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
        check_batch_aliasing(b, T);
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
            // units of every item (their partial slots in item order) and the block schedule
            const int64_t E = batch_unit_elems(py);
            std::vector<std::vector<coot_batch_unit_d>> per_item((size_t)b->n_items);
            std::vector<bool> small((size_t)b->n_items, false);
            int64_t n_units = 0;
            for (int i = 0; i < b->n_items; ++i) {
                coot_batch_item_d& d = P->h_items[(size_t)i];
                std::memset(&d, 0, sizeof d);
                d.rows = b->shapes[2 * i];
                d.cols = b->shapes[2 * i + 1];
                small[(size_t)i] = item_units(i, d.rows, d.cols, E, &per_item[(size_t)i]);
                d.nunits = (int64_t)per_item[(size_t)i].size();
                d.part0 = n_units;
                for (int64_t j = 0; j < d.nunits; ++j) per_item[(size_t)i][(size_t)j].part = (int)(n_units + j);
                n_units += d.nunits;
                if (n_units >= (int64_t)INT32_MAX) fail(COOT_ERR_SHAPE, "batch: more than 2^31 units");
                for (int s2 = 0; s2 < b->n_slots; ++s2) {
                    d.leaf[s2] = b->leaf_ptrs[(size_t)i * b->n_slots + s2];
                    if (!d.leaf[s2] && d.rows * d.cols > 0) fail(COOT_ERR_ARG, "batch: NULL operand pointer");
                }
                if (has_out) {
                    d.out = b->out_ptrs[i];
                    if (!d.out && d.rows * d.cols > 0) fail(COOT_ERR_ARG, "batch: NULL output pointer");
                }
            }
            std::vector<coot_batch_unit_d> units;
            std::vector<int> first;
            schedule_units(per_item, small, g_state.xcds, &units, &first);
            P->n_blocks = std::max<int64_t>(1, (int64_t)first.size() - 1);
            if (P->n_blocks > 0x7fffffff) fail(COOT_ERR_SHAPE, "batch: too many blocks");
            auto up = [](void** dst, const void* src, size_t bytes) {
                hipchk(hipMalloc(dst, std::max<size_t>(bytes, 16)), "hipMalloc(batch table)");
                if (bytes) hipchk(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy(batch table)");
            };
            up((void**)&P->d_items, P->h_items.data(), P->h_items.size() * sizeof(coot_batch_item_d));
            up((void**)&P->d_units, units.data(), units.size() * sizeof(coot_batch_unit_d));
            up((void**)&P->d_blk_first, first.data(), first.size() * sizeof(int));
            if (has_red) {
                (void)hipFree(P->d_part);
                P->d_part = nullptr;
                hipchk(hipMalloc((void**)&P->d_part, std::max<size_t>(16, (size_t)n_units * 2 * sizeof(double))),
                       "hipMalloc(batch partials)");
            }
            // kernels
            std::string name;
            std::string src = batch_kernel_source(py, has_red ? &pr : nullptr, has_out, b->out_dtype, b->red_dtype,
                                                  read_slot, &name);
            P->k = get_kernel(name, src, has_red);
            P->args = coot_bargs{P->d_items, P->d_units, P->d_blk_first, P->n_items, P->d_part, b->red_out};
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

int coot_eval_batched(const coot_batch* b, void* stream)
{
    return guard3([&] {
        if (!b) fail(COOT_ERR_ARG, "NULL batch");
        coot_batch_plan* P = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_eval_mu);
            for (size_t i = 0; i < g_eval_cache.size(); ++i) {
                KeyMatcher m{g_eval_cache[i].key};
                walk_batch(b, m);
                if (m.same && m.at == g_eval_cache[i].key.size()) {
                    P = g_eval_cache[i].plan;
                    std::rotate(g_eval_cache.begin(), g_eval_cache.begin() + (ptrdiff_t)i,
                                g_eval_cache.begin() + (ptrdiff_t)i + 1);
                    break;
                }
            }
        }
        if (!P) {
            int rc = coot_batch_create(b, stream, &P);
            if (rc) return rc;
            KeyWriter w;
            walk_batch(b, w);
            coot_batch_plan* evict = nullptr;
            {
                std::lock_guard<std::mutex> lk(g_eval_mu);
                g_eval_cache.insert(g_eval_cache.begin(), CachedPlan{std::move(w.key), P});
                if (g_eval_cache.size() > EVAL_CACHE_MAX) {
                    evict = g_eval_cache.back().plan;
                    g_eval_cache.pop_back();
                }
            }
            if (evict) {
                // its graph may still be running on some stream
                hipchk(hipDeviceSynchronize(), "hipDeviceSynchronize");
                int rc2 = coot_batch_destroy(evict);
                if (rc2) return rc2;
            }
        }
        return coot_batch_run(P, stream);
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
