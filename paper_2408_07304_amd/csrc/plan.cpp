// Mixed-shape plans: many ciphertexts of several contexts (ring degrees and
// moduli chains) encrypted by one persistent launch, captured once as a HIP
// graph and replayed.
#include <algorithm>
#include <cstring>
#include <functional>
#include <new>
#include <queue>
#include <string>
#include <vector>

#include "zinc_internal.h"

struct zinc_plan {
    std::vector<zinc_ctx*> ctxs;
    int scheme = 0;
    void* d_block = nullptr;            // contexts, items, units, counter, dummy outputs
    zinc::PlanDev dev{};
    size_t n_items = 0;
    uint64_t need_slots = 0;            // float64 words of slots the items read
    uint64_t need_ct = 0;               // uint64 words of output the items write
    // captured graph and what it was captured with
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream the graph is recorded on
    const double* cap_slots = nullptr;
    uint64_t* cap_ct = nullptr;
};

using namespace zinc;

namespace zinc {

uint32_t plan_units_per_group(uint32_t log_n) { return log_n == 12 ? 4u : log_n == 13 ? 2u : 1u; }

uint64_t plan_dummy_words(zinc_ctx* const* ctxs, uint32_t n_ctx) {
    uint64_t w = 0;
    for (uint32_t c = 0; c < n_ctx; ++c)
        w += (plan_units_per_group(ctxs[c]->log_n) - 1) * 2ull * ctxs[c]->L * ctxs[c]->n;
    return w;
}

int device_cu_count() {
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus > 0 ? cus : 256;
}

uint32_t limb_groups(const DevParams& p, uint32_t batch) {
    static const uint32_t cus = (uint32_t)device_cu_count();
    if (batch == 0 || 2 * batch > cus) return 1;
    return std::max(1u, std::min(p.L, cus / batch));
}

double plan_unit_cost(const zinc_ctx& c, const PlanUnit& u) {
    return (double)u.count * c.n * c.log_n * ((double)(u.l1 - u.l0) + 1.0);
}

// Completion time of units of the given costs on `round` workgroups that
// each take the next unit, longest first, when they become free (how k_plan
// runs a plan).
static double list_makespan(std::vector<double> costs, uint32_t round) {
    std::sort(costs.begin(), costs.end(), std::greater<double>());
    std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
    for (uint32_t i = 0; i < std::max(round, 1u); ++i) free_at.push(0.0);
    double end = 0.0;
    for (double c : costs) {
        const double t = free_at.top() + c;
        free_at.pop();
        free_at.push(t);
        end = std::max(end, t);
    }
    return end;
}

uint32_t plan_split_parts(const std::vector<double>& other_costs, uint32_t tail, uint32_t L, double unit,
                          uint32_t round) {
    uint32_t best = std::min(kPlanSplit, L);
    double best_end = 1e300;
    for (uint32_t parts = best; parts <= L; ++parts) {
        std::vector<double> costs = other_costs;
        for (uint32_t i = 0; i < tail; ++i)
            for (uint32_t j = 0; j < parts; ++j)
                costs.push_back(unit * ((double)((j + 1) * L / parts - j * L / parts) + 1.0));
        const double end = list_makespan(std::move(costs), round);
        if (end < best_end * (1.0 - 1e-9)) {
            best_end = end;
            best = parts;
        }
    }
    return best;
}

uint64_t build_plan_tables(zinc_ctx* const* ctxs, uint32_t n_ctx, const zinc_item* items, uint32_t n_items,
                           std::vector<PlanItem>& dev_items, std::vector<PlanUnit>& units, uint32_t round) {
    dev_items.clear();
    units.clear();
    uint64_t dummy_words = 0;
    std::vector<std::vector<uint32_t>> per_ctx(n_ctx);
    for (uint32_t i = 0; i < n_items; ++i) per_ctx[items[i].ctx_idx].push_back(i);
    // Ring degree 32768 (one ciphertext per unit): the ciphertexts beyond the
    // last whole round of `round` units would run in a partial round of their
    // own while the other workgroups idle; split into limb groups, they spread
    // over all workgroups (each group redraws the same noise and re-encodes
    // the message, about one limb's work).  The number of groups minimises the
    // estimated completion time of the plan (plan_split_parts): a few such
    // ciphertexts on an idle device take one limb per unit, a full device
    // keeps kPlanSplit.
    uint32_t n32 = 0;
    for (uint32_t c = 0; c < n_ctx; ++c)
        if (ctxs[c]->log_n == 15) n32 += (uint32_t)per_ctx[c].size();
    const uint32_t tail = round ? n32 % round : 0;
    // estimated costs of every unit but the tail's, and the tail per context
    std::vector<double> other_costs;
    std::vector<uint32_t> tail_of(n_ctx, 0);
    {
        uint32_t seen = 0;
        for (uint32_t c = 0; c < n_ctx; ++c) {
            const zinc_ctx* cx = ctxs[c];
            const uint32_t g = plan_units_per_group(cx->log_n);
            const double whole = plan_unit_cost(*cx, PlanUnit{c, cx->log_n, 0u, g, 0u, cx->L});
            for (size_t k = 0; k < per_ctx[c].size(); k += g) {
                if (cx->log_n == 15 && seen++ >= n32 - tail) ++tail_of[c];
                else other_costs.push_back(whole);
            }
        }
    }
    std::vector<uint32_t> parts_of(n_ctx, 1);
    for (uint32_t c = 0; c < n_ctx; ++c) {
        if (!tail_of[c]) continue;
        std::vector<double> others = other_costs;   // the other contexts' tails at the fewest groups
        for (uint32_t d = 0; d < n_ctx; ++d) {
            if (d == c || !tail_of[d]) continue;
            const uint32_t pd = std::min(kPlanSplit, ctxs[d]->L);
            for (uint32_t i = 0; i < tail_of[d]; ++i)
                for (uint32_t j = 0; j < pd; ++j)
                    others.push_back(plan_unit_cost(*ctxs[d], PlanUnit{d, 15u, 0u, 1u, j * ctxs[d]->L / pd,
                                                                       (j + 1) * ctxs[d]->L / pd}));
        }
        parts_of[c] = plan_split_parts(others, tail_of[c], ctxs[c]->L,
                                       plan_unit_cost(*ctxs[c], PlanUnit{c, 15u, 0u, 1u, 0u, 0u}), round);
    }
    uint32_t seen32 = 0;
    for (uint32_t c = 0; c < n_ctx; ++c) {
        const zinc_ctx* cx = ctxs[c];
        const uint32_t g = plan_units_per_group(cx->log_n);
        const uint64_t ct_words = 2ull * cx->L * cx->n;
        const auto& lst = per_ctx[c];
        for (size_t s = 0; s < lst.size(); s += g) {
            if (cx->log_n == 15 && seen32++ >= n32 - tail) {
                const uint32_t parts = parts_of[c];
                for (uint32_t j = 0; j < parts; ++j)
                    units.push_back(PlanUnit{c, cx->log_n, (uint32_t)dev_items.size(), 1u, j * cx->L / parts,
                                             (j + 1) * cx->L / parts});
            } else {
                units.push_back(PlanUnit{c, cx->log_n, (uint32_t)dev_items.size(), g, 0u, cx->L});
            }
            for (uint32_t k = 0; k < g; ++k) {
                if (s + k < lst.size()) {
                    const zinc_item& it = items[lst[s + k]];
                    dev_items.push_back(PlanItem{c, 0u, it.slot_off, it.ct_off, it.ct_id});
                } else {   // pad with a copy of the unit's first item writing into the dummy buffer
                    const zinc_item& it = items[lst[s]];
                    dev_items.push_back(PlanItem{c, 1u, it.slot_off, dummy_words, it.ct_id});
                    dummy_words += ct_words;
                }
            }
        }
    }
    // longest-processing-time order: the largest units start first
    std::stable_sort(units.begin(), units.end(), [&](const PlanUnit& a, const PlanUnit& b) {
        return plan_unit_cost(*ctxs[a.ctx], a) > plan_unit_cost(*ctxs[b.ctx], b);
    });
    return dummy_words;
}

}  // namespace zinc

static void drop_graph(zinc_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

extern "C" {

zinc_status zinc_plan_create(zinc_ctx* const* ctxs, uint32_t n_ctx, const zinc_item* items, uint32_t n_items,
                             int scheme, zinc_plan** out) {
    if (!out) return plan_fail(ZINC_E_INVAL, "zinc_plan_create: null output");
    *out = nullptr;
    if (!ctxs || n_ctx == 0 || (!items && n_items)) return plan_fail(ZINC_E_INVAL, "zinc_plan_create: null argument");
    if (scheme != ZINC_SCHEME_VANILLA && scheme != ZINC_SCHEME_ZINC)
        return plan_fail(ZINC_E_INVAL, "zinc_plan_create: scheme must be 0 (vanilla) or 1 (zinc)");
    for (uint32_t c = 0; c < n_ctx; ++c) {
        if (!ctxs[c]) return plan_fail(ZINC_E_INVAL, "zinc_plan_create: null context");
        if (!ctxs[c]->keyed) return plan_fail(ZINC_E_STATE, "zinc_plan_create: context without keys");
        if (ctxs[c]->dev.noise_t > 1)
            return plan_fail(ZINC_E_STATE, "zinc_plan_create: a BGV context encrypts integer plaintexts only");
        if (scheme == ZINC_SCHEME_ZINC && !ctxs[c]->precomputed)
            return plan_fail(ZINC_E_STATE, "zinc_plan_create: context without a cached Enc(0)");
    }
    uint64_t need_slots = 0, need_ct = 0;
    for (uint32_t i = 0; i < n_items; ++i) {
        if (items[i].ctx_idx >= n_ctx) return plan_fail(ZINC_E_INVAL, "zinc_plan_create: item context out of range");
        if (items[i].ct_id >= (1ull << 63)) return plan_fail(ZINC_E_INVAL, "zinc_plan_create: ct_id must be < 2^63");
        const zinc_ctx* cx = ctxs[items[i].ctx_idx];
        const uint64_t sw = cx->n / 2, cw = 2ull * cx->L * cx->n;
        if (items[i].slot_off > ~0ull - sw || items[i].ct_off > ~0ull - cw)
            return plan_fail(ZINC_E_INVAL, "zinc_plan_create: item offset out of range");
        need_slots = std::max(need_slots, items[i].slot_off + sw);
        need_ct = std::max(need_ct, items[i].ct_off + cw);
    }
    std::vector<PlanItem> dev_items;
    std::vector<PlanUnit> units;
    const int cus = device_cu_count();
    const uint64_t dummy_words = build_plan_tables(ctxs, n_ctx, items, n_items, dev_items, units, (uint32_t)cus);
    zinc_plan* p = new (std::nothrow) zinc_plan();
    if (!p) return plan_fail(ZINC_E_NOMEM, "host allocation failed");
    p->ctxs.assign(ctxs, ctxs + n_ctx);
    p->scheme = scheme;
    p->n_items = n_items;
    p->need_slots = need_slots;
    p->need_ct = need_ct;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t b_ctx = al(sizeof(DevParams) * n_ctx), b_items = al(sizeof(PlanItem) * std::max<size_t>(1, dev_items.size()));
    const size_t b_units = al(sizeof(PlanUnit) * std::max<size_t>(1, units.size())), b_cnt = 256;
    const size_t b_dummy = al(8 * std::max<uint64_t>(1, dummy_words));
    char* base = nullptr;
    if (hipMalloc(&base, b_ctx + b_items + b_units + b_cnt + b_dummy) != hipSuccess) {
        delete p;
        return plan_fail(ZINC_E_NOMEM, "zinc_plan_create: device allocation failed");
    }
    p->d_block = base;
    std::vector<DevParams> dp(n_ctx);
    for (uint32_t c = 0; c < n_ctx; ++c) dp[c] = ctxs[c]->dev;
    hipError_t e = hipMemcpy(base, dp.data(), sizeof(DevParams) * n_ctx, hipMemcpyHostToDevice);
    if (e == hipSuccess && !dev_items.empty())
        e = hipMemcpy(base + b_ctx, dev_items.data(), sizeof(PlanItem) * dev_items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !units.empty())
        e = hipMemcpy(base + b_ctx + b_items, units.data(), sizeof(PlanUnit) * units.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(base);
        delete p;
        return plan_fail(ZINC_E_HIP, std::string("zinc_plan_create: upload failed: ") + hipGetErrorString(e));
    }
    PlanDev& d = p->dev;
    d.ctxs = reinterpret_cast<const DevParams*>(base);
    d.items = reinterpret_cast<const PlanItem*>(base + b_ctx);
    d.units = reinterpret_cast<const PlanUnit*>(base + b_ctx + b_items);
    d.n_units = (uint32_t)units.size();
    d.counter = reinterpret_cast<uint32_t*>(base + b_ctx + b_items + b_units);
    d.dummy = reinterpret_cast<uint64_t*>(base + b_ctx + b_items + b_units + b_cnt);
    d.grid = (uint32_t)std::max(1, std::min<int>(cus, (int)std::max<uint32_t>(1, d.n_units)));
    *out = p;
    return ZINC_OK;
}

zinc_status zinc_plan_launch(zinc_plan* p, const double* slots, uint64_t n_slot_words, uint64_t* ct,
                             uint64_t n_ct_words, void* stream) {
    if (!p) return plan_fail(ZINC_E_INVAL, "zinc_plan_launch: null plan");
    if (p->n_items == 0) return ZINC_OK;
    if (!slots || !ct) return plan_fail(ZINC_E_INVAL, "zinc_plan_launch: null buffer");
    if (n_slot_words < p->need_slots)
        return plan_fail(ZINC_E_INVAL, "zinc_plan_launch: the slot buffer ends before an item's slots (" +
                                           std::to_string(n_slot_words) + " < " + std::to_string(p->need_slots) +
                                           " words)");
    if (n_ct_words < p->need_ct)
        return plan_fail(ZINC_E_INVAL, "zinc_plan_launch: the ciphertext buffer ends before an item's output (" +
                                           std::to_string(n_ct_words) + " < " + std::to_string(p->need_ct) +
                                           " words)");
    hipStream_t s = (hipStream_t)stream;
    if (!p->exec || p->cap_slots != slots || p->cap_ct != ct) {
        // Record the launch sequence on the plan's own stream (the caller's may
        // be the null stream, which cannot be captured); nothing runs here.
        drop_graph(p);
        hipError_t e = hipSuccess;
        if (!p->cap_stream) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return plan_fail(ZINC_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        hipError_t le = launch_plan(p->dev, p->scheme, slots, ct, p->cap_stream);
        e = hipStreamEndCapture(p->cap_stream, &p->graph);
        if (le != hipSuccess || e != hipSuccess) {
            drop_graph(p);
            return plan_fail(ZINC_E_HIP, std::string("graph capture: ") + hipGetErrorString(le != hipSuccess ? le : e));
        }
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(p);
            return plan_fail(ZINC_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        p->cap_slots = slots;
        p->cap_ct = ct;
    }
    hipError_t e = hipGraphLaunch(p->exec, s);
    if (e != hipSuccess) return plan_fail(ZINC_E_HIP, std::string("graph launch: ") + hipGetErrorString(e));
    return ZINC_OK;
}

zinc_status zinc_plan_destroy(zinc_plan* p) {
    if (!p) return ZINC_OK;
    (void)hipDeviceSynchronize();
    drop_graph(p);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->d_block) (void)hipFree(p->d_block);
    delete p;
    return ZINC_OK;
}

}  // extern "C"
