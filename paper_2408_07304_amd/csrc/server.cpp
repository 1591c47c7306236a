// Serving: requests of 1..max_batch plaintexts admitted against an HBM budget
// and encrypted by continuous batching on several streams.  Every batch is one
// launch of the mixed-shape persistent kernel over all its plaintexts,
// whatever their contexts, so a batch never waits for requests of one ring
// degree to accumulate.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "arena.h"
#include "zinc_internal.h"

using namespace zinc;

namespace {

constexpr uint32_t kMaxStreams = 16;
constexpr uint32_t kMaxBatch = 65536;
constexpr uint64_t kAlign = Arena::kAlign;

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum class ReqState : uint8_t { Waiting, Admitted, Running, Done };

struct Req {
    zinc_request r;
    zinc_request_times t;
    uint64_t bytes = 0;       // ciphertext bytes of the request
    uint64_t arena_off = 0;   // granted byte offset in the arena
    ReqState state = ReqState::Waiting;
    bool held = false;        // completed, output kept in the arena until released
};

struct Lane {                 // one stream and the buffers of the batch it runs
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t start = nullptr;    // timing events around the batch, for device times
    hipEvent_t end = nullptr;
    PlanItem* h_items = nullptr;   // pinned staging of the batch's tables
    PlanUnit* h_units = nullptr;
    PlanDev dev{};                 // device tables of the batch
    std::vector<uint64_t> tickets; // requests of the running batch
    bool busy = false;
};

}  // namespace

struct zinc_server {
    std::vector<zinc_ctx*> ctxs;
    zinc_server_config cfg{};
    uint64_t t0 = 0;
    void* d_block = nullptr;       // contexts + per-lane items, units, counter, dummy
    void* d_arena = nullptr;       // outputs when the caller gives no d_ct
    Arena arena;
    std::vector<Lane> lanes;
    std::vector<Req> reqs;
    std::deque<uint64_t> waiting, admitted;
    uint64_t outstanding = 0;
    uint32_t n_batches = 0;
    size_t item_cap = 0, unit_cap = 0;
    int cus = 256;
    // scratch reused by every batch
    std::vector<zinc_item> items;
    std::vector<PlanItem> dev_items;
    std::vector<PlanUnit> units;

    hipEvent_t ref = nullptr;      // recorded (and complete) at creation: origin of device times

    uint64_t now() const { return now_ns() - t0; }
};

namespace {

zinc_status release_all(zinc_server* s) {
    for (auto& l : s->lanes) {
        if (l.stream) (void)hipStreamSynchronize(l.stream);
        if (l.done) (void)hipEventDestroy(l.done);
        if (l.start) (void)hipEventDestroy(l.start);
        if (l.end) (void)hipEventDestroy(l.end);
        if (l.stream) (void)hipStreamDestroy(l.stream);
        if (l.h_items) (void)hipHostFree(l.h_items);
        if (l.h_units) (void)hipHostFree(l.h_units);
    }
    if (s->ref) (void)hipEventDestroy(s->ref);
    if (s->d_arena) (void)hipFree(s->d_arena);
    if (s->d_block) (void)hipFree(s->d_block);
    delete s;
    return ZINC_OK;
}

zinc_status hip_error(hipError_t e, const char* what) {
    return plan_fail(ZINC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Reap finished batches.
zinc_status reap(zinc_server* s, uint32_t* n_done) {
    for (size_t li = 0; li < s->lanes.size(); ++li) {
        Lane& l = s->lanes[li];
        if (!l.busy) continue;
        const hipError_t e = hipEventQuery(l.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return hip_error(e, "zinc_server_progress: batch failed");
        const uint64_t t = s->now();
        // device interval of the batch: its start and end events (both
        // complete once `done` is) against the creation-time reference
        float ms0 = 0.f, ms1 = 0.f;
        if (hipEventElapsedTime(&ms0, s->ref, l.start) != hipSuccess ||
            hipEventElapsedTime(&ms1, s->ref, l.end) != hipSuccess)
            return plan_fail(ZINC_E_HIP, "zinc_server_progress: device timing events");
        for (uint64_t tk : l.tickets) {
            Req& q = s->reqs[tk];
            q.t.done_ns = t;
            q.t.dev_start_ns = (uint64_t)((double)ms0 * 1e6);
            q.t.dev_end_ns = (uint64_t)((double)ms1 * 1e6);
            q.state = ReqState::Done;
            if (s->cfg.retain_outputs) q.held = true;     // released by zinc_server_release
            else s->arena.release(q.arena_off, q.bytes);
        }
        if (n_done) *n_done += (uint32_t)l.tickets.size();
        s->outstanding -= l.tickets.size();
        l.tickets.clear();
        l.busy = false;
    }
    return ZINC_OK;
}

void admit(zinc_server* s) {
    while (!s->waiting.empty()) {
        Req& q = s->reqs[s->waiting.front()];
        uint64_t off = 0;
        if (!s->arena.alloc(q.bytes, &off)) break;   // strict submission order
        q.arena_off = off;
        q.state = ReqState::Admitted;
        q.t.admit_ns = s->now();
        s->admitted.push_back(s->waiting.front());
        s->waiting.pop_front();
    }
}

zinc_status launch(zinc_server* s, uint32_t lane_idx) {
    Lane& l = s->lanes[lane_idx];
    s->items.clear();
    l.tickets.clear();
    uint32_t pts = 0;
    while (!s->admitted.empty()) {
        const uint64_t tk = s->admitted.front();
        const Req& q = s->reqs[tk];
        if (pts + q.r.n_pt > s->cfg.max_batch) break;
        const zinc_ctx* c = s->ctxs[q.r.ctx_idx];
        const uint64_t ct_words = 2ull * c->L * c->n;
        const uint64_t base = s->cfg.d_ct ? q.r.ct_off : q.arena_off / 8;
        for (uint32_t k = 0; k < q.r.n_pt; ++k)
            s->items.push_back(zinc_item{q.r.ctx_idx, 0u, q.r.slot_off + (uint64_t)k * (c->n / 2),
                                         base + k * ct_words, q.r.ct_id + k});
        pts += q.r.n_pt;
        l.tickets.push_back(tk);
        s->admitted.pop_front();
    }
    if (l.tickets.empty()) return ZINC_OK;
    (void)build_plan_tables(s->ctxs.data(), (uint32_t)s->ctxs.size(), s->items.data(), (uint32_t)s->items.size(),
                            s->dev_items, s->units, (uint32_t)s->cus);
    if (s->dev_items.size() > s->item_cap || s->units.size() > s->unit_cap)
        return plan_fail(ZINC_E_INVAL, "zinc_server_progress: batch tables exceed their capacity");
    std::memcpy(l.h_items, s->dev_items.data(), sizeof(PlanItem) * s->dev_items.size());
    std::memcpy(l.h_units, s->units.data(), sizeof(PlanUnit) * s->units.size());
    PlanDev d = l.dev;
    d.n_units = (uint32_t)s->units.size();
    d.grid = (uint32_t)std::max(1, std::min<int>(s->cus, (int)d.n_units));
    hipError_t e = hipMemcpyAsync((void*)d.items, l.h_items, sizeof(PlanItem) * s->dev_items.size(),
                                  hipMemcpyHostToDevice, l.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((void*)d.units, l.h_units, sizeof(PlanUnit) * s->units.size(), hipMemcpyHostToDevice,
                           l.stream);
    uint64_t* out = s->cfg.d_ct ? s->cfg.d_ct : (uint64_t*)s->d_arena;
    if (e == hipSuccess) e = hipEventRecord(l.start, l.stream);
    if (e == hipSuccess) e = launch_plan(d, s->cfg.scheme, s->cfg.d_slots, out, l.stream);
    if (e == hipSuccess) e = hipEventRecord(l.end, l.stream);
    if (e == hipSuccess) e = hipEventRecord(l.done, l.stream);
    if (e != hipSuccess) return hip_error(e, "zinc_server_progress: batch launch");
    const uint64_t t = s->now();
    const uint32_t b = s->n_batches++;
    for (uint64_t tk : l.tickets) {
        Req& q = s->reqs[tk];
        q.state = ReqState::Running;
        q.t.launch_ns = t;
        q.t.batch = b;
        q.t.stream = lane_idx;
    }
    l.busy = true;
    return ZINC_OK;
}

}  // namespace

extern "C" {

zinc_status zinc_server_create(zinc_ctx* const* ctxs, uint32_t n_ctx, const zinc_server_config* cfg,
                               zinc_server** out) {
    if (!out) return plan_fail(ZINC_E_INVAL, "zinc_server_create: null output");
    *out = nullptr;
    if (!ctxs || n_ctx == 0 || !cfg) return plan_fail(ZINC_E_INVAL, "zinc_server_create: null argument");
    if (cfg->scheme != ZINC_SCHEME_VANILLA && cfg->scheme != ZINC_SCHEME_ZINC)
        return plan_fail(ZINC_E_INVAL, "zinc_server_create: scheme must be 0 (vanilla) or 1 (zinc)");
    if (cfg->n_streams < 1 || cfg->n_streams > kMaxStreams)
        return plan_fail(ZINC_E_INVAL, "zinc_server_create: n_streams must be in [1, 16]");
    if (cfg->max_batch < 1 || cfg->max_batch > kMaxBatch)
        return plan_fail(ZINC_E_INVAL, "zinc_server_create: max_batch must be in [1, 65536]");
    if (!cfg->d_slots || cfg->slots_len == 0) return plan_fail(ZINC_E_INVAL, "zinc_server_create: null slot buffer");
    if (cfg->d_ct && cfg->ct_len == 0) return plan_fail(ZINC_E_INVAL, "zinc_server_create: empty output buffer");
    if (cfg->retain_outputs > 1 || (cfg->retain_outputs && cfg->d_ct))
        return plan_fail(ZINC_E_INVAL, "zinc_server_create: retain_outputs is 0 or 1, and 1 needs the arena (d_ct NULL)");
    for (uint32_t c = 0; c < n_ctx; ++c) {
        if (!ctxs[c]) return plan_fail(ZINC_E_INVAL, "zinc_server_create: null context");
        if (!ctxs[c]->keyed) return plan_fail(ZINC_E_STATE, "zinc_server_create: context without keys");
        if (ctxs[c]->dev.noise_t > 1)
            return plan_fail(ZINC_E_STATE, "zinc_server_create: a BGV context encrypts integer plaintexts only");
        if (cfg->scheme == ZINC_SCHEME_ZINC && !ctxs[c]->precomputed)
            return plan_fail(ZINC_E_STATE, "zinc_server_create: context without a cached Enc(0)");
    }
    uint64_t budget = cfg->hbm_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return plan_fail(ZINC_E_HIP, "zinc_server_create: hipMemGetInfo");
        budget = (uint64_t)fr / 2;
    }
    budget &= ~(kAlign - 1);
    if (budget == 0) return plan_fail(ZINC_E_INVAL, "zinc_server_create: empty HBM budget");

    zinc_server* s = new (std::nothrow) zinc_server();
    if (!s) return plan_fail(ZINC_E_NOMEM, "host allocation failed");
    s->ctxs.assign(ctxs, ctxs + n_ctx);
    s->cfg = *cfg;
    s->cfg.hbm_budget = budget;
    s->arena = Arena(budget);
    s->cus = device_cu_count();
    // Per-batch table capacity: every plaintext plus the padding of one
    // partial unit per context; a plaintext is at most max(kPlanSplit, L) units.
    s->item_cap = cfg->max_batch + 3ull * n_ctx;
    uint32_t max_split = kPlanSplit;            // a plaintext of ring degree 32768 is at most L units
    for (uint32_t c = 0; c < n_ctx; ++c)
        if (ctxs[c]->log_n == 15) max_split = std::max(max_split, ctxs[c]->L);
    s->unit_cap = (size_t)max_split * cfg->max_batch + (size_t)n_ctx;
    const uint64_t dummy_words = std::max<uint64_t>(1, plan_dummy_words(ctxs, n_ctx));
    auto al = [](size_t x) { return (x + kAlign - 1) & ~size_t(kAlign - 1); };
    const size_t b_ctx = al(sizeof(DevParams) * n_ctx), b_items = al(sizeof(PlanItem) * s->item_cap);
    const size_t b_units = al(sizeof(PlanUnit) * s->unit_cap), b_cnt = kAlign, b_dummy = al(8 * dummy_words);
    const size_t per_lane = b_items + b_units + b_cnt + b_dummy;
    char* base = nullptr;
    if (hipMalloc(&base, b_ctx + per_lane * cfg->n_streams) != hipSuccess) {
        delete s;
        return plan_fail(ZINC_E_NOMEM, "zinc_server_create: device allocation failed");
    }
    s->d_block = base;
    std::vector<DevParams> dp(n_ctx);
    for (uint32_t c = 0; c < n_ctx; ++c) dp[c] = ctxs[c]->dev;
    hipError_t e = hipMemcpy(base, dp.data(), sizeof(DevParams) * n_ctx, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release_all(s);
        return hip_error(e, "zinc_server_create: upload");
    }
    if (!cfg->d_ct && hipMalloc(&s->d_arena, budget) != hipSuccess) {
        release_all(s);
        return plan_fail(ZINC_E_NOMEM, "zinc_server_create: arena of hbm_budget bytes could not be allocated");
    }
    s->lanes.resize(cfg->n_streams);
    for (uint32_t i = 0; i < cfg->n_streams; ++i) {
        Lane& l = s->lanes[i];
        char* lb = base + b_ctx + per_lane * i;
        l.dev.ctxs = reinterpret_cast<const DevParams*>(base);
        l.dev.items = reinterpret_cast<const PlanItem*>(lb);
        l.dev.units = reinterpret_cast<const PlanUnit*>(lb + b_items);
        l.dev.counter = reinterpret_cast<uint32_t*>(lb + b_items + b_units);
        l.dev.dummy = reinterpret_cast<uint64_t*>(lb + b_items + b_units + b_cnt);
        e = hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&l.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreate(&l.start);
        if (e == hipSuccess) e = hipEventCreate(&l.end);
        if (e == hipSuccess) e = hipHostMalloc((void**)&l.h_items, sizeof(PlanItem) * s->item_cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&l.h_units, sizeof(PlanUnit) * s->unit_cap, hipHostMallocDefault);
        if (e != hipSuccess) {
            release_all(s);
            return hip_error(e, "zinc_server_create: stream resources");
        }
    }
    e = hipEventCreate(&s->ref);
    if (e == hipSuccess) e = hipEventRecord(s->ref, s->lanes[0].stream);
    if (e == hipSuccess) e = hipEventSynchronize(s->ref);
    if (e != hipSuccess) {
        release_all(s);
        return hip_error(e, "zinc_server_create: reference event");
    }
    s->t0 = now_ns();
    *out = s;
    return ZINC_OK;
}

zinc_status zinc_server_submit(zinc_server* s, const zinc_request* r, uint64_t* ticket) {
    if (!s || !r) return plan_fail(ZINC_E_INVAL, "zinc_server_submit: null argument");
    if (r->ctx_idx >= s->ctxs.size()) return plan_fail(ZINC_E_INVAL, "zinc_server_submit: context out of range");
    if (r->n_pt == 0) return plan_fail(ZINC_E_INVAL, "zinc_server_submit: empty request");
    if (r->n_pt > s->cfg.max_batch) return plan_fail(ZINC_E_RANGE, "zinc_server_submit: n_pt exceeds max_batch");
    if (r->ct_id >= (1ull << 63) || r->n_pt > (1ull << 63) - r->ct_id)
        return plan_fail(ZINC_E_INVAL, "zinc_server_submit: ct_id + n_pt must be <= 2^63");
    const zinc_ctx* c = s->ctxs[r->ctx_idx];
    const uint64_t slot_words = (uint64_t)r->n_pt * (c->n / 2), ct_words = (uint64_t)r->n_pt * 2ull * c->L * c->n;
    Req q;
    q.r = *r;
    q.bytes = ct_words * 8ull;
    if (((q.bytes + kAlign - 1) & ~(kAlign - 1)) > s->arena.size())
        return plan_fail(ZINC_E_RANGE, "zinc_server_submit: request output exceeds the HBM budget");
    if (r->slot_off > s->cfg.slots_len || slot_words > s->cfg.slots_len - r->slot_off)
        return plan_fail(ZINC_E_INVAL, "zinc_server_submit: the request's slots end beyond slots_len");
    if (s->cfg.d_ct && (r->ct_off > s->cfg.ct_len || ct_words > s->cfg.ct_len - r->ct_off))
        return plan_fail(ZINC_E_INVAL, "zinc_server_submit: the request's ciphertexts end beyond ct_len");
    std::memset(&q.t, 0, sizeof(q.t));
    q.t.submit_ns = s->now();
    const uint64_t tk = s->reqs.size();
    s->reqs.push_back(q);
    s->waiting.push_back(tk);
    ++s->outstanding;
    if (ticket) *ticket = tk;
    return ZINC_OK;
}

zinc_status zinc_server_progress(zinc_server* s, uint32_t* n_done) {
    if (!s) return plan_fail(ZINC_E_INVAL, "zinc_server_progress: null server");
    if (n_done) *n_done = 0;
    zinc_status st = reap(s, n_done);
    if (st != ZINC_OK) return st;
    admit(s);
    for (uint32_t i = 0; i < s->lanes.size() && !s->admitted.empty(); ++i) {
        if (s->lanes[i].busy) continue;
        st = launch(s, i);
        if (st != ZINC_OK) return st;
    }
    return ZINC_OK;
}

zinc_status zinc_server_query(zinc_server* s, uint64_t ticket, int* done, zinc_request_times* times) {
    if (!s || !done) return plan_fail(ZINC_E_INVAL, "zinc_server_query: null argument");
    if (ticket >= s->reqs.size()) return plan_fail(ZINC_E_INVAL, "zinc_server_query: unknown ticket");
    const Req& q = s->reqs[ticket];
    *done = q.state == ReqState::Done;
    if (times) *times = q.t;
    return ZINC_OK;
}

zinc_status zinc_server_output(zinc_server* s, uint64_t ticket, uint64_t** d_out) {
    if (!s || !d_out) return plan_fail(ZINC_E_INVAL, "zinc_server_output: null argument");
    *d_out = nullptr;
    if (!s->cfg.retain_outputs) return plan_fail(ZINC_E_STATE, "zinc_server_output: the server does not retain outputs");
    if (ticket >= s->reqs.size()) return plan_fail(ZINC_E_INVAL, "zinc_server_output: unknown ticket");
    const Req& q = s->reqs[ticket];
    if (q.state != ReqState::Done || !q.held)
        return plan_fail(ZINC_E_STATE, "zinc_server_output: the request has not completed or was released");
    *d_out = reinterpret_cast<uint64_t*>(static_cast<char*>(s->d_arena) + q.arena_off);
    return ZINC_OK;
}

zinc_status zinc_server_read_output(zinc_server* s, uint64_t ticket, uint64_t* d_dst, uint64_t dst_words,
                                    void* stream) {
    uint64_t* src = nullptr;
    if (!d_dst) return plan_fail(ZINC_E_INVAL, "zinc_server_read_output: null destination");
    if (zinc_status st = zinc_server_output(s, ticket, &src)) return st;
    const Req& q = s->reqs[ticket];
    if (dst_words < q.bytes / 8)
        return plan_fail(ZINC_E_INVAL, "zinc_server_read_output: the destination is shorter than the request's output");
    const hipError_t e = hipMemcpyAsync(d_dst, src, q.bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "zinc_server_read_output");
    return ZINC_OK;
}

zinc_status zinc_server_release(zinc_server* s, uint64_t ticket) {
    if (!s) return plan_fail(ZINC_E_INVAL, "zinc_server_release: null server");
    if (!s->cfg.retain_outputs) return plan_fail(ZINC_E_STATE, "zinc_server_release: the server does not retain outputs");
    if (ticket >= s->reqs.size()) return plan_fail(ZINC_E_INVAL, "zinc_server_release: unknown ticket");
    Req& q = s->reqs[ticket];
    if (q.state != ReqState::Done || !q.held)
        return plan_fail(ZINC_E_STATE, "zinc_server_release: the request has not completed or was released");
    q.held = false;
    s->arena.release(q.arena_off, q.bytes);
    return ZINC_OK;
}

zinc_status zinc_server_drain(zinc_server* s) {
    if (!s) return plan_fail(ZINC_E_INVAL, "zinc_server_drain: null server");
    while (s->outstanding) {
        zinc_status st = zinc_server_progress(s, nullptr);
        if (st != ZINC_OK) return st;
        bool running = false;
        for (const Lane& l : s->lanes) running |= l.busy;
        if (!running && s->admitted.empty() && !s->waiting.empty())   // only held outputs can free the arena
            return plan_fail(ZINC_E_STATE, "zinc_server_drain: waiting requests need retained outputs to be released");
    }
    return ZINC_OK;
}

zinc_status zinc_server_destroy(zinc_server* s) {
    if (!s) return ZINC_OK;
    return release_all(s);
}

zinc_status zinc_serve_trace(zinc_ctx* const* ctxs, uint32_t n_ctx, const zinc_server_config* cfg,
                             const zinc_request* reqs, const uint64_t* arrival_ns, uint32_t n_req,
                             zinc_request_times* times) {
    if ((!reqs || !arrival_ns || !times) && n_req) return plan_fail(ZINC_E_INVAL, "zinc_serve_trace: null argument");
    if (cfg && cfg->retain_outputs)
        return plan_fail(ZINC_E_INVAL, "zinc_serve_trace: a replay releases outputs as requests complete (retain_outputs 0)");
    for (uint32_t i = 1; i < n_req; ++i)
        if (arrival_ns[i] < arrival_ns[i - 1])
            return plan_fail(ZINC_E_INVAL, "zinc_serve_trace: arrivals must be non-decreasing");
    zinc_server* s = nullptr;
    zinc_status st = zinc_server_create(ctxs, n_ctx, cfg, &s);
    if (st != ZINC_OK) return st;
    s->reqs.reserve(n_req);
    // Validate the whole trace before the clock starts.
    for (uint32_t i = 0; i < n_req; ++i) {
        st = zinc_server_submit(s, &reqs[i], nullptr);
        if (st != ZINC_OK) {
            release_all(s);
            return st;
        }
    }
    s->reqs.clear();
    s->waiting.clear();
    s->outstanding = 0;
    const uint64_t start = s->now();
    uint32_t next = 0;
    while (next < n_req || s->outstanding) {
        const uint64_t t = s->now() - start;
        while (next < n_req && arrival_ns[next] <= t) {
            st = zinc_server_submit(s, &reqs[next], nullptr);
            if (st != ZINC_OK) break;
            s->reqs.back().t.submit_ns = start + arrival_ns[next];
            ++next;
        }
        if (st == ZINC_OK) st = zinc_server_progress(s, nullptr);
        if (st != ZINC_OK) {
            release_all(s);
            return st;
        }
    }
    for (uint32_t i = 0; i < n_req; ++i) {
        zinc_request_times t = s->reqs[i].t;
        t.submit_ns -= start;
        t.admit_ns -= start;
        t.launch_ns -= start;
        t.done_ns -= start;
        times[i] = t;
    }
    return release_all(s);
}

}  // extern "C"
