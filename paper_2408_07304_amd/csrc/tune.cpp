// Per-context tuning: form of the fused kernel (thread geometry, epilogue) and
// NTT arithmetic per limb, chosen by timing every combination, with an
// on-disk cache.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "zinc_internal.h"

using namespace zinc;

namespace {

// A candidate replaces an earlier (preferred) one only if it is faster by more
// than this fraction, so that near-ties resolve the same way run after run.
constexpr double kMinGain = 0.01;

// Kernel time (ms) spent before the first timed candidate (Bench::settle),
// and the number of sweeps over the candidates.
constexpr double kSettleMs = 200.0;
constexpr int kRounds = 2;

// Forms of the fused kernel: (coefficients per thread, register epilogue).
bool form_ok(uint32_t log_n, uint32_t tile, bool reg) {
    if (log_n == 15) return tile == 16 && !reg;
    if (tile == 16) return true;
    if (tile == 8) return log_n == 12 || log_n == 13;
    if (tile == 32) return !reg;
    return false;
}

uint32_t fp_eligible(const zinc_ctx* c) {
    uint32_t m = 0;
    for (uint32_t l = 0; l < c->M; ++l)
        if (c->q[l] < kFpBound) m |= 1u << l;
    return m;
}

// Rewrite the limb constants' arithmetic field and upload them.
zinc_status apply_arith(zinc_ctx* c, uint32_t mask) {
    for (uint32_t l = 0; l < c->M; ++l) {
        const uint64_t q = c->q[l];
        c->h_limbs[l].fp = (mask >> l & 1u) ? (q >= kFpNoReduceBound ? 2u : 1u) : 0u;
    }
    const hipError_t e = hipMemcpy(const_cast<LimbConst*>(c->dev.limbs), c->h_limbs, sizeof(LimbConst) * c->M,
                                   hipMemcpyHostToDevice);
    if (e != hipSuccess) return plan_fail(ZINC_E_HIP, std::string("limb table upload: ") + hipGetErrorString(e));
    c->fp64_mask = mask;
    return ZINC_OK;
}

std::string cache_key(const zinc_ctx* c, uint32_t batch) {
    hipDeviceProp_t prop;
    std::memset(&prop, 0, sizeof(prop));
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    std::ostringstream k;
    std::string arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == ' ') ch = '_';
    k << arch << ' ' << prop.multiProcessorCount << ' ' << c->log_n << ' ' << batch << ' ';
    for (uint32_t l = 0; l < c->M; ++l) k << (l ? "," : "") << c->q[l];
    return k.str();
}

// Cache file: one line per result,
// "zinc-tune-2 <key fields> : <tile_v> <tile_z> <mask> <reg_epilogue>".
bool cache_lookup(const char* path, const std::string& key, zinc_tuning* t) {
    std::ifstream f(path);
    std::string line;
    const std::string head = "zinc-tune-2 " + key + " : ";
    while (std::getline(f, line)) {
        if (line.compare(0, head.size(), head) != 0) continue;
        std::istringstream v(line.substr(head.size()));
        zinc_tuning r{};
        if (v >> r.tile[0] >> r.tile[1] >> r.ntt_fp64_mask >> r.reg_epilogue) {
            *t = r;
            return true;
        }
    }
    return false;
}

void cache_store(const char* path, const std::string& key, const zinc_tuning& t) {
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        const std::string head = "zinc-tune-2 " + key + " : ";
        while (std::getline(f, line))
            if (!line.empty() && line.compare(0, head.size(), head) != 0) keep.push_back(line);
    }
    std::ostringstream o;
    o << "zinc-tune-2 " << key << " : " << t.tile[0] << ' ' << t.tile[1] << ' ' << t.ntt_fp64_mask << ' '
      << t.reg_epilogue;
    keep.push_back(o.str());
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        for (const auto& l : keep) f << l << '\n';
        if (!f) return;   // the cache is an optimisation: failures to write it are ignored
    }
    std::rename(tmp.c_str(), path);
}

struct Bench {
    zinc_ctx* c;
    uint32_t batch;
    double* slots;
    uint64_t* ids;
    uint64_t* ct;
    hipStream_t s;
    hipEvent_t a, b;

    // Median time of one batch in ms, or a negative value on failure.
    double time(int scheme) {
        constexpr int kWarm = 2, kRuns = 9;
        std::vector<double> ms;
        for (int i = 0; i < kWarm + kRuns; ++i) {
            if (hipEventRecord(a, s) != hipSuccess) return -1;
            if (zinc_encrypt_slots(c, scheme, slots, c->n / 2, batch, ids, ct, s) != ZINC_OK) return -1;
            if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return -1;
            float t = 0;
            if (hipEventElapsedTime(&t, a, b) != hipSuccess) return -1;
            if (i >= kWarm) ms.push_back(t);
        }
        std::sort(ms.begin(), ms.end());
        return ms[ms.size() / 2];
    }

    // The GPU's clocks rise over the first tens of milliseconds under load:
    // run `scheme` until about `target_ms` of kernel time has passed, so that
    // the first candidates are not timed at lower clocks than the last.
    bool settle(int scheme, double target_ms) {
        double done = 0;
        for (int round = 0; round < 4096 && done < target_ms; ++round) {
            if (hipEventRecord(a, s) != hipSuccess) return false;
            for (int i = 0; i < 4; ++i)
                if (zinc_encrypt_slots(c, scheme, slots, c->n / 2, batch, ids, ct, s) != ZINC_OK) return false;
            if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return false;
            float t = 0;
            if (hipEventElapsedTime(&t, a, b) != hipSuccess) return false;
            done += t;
        }
        return true;
    }
};

}  // namespace

extern "C" {

zinc_status zinc_set_tuning(zinc_ctx* c, const zinc_tuning* t) {
    if (!c || !t) return plan_fail(ZINC_E_INVAL, "zinc_set_tuning: null argument");
    if (t->reg_epilogue & ~3u) return plan_fail(ZINC_E_INVAL, "zinc_set_tuning: reg_epilogue has bits 0 and 1 only");
    for (int s = 0; s < 2; ++s)
        if (!form_ok(c->log_n, t->tile[s], (t->reg_epilogue >> s) & 1u))
            return plan_fail(ZINC_E_INVAL, "zinc_set_tuning: kernel form not available for this ring degree");
    if (t->ntt_fp64_mask & ~fp_eligible(c))
        return plan_fail(ZINC_E_INVAL, "zinc_set_tuning: FP64 arithmetic needs a modulus below 2^50");
    if (t->ntt_fp64_mask != c->fp64_mask) {
        if (zinc_status st = apply_arith(c, t->ntt_fp64_mask)) return st;
    }
    c->tile[0] = t->tile[0];
    c->tile[1] = t->tile[1];
    c->reg_epilogue = t->reg_epilogue;
    return ZINC_OK;
}

zinc_status zinc_get_tuning(const zinc_ctx* c, zinc_tuning* t) {
    if (!c || !t) return plan_fail(ZINC_E_INVAL, "zinc_get_tuning: null argument");
    *t = zinc_tuning{{c->tile[0], c->tile[1]}, c->fp64_mask, c->reg_epilogue};
    return ZINC_OK;
}

zinc_status zinc_autotune(zinc_ctx* c, uint32_t batch, const char* cache_path, zinc_tune_result* out) {
    if (!c || !out) return plan_fail(ZINC_E_INVAL, "zinc_autotune: null argument");
    if (batch == 0 || batch > 65536) return plan_fail(ZINC_E_INVAL, "zinc_autotune: batch must be in [1, 65536]");
    if (!c->keyed) return plan_fail(ZINC_E_STATE, "zinc_autotune before zinc_keygen");
    if (c->dev.noise_t > 1) return plan_fail(ZINC_E_STATE, "zinc_autotune: a BGV context has no slot encryption");
    std::memset(out, 0, sizeof(*out));
    const std::string key = cache_key(c, batch);
    if (cache_path) {
        zinc_tuning t{};
        if (cache_lookup(cache_path, key, &t) && zinc_set_tuning(c, &t) == ZINC_OK) {
            out->chosen = t;
            out->from_cache = 1;
            return ZINC_OK;
        }
    }
    const uint32_t eligible = fp_eligible(c), default_mask = c->fp64_mask;
    std::vector<uint32_t> masks{default_mask};
    if (default_mask != 0) masks.push_back(0u);
    if (default_mask != eligible) masks.push_back(eligible);
    struct Form {
        uint32_t tile;
        bool reg;
    };
    std::vector<Form> forms;
    for (uint32_t t : {16u, 8u, 32u})
        for (bool r : {false, true})
            if (form_ok(c->log_n, t, r)) forms.push_back(Form{t, r});
    const int n_schemes = c->precomputed ? 2 : 1;

    Bench bn{c, batch, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    const size_t b_slots = sizeof(double) * batch * (c->n / 2), b_ids = 8ull * batch;
    const size_t b_ct = 16ull * batch * c->L * c->n;
    char* mem = nullptr;
    hipError_t e = hipMalloc(&mem, b_slots + b_ids + b_ct);
    if (e != hipSuccess) return plan_fail(ZINC_E_NOMEM, "zinc_autotune: scratch allocation failed");
    bn.slots = reinterpret_cast<double*>(mem);
    bn.ids = reinterpret_cast<uint64_t*>(mem + b_slots);
    bn.ct = reinterpret_cast<uint64_t*>(mem + b_slots + b_ids);
    e = hipStreamCreateWithFlags(&bn.s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&bn.a);
    if (e == hipSuccess) e = hipEventCreate(&bn.b);
    if (e == hipSuccess) {
        // slot values uniform on [-1, 1) (a fixed splitmix64 sequence): timing on
        // zeros would flatter every candidate (lower switching power, higher clocks)
        std::vector<double> z((size_t)batch * (c->n / 2));
        uint64_t x = 0x9E3779B97F4A7C15ull;
        for (double& v : z) {
            uint64_t r = (x += 0x9E3779B97F4A7C15ull);
            r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ull;
            r = (r ^ (r >> 27)) * 0x94D049BB133111EBull;
            r ^= r >> 31;
            v = (double)(r >> 11) * 0x1p-52 - 1.0;
        }
        e = hipMemcpy(bn.slots, z.data(), b_slots, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
        std::vector<uint64_t> ids(batch);
        for (uint32_t i = 0; i < batch; ++i) ids[i] = i;
        e = hipMemcpy(bn.ids, ids.data(), b_ids, hipMemcpyHostToDevice);
    }
    const uint32_t saved_tile[2] = {c->tile[0], c->tile[1]}, saved_reg = c->reg_epilogue;
    zinc_status st = ZINC_OK;
    double best_total = -1;
    zinc_tuning best{{saved_tile[0], saved_tile[1]}, default_mask, saved_reg};
    if (e != hipSuccess) st = plan_fail(ZINC_E_HIP, std::string("zinc_autotune: setup: ") + hipGetErrorString(e));
    if (st == ZINC_OK && !bn.settle(0, kSettleMs))
        st = plan_fail(ZINC_E_HIP, "zinc_autotune: warm-up launch failed");
    // Every candidate is timed in each of kRounds sweeps and keeps its best
    // median, so that a slow moment of the GPU does not decide the choice.
    const size_t nf = forms.size();
    std::vector<double> ms((size_t)masks.size() * 2 * nf, -1.0);
    auto at = [&](size_t mi, int sc, size_t fi) -> double& { return ms[(mi * 2 + (size_t)sc) * nf + fi]; };
    for (int round = 0; st == ZINC_OK && round < kRounds; ++round) {
        for (size_t mi = 0; st == ZINC_OK && mi < masks.size(); ++mi) {
            st = apply_arith(c, masks[mi]);
            for (int sc = 0; st == ZINC_OK && sc < n_schemes; ++sc) {
                for (size_t fi = 0; fi < nf; ++fi) {
                    c->tile[sc] = forms[fi].tile;
                    c->reg_epilogue = (c->reg_epilogue & ~(1u << sc)) | ((forms[fi].reg ? 1u : 0u) << sc);
                    const double t = bn.time(sc);
                    ++out->n_timed;
                    if (t < 0) {
                        st = plan_fail(ZINC_E_HIP, "zinc_autotune: timed launch failed");
                        break;
                    }
                    double& m = at(mi, sc, fi);
                    if (m < 0 || t < m) m = t;
                }
            }
        }
    }
    for (size_t mi = 0; st == ZINC_OK && mi < masks.size(); ++mi) {
        double total = 0;
        Form pick[2] = {{16u, false}, {16u, false}};
        double pick_ms[2] = {0, 0};
        for (int sc = 0; sc < n_schemes; ++sc) {
            double bm = -1;
            for (size_t fi = 0; fi < nf; ++fi) {
                const Form& f = forms[fi];
                const double t = at(mi, sc, fi);
                if (mi == 0 && f.tile == 16 && !f.reg) out->default_ms[sc] = t;
                // candidates come in order of preference (default form first);
                // a later one must be faster by more than the timing noise
                if (bm < 0 || t < bm * (1.0 - kMinGain)) {
                    bm = t;
                    pick[sc] = f;
                }
            }
            pick_ms[sc] = bm;
            total += bm;
        }
        if (best_total < 0 || total < best_total * (1.0 - kMinGain)) {
            best_total = total;
            const uint32_t reg = (pick[0].reg ? 1u : 0u) |
                                 (n_schemes == 2 ? (pick[1].reg ? 2u : 0u) : (saved_reg & 2u));
            best = zinc_tuning{{pick[0].tile, n_schemes == 2 ? pick[1].tile : saved_tile[1]}, masks[mi], reg};
            out->best_ms[0] = pick_ms[0];
            out->best_ms[1] = pick_ms[1];
        }
    }
    if (bn.a) (void)hipEventDestroy(bn.a);
    if (bn.b) (void)hipEventDestroy(bn.b);
    if (bn.s) (void)hipStreamDestroy(bn.s);
    (void)hipFree(mem);
    if (st != ZINC_OK) {
        c->tile[0] = saved_tile[0];
        c->tile[1] = saved_tile[1];
        c->reg_epilogue = saved_reg;
        (void)apply_arith(c, default_mask);
        return st;
    }
    c->tile[0] = best.tile[0];
    c->tile[1] = best.tile[1];
    c->reg_epilogue = best.reg_epilogue;
    st = apply_arith(c, best.ntt_fp64_mask);
    if (st != ZINC_OK) return st;
    out->chosen = best;
    if (cache_path) cache_store(cache_path, key, best);
    return ZINC_OK;
}

}  // extern "C"
