// C ABI of the library: parameter validation, context construction (moduli,
// roots of unity, twiddle / FFT / sampler tables), the Gen -> precompute ->
// Enc / Enc_z state machine and the argument checks of every entry point.
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "zinc_internal.h"

namespace zinc {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

static zinc_status fail(zinc_status code, const std::string& msg) {
    set_error(msg);
    return code;
}

zinc_status plan_fail(zinc_status code, const std::string& msg) { return fail(code, msg); }

static zinc_status hip_fail(hipError_t e, const char* what) {
    return fail(ZINC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static uint32_t bitrev(uint32_t x, int bits) {
    uint32_t r = 0;
    for (int i = 0; i < bits; ++i) r = (r << 1) | ((x >> i) & 1u);
    return r;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace zinc

using namespace zinc;

extern "C" {

const char* zinc_last_error(void) { return g_last_error.c_str(); }

zinc_status zinc_ctx_create(const zinc_params* p, zinc_ctx** out) {
    if (!p || !out) return fail(ZINC_E_INVAL, "zinc_ctx_create: null argument");
    *out = nullptr;
    if (p->log_n < 12 || p->log_n > 15)
        return fail(ZINC_E_PARAM, "log_n must be in [12, 15] (ring degree 4096..32768)");
    if (p->n_moduli < 2 || p->n_moduli > ZINC_MAX_MODULI)
        return fail(ZINC_E_PARAM, "n_moduli must be in [2, 32] (data limbs plus the special prime)");
    if (!(p->scale > 0.0) || !std::isfinite(p->scale) || p->scale >= 4611686018427387904.0)
        return fail(ZINC_E_PARAM, "scale must be finite, positive and below 2^62");
    if (std::fabs(p->sigma - 3.2) > 1e-12)
        return fail(ZINC_E_PARAM, "sigma must be 3.2 (the error distribution's standard deviation)");
    const uint32_t M = p->n_moduli, n = 1u << p->log_n;
    const uint64_t two_n = 2ull * n;
    uint64_t q[ZINC_MAX_MODULI];
    if (p->moduli) {
        for (uint32_t i = 0; i < M; ++i) {
            q[i] = p->moduli[i];
            if (q[i] >= (1ull << 60) || q[i] <= two_n || q[i] % two_n != 1 || !is_prime(q[i]))
                return fail(ZINC_E_PARAM, "modulus " + std::to_string(i) +
                                              " is not a prime = 1 mod 2N below 2^60");
            for (uint32_t j = 0; j < i; ++j)
                if (q[j] == q[i]) return fail(ZINC_E_PARAM, "moduli must be distinct");
        }
    } else {
        if (!p->bit_sizes) return fail(ZINC_E_INVAL, "either moduli or bit_sizes must be given");
        for (uint32_t i = 0; i < M; ++i)
            if (p->bit_sizes[i] < 20 || p->bit_sizes[i] > 60 || p->bit_sizes[i] < p->log_n + 2)
                return fail(ZINC_E_PARAM, "bit sizes must be in [20, 60]");
        if (!choose_moduli(p->log_n, M, p->bit_sizes, q))
            return fail(ZINC_E_PARAM, "not enough primes = 1 mod 2N for the requested bit sizes");
    }

    zinc_ctx* c = new (std::nothrow) zinc_ctx();
    if (!c) return fail(ZINC_E_NOMEM, "host allocation failed");
    (void)hipGetDevice(&c->device);
    c->log_n = p->log_n;
    c->n = n;
    c->M = M;
    c->L = M - 1;
    c->scale = p->scale;
    c->sigma = p->sigma;
    c->seed = p->seed;
    for (uint32_t i = 0; i < M; ++i) {
        c->q[i] = q[i];
        c->psi[i] = smallest_psi(q[i], p->log_n);
    }
    gaussian_cdt(p->sigma, c->cdt);

    // ---- host tables ----
    const uint32_t H = n / 2;
    const int logh = (int)p->log_n - 1;
    std::vector<LimbConst> limbs(M);
    std::vector<uint64_t> tw((size_t)M * n * 2), itw((size_t)M * n * 2);
    std::vector<double> tw_fp((size_t)M * n * 2);
    // ZINC_NTT_ARITH=int forces the integer path for every modulus.
    const char* arith = std::getenv("ZINC_NTT_ARITH");
    const bool force_int = arith && std::strcmp(arith, "int") == 0;
    std::vector<uint64_t> pw(n);
    for (uint32_t l = 0; l < M; ++l) {
        const uint64_t ql = q[l];
        limbs[l].q = ql;
        limbs[l].q2 = 2 * ql;
        limbs[l].bar = shoup_companion(1, ql);
        limbs[l].ninv = powmod_host(n, ql - 2, ql);
        limbs[l].ninv_sh = shoup_companion(limbs[l].ninv, ql);
        limbs[l].half = (ql - 1) / 2;
        if (l + 1 < M) {
            limbs[l].pinv = powmod_host(q[M - 1] % ql, ql - 2, ql);
            limbs[l].pinv_sh = shoup_companion(limbs[l].pinv, ql);
        }
        limbs[l].qd = (double)ql;
        limbs[l].qinv = (double)(1.0L / (long double)ql);
        limbs[l].fp = force_int || ql >= kFpBound ? 0u : (ql >= kFpNoReduceBound ? 2u : 1u);
        if (limbs[l].fp) c->fp64_mask |= 1u << l;
        c->h_limbs[l] = limbs[l];
        for (int inv = 0; inv < 2; ++inv) {
            const uint64_t root = inv ? powmod_host(c->psi[l], ql - 2, ql) : c->psi[l];
            pw[0] = 1;
            for (uint32_t i = 1; i < n; ++i) pw[i] = mulmod_host(pw[i - 1], root, ql);
            uint64_t* dst = (inv ? itw.data() : tw.data()) + (size_t)l * n * 2;
            for (uint32_t k = 0; k < n; ++k) {
                const uint64_t w = pw[bitrev(k, (int)p->log_n)];
                dst[2 * k] = w;
                dst[2 * k + 1] = shoup_companion(w, ql);
                if (!inv && ql < kFpBound) {
                    tw_fp[((size_t)l * n + k) * 2] = (double)w;
                    tw_fp[((size_t)l * n + k) * 2 + 1] = (double)((long double)w / (long double)ql);
                }
            }
        }
    }
    const long double pi = 3.14159265358979323846264338327950288L;
    std::vector<double> fft_tw(H), twist(2 * H);
    for (uint32_t k = 0; k < H / 2; ++k) {
        const long double a = -2.0L * pi * (long double)k / (long double)H;
        fft_tw[2 * k] = (double)cosl(a);
        fft_tw[2 * k + 1] = (double)sinl(a);
    }
    for (uint32_t i = 0; i < H; ++i) {
        const long double a = -pi * (long double)i / (long double)n;
        twist[2 * i] = (double)cosl(a);
        twist[2 * i + 1] = (double)sinl(a);
    }
    std::vector<uint32_t> slot_pos(H);
    uint64_t g = 1;
    for (uint32_t j = 0; j < H; ++j) {
        slot_pos[j] = bitrev((uint32_t)((g - 1) / 4), logh);
        g = g * 5 % two_n;
    }
    uint64_t cdt[kCdtTab];
    for (int i = 0; i < kCdtPad; ++i) cdt[i] = i < kCdtLen ? c->cdt[i] : ~0ull;
    gaussian_buckets(c->cdt, cdt + kCdtPad);

    // ---- one device block ----
    const size_t nb = (size_t)n * 8, L = c->L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    const size_t o_limbs = take(sizeof(LimbConst) * M);
    const size_t o_tw = take(nb * 2 * M), o_itw = take(nb * 2 * M), o_twfp = take(nb * 2 * M);
    const size_t o_fft = take(sizeof(double) * H), o_twist = take(sizeof(double) * 2 * H);
    const size_t o_pos = take(4 * H), o_cdt = take(8 * kCdtTab);
    const size_t o_sk = take(nb * M), o_sks = take(nb * M);
    const size_t o_pk = take(nb * 2 * M), o_pks = take(nb * 2 * M);
    const size_t o_zero = take(nb * 2 * L), o_pkp = take(nb * 2 * L), o_pkps = take(nb * 2 * L);
    const size_t o_err = take(256);
    const size_t o_self = take(sizeof(DevParams));
    char* base = nullptr;
    hipError_t e = hipMalloc(&base, off);
    if (e != hipSuccess) {
        delete c;
        return fail(ZINC_E_NOMEM, std::string("hipMalloc of the context tables failed: ") + hipGetErrorString(e));
    }
    c->d_block = base;
    struct Up { size_t o; const void* src; size_t bytes; } ups[] = {
        {o_limbs, limbs.data(), sizeof(LimbConst) * M}, {o_tw, tw.data(), nb * 2 * M},
        {o_itw, itw.data(), nb * 2 * M}, {o_twfp, tw_fp.data(), nb * 2 * M},
        {o_fft, fft_tw.data(), sizeof(double) * H},
        {o_twist, twist.data(), sizeof(double) * 2 * H}, {o_pos, slot_pos.data(), 4 * H},
        {o_cdt, cdt, 8 * kCdtTab}};
    for (const Up& u : ups) {
        e = hipMemcpy(base + u.o, u.src, u.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(base);
            delete c;
            return hip_fail(e, "table upload");
        }
    }
    e = hipMemset(base + o_sk, 0, o_err + 256 - o_sk);
    if (e != hipSuccess) {
        (void)hipFree(base);
        delete c;
        return hip_fail(e, "hipMemset");
    }
    DevParams& d = c->dev;
    d.log_n = c->log_n;
    d.n = n;
    d.M = M;
    d.L = c->L;
    d.seed = c->seed;
    d.scale = c->scale;
    d.noise_t = 1;
    d.limbs = reinterpret_cast<const LimbConst*>(base + o_limbs);
    d.tw = reinterpret_cast<const uint64_t*>(base + o_tw);
    d.itw = reinterpret_cast<const uint64_t*>(base + o_itw);
    d.tw_fp = reinterpret_cast<const double*>(base + o_twfp);
    d.fft_tw = reinterpret_cast<const double*>(base + o_fft);
    d.twist = reinterpret_cast<const double*>(base + o_twist);
    d.slot_pos = reinterpret_cast<const uint32_t*>(base + o_pos);
    d.cdt = reinterpret_cast<const uint64_t*>(base + o_cdt);
    d.sk = reinterpret_cast<const uint64_t*>(base + o_sk);
    d.sk_sh = reinterpret_cast<const uint64_t*>(base + o_sks);
    d.pk = reinterpret_cast<const uint64_t*>(base + o_pk);
    d.pk_sh = reinterpret_cast<const uint64_t*>(base + o_pks);
    d.zero = reinterpret_cast<const uint64_t*>(base + o_zero);
    d.pkp = reinterpret_cast<const uint64_t*>(base + o_pkp);
    d.pkp_sh = reinterpret_cast<const uint64_t*>(base + o_pkps);
    d.err = reinterpret_cast<uint32_t*>(base + o_err);
    d.self = reinterpret_cast<const DevParams*>(base + o_self);
    e = hipMemcpy(base + o_self, &d, sizeof(DevParams), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(base);
        delete c;
        return hip_fail(e, "parameter upload");
    }
    *out = c;
    return ZINC_OK;
}

zinc_status zinc_ctx_destroy(zinc_ctx* c) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_ctx_destroy: null context");
    (void)hipDeviceSynchronize();
    if (c->d_block) (void)hipFree(c->d_block);
    for (const auto& b : c->batch_tables) (void)hipFree(b.d);
    delete c;
    return ZINC_OK;
}

zinc_status zinc_ctx_info(const zinc_ctx* c, zinc_info* o) {
    if (!c || !o) return fail(ZINC_E_INVAL, "zinc_ctx_info: null argument");
    std::memset(o, 0, sizeof(*o));
    o->n = c->n;
    o->log_n = c->log_n;
    o->n_moduli = c->M;
    o->limbs = c->L;
    for (uint32_t i = 0; i < c->M; ++i) {
        o->moduli[i] = c->q[i];
        o->psi[i] = c->psi[i];
    }
    o->scale = c->scale;
    o->seed = c->seed;
    for (int i = 0; i < kCdtLen; ++i) o->cdt[i] = c->cdt[i];
    o->plaintext_bytes = (size_t)c->L * c->n * 8;
    o->ciphertext_bytes = 2 * (size_t)c->L * c->n * 8;
    o->keyed = c->keyed;
    o->precomputed = c->precomputed;
    o->ntt_fp64_mask = c->fp64_mask;
    o->tile[0] = c->tile[0];
    o->tile[1] = c->tile[1];
    o->reg_epilogue = c->reg_epilogue;
    o->bgv_t = c->dev.noise_t > 1 ? c->dev.noise_t : 0;
    return ZINC_OK;
}

static zinc_status launched(hipError_t e, const char* what) {
    if (e != hipSuccess) return hip_fail(e, what);
    return ZINC_OK;
}

zinc_status zinc_keygen(zinc_ctx* c, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_keygen: null context");
    DevParams& d = c->dev;
    zinc_status st = launched(launch_keygen(d, const_cast<uint64_t*>(d.sk), const_cast<uint64_t*>(d.sk_sh),
                                            const_cast<uint64_t*>(d.pk), const_cast<uint64_t*>(d.pk_sh),
                                            (hipStream_t)stream),
                              "keygen launch");
    if (st == ZINC_OK)
        st = launched(launch_scale_pk(d, const_cast<uint64_t*>(d.pkp), const_cast<uint64_t*>(d.pkp_sh),
                                      (hipStream_t)stream),
                      "keygen launch");
    if (st == ZINC_OK) {
        c->keyed = true;
        c->precomputed = false;
    }
    return st;
}

zinc_status zinc_precompute(zinc_ctx* c, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_precompute: null context");
    if (!c->keyed) return fail(ZINC_E_STATE, "zinc_precompute before zinc_keygen");
    hipStream_t s = (hipStream_t)stream;
    uint64_t* tmp = nullptr;
    const size_t words = (size_t)c->L * c->n + 1;
    hipError_t e = hipMalloc(&tmp, words * 8);
    if (e != hipSuccess) return fail(ZINC_E_NOMEM, "zinc_precompute: scratch allocation failed");
    const uint64_t id = ZINC_ZERO_ID;
    e = hipMemsetAsync(tmp, 0, (words - 1) * 8, s);
    if (e == hipSuccess) e = hipMemcpyAsync(tmp + words - 1, &id, 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_encrypt_pt(c->dev, ZINC_SCHEME_VANILLA, tmp, 1, tmp + words - 1,
                              const_cast<uint64_t*>(c->dev.zero), s, true);
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "zinc_precompute");
    if (e2 != hipSuccess) return hip_fail(e2, "zinc_precompute (synchronise)");
    c->precomputed = true;
    return ZINC_OK;
}

static zinc_status check_batch(const char* fn, uint32_t batch, std::initializer_list<const void*> ptrs) {
    if (batch == 0) return ZINC_OK;
    for (const void* q : ptrs)
        if (!q) return fail(ZINC_E_INVAL, std::string(fn) + ": null buffer");
    return ZINC_OK;
}

// Special-prime vanilla: scratch of [batch][3][N] int64 (message and the two
// rounding offsets), allocated and freed in stream order around the launch.
static zinc_status encrypt_sp(zinc_ctx* c, bool from_slots, const double* slots, uint32_t n_slots,
                              const uint64_t* pt, uint32_t batch, const uint64_t* ids, uint64_t* ct, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    int64_t* ws = nullptr;
    hipError_t e = hipMallocAsync((void**)&ws, (size_t)batch * 3 * c->n * sizeof(int64_t), s);
    if (e != hipSuccess) return fail(ZINC_E_NOMEM, "special-prime vanilla: scratch allocation failed");
    const hipError_t le = launch_encrypt_sp(c->dev, from_slots, slots, n_slots, pt, batch, ids, ct, ws, s);
    e = hipFreeAsync(ws, s);
    if (le != hipSuccess) return hip_fail(le, "special-prime vanilla launch");
    if (e != hipSuccess) return hip_fail(e, "special-prime vanilla: scratch release");
    return ZINC_OK;
}

zinc_status zinc_encode(zinc_ctx* c, const double* slots, uint32_t n_slots, uint32_t batch, uint64_t* pt,
                        void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_encode: null context");
    if (n_slots > c->n / 2) return fail(ZINC_E_RANGE, "zinc_encode: n_slots exceeds N/2");
    if (zinc_status s = check_batch("zinc_encode", batch, {slots, pt})) return s;
    if (batch == 0) return ZINC_OK;
    return launched(launch_encode(c->dev, slots, n_slots, batch, pt, (hipStream_t)stream), "encode launch");
}

zinc_status zinc_encrypt_vanilla(zinc_ctx* c, const uint64_t* pt, uint32_t batch, const uint64_t* ids,
                                 uint64_t* ct, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_encrypt_vanilla: null context");
    if (!c->keyed) return fail(ZINC_E_STATE, "zinc_encrypt_vanilla before zinc_keygen");
    if (zinc_status s = check_batch("zinc_encrypt_vanilla", batch, {pt, ids, ct})) return s;
    if (batch == 0) return ZINC_OK;
    return launched(launch_encrypt_pt(c->dev, ZINC_SCHEME_VANILLA, pt, batch, ids, ct, (hipStream_t)stream),
                    "vanilla encrypt launch");
}

zinc_status zinc_encrypt(zinc_ctx* c, const uint64_t* pt, uint32_t batch, const uint64_t* ids, uint64_t* ct,
                         void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_encrypt: null context");
    if (!c->precomputed) return fail(ZINC_E_STATE, "zinc_encrypt before zinc_precompute");
    if (zinc_status s = check_batch("zinc_encrypt", batch, {pt, ids, ct})) return s;
    if (batch == 0) return ZINC_OK;
    return launched(launch_encrypt_pt(c->dev, ZINC_SCHEME_ZINC, pt, batch, ids, ct, (hipStream_t)stream),
                    "zinc encrypt launch");
}

zinc_status zinc_encrypt_slots(zinc_ctx* c, int scheme, const double* slots, uint32_t n_slots, uint32_t batch,
                               const uint64_t* ids, uint64_t* ct, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_encrypt_slots: null context");
    if (scheme != ZINC_SCHEME_VANILLA && scheme != ZINC_SCHEME_ZINC && scheme != ZINC_SCHEME_VANILLA_SP)
        return fail(ZINC_E_INVAL, "zinc_encrypt_slots: scheme must be 0 (vanilla), 1 (zinc) or 2 (vanilla_sp)");
    if (!c->keyed) return fail(ZINC_E_STATE, "zinc_encrypt_slots before zinc_keygen");
    if (c->dev.noise_t > 1) return fail(ZINC_E_STATE, "zinc_encrypt_slots: a BGV context encrypts integer plaintexts");
    if (scheme == ZINC_SCHEME_ZINC && !c->precomputed)
        return fail(ZINC_E_STATE, "zinc_encrypt_slots (zinc) before zinc_precompute");
    if (n_slots > c->n / 2) return fail(ZINC_E_RANGE, "zinc_encrypt_slots: n_slots exceeds N/2");
    if (zinc_status s = check_batch("zinc_encrypt_slots", batch, {slots, ids, ct})) return s;
    if (batch == 0) return ZINC_OK;
    if (scheme == ZINC_SCHEME_VANILLA_SP) return encrypt_sp(c, true, slots, n_slots, nullptr, batch, ids, ct, stream);
    const uint32_t tile = c->tile[scheme];
    const bool reg = (c->reg_epilogue >> scheme) & 1u;
    if (tile != 16 || reg)
        return launched(launch_encrypt_slots_tile(c->dev, scheme, tile == 8 ? kTileR8 : tile == 32 ? kTileR32 : kTileR16,
                                                  reg, slots, n_slots, batch, ids, ct, (hipStream_t)stream),
                        "fused encrypt launch");
    return launched(launch_encrypt_slots(c->dev, scheme, slots, n_slots, batch, ids, ct, (hipStream_t)stream),
                    "fused encrypt launch");
}

zinc_status zinc_encrypt_vanilla_sp(zinc_ctx* c, const uint64_t* pt, uint32_t batch, const uint64_t* ids,
                                    uint64_t* ct, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_encrypt_vanilla_sp: null context");
    if (!c->keyed) return fail(ZINC_E_STATE, "zinc_encrypt_vanilla_sp before zinc_keygen");
    if (c->dev.noise_t > 1) return fail(ZINC_E_STATE, "zinc_encrypt_vanilla_sp: not built for BGV contexts");
    if (zinc_status s = check_batch("zinc_encrypt_vanilla_sp", batch, {pt, ids, ct})) return s;
    if (batch == 0) return ZINC_OK;
    return encrypt_sp(c, false, nullptr, 0, pt, batch, ids, ct, stream);
}

// The same encryption with the scratch rows in the library's static device
// array instead of stream-ordered allocations (callers that cannot allocate).
zinc_status zinc_encrypt_vanilla_sp_noalloc(zinc_ctx* c, const uint64_t* pt, uint32_t batch, const uint64_t* ids,
                                            uint64_t* ct, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_encrypt_vanilla_sp_noalloc: null context");
    if (!c->keyed) return fail(ZINC_E_STATE, "zinc_encrypt_vanilla_sp_noalloc before zinc_keygen");
    if (c->dev.noise_t > 1) return fail(ZINC_E_STATE, "zinc_encrypt_vanilla_sp_noalloc: not built for BGV contexts");
    if (zinc_status s = check_batch("zinc_encrypt_vanilla_sp_noalloc", batch, {pt, ids, ct})) return s;
    if (batch == 0) return ZINC_OK;
    const size_t per_ct = (size_t)3 * c->n * sizeof(int64_t);
    if ((size_t)batch * per_ct > kSpScratchBytes)
        return fail(ZINC_E_RANGE, "zinc_encrypt_vanilla_sp_noalloc: at most " +
                                      std::to_string(kSpScratchBytes / per_ct) + " ciphertexts of ring degree " +
                                      std::to_string(c->n) + " per call (" +
                                      std::to_string(kSpScratchBytes >> 20) + " MiB of static scratch)");
    long long* ws = nullptr;
    const hipError_t e = sp_scratch(c->device, &ws);
    if (e != hipSuccess) return hip_fail(e, "zinc_encrypt_vanilla_sp_noalloc: static scratch (is the context's device current?)");
    return launched(launch_encrypt_sp(c->dev, false, nullptr, 0, pt, batch, ids, ct, reinterpret_cast<int64_t*>(ws),
                                      (hipStream_t)stream),
                    "special-prime vanilla launch");
}

// Constants of the BFV encoding / decoding for plaintext modulus t.
static zinc_status bfv_consts(const zinc_ctx* c, uint64_t t, BfvConsts* k, const char* fn) {
    if (c->dev.noise_t > 1) return fail(ZINC_E_STATE, std::string(fn) + ": the context is in BGV form");
    if (t < 2 || t >= (1ull << 32)) return fail(ZINC_E_INVAL, std::string(fn) + ": t must be in [2, 2^32)");
    const uint32_t L = c->L;
    for (uint32_t l = 0; l < L; ++l)
        if (t >= c->q[l]) return fail(ZINC_E_INVAL, std::string(fn) + ": t must be below every data modulus");
    std::memset(k, 0, sizeof(*k));
    k->t = t;
    uint64_t q_mod_t = 1 % t;                                  // Q mod t
    for (uint32_t l = 0; l < L; ++l) q_mod_t = (uint64_t)((unsigned __int128)q_mod_t * (c->q[l] % t) % t);
    for (uint32_t l = 0; l < L; ++l) {
        const uint64_t q = c->q[l];
        uint64_t prod = 1;                                     // (Q / q_l) mod q_l
        for (uint32_t j = 0; j < L; ++j)
            if (j != l) prod = mulmod_host(prod, c->q[j] % q, q);
        const uint64_t qt = powmod_host(prod, q - 2, q);        // Qt_l
        const unsigned __int128 tq = (unsigned __int128)t * qt;
        k->b[l] = (uint64_t)(tq % q);
        k->b_sh[l] = shoup_companion(k->b[l], q);
        k->w_mod_t[l] = (uint64_t)((tq / q) % t);
        const uint64_t tinv = powmod_host(t % q, q - 2, q);
        k->delta[l] = mulmod_host((q - q_mod_t % q) % q, tinv, q); // (Q - (Q mod t)) / t mod q_l
        k->delta_sh[l] = shoup_companion(k->delta[l], q);
    }
    return ZINC_OK;
}

zinc_status zinc_bfv_encode(zinc_ctx* c, uint64_t t, const int64_t* m, uint32_t batch, uint64_t* pt, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_bfv_encode: null context");
    if (zinc_status s = check_batch("zinc_bfv_encode", batch, {m, pt})) return s;
    BfvConsts k;
    if (zinc_status s = bfv_consts(c, t, &k, "zinc_bfv_encode")) return s;
    if (batch == 0) return ZINC_OK;
    return launched(launch_bfv_encode(c->dev, k, m, batch, pt, (hipStream_t)stream), "BFV encode launch");
}

zinc_status zinc_bfv_decode(zinc_ctx* c, uint64_t t, const uint64_t* pt, uint32_t batch, int64_t* m, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_bfv_decode: null context");
    if (zinc_status s = check_batch("zinc_bfv_decode", batch, {pt, m})) return s;
    BfvConsts k;
    if (zinc_status s = bfv_consts(c, t, &k, "zinc_bfv_decode")) return s;
    if (batch == 0) return ZINC_OK;
    return launched(launch_bfv_decode(c->dev, k, pt, batch, m, (hipStream_t)stream), "BFV decode launch");
}

// BGV (Eq. 13): the plaintext modulus scales every error from the next keygen.
zinc_status zinc_set_bgv(zinc_ctx* c, uint64_t t) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_set_bgv: null context");
    if (t != 1) {
        if (t < 2 || t >= (1ull << 32)) return fail(ZINC_E_INVAL, "zinc_set_bgv: t must be 1 or in [2, 2^32)");
        for (uint32_t l = 0; l < c->L; ++l)
            if (t >= c->q[l]) return fail(ZINC_E_INVAL, "zinc_set_bgv: t must be below every data modulus");
    }
    c->dev.noise_t = t;
    c->keyed = false;
    c->precomputed = false;
    const hipError_t e = hipMemcpy(const_cast<DevParams*>(c->dev.self), &c->dev, sizeof(DevParams),
                                   hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "zinc_set_bgv: parameter upload");
    return ZINC_OK;
}

zinc_status zinc_bgv_encode(zinc_ctx* c, const int64_t* m, uint32_t batch, uint64_t* pt, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_bgv_encode: null context");
    if (c->dev.noise_t < 2) return fail(ZINC_E_STATE, "zinc_bgv_encode: the context is not in BGV form");
    if (zinc_status s = check_batch("zinc_bgv_encode", batch, {m, pt})) return s;
    if (batch == 0) return ZINC_OK;
    BfvConsts k;                                   // the BFV encoder with Delta = 1: m mod t on every limb
    std::memset(&k, 0, sizeof(k));
    k.t = c->dev.noise_t;
    for (uint32_t l = 0; l < c->L; ++l) {
        k.delta[l] = 1;
        k.delta_sh[l] = shoup_companion(1, c->q[l]);
    }
    return launched(launch_bfv_encode(c->dev, k, m, batch, pt, (hipStream_t)stream), "BGV encode launch");
}

zinc_status zinc_bgv_decode(zinc_ctx* c, const uint64_t* pt, uint32_t batch, int64_t* m, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_bgv_decode: null context");
    if (c->dev.noise_t < 2) return fail(ZINC_E_STATE, "zinc_bgv_decode: the context is not in BGV form");
    if (zinc_status s = check_batch("zinc_bgv_decode", batch, {pt, m})) return s;
    if (batch == 0) return ZINC_OK;
    const uint64_t t = c->dev.noise_t;
    const uint32_t L = c->L;
    BgvConsts k;
    std::memset(&k, 0, sizeof(k));
    k.t = t;
    k.q_mod_t = 1 % t;
    for (uint32_t l = 0; l < L; ++l) k.q_mod_t = (uint64_t)((unsigned __int128)k.q_mod_t * (c->q[l] % t) % t);
    for (uint32_t l = 0; l < L; ++l) {
        const uint64_t q = c->q[l];
        uint64_t prod = 1, prod_t = 1 % t;                  // (Q / q_l) mod q_l and mod t
        for (uint32_t j = 0; j < L; ++j)
            if (j != l) {
                prod = mulmod_host(prod, c->q[j] % q, q);
                prod_t = (uint64_t)((unsigned __int128)prod_t * (c->q[j] % t) % t);
            }
        k.qt[l] = powmod_host(prod, q - 2, q);
        k.qt_sh[l] = shoup_companion(k.qt[l], q);
        k.qhat_mod_t[l] = prod_t;
    }
    return launched(launch_bgv_decode(c->dev, k, pt, batch, m, (hipStream_t)stream), "BGV decode launch");
}

// The batch-encoding tables for t, built and uploaded on first use and kept
// (never rewritten) until the context is destroyed.
static zinc_status batch_args(zinc_ctx* c, uint64_t t, BatchArgs* g, const char* fn) {
    const uint32_t n = c->n, log_n = c->log_n;
    if (t < 3 || t >= (1ull << 31) || t % (2ull * n) != 1 || !is_prime(t))
        return fail(ZINC_E_INVAL, std::string(fn) + ": t must be a prime below 2^31 with t = 1 mod 2N");
    std::lock_guard<std::mutex> lock(c->batch_mu);
    const zinc_ctx::BatchTable* found = nullptr;
    for (const auto& b : c->batch_tables)
        if (b.t == t) found = &b;
    if (!found) {
        const uint64_t zeta = smallest_psi(t, log_n), zinv = powmod_host(zeta, t - 2, t);
        std::vector<uint32_t> h((size_t)5 * n);
        uint32_t* tw = h.data();
        uint32_t* itw = tw + 2 * (size_t)n;
        uint32_t* pos = itw + 2 * (size_t)n;
        for (uint32_t k = 0; k < n; ++k) {
            uint32_t r = 0;                                       // brv(k) over log_n bits
            for (uint32_t b = 0; b < log_n; ++b) r |= ((k >> b) & 1u) << (log_n - 1 - b);
            const uint64_t w = powmod_host(zeta, r, t), wi = powmod_host(zinv, r, t);
            tw[2 * k] = (uint32_t)w;
            tw[2 * k + 1] = (uint32_t)((w << 32) / t);
            itw[2 * k] = (uint32_t)wi;
            itw[2 * k + 1] = (uint32_t)((wi << 32) / t);
        }
        uint64_t e = 1;                                           // 3^i mod 2N
        for (uint32_t i = 0; i < n / 2; ++i) {
            const uint64_t es[2] = {e, 2ull * n - e};             // slots i and N/2 + i
            for (int half = 0; half < 2; ++half) {
                const uint32_t x = (uint32_t)((es[half] - 1) / 2);
                uint32_t r = 0;
                for (uint32_t b = 0; b < log_n; ++b) r |= ((x >> b) & 1u) << (log_n - 1 - b);
                pos[i + half * (n / 2)] = r;
            }
            e = e * 3 % (2ull * n);
        }
        void* d = nullptr;
        if (hipMalloc(&d, h.size() * 4) != hipSuccess) return fail(ZINC_E_NOMEM, std::string(fn) + ": table allocation");
        const hipError_t ce = hipMemcpy(d, h.data(), h.size() * 4, hipMemcpyHostToDevice);
        if (ce != hipSuccess) {
            (void)hipFree(d);
            return hip_fail(ce, fn);
        }
        const uint64_t ninv = powmod_host(n % t, t - 2, t);
        c->batch_tables.push_back({t, d, (uint32_t)ninv, (uint32_t)((ninv << 32) / t)});
        found = &c->batch_tables.back();
    }
    const uint32_t* base = static_cast<const uint32_t*>(found->d);
    g->tw = base;
    g->itw = base + 2 * (size_t)n;
    g->pos = base + 4 * (size_t)n;
    g->t = (uint32_t)t;
    g->ninv = found->ninv;
    g->ninv_sh = found->ninv_sh;
    return ZINC_OK;
}

static zinc_status batch_codec(zinc_ctx* c, uint64_t t, bool decode, const int64_t* in, uint32_t batch, int64_t* out,
                               void* stream, const char* fn) {
    if (!c) return fail(ZINC_E_INVAL, std::string(fn) + ": null context");
    if (zinc_status s = check_batch(fn, batch, {in, out})) return s;
    BatchArgs g;
    if (zinc_status s = batch_args(c, t, &g, fn)) return s;
    if (batch == 0) return ZINC_OK;
    return launched(launch_batch_codec(g, c->log_n, decode, in, batch, out, (hipStream_t)stream), fn);
}

zinc_status zinc_batch_encode(zinc_ctx* c, uint64_t t, const int64_t* slots, uint32_t batch, int64_t* m,
                              void* stream) {
    return batch_codec(c, t, false, slots, batch, m, stream, "zinc_batch_encode");
}

zinc_status zinc_batch_decode(zinc_ctx* c, uint64_t t, const int64_t* m, uint32_t batch, int64_t* slots,
                              void* stream) {
    return batch_codec(c, t, true, m, batch, slots, stream, "zinc_batch_decode");
}

zinc_status zinc_elementwise_zinc(zinc_ctx* c, const uint64_t* hat, uint32_t batch, uint64_t* ct, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_elementwise_zinc: null context");
    if (!c->precomputed) return fail(ZINC_E_STATE, "zinc_elementwise_zinc before zinc_precompute");
    if (zinc_status s = check_batch("zinc_elementwise_zinc", batch, {hat, ct})) return s;
    if ((uint64_t)batch * 2 * c->L >= (1ull << 31)) return fail(ZINC_E_INVAL, "zinc_elementwise_zinc: batch too large");
    if (batch == 0) return ZINC_OK;
    return launched(launch_elementwise_zinc(c->dev, hat, batch, ct, (hipStream_t)stream), "element-wise launch");
}

zinc_status zinc_elementwise_vanilla(zinc_ctx* c, const uint64_t* uhat, const uint64_t* hat, uint32_t batch,
                                     uint64_t* ct, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_elementwise_vanilla: null context");
    if (!c->keyed) return fail(ZINC_E_STATE, "zinc_elementwise_vanilla before zinc_keygen");
    if (zinc_status s = check_batch("zinc_elementwise_vanilla", batch, {uhat, hat, ct})) return s;
    if ((uint64_t)batch * c->L >= (1ull << 31)) return fail(ZINC_E_INVAL, "zinc_elementwise_vanilla: batch too large");
    if (batch == 0) return ZINC_OK;
    return launched(launch_elementwise_vanilla(c->dev, uhat, hat, batch, ct, (hipStream_t)stream),
                    "element-wise launch");
}

zinc_status zinc_decrypt(zinc_ctx* c, const uint64_t* ct, uint32_t batch, uint64_t* pt, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_decrypt: null context");
    if (!c->keyed) return fail(ZINC_E_STATE, "zinc_decrypt before zinc_keygen");
    if (zinc_status s = check_batch("zinc_decrypt", batch, {ct, pt})) return s;
    if (batch == 0) return ZINC_OK;
    return launched(launch_decrypt(c->dev, ct, batch, pt, (hipStream_t)stream), "decrypt launch");
}

zinc_status zinc_decode(zinc_ctx* c, const uint64_t* pt, uint32_t batch, double* slots, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_decode: null context");
    if (zinc_status s = check_batch("zinc_decode", batch, {pt, slots})) return s;
    if (batch == 0) return ZINC_OK;
    return launched(launch_decode(c->dev, pt, batch, slots, (hipStream_t)stream), "decode launch");
}

zinc_status zinc_add(zinc_ctx* c, const uint64_t* a, const uint64_t* b, uint32_t batch, uint64_t* out,
                     void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_add: null context");
    if (zinc_status s = check_batch("zinc_add", batch, {a, b, out})) return s;
    if (batch == 0) return ZINC_OK;
    return launched(launch_add(c->dev, a, b, batch, out, (hipStream_t)stream), "add launch");
}

zinc_status zinc_device_errors(zinc_ctx* c, uint32_t* flags) {
    if (!c || !flags) return fail(ZINC_E_INVAL, "zinc_device_errors: null argument");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(flags, c->dev.err, 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemset(c->dev.err, 0, 4);
    if (e != hipSuccess) return hip_fail(e, "zinc_device_errors");
    return ZINC_OK;
}

zinc_status zinc_ntt_forward(zinc_ctx* c, uint32_t limb, uint64_t* poly, uint32_t n_polys, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_ntt_forward: null context");
    if (limb >= c->M) return fail(ZINC_E_INVAL, "zinc_ntt_forward: limb out of range");
    if (zinc_status s = check_batch("zinc_ntt_forward", n_polys, {poly})) return s;
    if (n_polys == 0) return ZINC_OK;
    return launched(launch_ntt(c->dev, false, limb, poly, n_polys, (hipStream_t)stream), "ntt launch");
}

zinc_status zinc_ntt_inverse(zinc_ctx* c, uint32_t limb, uint64_t* poly, uint32_t n_polys, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_ntt_inverse: null context");
    if (limb >= c->M) return fail(ZINC_E_INVAL, "zinc_ntt_inverse: limb out of range");
    if (zinc_status s = check_batch("zinc_ntt_inverse", n_polys, {poly})) return s;
    if (n_polys == 0) return ZINC_OK;
    return launched(launch_ntt(c->dev, true, limb, poly, n_polys, (hipStream_t)stream), "intt launch");
}

zinc_status zinc_sample(zinc_ctx* c, int kind, uint32_t tag, uint32_t limb, const uint64_t* ids, uint32_t batch,
                        void* out, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_sample: null context");
    if (kind < 0 || kind > 2) return fail(ZINC_E_INVAL, "zinc_sample: kind must be 0, 1 or 2");
    if (tag == 0 || tag > 255) return fail(ZINC_E_INVAL, "zinc_sample: tag must be in [1, 255]");
    if (limb >= c->M) return fail(ZINC_E_INVAL, "zinc_sample: limb out of range");
    if (zinc_status s = check_batch("zinc_sample", batch, {ids, out})) return s;
    if (batch == 0) return ZINC_OK;
    return launched(launch_sample(c->dev, kind, tag, limb, ids, batch, out, (hipStream_t)stream),
                    "sample launch");
}

zinc_status zinc_export_keys(zinc_ctx* c, uint64_t* sk, uint64_t* pk, uint64_t* zero, void* stream) {
    if (!c) return fail(ZINC_E_INVAL, "zinc_export_keys: null context");
    if (!c->keyed) return fail(ZINC_E_STATE, "zinc_export_keys before zinc_keygen");
    if (zero && !c->precomputed) return fail(ZINC_E_STATE, "zinc_export_keys: no cached Enc(0) yet");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = (size_t)c->n * 8;
    hipError_t e = hipSuccess;
    if (sk) e = hipMemcpyAsync(sk, c->dev.sk, nb * c->M, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && pk) e = hipMemcpyAsync(pk, c->dev.pk, nb * 2 * c->M, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && zero)
        e = hipMemcpyAsync(zero, c->dev.zero, nb * 2 * c->L, hipMemcpyDeviceToDevice, s);
    return launched(e, "zinc_export_keys");
}

}  // extern "C"
