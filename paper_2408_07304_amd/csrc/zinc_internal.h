// Internal declarations shared by the host runtime (capi.cpp, host_math.cpp)
// and the HIP kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/zinc.h"

namespace zinc {

constexpr int kCdtLen = 38;       // support [-19, 19] -> 38 thresholds
constexpr int kCdtPad = 64;       // padded to a power of two for the device search
constexpr int kCdtBucketBits = 10;                // first-level table over the top 10 bits of the uniform
constexpr int kCdtBuckets = 1 << kCdtBucketBits;
constexpr int kCdtShift = 64 - kCdtBucketBits;   // bucket = u >> kCdtShift
constexpr uint64_t kCdtLowMask = (1ull << kCdtShift) - 1;
constexpr int kCdtTab = kCdtPad + kCdtBuckets;   // words of the device table
constexpr int kTail = 19;

enum Tag : uint32_t { TAG_SK = 1, TAG_A = 2, TAG_EPK = 3, TAG_U = 4, TAG_E1 = 5, TAG_E2 = 6,
                      TAG_E1Z = 7, TAG_E2Z = 8 };

// Per-modulus constants read by the kernels (one entry per limb).
struct LimbConst {
    uint64_t q;         // modulus
    uint64_t q2;        // 2q
    uint64_t bar;       // floor(2^64 / q): Shoup companion of 1, used to reduce < 2^64 values
    uint64_t ninv;      // N^-1 mod q
    uint64_t ninv_sh;   // Shoup companion of N^-1
    uint64_t half;      // (q - 1) / 2, centred-lift threshold
    uint64_t pinv;      // p^-1 mod q for the special prime p = q_{M-1} (data limbs)
    uint64_t pinv_sh;   // Shoup companion of pinv
    double qd;          // q as a double (exact)
    double qinv;        // 1/q rounded to double
    uint32_t fp;        // forward-NTT arithmetic: 0 integer (Shoup), 1 FP64, 2 FP64 with per-pass rounding
    uint32_t reserved;
};

// FP64 arithmetic is used for moduli below these bounds (see device.h).
constexpr uint64_t kFpNoReduceBound = 1ull << 47;
constexpr uint64_t kFpBound = 1ull << 50;

// Everything a kernel needs about one parameter set, as device pointers.
struct DevParams {
    uint32_t log_n, n, M, L;
    uint64_t seed;
    double scale;
    uint64_t noise_t;             // 1; BGV: the plaintext modulus t scaling every error (Eq. 13)
    const LimbConst* limbs;       // [M]
    const uint64_t* tw;           // [M][N][2]  (psi^brv(k), Shoup companion)
    const uint64_t* itw;          // [M][N][2]  (psi^-brv(k), Shoup companion)
    const double* tw_fp;          // [M][N][2]  (psi^brv(k), psi^brv(k) / q) as doubles
    const double* fft_tw;         // [N/4][2]   exp(-2 pi i k / (N/2)), k < N/4
    const double* twist;          // [N/2][2]   exp(-i pi k / N),       k < N/2
    const uint32_t* slot_pos;     // [N/2]      brv_{log N - 1}((5^j mod 2N - 1) / 4)
    const uint64_t* cdt;          // [kCdtTab]  cumulative table padded with 2^64-1, then bucket entries
    const uint64_t* sk;           // [M][N]     s_hat
    const uint64_t* sk_sh;        // [M][N]     Shoup companions of s_hat
    const uint64_t* pk;           // [2][M][N]
    const uint64_t* pk_sh;        // [2][M][N]
    const uint64_t* zero;         // [2][L][N]  cached Enc(0)
    const uint64_t* pkp;          // [2][L][N]  pk_j p^-1 on the data limbs (special-prime vanilla)
    const uint64_t* pkp_sh;       // [2][L][N]  Shoup companions
    uint32_t* err;                // sticky device error flags
    // This struct's copy in device memory.  The largest kernels (ring degree
    // 16384 and the split 32768 ones) read their parameters through it, field
    // by field with scalar loads, which frees registers (by value the split
    // kernels spill); the others take the kernel argument, whose first words
    // the hardware preloads, which saves latency on short workgroups.
    const DevParams* self;
};

// Per-call constants of the BFV integer encoding and decoding for plaintext
// modulus t (kernels_bfv.hip), one entry per data limb.
struct BfvConsts {
    uint64_t t;
    uint64_t delta[ZINC_MAX_MODULI];      // floor(Q / t) mod q_l
    uint64_t delta_sh[ZINC_MAX_MODULI];
    uint64_t b[ZINC_MAX_MODULI];          // t Qt_l mod q_l, Qt_l = (Q / q_l)^-1 mod q_l
    uint64_t b_sh[ZINC_MAX_MODULI];
    uint64_t w_mod_t[ZINC_MAX_MODULI];    // floor(t Qt_l / q_l) mod t
};

// Tables of the batch (slot) encoding for a prime t = 1 mod 2N, t < 2^31
// (kernels_batch.hip); the pointers are device memory owned by the context.
struct BatchArgs {
    const uint32_t* tw;      // [N][2] (zeta^brv(k), floor(zeta^brv(k) 2^32 / t))
    const uint32_t* itw;     // [N][2] (zeta^-brv(k), companion)
    const uint32_t* pos;     // [N]    entry of the forward transform holding slot j
    uint32_t t, ninv, ninv_sh;
};

// Constants of BGV decoding for plaintext modulus t (kernels_bfv.hip).
struct BgvConsts {
    uint64_t t;
    uint64_t q_mod_t;                     // Q mod t
    uint64_t qt[ZINC_MAX_MODULI];         // Qt_l = (Q / q_l)^-1 mod q_l
    uint64_t qt_sh[ZINC_MAX_MODULI];
    uint64_t qhat_mod_t[ZINC_MAX_MODULI]; // (Q / q_l) mod t
};

// One ciphertext of a mixed-shape plan (device copy of a zinc_item).
struct PlanItem {
    uint32_t ctx;            // index into the plan's contexts
    uint32_t dummy;          // 1: padding of a partial unit, output goes to the plan's dummy buffer
    uint64_t slot_off;       // float64 offset of the slot vector (N/2 values)
    uint64_t ct_off;         // uint64 offset of the ciphertext ([2][L][N])
    uint64_t ct_id;
};

// A unit of work: `count` consecutive items of one context, all encrypted by
// one workgroup (4, 2, 1, 1 items for ring degree 4096, 8192, 16384, 32768),
// over data limbs [l0, l1) (all of them, except for ring degree 32768, where
// the ciphertexts of a last partial round of units are split into limb groups).
struct PlanUnit {
    uint32_t ctx;
    uint32_t log_n;
    uint32_t first;
    uint32_t count;
    uint32_t l0, l1;
};

struct PlanDev {
    const DevParams* ctxs;
    const PlanItem* items;
    const PlanUnit* units;
    uint32_t n_units;
    uint32_t grid;           // persistent workgroups
    uint32_t* counter;
    uint64_t* dummy;
};

}  // namespace zinc

struct zinc_ctx {
    int device = 0;
    uint32_t log_n = 0, n = 0, M = 0, L = 0;
    double scale = 0, sigma = 0;
    uint64_t seed = 0;
    uint64_t q[ZINC_MAX_MODULI] = {};
    uint64_t psi[ZINC_MAX_MODULI] = {};
    uint64_t cdt[zinc::kCdtLen] = {};
    uint32_t fp64_mask = 0;       // limbs whose forward NTT uses FP64 arithmetic
    uint32_t tile[2] = {16, 16};  // coefficients per thread of the fused kernel, per scheme
    uint32_t reg_epilogue = 0;    // bit s: scheme s stores from the last pass's registers
    zinc::LimbConst h_limbs[ZINC_MAX_MODULI] = {};   // host copy of the limb constants
    bool keyed = false, precomputed = false;
    struct BatchTable {           // batch-encoding tables per plaintext modulus t
        uint64_t t;
        void* d;                  // device block: tw [N][2], itw [N][2], pos [N] (uint32)
        uint32_t ninv, ninv_sh;
    };
    std::vector<BatchTable> batch_tables;
    std::mutex batch_mu;          // guards batch_tables (first use of a t may come from any thread)
    // device allocations owned by the context
    void* d_block = nullptr;      // one allocation holding every table and key
    zinc::DevParams dev{};
};

namespace zinc {

// host_math.cpp
bool is_prime(uint64_t n);
bool choose_moduli(uint32_t log_n, uint32_t count, const uint32_t* bits, uint64_t* out);
uint64_t smallest_psi(uint64_t q, uint32_t log_n);
uint64_t mulmod_host(uint64_t a, uint64_t b, uint64_t q);
uint64_t powmod_host(uint64_t b, uint64_t e, uint64_t q);
uint64_t shoup_companion(uint64_t w, uint64_t q);
void gaussian_cdt(double sigma, uint64_t out[kCdtLen]);
void gaussian_buckets(const uint64_t cdt[kCdtLen], uint64_t out[kCdtBuckets]);

void set_error(const std::string& msg);

// kernel launchers (return hipError_t of the launch)
hipError_t launch_keygen(const DevParams& p, uint64_t* sk, uint64_t* sk_sh, uint64_t* pk,
                         uint64_t* pk_sh, hipStream_t s);
// reserved_ok: the identifiers may be reserved ones (the cached Enc(0) only)
// Workgroups per ciphertext of the fused kernels for N <= 16384: a batch of
// fewer than half as many ciphertexts as the device has CUs leaves CUs idle
// with one workgroup per ciphertext, so each ciphertext's data limbs are
// spread over up to CUs / batch workgroups (at most one limb each).
uint32_t limb_groups(const DevParams& p, uint32_t batch);
hipError_t launch_encrypt_pt(const DevParams& p, int scheme, const uint64_t* pt, uint32_t batch,
                             const uint64_t* ct_ids, uint64_t* ct, hipStream_t s, bool reserved_ok = false);
hipError_t launch_encrypt_slots(const DevParams& p, int scheme, const double* slots,
                                uint32_t n_slots, uint32_t batch, const uint64_t* ct_ids,
                                uint64_t* ct, hipStream_t s);
hipError_t launch_encode(const DevParams& p, const double* slots, uint32_t n_slots, uint32_t batch,
                         uint64_t* pt, hipStream_t s);
hipError_t launch_decrypt(const DevParams& p, const uint64_t* ct, uint32_t batch, uint64_t* pt,
                          hipStream_t s);
hipError_t launch_decode(const DevParams& p, const uint64_t* pt, uint32_t batch, double* slots,
                         hipStream_t s);
hipError_t launch_add(const DevParams& p, const uint64_t* a, const uint64_t* b, uint32_t batch,
                      uint64_t* out, hipStream_t s);
hipError_t launch_ntt(const DevParams& p, bool inverse, uint32_t limb, uint64_t* poly,
                      uint32_t n_polys, hipStream_t s);
hipError_t launch_sample(const DevParams& p, int kind, uint32_t tag, uint32_t limb,
                         const uint64_t* ct_ids, uint32_t batch, void* out, hipStream_t s);

// vanilla with division by the special prime (kernels_sp.hip); ws holds
// [batch][3][N] int64 of scratch
hipError_t launch_scale_pk(const DevParams& p, uint64_t* pkp, uint64_t* pkp_sh, hipStream_t s);
hipError_t launch_encrypt_sp(const DevParams& p, bool from_slots, const double* slots, uint32_t n_slots,
                             const uint64_t* pt, uint32_t batch, const uint64_t* ct_ids, uint64_t* ct, int64_t* ws,
                             hipStream_t s);
// Static scratch of zinc_encrypt_vanilla_sp_noalloc: its size, and its device
// address on `device`, which must be the current device (looked up once per
// device; hipErrorInvalidDevice otherwise).
constexpr size_t kSpScratchBytes = 64ull << 20;
hipError_t sp_scratch(int device, long long** out);

// BFV integer encoding / decoding (kernels_bfv.hip)
hipError_t launch_bfv_encode(const DevParams& p, const BfvConsts& k, const int64_t* m, uint32_t batch, uint64_t* pt,
                             hipStream_t s);
hipError_t launch_bfv_decode(const DevParams& p, const BfvConsts& k, const uint64_t* pt, uint32_t batch, int64_t* m,
                             hipStream_t s);
hipError_t launch_batch_codec(const BatchArgs& g, uint32_t log_n, bool decode, const int64_t* in, uint32_t batch,
                              int64_t* out, hipStream_t s);
hipError_t launch_bgv_decode(const DevParams& p, const BgvConsts& k, const uint64_t* pt, uint32_t batch, int64_t* m,
                             hipStream_t s);

// element-wise steps alone (kernels_elementwise.hip)
hipError_t launch_elementwise_zinc(const DevParams& p, const uint64_t* hat, uint32_t batch, uint64_t* ct,
                                   hipStream_t s);
hipError_t launch_elementwise_vanilla(const DevParams& p, const uint64_t* uhat, const uint64_t* hat, uint32_t batch,
                                      uint64_t* ct, hipStream_t s);

// thread geometries of the fused encode + encrypt kernel (coefficients per
// thread); kTileR16 is the default kernel, the others are kernels_tiles*.hip
constexpr int kTileR16 = 0, kTileR8 = 1, kTileR32 = 2;
hipError_t launch_encrypt_slots_tile(const DevParams& p, int scheme, int tile, bool reg, const double* slots,
                                     uint32_t n_slots, uint32_t batch, const uint64_t* ct_ids, uint64_t* ct,
                                     hipStream_t s);

// mixed-shape plans (kernels_plan*.hip)
hipError_t launch_plan(const PlanDev& d, int scheme, const double* slots, uint64_t* ct, hipStream_t s);

// plan tables (plan.cpp), shared by plans and the server
uint32_t plan_units_per_group(uint32_t log_n);
// Group items by context and cut each group into units of
// plan_units_per_group items; a partial unit is padded with copies of its
// first item whose outputs go to a dummy buffer.  Ciphertexts of ring degree
// 32768 that would form a last partial round of `round` units (one per
// workgroup of the persistent launch) are split into up to four limb groups.
// Units are ordered by decreasing estimated cost (plan_unit_cost), so the
// largest start first.  Returns the dummy buffer's size in words (at most
// plan_dummy_words).
uint64_t build_plan_tables(zinc_ctx* const* ctxs, uint32_t n_ctx, const zinc_item* items, uint32_t n_items,
                           std::vector<PlanItem>& dev_items, std::vector<PlanUnit>& units, uint32_t round);
// Estimated cost of a unit (relative): per item, N log N times the unit's
// limbs plus one limb's worth for the encoding and sampling every unit does.
// Limb groups of each of the `tail` ring-degree-32768 ciphertexts of a last
// partial round of a plan: the count in [kPlanSplit, L] that minimises the
// plan's completion time on `round` workgroups that take units longest first
// (costs as plan_unit_cost: `unit` is one limb's cost, a group of g limbs costs
// unit * (g + 1); `other_costs` are the plan's other units); ties go to fewer
// groups.
uint32_t plan_split_parts(const std::vector<double>& other_costs, uint32_t tail, uint32_t L, double unit,
                          uint32_t round);
double plan_unit_cost(const zinc_ctx& c, const PlanUnit& u);
constexpr uint32_t kPlanSplit = 4;        // fewest limb groups of a split ring-degree-32768 ciphertext
uint64_t plan_dummy_words(zinc_ctx* const* ctxs, uint32_t n_ctx);
int device_cu_count();
zinc_status plan_fail(zinc_status code, const std::string& msg);

// ring degree 32768 (kernels_split.hip)
hipError_t launch_split_keygen(const DevParams& p, uint64_t* sk, uint64_t* sk_sh, uint64_t* pk,
                               uint64_t* pk_sh, hipStream_t s);
hipError_t launch_split_encrypt(const DevParams& p, int scheme, bool from_slots, const double* slots,
                                uint32_t n_slots, const uint64_t* pt, uint32_t batch,
                                const uint64_t* ct_ids, uint64_t* ct, hipStream_t s, bool reserved_ok = false);
hipError_t launch_split_encode(const DevParams& p, const double* slots, uint32_t n_slots,
                               uint32_t batch, uint64_t* pt, hipStream_t s);
hipError_t launch_split_decrypt(const DevParams& p, const uint64_t* ct, uint32_t batch,
                                uint64_t* pt, hipStream_t s);
hipError_t launch_split_decode(const DevParams& p, const uint64_t* pt, uint32_t batch,
                               double* slots, hipStream_t s);
hipError_t launch_split_ntt(const DevParams& p, bool inverse, uint32_t limb, uint64_t* poly,
                            uint32_t n_polys, hipStream_t s);
hipError_t launch_split_encrypt_sp(const DevParams& p, bool from_slots, const double* slots, uint32_t n_slots,
                                   const uint64_t* pt, uint32_t batch, const uint64_t* ct_ids, uint64_t* ct,
                                   int64_t* ws, hipStream_t s);

}  // namespace zinc
