// Brute-force check, on the CPU, of the index layouts that let the kernels
// exchange data through LDS without workgroup barriers.  Compiled as HIP
// source (the layouts are the kernels' own constexpr host/device functions)
// but runs no GPU code.  Prints "ok" or the first failing case.
//
// For every thread geometry and FFT shape the kernels instantiate:
//  * wave_local<G>(P1, P2) true => every wave holds the same set of indices in
//    passes P1 and P2 (so its LDS words before and after are its own);
//  * a forward transform's first exchange is never wave-local;
//  * wave_pair_index<G> hands each wave exactly its own indices of the last
//    pass, as pairs (k, k + 1), every index once;
//  * fft_wave_local<LOGH, LOGT, P> true => every wave touches the same set of
//    FFT points in passes P and P + 1, and every point of the transform is
//    held by exactly one thread in each pass.
#include <stdio.h>
#include <stdlib.h>

#include <set>
#include <vector>

#include "device.h"

using namespace zinc;

static int fails = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            if (fails++ < 10) fprintf(stderr, __VA_ARGS__); \
        }                                                 \
    } while (0)

// indices held by wave w in pass p of geometry G
template <class G>
static std::set<uint32_t> wave_set(int p, uint32_t w) {
    std::set<uint32_t> s;
    for (uint32_t t = w * 64; t < (w + 1) * 64 && t < (uint32_t)G::T; ++t)
        for (int c = 0; c < G::R; ++c) s.insert(G::spread(p, t) | G::cpart(p, c));
    return s;
}

template <class G>
static void check_geom(const char* name) {
    const uint32_t waves = (G::T + 63) / 64;
    // every pass is a bijection of (thread, register) onto the indices
    for (int p = 0; p < G::NPASS; ++p) {
        std::vector<int> seen(G::N, 0);
        for (uint32_t t = 0; t < (uint32_t)G::T; ++t)
            for (int c = 0; c < G::R; ++c) seen[G::spread(p, t) | G::cpart(p, c)]++;
        for (int i = 0; i < G::N; ++i) CHECK(seen[i] == 1, "%s: pass %d index %d held %d times\n", name, p, i, seen[i]);
    }
    for (int p = 0; p + 1 < G::NPASS; ++p) {
        const bool wl = wave_local<G>(p, p + 1);
        CHECK((wl == wave_local<G>(p + 1, p)), "%s: wave_local not symmetric at %d\n", name, p);
        if (p == 0) CHECK(!wl, "%s: first exchange is wave-local\n", name);
        if (!wl) continue;
        for (uint32_t w = 0; w < waves; ++w)
            CHECK((wave_set<G>(p, w) == wave_set<G>(p + 1, w)), "%s: passes %d/%d differ on wave %u\n", name, p, p + 1, w);
    }
    constexpr int PL = G::NPASS - 1;
    for (uint32_t w = 0; w < waves; ++w) {
        const std::set<uint32_t> own = wave_set<G>(PL, w);
        std::multiset<uint32_t> got;
        for (uint32_t t = w * 64; t < (w + 1) * 64; ++t)
            for (int i = 0; i < G::R / 2; ++i) {
                const uint32_t k = wave_pair_index<G>(t, i);
                CHECK(k % 2 == 0, "%s: odd pair index %u\n", name, k);
                got.insert(k);
                got.insert(k + 1);
            }
        CHECK(std::set<uint32_t>(got.begin(), got.end()) == own && got.size() == own.size(),
              "%s: wave %u pairs are not its own last-pass indices\n", name, w);
    }
}

// points touched by wave w in pass P of an FFT of 2^LOGH points on 2^LOGT threads
template <int LOGH, int LOGT, int P>
static std::set<uint32_t> fft_wave_set(uint32_t w) {
    using F = FftPass<LOGH, LOGT, P>;
    std::set<uint32_t> s;
    for (uint32_t t = w * 64; t < (w + 1) * 64 && t < (1u << LOGT); ++t)
        for (int e = 0; e < F::R; ++e) s.insert(F::idx(t, e));
    return s;
}

template <int LOGH, int LOGT, int P>
static void check_fft_pass(const char* name) {
    using F = FftPass<LOGH, LOGT, P>;
    if constexpr (F::B < LOGH) {
        std::vector<int> seen(1u << LOGH, 0);
        for (uint32_t t = 0; t < (1u << LOGT); ++t)
            for (int e = 0; e < F::R; ++e) seen[F::idx(t, e)]++;
        for (uint32_t i = 0; i < (1u << LOGH); ++i) CHECK(seen[i] == 1, "%s: FFT pass %d point %u held %d times\n", name, P, i, seen[i]);
        if constexpr (F::B + F::LOGR < LOGH) {
            if (fft_wave_local<LOGH, LOGT, P>()) {
                const uint32_t waves = ((1u << LOGT) + 63) / 64;
                for (uint32_t w = 0; w < waves; ++w)
                    CHECK((fft_wave_set<LOGH, LOGT, P>(w) == fft_wave_set<LOGH, LOGT, P + 1>(w)),
                          "%s: FFT passes %d/%d differ on wave %u\n", name, P, P + 1, w);
            }
            check_fft_pass<LOGH, LOGT, P + 1>(name);
        }
    }
}

// the encoder's FFT: N/4 points on min(N/32, T) threads
template <class G>
static void check_encode_fft(const char* name) {
    constexpr int LOGQ = G::LOGN - 2, TF = (1 << LOGQ) / 8 < G::T ? (1 << LOGQ) / 8 : G::T;
    check_fft_pass<LOGQ, ilog2(TF), 0>(name);
}

int main() {
    check_geom<Geom<12, 8>>("N4096 T256");
    check_geom<Geom<12, 9>>("N4096 T512");
    check_geom<Geom<12, 7>>("N4096 T128");
    check_geom<Geom<13, 9>>("N8192 T512");
    check_geom<Geom<13, 10>>("N8192 T1024");
    check_geom<Geom<13, 8>>("N8192 T256");
    check_geom<Geom<14, 10>>("N16384 T1024 (and each half of N32768)");
    check_geom<Geom<14, 9>>("N16384 T512");
    check_encode_fft<Geom<12, 8>>("encode N4096 T256");
    check_encode_fft<Geom<12, 9>>("encode N4096 T512");
    check_encode_fft<Geom<12, 7>>("encode N4096 T128");
    check_encode_fft<Geom<13, 9>>("encode N8192 T512");
    check_encode_fft<Geom<13, 10>>("encode N8192 T1024");
    check_encode_fft<Geom<13, 8>>("encode N8192 T256");
    check_encode_fft<Geom<14, 10>>("encode N16384 T1024");
    check_encode_fft<Geom<14, 9>>("encode N16384 T512");
    check_fft_pass<13, 10, 0>("encode N32768 T1024");
    // at least one barrier-free transition is exercised by these shapes
    CHECK((fft_wave_local<11, 8, 0>()), "the N8192 encoder's first FFT passes are expected wave-local\n");
    CHECK((wave_local<Geom<13, 9>>(2, 3)), "the N8192 transform's last exchange is expected wave-local\n");
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
