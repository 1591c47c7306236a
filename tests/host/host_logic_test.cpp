// Host-side logic of the library, checked on the CPU: the serving budget's
// first-fit arena, the mixed-plan unit tables, and the chi sampler's bucket
// table against the count it stands for.  Prints "ok" and exits 0 on success.
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "arena.h"
#include "zinc_internal.h"

#define CHECK(c)                                                     \
    do {                                                             \
        if (!(c)) {                                                  \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                \
        }                                                            \
    } while (0)

static int test_arena() {
    std::mt19937_64 rng(1);
    const uint64_t size = 1 << 20;
    zinc::Arena a(size);
    struct Block { uint64_t off, bytes; };
    std::vector<Block> live;
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 3) {
            const uint64_t bytes = 1 + rng() % 40000;
            uint64_t off = 0;
            if (a.alloc(bytes, &off)) {
                const uint64_t r = (bytes + 255) & ~255ull;
                CHECK(off % 256 == 0 && off + r <= size);
                for (const Block& b : live) CHECK(off + r <= b.off || b.off + ((b.bytes + 255) & ~255ull) <= off);
                live.push_back({off, bytes});
            }
        } else {
            const size_t i = rng() % live.size();
            a.release(live[i].off, live[i].bytes);
            live.erase(live.begin() + (long)i);
        }
        uint64_t used = 0;
        for (const Block& b : live) used += (b.bytes + 255) & ~255ull;
        CHECK(a.used() == used);
    }
    for (const Block& b : live) a.release(b.off, b.bytes);
    uint64_t off = 1;
    CHECK(a.used() == 0 && a.alloc(size, &off) && off == 0);   // everything merged back
    return 0;
}

static int test_plan_tables() {
    const uint32_t logs[4] = {14, 12, 15, 13}, limbs[4] = {7, 2, 14, 3};
    std::vector<zinc_ctx> ctx(4);
    std::vector<zinc_ctx*> cp;
    for (int c = 0; c < 4; ++c) {
        ctx[c].log_n = logs[c];
        ctx[c].n = 1u << logs[c];
        ctx[c].L = limbs[c];
        cp.push_back(&ctx[c]);
    }
    std::mt19937 rng(2);
    std::vector<zinc_item> items;
    for (uint32_t i = 0; i < 301; ++i)
        items.push_back(zinc_item{(uint32_t)(rng() % 4), 0u, 1000ull * i, 7000ull * i, 5ull * i + 1});
    std::vector<zinc::PlanItem> di;
    std::vector<zinc::PlanUnit> un;
    const uint32_t round = 16;                           // workgroups of the persistent launch
    const uint64_t dummy =
        zinc::build_plan_tables(cp.data(), 4, items.data(), (uint32_t)items.size(), di, un, round);
    CHECK(dummy <= zinc::plan_dummy_words(cp.data(), 4));
    std::map<uint64_t, uint32_t> limbs_done;             // ct_id -> limbs covered (each limb once)
    double last_cost = 1e300;
    uint32_t n32 = 0, split_units = 0;
    for (const zinc_item& it : items) n32 += ctx[it.ctx_idx].log_n == 15;
    for (const zinc::PlanUnit& u : un) {
        const zinc_ctx& c = ctx[u.ctx];
        CHECK(u.log_n == c.log_n && u.count == zinc::plan_units_per_group(c.log_n));
        CHECK(u.l0 < u.l1 && u.l1 <= c.L);
        if (u.l1 - u.l0 < c.L) {
            CHECK(c.log_n == 15);                        // only ring degree 32768 is split
            ++split_units;
        }
        const double cost = zinc::plan_unit_cost(c, u);
        CHECK(cost <= last_cost);                        // longest units first
        last_cost = cost;
        for (uint32_t k = 0; k < u.count; ++k) {
            const zinc::PlanItem& it = di[u.first + k];
            CHECK(it.ctx == u.ctx);
            if (it.dummy) {
                CHECK(it.ct_off + 2ull * c.L * c.n <= dummy);
            } else {
                uint32_t& m = limbs_done[it.ct_id];
                for (uint32_t l = u.l0; l < u.l1; ++l) {
                    CHECK(!((m >> l) & 1u));
                    m |= 1u << l;
                }
            }
        }
        CHECK(!di[u.first].dummy);                       // a unit starts with a real item
    }
    // the ciphertexts beyond the last whole round of 16 are split, here (many
    // units of work per workgroup) into the fewest groups
    CHECK(split_units == (n32 % round) * zinc::kPlanSplit);
    CHECK(limbs_done.size() == items.size());
    for (const zinc_item& it : items) CHECK(limbs_done[it.ct_id] == (1u << ctx[it.ctx_idx].L) - 1u);

    // a light batch (a few ciphertexts, idle workgroups): one limb per unit
    std::vector<zinc_item> few;
    for (uint32_t i = 0; i < 3; ++i) few.push_back(zinc_item{2u, 0u, 1000ull * i, 7000ull * i, 900ull + i});
    few.push_back(zinc_item{1u, 0u, 5000ull, 9000ull, 990ull});
    zinc::build_plan_tables(cp.data(), 4, few.data(), (uint32_t)few.size(), di, un, 256);
    uint32_t n_split = 0;
    std::map<uint64_t, uint32_t> covered;
    for (const zinc::PlanUnit& u : un) {
        if (ctx[u.ctx].log_n == 15) {
            CHECK(u.l1 - u.l0 == 1u);
            ++n_split;
        }
        for (uint32_t l = u.l0; l < u.l1; ++l) covered[di[u.first].ct_id] |= 1u << l;
    }
    CHECK(n_split == 3u * ctx[2].L);
    for (const zinc_item& it : few) CHECK(covered[it.ct_id] == (1u << ctx[it.ctx_idx].L) - 1u);

    // the rule itself: a lone ciphertext on an idle device takes one limb per
    // unit; 64 on 256 workgroups keep four groups (256 units, one round: five
    // groups would need a second round); a long queue keeps the fewest
    const std::vector<double> none;
    CHECK(zinc::plan_split_parts(none, 1, 14, 1.0, 256) == 14u);
    CHECK(zinc::plan_split_parts(none, 64, 14, 1.0, 256) == zinc::kPlanSplit);
    CHECK(zinc::plan_split_parts(none, 16, 14, 1.0, 256) == 14u);
    CHECK(zinc::plan_split_parts(std::vector<double>(4000, 15.0), 100, 14, 1.0, 16) == zinc::kPlanSplit);
    CHECK(zinc::plan_split_parts(none, 1, 3, 1.0, 256) == 3u);   // never more groups than limbs
    return 0;
}

static int test_gaussian_buckets() {
    uint64_t cdt[zinc::kCdtLen], bucket[zinc::kCdtBuckets];
    zinc::gaussian_cdt(3.2, cdt);
    zinc::gaussian_buckets(cdt, bucket);
    std::vector<uint64_t> us;
    std::mt19937_64 rng(3);
    for (int i = 0; i < 200000; ++i) us.push_back(rng());
    for (int i = 0; i < zinc::kCdtLen; ++i)
        for (int d = -1; d <= 1; ++d) us.push_back(cdt[i] + (uint64_t)(int64_t)d);
    for (uint64_t b = 0; b < (uint64_t)zinc::kCdtBuckets; ++b) {
        us.push_back(b << zinc::kCdtShift);
        us.push_back(((b + 1) << zinc::kCdtShift) - 1);
    }
    int fallback = 0;
    for (uint64_t u : us) {
        int count = 0;
        for (int i = 0; i < zinc::kCdtLen; ++i) count += u >= cdt[i];
        const uint64_t e = bucket[u >> zinc::kCdtShift];
        if (e >> 63) {
            ++fallback;
            continue;
        }
        const uint64_t thr = (u & ~zinc::kCdtLowMask) | (e & zinc::kCdtLowMask);
        CHECK((int)((e >> 56) & 63) + (u >= thr ? 1 : 0) == count);
    }
    int flagged = 0;
    for (int b = 0; b < zinc::kCdtBuckets; ++b) flagged += (int)(bucket[b] >> 63);
    CHECK(flagged == 2 && (bucket[0] >> 63) && (bucket[zinc::kCdtBuckets - 1] >> 63));
    CHECK(fallback > 0);
    return 0;
}

int main() {
    if (test_arena()) return 1;
    if (test_plan_tables()) return 1;
    if (test_gaussian_buckets()) return 1;
    printf("ok\n");
    return 0;
}
