// Host-only checks of the capacity planner (capacity.h): totals beyond what
// 32-bit offsets can index must fail the call, never wrap into a capacity.
#include <cstdio>

#include "capacity.h"

using namespace emt;

static int failures = 0;

#define CHECK(cond)                                                  \
    do {                                                             \
        if (!(cond)) {                                               \
            std::printf("FAIL line %d: %s\n", __LINE__, #cond);      \
            ++failures;                                              \
        }                                                            \
    } while (0)

int main() {
    const Ratios r0{256.0, 8.0, 24.0};
    const unsigned long long two32 = 1ull << 32;
    for (unsigned long long k : {0ull, 1ull, 5ull, 4096ull, 1ull << 20}) {
        // seeds at 2^32 + k: a uint32 total would read k and look like a fit
        CapSizes c{4096, 1024, 1024};
        Ratios r = r0;
        const Needs h{two32 + k, 0, 0};
        CHECK(!fits(h, c));
        CHECK(!plan_retry(h, 100000, c, r));
        // members at 2^32 + k likewise
        CapSizes c2{1u << 20, 1024, 1024};
        Ratios r2 = r0;
        const Needs h2{1000, two32 + k, 1000};
        CHECK(!fits(h2, c2));
        CHECK(!plan_retry(h2, 100000, c2, r2));
    }
    {
        // the largest seed total that fits 31 bits is served
        CapSizes c{4096, 1024, 1024};
        Ratios r = r0;
        const Needs h{kSeedCapMax, 0, 0};
        CHECK(plan_retry(h, 1000, c, r));
        CHECK(c.seed_cap == kSeedCapMax);
        CHECK(fits(h, c));
        // one more is not
        CapSizes c2{4096, 1024, 1024};
        const Needs h2{kSeedCapMax + 1, 0, 0};
        CHECK(!plan_retry(h2, 1000, c2, r));
    }
    {
        // an ordinary overflow grows the stage to its exact need plus margin
        CapSizes c{4096, 1024, 1024};
        Ratios r = r0;
        const Needs h{100000, 0, 0};
        CHECK(plan_retry(h, 1000, c, r));
        CHECK(c.seed_cap >= 100000 && c.seed_cap < 200000);
        CHECK(r.seeds_per_grain >= 100.0);
        CHECK(fits(Needs{100000, 0, 0}, c));
    }
    {
        // too few candidate slots: members are sized from the listed ones
        CapSizes c{1u << 20, 1024, 1u << 20};
        Ratios r = r0;
        const Needs h{50000, 1024 * 30, 5000};
        CHECK(plan_retry(h, 1000, c, r));
        CHECK(c.cand_cap >= 5000);
        CHECK(c.mem_cap >= 30u * 5000u);
    }
    if (failures == 0) std::printf("capacity ok\n");
    return failures ? 1 : 0;
}
