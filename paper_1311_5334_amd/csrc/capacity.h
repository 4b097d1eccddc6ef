// capacity.h -- how the buffers of a call that overflowed are resized.
//
// Device counters keep counting past a buffer's capacity, with the seed and
// member totals summed in 64 bits, so after an attempt the host knows what
// each stage needed. Plain C++ (no HIP): the host tests compile it alone.
#ifndef EMT_CAPACITY_H
#define EMT_CAPACITY_H

#include <stdint.h>

#include <algorithm>

namespace emt {

// Seeds and member entries are indexed and scanned in uint32 on the device;
// capacities stay below 2^31 so every offset and total fits.
constexpr unsigned long long kSeedCapMax = (1ull << 31) - 1;
constexpr unsigned long long kMemCapMax = (1ull << 31) - 1;

// What the device counted in one attempt (exact totals). A stage behind an
// overflowed one takes no input, so its count is 0 then.
struct Needs {
    unsigned long long seeds;
    unsigned long long members;
    uint32_t cand;
};

// Capacities of an attempt.
struct CapSizes {
    unsigned long long seed_cap;
    uint32_t cand_cap;
    uint32_t mem_cap;
};

// Ratios a context learns for sizing its next calls.
struct Ratios {
    double seeds_per_grain;
    double cand_per_grain;
    double mem_per_cand;
};

inline uint32_t clamp_cap(double x) {
    if (x < 1024.0) return 1024u;
    if (x > 2147483647.0) return 2147483647u;
    return (uint32_t)x;
}

inline bool fits(const Needs &h, const CapSizes &c) {
    return h.seeds <= c.seed_cap && h.cand <= c.cand_cap && h.members <= c.mem_cap;
}

// Capacities for re-running an attempt whose needs did not fit. The stage
// that overflowed is sized from its exact count, the later ones from the
// learned ratios. Returns false when no capacity can hold the needs (the
// call then fails with EMT_EOVERFLOW).
inline bool plan_retry(const Needs &h, uint32_t n_total, CapSizes &c, Ratios &r) {
    const double grains = std::max(1.0, (double)n_total);
    if (h.seeds > c.seed_cap) {
        if (h.seeds > kSeedCapMax) return false;
        c.seed_cap = std::min<unsigned long long>(kSeedCapMax, h.seeds + h.seeds / 8 + 1024);
        r.seeds_per_grain = std::max(r.seeds_per_grain, 1.125 * (double)h.seeds / grains);
    }
    const bool cand_over = h.cand > c.cand_cap;
    const uint32_t cand_seen = cand_over ? c.cand_cap : h.cand;  // candidates with members
    if (cand_over) {
        c.cand_cap = clamp_cap((double)h.cand * 1.125 + 1024);
        r.cand_per_grain = std::max(r.cand_per_grain, 1.125 * (double)h.cand / grains);
    }
    // with too few candidate slots the member count covers only the first
    // cand_cap candidates: size the members from the ratio as well
    if (h.members > c.mem_cap || cand_over) {
        if (h.members > kMemCapMax) return false;
        const double per = cand_seen ? (double)h.members / (double)cand_seen : r.mem_per_cand;
        r.mem_per_cand = std::max(r.mem_per_cand, 1.125 * per);
        c.mem_cap = clamp_cap(std::max((double)h.members * 1.125 + 1024,
                                       r.mem_per_cand * (double)c.cand_cap));
    }
    return true;
}

}  // namespace emt

#endif
