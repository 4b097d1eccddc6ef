// emt_dev.h -- device-side structures and launchers of the track finder.
//
// Library-internal: shared by the kernels (kernels.hip) and the host
// implementation of the C ABI (api.hip). Nothing here is part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "emt.h"
#include "tile_table.h"

namespace emt {

constexpr int kSpanMax = 1 << 18;  // per-axis coordinate span limit (units)
constexpr uint32_t kNMax = 1u << 20;
constexpr int kRMax = 4096;
constexpr int kBlock = 256;
// Cells a view may use: kCellsPerGrain per grain plus kCellsBase; cell edges
// are doubled until the grid fits.
constexpr uint32_t kCellsPerGrain = EMT_CELLS_PER_GRAIN;
constexpr uint32_t kCellsBase = 4096;
// Entries of the sorted-grain array past the last grain: kernels that load
// a fixed group of consecutive grains may read (and then ignore) them.
constexpr uint32_t kSortedSpare = 8;

// Per view. Host fills grain_off, n, cell_off, cell_cap and resets lo/hi;
// the device fills the rest (bounding box, then cell geometry).
struct ViewGrid {
    int32_t lo[3];       // bounding box min (absolute units) = grid origin
    int32_t hi[3];       // bounding box max
    int32_t cell[3];     // cell edge per axis (units)
    int32_t dims[3];     // cells per axis
    uint32_t grain_off;  // first grain of the view in the packed arrays
    uint32_t n;          // grains of the view (0 if rejected on device)
    uint32_t cell_off;   // first cell of the view in cell_start
    uint32_t cell_cap;   // cells the view may use
    int32_t err;         // 1: coordinate span above kSpanMax
    int32_t pad[3];
};

// Sizes of the batch in flight, in device memory so that one captured launch
// sequence serves every batch within its capacities.
struct BatchDesc {
    uint32_t n_total;     // grains
    uint32_t n_views;
    uint32_t n_cells;     // cell table entries in use
    uint32_t n_cells_m1;  // n_cells - 1 (scan length of the cell table)
};

// Cell edges by grain density: bucket b holds views with at least
// kCellEdge0 * 2^(b-1) grains per 1000 um^3 (b = 0: below kCellEdge0).
// Per-XCD seed-range counters of the counting kernel, 64 B apart.
// two sets (counting, then listing the candidates' members), 16 words per XCD
constexpr int kGrabWords = 2 * 8 * 16;
constexpr int kCellBuckets = 8;
// Partial sums of four 64-bit totals (seeds, member entries, counting tests,
// counting hits): kPartSlots counters per total, one 128-byte line apart, so
// that the workgroups' atomic adds spread over many L2 addresses instead of
// serialising on one.
constexpr int kPartSlots = 64;
constexpr int kPartStride = 16;
constexpr int kPartWords = 4 * kPartSlots * kPartStride;
constexpr double kCellEdge0 = 0.75;

struct Params {
    int32_t R, r, n_min, pad0;
    // acceptance variants: cyl_ext < 0 the infinite line, else a finite
    // cylinder reaching cyl_ext units beyond each seed grain; thr_num > 0
    // a threshold n_min + ceil(thr_num / thr_den tan(theta)), capped at
    // thr_max when thr_max > 0
    int32_t cyl_ext, thr_num, thr_den, thr_max;
    int32_t cell_req[3];  // fixed cell edges, used when auto_cells == 0
    uint32_t flags;
    int32_t auto_cells;   // 1: per view from cell_tab by density
    int32_t cell_tab[kCellBuckets][3];
};

// Device counters of one call. Totals keep counting past capacities so the
// host learns what a retry needs.
// Seed and member totals come from uint32 scans; their exact 64-bit sums are
// kept beside them, and a scan total that wrapped is saturated to 2^32 - 1,
// so a wrapped total always reads as an overflow.
struct Counters {
    uint32_t n_seeds;
    uint32_t n_seeds_ok;  // seeds the later stages take: n_seeds if it fits, else 0
    unsigned long long tests;
    unsigned long long hits;
    uint32_t n_cand;
    uint32_t n_members;
    uint32_t n_act[2];  // [0]: candidates taking part in the merge
    uint32_t n_acc;
    uint32_t n_track_grains;
    uint32_t rounds;
    uint32_t n_fp64;
    uint32_t err;
    uint32_t pass_words;  // words of the candidate bit mask: ceil(n_seeds_ok / 32)
    unsigned long long seeds64;    // exact number of seeds
    unsigned long long members64;  // exact number of member entries
};

struct Cand {
    uint32_t p, q;  // sorted positions of the seed grains
    uint32_t n;     // grains within r of the seed line
    uint32_t v;     // view
};

// Candidate priority: smaller key = taken earlier. Grain count descending,
// then the seed's input indices i, j ascending (all below 2^20).
__host__ __device__ inline unsigned long long cand_key(uint32_t n, uint32_t i,
                                                       uint32_t j) {
    return ((unsigned long long)(kNMax - 1u - n) << 40) |
           ((unsigned long long)i << 20) | (unsigned long long)j;
}

// kCertain: undecided, but sure to be accepted (it already holds n_min of
// its grains); it has taken those and waits for the others to be settled.
enum : uint8_t { kUndecided = 0, kAccepted = 1, kRejected = 2, kCertain = 3 };

// Results, written by the last kernel straight into mapped pinned host
// memory (device-side addresses of host buffers).
struct HostOut {
    Counters *cnt;
    unsigned long long *view_seeds;
    uint32_t *view_cand;
    uint32_t *view_ntr;
    uint32_t *view_tr_off;
    int32_t *view_err;
    emt_track *tracks;     // cand_cap
    uint32_t *grains;      // mem_cap
    uint32_t *cands;       // 3 cand_cap (i, j, n), or null when not kept
};

// All device buffers of one call, as raw pointers.
struct DevPtrs {
    const int32_t *xyz;   // packed input, N x 3
    ViewGrid *grids;
    uint32_t *view_of;    // N
    uint32_t *cell_of;    // N
    uint32_t *rank;       // N
    uint32_t *cell_count; // C
    uint32_t *cell_start; // C
    int4 *sg;             // N (+ kSortedSpare) sorted grains: x, y, z relative to lo; w = input index
    float4 *sgf;          // N (+ kSortedSpare): x, y, z of sg as floats (exact), w = 0
    uint32_t *seed_cnt;   // N: seeds per anchor
    uint32_t *seed_off;   // N + 1
    uint2 *seeds;         // seed_cap
    uint32_t *seed_n;     // seed_cap: count if >= n_min, else 0
    uint32_t *pass;       // seed_cap / 32 + 1 words: bit s % 32 of word s / 32
                          // set when seed s reaches its threshold
    uint32_t *pass_pos;   // seed_cap / 32 + 2: candidates in the words before
    Cand *cand;           // cand_cap
    unsigned long long *key;  // cand_cap
    uint32_t *cand_n;     // cand_cap + 1
    uint32_t *cand_thr;   // cand_cap: grain-count threshold of each candidate
    uint32_t *mem_off;    // cand_cap + 1
    uint32_t *members;    // mem_cap
    uint8_t *taken;       // mem_cap
    uint8_t *status;      // cand_cap
    uint32_t *mcount;     // cand_cap
    unsigned long long *owner;  // N
    uint32_t *undecided;  // per merge round: candidates it left undecided
    uint32_t *grab;       // kGrabWords: item-range counters of the counting kernel
    uint32_t *act;        // cand_cap: undecided candidates handed to the tail
    uint32_t *act2;       // cand_cap
    uint32_t *acc;        // cand_cap
    uint32_t *grouped;    // cand_cap
    uint32_t *track_cand; // cand_cap
    uint32_t *tg_n;       // cand_cap + 1
    uint32_t *tg_off;     // cand_cap + 1
    long long *tvals;     // mem_cap
    uint32_t *tord;       // mem_cap
    emt_track *tracks;    // cand_cap
    uint32_t *out_grains; // mem_cap
    unsigned long long *view_seeds;  // V
    uint32_t *view_cand;  // V
    uint32_t *view_ntr;   // V
    uint32_t *view_tr_off;  // V + 1
    uint32_t *view_cursor;  // V
    uint32_t *view_tail;    // V: candidates of each view handed to its merge tail
    unsigned long long *part64;  // kPartWords: spread partial sums of four 64-bit totals
    uint32_t *scan_part;  // scan scratch
    Counters *cnt;
    const BatchDesc *desc;
    HostOut out;
};

// Capacities a launch sequence is built for (the actual sizes are in
// BatchDesc and never exceed these).
struct Caps {
    uint32_t n_total;         // grains
    uint32_t n_views;
    uint32_t n_cells;         // cell table entries
    uint32_t max_view_n;      // grains of the largest view
    unsigned long long seed_cap;
    uint32_t cand_cap;
    uint32_t mem_cap;
    int32_t wide_rounds;      // grid-wide merge rounds before the tail kernel
    int32_t pad;
};

// Grain recognition: stack geometry and the device buffers of one call.
struct StackGeom {
    uint32_t nx, ny, nz;  // pixels per row, rows per frame, frames; nx % 4 == 0
    uint32_t thr;         // pulse-height threshold (strict)
    uint32_t pnum[3], pden[3];  // pitch of x, y, z in 0.01 um units: num/den
    double inv_nx, inv_ny;      // 1 / nx, 1 / ny
};

struct GrainBufs {
    uint32_t *tile_cnt;   // grains per tile, grain_tile_count(G) entries
    uint32_t *group_cnt;  // grains per 64 tiles, grain_group_count(G) entries
    uint16_t *stage;      // grain_stage_slots(G): grain offsets within their tile
    uint32_t *total;      // grains found (may exceed max_out)
    int32_t *out;         // 3 * max_out: x, y, z per grain, 0.01 um units
    uint32_t max_out;
};

// Tiles of the grain recognition: pixels a tile streams, staging slots (two
// bytes each) per tile, tiles summed per group.
constexpr uint32_t kGrainTilePix = 8192;
constexpr uint32_t kGrainTileGrains = kGrainTilePix / 2;
constexpr uint32_t kGrainTileGroup = 64;

size_t grain_tile_count(const StackGeom &G);
size_t grain_group_count(const StackGeom &G);
size_t grain_stage_slots(const StackGeom &G);
void launch_find_grains(const uint8_t *img, const StackGeom &G, const GrainBufs &b,
                        hipStream_t s);

// Image filtering of an nx x ny x nz stack with per-pixel maps (ny x nx).
// vec16: every pointer 16-byte aligned (the 16-pixel form is used when the
// frame size allows it). Returns false if nx * ny is not a multiple of 4.
bool launch_filter(const uint8_t *raw, const uint16_t *gain, const uint8_t *thr, uint8_t *out,
                   uint32_t nx, uint32_t ny, uint32_t nz, bool vec16, hipStream_t s);

// Launchers (kernels.hip). All run on `s` and only enqueue work.
void launch_prepare(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s);
void launch_bin(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s);
void launch_seeds(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s);
void launch_count(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s);
void launch_candidates(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s);
void launch_members(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s);
void launch_merge_init(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s);
void launch_merge(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s);
void launch_fit(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s);
void launch_copy_out(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s);

size_t scan_scratch_words(uint32_t n_cap);
int max_merge_rounds();
int max_wide_rounds();

}  // namespace emt
