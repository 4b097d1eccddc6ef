// api.hip -- host implementation of the C ABI declared in include/emt.h.
//
// A context owns a stream, device buffers sized by capacities that only
// grow, pinned host buffers for staging and results, and timing events.
// One call packs the views, runs the stage sequence of kernels.hip on the
// stream, and copies the tracks back. Device-side counters keep counting
// past a capacity, so an overflow is repaired by one re-run with the exact
// sizes the first run reported.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "capacity.h"
#include "cell_table.h"
#include "emt_dev.h"
#include "emt_host.h"

using namespace emt;

namespace {

constexpr uint32_t kKnownFlags =
    EMT_F_STATS | EMT_F_FP64_FIT_ALWAYS | EMT_F_DEVICE_PTRS | EMT_F_CANDIDATES;
// Cell edges (units) for an axis left at 0 when the others are given:
// short along x, where a cell row is one contiguous run, and about the
// paper's 7.5 um hash cell across it.
constexpr int kDefaultCell[3] = {250, 750, 500};
constexpr int kMaxAttempts = 4;

struct DevArena {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace



struct emt_ctx {
    emt_config cfg{};
    Params P{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool poisoned = false;
    hipEvent_t ev[EMT_N_STAGES + 1] = {};
    hipEvent_t done = nullptr;  // end of the last enqueued attempt
    size_t budget = 0;
    size_t held = 0;

    // device buffers, grown on demand
    DevArena grain_buf, cell_buf, seed_buf, cand_buf, mem_buf, view_buf, misc_buf;
    DevArena stack_buf;  // grain recognition: stack copy, block counts, scan, output
    uint32_t *h_small = nullptr;  // pinned: two words exchanged with the device
    DevPtrs d{};
    // capacities the buffers currently hold
    uint32_t cap_n = 0, cap_cells = 0, cap_views = 0, cap_cand = 0, cap_mem = 0;
    unsigned long long cap_seeds = 0;
    // capacities learned from earlier calls
    double seeds_per_grain = 256.0, cand_per_grain = 8.0, mem_per_cand = 24.0;
    // grid-wide merge rounds for the next call: two more than the last call
    // needed in all (the single-workgroup tail finishes any rest)
    int next_wide = 0;

    // pinned host buffers
    int32_t *h_xyz = nullptr;
    size_t h_xyz_cap = 0;
    ViewGrid *h_grids = nullptr;
    uint32_t h_views_cap = 0;
    // results, in mapped pinned memory written by the device
    HostOut h{};                  // host addresses
    size_t cap_out_views = 0, cap_out_cnt = 0, cap_out_tracks = 0, cap_out_grains = 0;
    size_t cap_vs = 0, cap_vc = 0, cap_vn = 0, cap_vo = 0, cap_ve = 0, cap_cands = 0;
    // candidates kept (EMT_F_CANDIDATES): first candidate of each view of
    // the last call, and the number of views it had
    std::vector<uint32_t> cand_off;
    uint32_t last_views = 0;

    emt_call_stats last{};

    // the batch between begin and finish
    struct Pending {
        const emt_view_in *views = nullptr;
        uint32_t n_views = 0;
        Caps caps{};
        bool active = false;
    } pend;

    // captured launch sequences, keyed by capacities and buffer generation
    struct GraphEntry {
        Caps caps;
        unsigned gen;
        int stage;  // -1: the whole sequence
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    unsigned gen = 0;        // bumped whenever a device buffer moves
    bool use_graphs = true;
    BatchDesc *h_desc = nullptr;
};

namespace {

int check_config(const emt_config *c) {
    if (!c) return EMT_EINVAL;
    if (c->abi_version != EMT_ABI_VERSION) return EMT_EINVAL;
    if ((c->flags & ~kKnownFlags) != 0) return EMT_EINVAL;
    if (c->cell[0] < 0 || c->cell[1] < 0 || c->cell[2] < 0) return EMT_EINVAL;
    if (c->device < 0) return EMT_EINVAL;
    if (c->seed_dist < 1 || c->seed_dist > kRMax) return EMT_ERANGE;
    if (c->tol_radius < 0 || c->tol_radius >= c->seed_dist) return EMT_ERANGE;
    if (c->min_grains < 2 || (uint32_t)c->min_grains >= kNMax) return EMT_ERANGE;
    if (c->cell[0] > kSpanMax || c->cell[1] > kSpanMax || c->cell[2] > kSpanMax) return EMT_ERANGE;
    if (c->cyl_ext < -1 || c->cyl_ext > kSpanMax) return EMT_ERANGE;
    if (c->thr_slope[0] < 0 || c->thr_slope[0] > 1024 || c->thr_slope[1] < 1 ||
        c->thr_slope[1] > 1024)
        return EMT_ERANGE;
    if (c->thr_max < 0 ||
        (c->thr_max > 0 && (c->thr_max < c->min_grains || (uint32_t)c->thr_max >= kNMax)))
        return EMT_ERANGE;
    return EMT_OK;
}

int check_views(const emt_config *c, const emt_view_in *v, uint32_t nv) {
    if (nv > 0 && !v) return EMT_EINVAL;
    unsigned long long total = 0;
    for (uint32_t i = 0; i < nv; ++i) {
        if (v[i].n_grains > 0 && !v[i].xyz) return EMT_EINVAL;
        if (v[i].n_grains >= kNMax) return EMT_ERANGE;
        total += v[i].n_grains;
        if (c->flags & EMT_F_DEVICE_PTRS) continue;
        const int32_t *x = v[i].xyz;
        for (int m = 0; m < 3 && v[i].n_grains; ++m) {
            int32_t lo = x[m], hi = x[m];
            for (uint32_t k = 1; k < v[i].n_grains; ++k) {
                const int32_t q = x[3 * (size_t)k + m];
                lo = q < lo ? q : lo;
                hi = q > hi ? q : hi;
            }
            if ((long long)hi - (long long)lo > kSpanMax) return EMT_ERANGE;
        }
    }
    if (total >= (1ull << 31)) return EMT_ERANGE;
    return EMT_OK;
}

template <class T>
T *carve(char *&p, size_t n) {
    T *r = reinterpret_cast<T *>(p);
    p += ((n * sizeof(T) + 255) / 256) * 256;
    return r;
}

template <class T>
size_t bytes_of(size_t n) {
    return ((n * sizeof(T) + 255) / 256) * 256;
}

#define HIP_OK(expr)                        \
    do {                                    \
        if ((expr) != hipSuccess) {         \
            ctx->poisoned = true;           \
            return EMT_EDEVICE;             \
        }                                   \
    } while (0)

int arena(emt_ctx *ctx, DevArena &a, size_t bytes) {
    if (a.bytes >= bytes) return EMT_OK;
    if (a.p) {
        if (hipFree(a.p) != hipSuccess) {
            ctx->poisoned = true;
            return EMT_EDEVICE;
        }
        ctx->held -= a.bytes;
        a.p = nullptr;
        a.bytes = 0;
    }
    if (ctx->held + bytes > ctx->budget) return EMT_ENOMEM;
    ctx->gen++;
    if (hipMalloc(&a.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return EMT_ENOMEM;
    }
    a.bytes = bytes;
    ctx->held += bytes;
    return EMT_OK;
}

template <class T>
int pinned(emt_ctx *ctx, T *&p, size_t &cap, size_t n) {
    if (cap >= n && p) return EMT_OK;
    if (p) {
        if (hipHostFree(p) != hipSuccess) {
            ctx->poisoned = true;
            return EMT_EDEVICE;
        }
        p = nullptr;
        cap = 0;
    }
    size_t want = std::max<size_t>(n, 1024);
    want += want / 4;
    if (hipHostMalloc((void **)&p, want * sizeof(T), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return EMT_ENOMEM;
    }
    cap = want;
    return EMT_OK;
}

// Mapped pinned host memory the device writes results into.
template <class T>
int mapped(emt_ctx *ctx, T *&host, T *&dev, size_t &cap, size_t n) {
    if (cap >= n && host) return EMT_OK;
    if (host) {
        if (hipHostFree(host) != hipSuccess) {
            ctx->poisoned = true;
            return EMT_EDEVICE;
        }
        host = nullptr;
        dev = nullptr;
        cap = 0;
    }
    ctx->gen++;
    size_t want = std::max<size_t>(n, 64);
    if (hipHostMalloc((void **)&host, want * sizeof(T), hipHostMallocMapped) != hipSuccess) {
        (void)hipGetLastError();
        host = nullptr;
        return EMT_ENOMEM;
    }
    if (hipHostGetDevicePointer((void **)&dev, host, 0) != hipSuccess) {
        (void)hipGetLastError();
        return EMT_EDEVICE;
    }
    cap = want;
    return EMT_OK;
}

// Device bytes of each arena for a capacity (ensure carves them in this
// layout).
size_t grain_bytes(size_t n) {
    return bytes_of<int32_t>(3 * n) + 4 * bytes_of<uint32_t>(n) + bytes_of<uint32_t>(n + 1) +
           2 * bytes_of<int4>(n + kSortedSpare) + bytes_of<unsigned long long>(n);
}
size_t seed_bytes(size_t n) {
    return bytes_of<uint2>(n) + bytes_of<uint32_t>(n) + bytes_of<uint32_t>(n / 32 + 1) +
           bytes_of<uint32_t>(n / 32 + 2);
}
size_t cand_bytes(size_t n) {
    return bytes_of<Cand>(n) + bytes_of<unsigned long long>(n) + 4 * bytes_of<uint32_t>(n + 1) +
           7 * bytes_of<uint32_t>(n) + bytes_of<uint8_t>(n) + bytes_of<emt_track>(n);
}
size_t mem_bytes(size_t n) {
    return 3 * bytes_of<uint32_t>(n) + bytes_of<uint8_t>(n) + bytes_of<long long>(n);
}
size_t cell_bytes(size_t n) {
    return 2 * bytes_of<uint32_t>(n) + bytes_of<uint32_t>(scan_scratch_words((uint32_t)n));
}
size_t view_bytes(size_t n) {
    return bytes_of<ViewGrid>(n) + bytes_of<unsigned long long>(n) + 5 * bytes_of<uint32_t>(n + 1) +
           bytes_of<Counters>(1) + bytes_of<uint32_t>((size_t)max_merge_rounds()) +
           bytes_of<uint32_t>(kGrabWords) + bytes_of<unsigned long long>(kPartWords) +
           bytes_of<BatchDesc>(1);
}
// the scan scratch serves every scan: cells, anchors, seeds, candidates
uint32_t scan_words(const Caps &c) {
    return std::max<uint32_t>(std::max<uint32_t>(c.n_cells, c.cand_cap),
                              std::max<uint32_t>((uint32_t)(c.seed_cap / 32 + 1), c.n_total)) + 1;
}

// Make every buffer hold the capacities in c, carve the pointer table, and
// raise c to what the buffers hold.
int ensure(emt_ctx *ctx, Caps &c) {
    int rc;
    DevPtrs &d = ctx->d;
    if (c.n_total > ctx->cap_n || !ctx->grain_buf.p) {
        const size_t n = std::max<uint32_t>(c.n_total, 1024);
        const size_t b = grain_bytes(n);
        if ((rc = arena(ctx, ctx->grain_buf, b))) return rc;
        char *p = (char *)ctx->grain_buf.p;
        d.xyz = carve<int32_t>(p, 3 * n);
        d.view_of = carve<uint32_t>(p, n);
        d.cell_of = carve<uint32_t>(p, n);
        d.rank = carve<uint32_t>(p, n);
        d.seed_cnt = carve<uint32_t>(p, n);
        d.seed_off = carve<uint32_t>(p, n + 1);
        d.sg = carve<int4>(p, n + kSortedSpare);
        d.sgf = carve<float4>(p, n + kSortedSpare);
        d.owner = carve<unsigned long long>(p, n);
        ctx->cap_n = (uint32_t)n;
    }
    if (c.seed_cap > ctx->cap_seeds || !ctx->seed_buf.p) {
        const size_t n = c.seed_cap;
        const size_t b = seed_bytes(n);
        if ((rc = arena(ctx, ctx->seed_buf, b))) return rc;
        char *p = (char *)ctx->seed_buf.p;
        d.seeds = carve<uint2>(p, n);
        d.seed_n = carve<uint32_t>(p, n);
        d.pass = carve<uint32_t>(p, n / 32 + 1);
        d.pass_pos = carve<uint32_t>(p, n / 32 + 2);
        ctx->cap_seeds = c.seed_cap;
    }
    if (c.cand_cap > ctx->cap_cand || !ctx->cand_buf.p) {
        const size_t n = c.cand_cap;
        const size_t b = cand_bytes(n);
        if ((rc = arena(ctx, ctx->cand_buf, b))) return rc;
        char *p = (char *)ctx->cand_buf.p;
        d.cand = carve<Cand>(p, n);
        d.key = carve<unsigned long long>(p, n);
        d.cand_n = carve<uint32_t>(p, n + 1);
        d.cand_thr = carve<uint32_t>(p, n);
        d.mem_off = carve<uint32_t>(p, n + 1);
        d.tg_n = carve<uint32_t>(p, n + 1);
        d.tg_off = carve<uint32_t>(p, n + 1);
        d.mcount = carve<uint32_t>(p, n);
        d.act = carve<uint32_t>(p, n);
        d.act2 = carve<uint32_t>(p, n);
        d.acc = carve<uint32_t>(p, n);
        d.grouped = carve<uint32_t>(p, n);
        d.track_cand = carve<uint32_t>(p, n);
        d.status = carve<uint8_t>(p, n);
        d.tracks = carve<emt_track>(p, n);
        ctx->cap_cand = (uint32_t)n;
    }
    if (c.mem_cap > ctx->cap_mem || !ctx->mem_buf.p) {
        const size_t n = c.mem_cap;
        const size_t b = mem_bytes(n);
        if ((rc = arena(ctx, ctx->mem_buf, b))) return rc;
        char *p = (char *)ctx->mem_buf.p;
        d.members = carve<uint32_t>(p, n);
        d.tord = carve<uint32_t>(p, n);
        d.out_grains = carve<uint32_t>(p, n);
        d.taken = carve<uint8_t>(p, n);
        d.tvals = carve<long long>(p, n);
        ctx->cap_mem = (uint32_t)n;
    }
    c.seed_cap = std::max<unsigned long long>(c.seed_cap, ctx->cap_seeds);
    c.cand_cap = std::max(c.cand_cap, ctx->cap_cand);
    c.mem_cap = std::max(c.mem_cap, ctx->cap_mem);
    const uint32_t scan_cap = scan_words(c);
    if (scan_cap > ctx->cap_cells || !ctx->cell_buf.p) {
        const size_t n = std::max<uint32_t>(scan_cap, 1u << 16);
        const size_t b = cell_bytes(n);
        if ((rc = arena(ctx, ctx->cell_buf, b))) return rc;
        char *p = (char *)ctx->cell_buf.p;
        d.cell_count = carve<uint32_t>(p, n);
        d.cell_start = carve<uint32_t>(p, n);
        d.scan_part = carve<uint32_t>(p, scan_scratch_words((uint32_t)n));
        ctx->cap_cells = (uint32_t)n;
    }
    if (c.n_views > ctx->cap_views || !ctx->view_buf.p) {
        const size_t n = std::max<uint32_t>(c.n_views, 64);
        const size_t b = view_bytes(n);
        if ((rc = arena(ctx, ctx->view_buf, b))) return rc;
        char *p = (char *)ctx->view_buf.p;
        d.grids = carve<ViewGrid>(p, n);
        d.view_seeds = carve<unsigned long long>(p, n);
        d.view_cand = carve<uint32_t>(p, n + 1);
        d.view_ntr = carve<uint32_t>(p, n + 1);
        d.view_tr_off = carve<uint32_t>(p, n + 1);
        d.view_cursor = carve<uint32_t>(p, n + 1);
        d.view_tail = carve<uint32_t>(p, n + 1);
        d.cnt = carve<Counters>(p, 1);
        d.undecided = carve<uint32_t>(p, (size_t)max_merge_rounds());
        d.grab = carve<uint32_t>(p, kGrabWords);
        d.part64 = carve<unsigned long long>(p, kPartWords);
        d.desc = carve<BatchDesc>(p, 1);
        ctx->cap_views = (uint32_t)n;
        // matching pinned staging of the view table
        size_t cap = 0;
        if (ctx->h_grids) {
            (void)hipHostFree(ctx->h_grids);
            ctx->h_grids = nullptr;
        }
        if ((rc = pinned(ctx, ctx->h_grids, cap, n))) return rc;
        ctx->h_views_cap = (uint32_t)n;
    }
    if (!ctx->h_desc) {
        size_t cap = 0;
        if ((rc = pinned(ctx, ctx->h_desc, cap, 1))) return rc;
    }
    {
        const size_t nv = ctx->cap_views + 1;
        HostOut &h = ctx->h;
        HostOut &o = d.out;
        if ((rc = mapped(ctx, h.cnt, o.cnt, ctx->cap_out_cnt, 1))) return rc;
        if ((rc = mapped(ctx, h.view_seeds, o.view_seeds, ctx->cap_vs, nv))) return rc;
        if ((rc = mapped(ctx, h.view_cand, o.view_cand, ctx->cap_vc, nv))) return rc;
        if ((rc = mapped(ctx, h.view_ntr, o.view_ntr, ctx->cap_vn, nv))) return rc;
        if ((rc = mapped(ctx, h.view_tr_off, o.view_tr_off, ctx->cap_vo, nv))) return rc;
        if ((rc = mapped(ctx, h.view_err, o.view_err, ctx->cap_ve, nv))) return rc;
        if ((rc = mapped(ctx, h.tracks, o.tracks, ctx->cap_out_tracks, c.cand_cap))) return rc;
        if ((rc = mapped(ctx, h.grains, o.grains, ctx->cap_out_grains, c.mem_cap))) return rc;
        if (ctx->cfg.flags & EMT_F_CANDIDATES) {
            if ((rc = mapped(ctx, h.cands, o.cands, ctx->cap_cands, 3 * (size_t)c.cand_cap)))
                return rc;
        }
    }
    return EMT_OK;
}

void record(emt_ctx *ctx, int i) {
    if (ctx->cfg.flags & EMT_F_STATS) (void)hipEventRecord(ctx->ev[i], ctx->stream);
}

// The kernel sequence of one batch, in stages: 0 bin, 1 seeds, 2 count,
// 3 candidates and members, 4 merge, 5 fit, 6 results to the host; -1 runs
// them all.
constexpr int kStages = 7;

void launch_stage(emt_ctx *ctx, const DevPtrs &run, const Caps &c, hipStream_t s, int stage) {
    switch (stage) {
        case 0:
            launch_prepare(run, c, ctx->P, s);
            launch_bin(run, c, ctx->P, s);
            break;
        case 1:
            launch_seeds(run, c, ctx->P, s);
            break;
        case 2:
            launch_count(run, c, ctx->P, s);
            break;
        case 3:
            launch_candidates(run, c, ctx->P, s);
            launch_members(run, c, ctx->P, s);
            break;
        case 4:
            launch_merge_init(run, c, ctx->P, s);
            launch_merge(run, c, ctx->P, s);
            break;
        case 5:
            launch_fit(run, c, ctx->P, s);
            break;
        default:
            launch_copy_out(run, c, ctx->P, s);
            break;
    }
}

void launch_stages(emt_ctx *ctx, const Caps &c, hipStream_t s, int stage) {
    if (stage >= 0) {
        launch_stage(ctx, ctx->d, c, s, stage);
        return;
    }
    for (int k = 0; k < kStages; ++k) launch_stage(ctx, ctx->d, c, s, k);
}

bool same_caps(const Caps &a, const Caps &b) {
    return a.n_total == b.n_total && a.n_views == b.n_views && a.n_cells == b.n_cells &&
           a.max_view_n == b.max_view_n && a.seed_cap == b.seed_cap &&
           a.cand_cap == b.cand_cap && a.mem_cap == b.mem_cap &&
           a.wide_rounds == b.wide_rounds;
}

void drop_graphs(emt_ctx *ctx) {
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
    ctx->graphs.clear();
}

// Run one stage (or all, stage -1): replay the graph captured for these
// capacities, capturing it first if needed; eager launches if graphs are off
// or capture fails.
int launch_graph(emt_ctx *ctx, const Caps &c, int stage) {
    hipStream_t s = ctx->stream;
    if (ctx->use_graphs) {
        for (auto &g : ctx->graphs) {
            if (g.gen == ctx->gen && g.stage == stage && same_caps(g.caps, c)) {
                HIP_OK(hipGraphLaunch(g.exec, s));
                return EMT_OK;
            }
        }
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            launch_stages(ctx, c, s, stage);
            ok = hipStreamEndCapture(s, &graph) == hipSuccess && graph != nullptr;
        }
        if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        if (ok) {
            if (ctx->graphs.size() >= 16) {
                (void)hipGraphExecDestroy(ctx->graphs.front().exec);
                ctx->graphs.erase(ctx->graphs.begin());
            }
            ctx->graphs.push_back({c, ctx->gen, stage, exec});
            HIP_OK(hipGraphLaunch(exec, s));
            return EMT_OK;
        }
        // capture is not available here: run eagerly from now on
        (void)hipGetLastError();
        ctx->use_graphs = false;
    }
    launch_stages(ctx, c, s, stage);
    return hipGetLastError() == hipSuccess ? EMT_OK : EMT_EDEVICE;
}

// The whole kernel sequence. With EMT_F_STATS each stage is its own graph
// and the timing events are recorded between them.
int launch_sequence(emt_ctx *ctx, const Caps &c) {
    if (!(ctx->cfg.flags & EMT_F_STATS)) return launch_graph(ctx, c, -1);
    for (int k = 0; k < kStages; ++k) {
        int rc = launch_graph(ctx, c, k);
        if (rc) return rc;
        record(ctx, k + 2);  // events 2..8 close stages bin..out
    }
    return EMT_OK;
}

// Enqueue one attempt at the whole batch on the context's stream: staging
// copies, then the kernel sequence. Nothing waits.
int run_launch(emt_ctx *ctx, const emt_view_in *views, uint32_t nv, const Caps &c) {
    DevPtrs &d = ctx->d;
    hipStream_t s = ctx->stream;
    record(ctx, 0);
    // stage the grains into the packed buffer
    const bool dev = (ctx->cfg.flags & EMT_F_DEVICE_PTRS) != 0;
    if (dev) {
        for (uint32_t v = 0; v < nv; ++v) {
            if (!views[v].n_grains) continue;
            HIP_OK(hipMemcpyAsync((void *)(d.xyz + 3 * (size_t)ctx->h_grids[v].grain_off),
                                  views[v].xyz, 12 * (size_t)views[v].n_grains,
                                  hipMemcpyDeviceToDevice, s));
        }
    } else if (ctx->h_desc->n_total) {
        HIP_OK(hipMemcpyAsync((void *)d.xyz, ctx->h_xyz, 12 * (size_t)ctx->h_desc->n_total,
                              hipMemcpyHostToDevice, s));
    }
    HIP_OK(hipMemcpyAsync(d.grids, ctx->h_grids, sizeof(ViewGrid) * nv, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync((void *)d.desc, ctx->h_desc, sizeof(BatchDesc), hipMemcpyHostToDevice, s));
    record(ctx, 1);
    int rc = launch_sequence(ctx, c);
    if (rc) {
        ctx->poisoned = true;
        return rc;
    }
    HIP_OK(hipEventRecord(ctx->done, s));
    return EMT_OK;
}

// Wait for the attempt enqueued by run_launch. Returns EMT_OK,
// EMT_EOVERFLOW (caps too small: ctx->h.cnt holds the needs) or an error.
int run_check(emt_ctx *ctx, const Caps &c, bool *overflow) {
    *overflow = false;
    HIP_OK(hipEventSynchronize(ctx->done));
    const Counters &h = *ctx->h.cnt;
    const Needs need{h.seeds64, h.members64, h.n_cand};
    const CapSizes have{c.seed_cap, c.cand_cap, c.mem_cap};
    if (!fits(need, have)) {
        *overflow = true;
        return EMT_EOVERFLOW;
    }
    if (h.err & 4u) {
        ctx->poisoned = true;
        return EMT_EDEVICE;
    }
    return EMT_OK;
}

// Per-view grid records for one attempt (the device overwrites them).
void fill_grids(emt_ctx *ctx, const emt_view_in *views, uint32_t n_views) {
    uint32_t go = 0, co = 0;
    for (uint32_t v = 0; v < n_views; ++v) {
        ViewGrid &G = ctx->h_grids[v];
        G = ViewGrid{};
        for (int m = 0; m < 3; ++m) {
            G.lo[m] = INT32_MAX;
            G.hi[m] = INT32_MIN;
        }
        G.grain_off = go;
        G.n = views[v].n_grains;
        G.cell_off = co;
        G.cell_cap = kCellsPerGrain * views[v].n_grains + kCellsBase;
        go += G.n;
        co += G.cell_cap + 1;
    }
}

// Capacity bucket: the next power of two, at least lo.
uint32_t bucket(uint64_t n, uint32_t lo) {
    uint64_t b = lo;
    while (b < n) b <<= 1;
    return (uint32_t)std::min<uint64_t>(b, 0x80000000ull);
}

// Capacities for a batch: power-of-two buckets of the sizes (so launch
// shapes and captured graphs repeat) and learned per-grain ratios.
int batch_caps(const emt_ctx *ctx, unsigned long long n_total, uint32_t n_views, uint32_t max_n,
               Caps *out) {
    Caps c{};
    c.n_total = bucket(n_total, 1024);
    c.n_views = bucket(n_views, 1);
    const unsigned long long cells_cap =
        (unsigned long long)kCellsPerGrain * c.n_total + (kCellsBase + 1ull) * c.n_views;
    if (cells_cap >= (1ull << 31)) return EMT_ERANGE;
    c.n_cells = (uint32_t)cells_cap;
    c.max_view_n = std::min(c.n_total, bucket(max_n, 64));
    c.seed_cap = std::min<unsigned long long>(
        kSeedCapMax, std::max<unsigned long long>(
                         4096, (unsigned long long)(ctx->seeds_per_grain * (double)c.n_total)));
    c.cand_cap = clamp_cap(ctx->cand_per_grain * (double)c.n_total);
    c.mem_cap = clamp_cap(ctx->mem_per_cand * (double)c.cand_cap);
    c.wide_rounds = ctx->next_wide > 0 ? ctx->next_wide : max_wide_rounds();
    *out = c;
    return EMT_OK;
}

// Scratch of emt_find_grains_noalloc: the per-tile grain counts, per-group
// sums, staging slots and the grain total of one recognition call, carved
// in that order (1 byte a stack pixel plus ~0.1 %). One copy per device,
// held until the process ends; every call on a device shares it and keeps
// the last call's contents (the per-group sums, the only words read before
// they are written, are cleared by a kernel at the start of each call).
// Host code never passes the array's name to a kernel: it uses the device
// address emt_create resolves for each device (scratch_dev).
constexpr size_t kNoAllocScratchBytes = (size_t)EMT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxScratchDevices = 256;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxScratchDevices];  // address of scratch on each device

// With the device current: resolve the array's address on it (once).
int resolve_scratch(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return EMT_OK;  // variant unavailable
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return EMT_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return EMT_EDEVICE;
    }
    g_scratch_dev[device] = ptr;
    return EMT_OK;
}

void *scratch_dev(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[device];
}

// Bytes the recognition buffers take when carved from one block.
size_t grain_scratch_bytes(const StackGeom &G) {
    auto r = [](size_t b) { return ((b + 255) / 256) * 256; };
    return r(bytes_of<uint32_t>(grain_tile_count(G))) +
           r(bytes_of<uint32_t>(grain_group_count(G))) +
           r(bytes_of<uint16_t>(grain_stage_slots(G))) + r(bytes_of<uint32_t>(1));
}

}  // namespace

extern "C" {

void emt_default_config(emt_config *cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->abi_version = EMT_ABI_VERSION;
    cfg->seed_dist = 2500;
    cfg->tol_radius = 50;
    cfg->min_grains = 8;
    cfg->cell[0] = cfg->cell[1] = cfg->cell[2] = 0;
    cfg->device = 0;
    cfg->flags = 0;
    cfg->hbm_budget = 0;
    cfg->stream = nullptr;
    cfg->cyl_ext = -1;
    cfg->thr_slope[0] = 0;
    cfg->thr_slope[1] = 1;
    cfg->thr_max = 0;
}

int emt_validate(const emt_config *cfg, const emt_view_in *views, uint32_t n_views) {
    int rc = check_config(cfg);
    if (rc) return rc;
    return check_views(cfg, views, n_views);
}

const char *emt_strerror(int code) {
    switch (code) {
        case EMT_OK: return "ok";
        case EMT_EINVAL: return "invalid argument";
        case EMT_ERANGE: return "value out of range (span, grain count, R or r)";
        case EMT_ENOMEM: return "out of memory or HBM budget";
        case EMT_EDEVICE: return "HIP device error (context poisoned)";
        case EMT_EOVERFLOW: return "internal capacity overflow after retries";
        default: return "unknown error";
    }
}

int emt_create(const emt_config *cfg, emt_ctx **out) {
    if (!out) return EMT_EINVAL;
    *out = nullptr;
    int rc = check_config(cfg);
    if (rc) return rc;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device >= ndev) {
        (void)hipGetLastError();
        return EMT_EDEVICE;
    }
    if (hipSetDevice(cfg->device) != hipSuccess) return EMT_EDEVICE;
    emt_ctx *ctx = new (std::nothrow) emt_ctx();
    if (!ctx) return EMT_ENOMEM;
    ctx->cfg = *cfg;
    ctx->P.R = cfg->seed_dist;
    ctx->P.r = cfg->tol_radius;
    ctx->P.n_min = cfg->min_grains;
    ctx->P.cyl_ext = cfg->cyl_ext;
    ctx->P.thr_num = cfg->thr_slope[0];
    ctx->P.thr_den = cfg->thr_slope[1];
    ctx->P.thr_max = cfg->thr_max;
    // cell edges: per view from the tuned density table when none is given
    ctx->P.auto_cells = (cfg->cell[0] || cfg->cell[1] || cfg->cell[2]) ? 0 : 1;
    for (int m = 0; m < 3; ++m) ctx->P.cell_req[m] = cfg->cell[m] ? cfg->cell[m] : kDefaultCell[m];
    for (int b = 0; b < kCellBuckets; ++b)
        for (int m = 0; m < 3; ++m) ctx->P.cell_tab[b][m] = kTunedCells[b][m];
    ctx->P.flags = cfg->flags;
    // Tuning hook: fixed cell edges "x,y,z" in units.
    if (const char *e = std::getenv("EMT_CELL")) {
        int v[3];
        if (std::sscanf(e, "%d,%d,%d", &v[0], &v[1], &v[2]) == 3 && v[0] > 0 && v[1] > 0 &&
            v[2] > 0 && v[0] <= kSpanMax && v[1] <= kSpanMax && v[2] <= kSpanMax) {
            for (int m = 0; m < 3; ++m) ctx->P.cell_req[m] = v[m];
            ctx->P.auto_cells = 0;
        }
    }
    if (const char *e = std::getenv("EMT_NO_GRAPH")) ctx->use_graphs = (std::atoi(e) == 0);
    // Test hook: start from tiny capacities so the first call overflows and
    // the retry path runs.
    if (const char *e = std::getenv("EMT_INITIAL_CAPS")) {
        if (std::strcmp(e, "tiny") == 0) {
            ctx->seeds_per_grain = 0.5;
            ctx->cand_per_grain = 0.01;
            ctx->mem_per_cand = 1.0;
        }
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        delete ctx;
        return EMT_EDEVICE;
    }
    ctx->budget = cfg->hbm_budget ? (size_t)cfg->hbm_budget : (size_t)(0.8 * (double)free_b);
    if (cfg->stream) {
        ctx->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return EMT_EDEVICE;
        }
        ctx->own_stream = true;
    }
    for (int i = 0; i <= EMT_N_STAGES; ++i) {
        if (hipEventCreate(&ctx->ev[i]) != hipSuccess) {
            emt_destroy(ctx);
            return EMT_EDEVICE;
        }
    }
    if (hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming) != hipSuccess) {
        emt_destroy(ctx);
        return EMT_EDEVICE;
    }
    // set-up of the no-allocation variant: the scratch array's address on
    // this device, and the pinned words results come back through
    if ((rc = resolve_scratch(cfg->device)) != EMT_OK) {
        emt_destroy(ctx);
        return rc;
    }
    size_t small_cap = 0;
    if ((rc = pinned(ctx, ctx->h_small, small_cap, 4)) != EMT_OK) {
        emt_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return EMT_OK;
}

}  // extern "C"

namespace emt {

// Device bytes a context needs for a batch of these sizes (its arenas only
// grow, so this bounds what the batch adds to the context's holdings).
size_t batch_bytes(const emt_ctx *ctx, unsigned long long n_total, uint32_t n_views,
                   uint32_t max_n) {
    Caps c{};
    if (batch_caps(ctx, n_total, n_views, max_n, &c)) return SIZE_MAX;
    return grain_bytes(std::max<uint32_t>(c.n_total, 1024)) + seed_bytes(c.seed_cap) +
           cand_bytes(c.cand_cap) + mem_bytes(c.mem_cap) +
           cell_bytes(std::max<uint32_t>(scan_words(c), 1u << 16)) +
           view_bytes(std::max<uint32_t>(c.n_views, 64));
}

size_t held_bytes(const emt_ctx *ctx) { return ctx->held; }

// First half of a call: check, size, stage and enqueue the first attempt.
// The views (and, for host input, their grains) must stay valid until
// finish_views returns.
int begin_views(emt_ctx *ctx, const emt_view_in *views, uint32_t n_views) {
    if (!ctx) return EMT_EINVAL;
    if (ctx->poisoned) return EMT_EDEVICE;
    if (ctx->pend.active) return EMT_EINVAL;
    int rc = check_views(&ctx->cfg, views, n_views);
    if (rc) return rc;
    if (hipSetDevice(ctx->cfg.device) != hipSuccess) {
        ctx->poisoned = true;
        return EMT_EDEVICE;
    }
    // batch sizes (to the device) and capacity buckets (launch shapes)
    unsigned long long n_total = 0, n_cells = 0;
    uint32_t max_n = 0;
    for (uint32_t v = 0; v < n_views; ++v) {
        n_total += views[v].n_grains;
        n_cells += (unsigned long long)kCellsPerGrain * views[v].n_grains + kCellsBase + 1;
        max_n = std::max(max_n, views[v].n_grains);
    }
    Caps c{};
    if ((rc = batch_caps(ctx, n_total, n_views, max_n, &c))) return rc;

    // ensure the view tables exist before filling pinned staging
    if ((rc = ensure(ctx, c))) return rc;
    ctx->h_desc->n_total = (uint32_t)n_total;
    ctx->h_desc->n_views = n_views;
    ctx->h_desc->n_cells = (uint32_t)n_cells;
    ctx->h_desc->n_cells_m1 = (uint32_t)n_cells - 1u;
    if (!(ctx->cfg.flags & EMT_F_DEVICE_PTRS)) {
        if ((rc = pinned(ctx, ctx->h_xyz, ctx->h_xyz_cap, 3 * (size_t)std::max<unsigned long long>(n_total, 1))))
            return rc;
        uint32_t goff = 0;
        for (uint32_t v = 0; v < n_views; ++v) {
            if (views[v].n_grains)
                std::memcpy(ctx->h_xyz + 3 * (size_t)goff, views[v].xyz,
                            12 * (size_t)views[v].n_grains);
            goff += views[v].n_grains;
        }
    }
    fill_grids(ctx, views, n_views);
    if ((rc = run_launch(ctx, views, n_views, c))) return rc;
    ctx->pend.views = views;
    ctx->pend.n_views = n_views;
    ctx->pend.caps = c;
    ctx->pend.active = true;
    return EMT_OK;
}

// True once the enqueued attempt has finished on the device.
bool views_ready(emt_ctx *ctx) {
    return !ctx->pend.active || hipEventQuery(ctx->done) != hipErrorNotReady;
}

// Second half: wait, repair an overflow by re-running with the sizes the
// counters report, and fill out[] with per-view slices of the results.
int finish_views(emt_ctx *ctx, emt_view_out *out) {
    if (!ctx || !ctx->pend.active) return EMT_EINVAL;
    ctx->pend.active = false;
    const emt_view_in *views = ctx->pend.views;
    const uint32_t n_views = ctx->pend.n_views;
    Caps c = ctx->pend.caps;
    int rc;
    uint32_t retries = 0;
    for (int attempt = 0;; ++attempt) {
        bool overflow = false;
        rc = run_check(ctx, c, &overflow);
        if (rc == EMT_OK) break;
        if (!overflow) return rc;
        if (attempt + 1 >= kMaxAttempts) return EMT_EOVERFLOW;
        ++retries;
        const Counters h = *ctx->h.cnt;
        const Needs need{h.seeds64, h.members64, h.n_cand};
        CapSizes next{c.seed_cap, c.cand_cap, c.mem_cap};
        Ratios ratios{ctx->seeds_per_grain, ctx->cand_per_grain, ctx->mem_per_cand};
        if (!plan_retry(need, c.n_total, next, ratios)) return EMT_EOVERFLOW;
        c.seed_cap = next.seed_cap;
        c.cand_cap = next.cand_cap;
        c.mem_cap = next.mem_cap;
        ctx->seeds_per_grain = ratios.seeds_per_grain;
        ctx->cand_per_grain = ratios.cand_per_grain;
        ctx->mem_per_cand = ratios.mem_per_cand;
        if ((rc = ensure(ctx, c))) return rc;
        fill_grids(ctx, views, n_views);
        if ((rc = run_launch(ctx, views, n_views, c))) return rc;
    }

    // device-side rejections (span of device-resident views)
    for (uint32_t v = 0; v < n_views; ++v)
        if (ctx->h.view_err[v]) return EMT_ERANGE;
    if (ctx->h.cnt->err & 2u) {
        // member lists disagreed with the counts: an internal fault
        ctx->poisoned = true;
        return EMT_EDEVICE;
    }

    // outputs: per-view slices of the track and grain arrays
    const Counters &h = *ctx->h.cnt;
    for (uint32_t v = 0; v < n_views; ++v) {
        emt_view_out &o = out[v];
        const uint32_t t0 = ctx->h.view_tr_off[v], nt = ctx->h.view_ntr[v];
        o.view_id = views[v].view_id;
        o.n_tracks = nt;
        o.tracks = ctx->h.tracks + t0;
        const uint32_t g0 = nt ? ctx->h.tracks[t0].grain_offset : 0;
        uint32_t ng = 0;
        for (uint32_t t = 0; t < nt; ++t) {
            emt_track &tr = ctx->h.tracks[t0 + t];
            tr.grain_offset -= g0;
            ng += tr.n_grains;
        }
        o.n_track_grains = ng;
        o.grains = ctx->h.grains + g0;
        o.stats.n_seeds = ctx->h.view_seeds[v];
        o.stats.n_candidates = ctx->h.view_cand[v];
        o.stats.n_tracks = nt;
    }
    if (ctx->cfg.flags & EMT_F_CANDIDATES) {
        try {
            ctx->cand_off.resize((size_t)n_views + 1);
        } catch (...) {
            return EMT_ENOMEM;
        }
        uint32_t o = 0;
        for (uint32_t v = 0; v < n_views; ++v) {
            ctx->cand_off[v] = o;
            o += ctx->h.view_cand[v];
        }
        ctx->cand_off[n_views] = o;
        ctx->last_views = n_views;
    }
    ctx->next_wide = std::max(std::min(6, max_wide_rounds()),
                              std::min(max_wide_rounds(), (int)h.rounds + 2));
    emt_call_stats &st = ctx->last;
    st = emt_call_stats{};
    st.n_seeds = h.seeds64;
    st.n_tests = h.tests;
    st.n_hits = h.hits;
    st.n_candidates = h.n_cand;
    st.n_tracks = h.n_acc;
    st.merge_rounds = h.rounds;
    st.n_fp64_fits = h.n_fp64;
    st.retries = retries;
    st.n_views = n_views;
    if (ctx->cfg.flags & EMT_F_STATS) {
        float tot = 0.0f;
        for (int i = 0; i < EMT_N_STAGES; ++i) {
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]);
            st.ms[i] = ms;
            tot += ms;
        }
        st.ms_total = tot;
    }
    return EMT_OK;
}

}  // namespace emt

extern "C" {

int emt_track_views(emt_ctx *ctx, const emt_view_in *views, uint32_t n_views, emt_view_out *out) {
    int rc;
    if (!ctx) {
        rc = EMT_EINVAL;
    } else if (n_views > 0 && !out) {
        rc = EMT_EINVAL;
    } else if (n_views == 0) {
        rc = ctx->poisoned ? EMT_EDEVICE : check_views(&ctx->cfg, views, 0);
    } else {
        rc = begin_views(ctx, views, n_views);
        if (rc == EMT_OK) rc = finish_views(ctx, out);
    }
    // return codes carry every failure: leave no sticky HIP error behind
    (void)hipGetLastError();
    return rc;
}


// static_buf: null for emt_find_grains (buffers from the context's arena,
// grown as needed); the device address of scratch for the no-allocation
// variant (device pointers only, no allocation, stacks up to its size).
static int find_grains_impl(emt_ctx *ctx, const uint8_t *stack, const emt_stack_geom *g,
                            int32_t *xyz_out, uint32_t max_out, uint32_t *n_out,
                            void *static_buf = nullptr) {
    if (!ctx || !g || !n_out) return EMT_EINVAL;
    *n_out = 0;
    if (ctx->poisoned) return EMT_EDEVICE;
    if (g->nx < 4 || (g->nx & 3u) || g->nx > 65536u || g->ny < 1 || g->ny > 65536u ||
        g->nz < 1 || g->nz > 4096u || g->threshold > 255u)
        return EMT_ERANGE;
    for (int m = 0; m < 3; ++m)
        if (g->pitch_num[m] < 1 || g->pitch_num[m] > 65536u || g->pitch_den[m] < 1 ||
            g->pitch_den[m] > 65536u)
            return EMT_ERANGE;
    const unsigned long long npix = (unsigned long long)g->nx * g->ny * g->nz;
    if (npix > (1ull << 31)) return EMT_ERANGE;  // four-pixel groups then fit 32 bits
    if (!stack || (max_out > 0 && !xyz_out)) return EMT_EINVAL;
    if (max_out > (1u << 28)) return EMT_ERANGE;
    if (hipSetDevice(ctx->cfg.device) != hipSuccess) {
        ctx->poisoned = true;
        return EMT_EDEVICE;
    }
    const bool dev = (ctx->cfg.flags & EMT_F_DEVICE_PTRS) != 0;
    // the stack is read as aligned 16-byte vectors (host stacks are copied
    // into an aligned buffer; device ones must start on a 16-byte boundary)
    if (dev && ((uintptr_t)stack & 15u)) return EMT_EINVAL;
    if (dev && max_out > 0 && ((uintptr_t)xyz_out & 3u)) return EMT_EINVAL;
    StackGeom G{};
    G.nx = g->nx;
    G.ny = g->ny;
    G.nz = g->nz;
    G.thr = g->threshold;
    for (int m = 0; m < 3; ++m) {
        G.pnum[m] = g->pitch_num[m];
        G.pden[m] = g->pitch_den[m];
    }
    G.inv_nx = 1.0 / (double)G.nx;
    G.inv_ny = 1.0 / (double)G.ny;
    const size_t nt = grain_tile_count(G), ng = grain_group_count(G);
    char *p = nullptr;
    if (static_buf) {
        if (!dev) return EMT_EINVAL;
        if (grain_scratch_bytes(G) > kNoAllocScratchBytes) return EMT_ERANGE;
        if (!ctx->h_small) return EMT_EDEVICE;  // made by emt_create
        p = (char *)static_buf;
    } else {
        const size_t bytes = (dev ? 0 : bytes_of<uint8_t>((size_t)npix)) + bytes_of<uint32_t>(nt) +
                             bytes_of<uint32_t>(ng) + bytes_of<uint16_t>(grain_stage_slots(G)) +
                             bytes_of<uint32_t>(1) +
                             (dev ? 0 : bytes_of<int32_t>(3 * (size_t)max_out));
        int rc;
        if ((rc = arena(ctx, ctx->stack_buf, bytes))) return rc;
        size_t cap = 0;
        if (!ctx->h_small && (rc = pinned(ctx, ctx->h_small, cap, 4))) return rc;
        p = (char *)ctx->stack_buf.p;
    }
    const uint8_t *img = stack;
    if (!dev) img = carve<uint8_t>(p, (size_t)npix);
    GrainBufs b{};
    b.tile_cnt = carve<uint32_t>(p, nt);
    b.group_cnt = carve<uint32_t>(p, ng);
    b.stage = carve<uint16_t>(p, grain_stage_slots(G));
    b.total = carve<uint32_t>(p, 1);
    b.out = dev ? xyz_out : carve<int32_t>(p, 3 * (size_t)max_out);
    b.max_out = max_out;
    hipStream_t s = ctx->stream;
    if (!dev)
        HIP_OK(hipMemcpyAsync((void *)img, stack, (size_t)npix, hipMemcpyHostToDevice, s));
    const bool stats = (ctx->cfg.flags & EMT_F_STATS) != 0;
    if (stats) HIP_OK(hipEventRecord(ctx->ev[0], s));
    launch_find_grains(img, G, b, s);
    HIP_OK(hipGetLastError());
    if (stats) HIP_OK(hipEventRecord(ctx->ev[1], s));
    HIP_OK(hipMemcpyAsync(ctx->h_small + 1, b.total, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const uint32_t total = ctx->h_small[1];
    *n_out = total;
    ctx->last = emt_call_stats{};
    if (stats) (void)hipEventElapsedTime(&ctx->last.ms_total, ctx->ev[0], ctx->ev[1]);
    const uint32_t n = total < max_out ? total : max_out;
    if (!dev && n) {
        HIP_OK(hipMemcpyAsync(xyz_out, b.out, 12 * (size_t)n, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    return total > max_out ? EMT_EOVERFLOW : EMT_OK;
}

static int filter_impl(emt_ctx *ctx, const uint8_t *raw, const emt_stack_geom *g,
                       const uint16_t *gain, const uint8_t *thr, uint8_t *out) {
    if (!ctx || !g) return EMT_EINVAL;
    if (ctx->poisoned) return EMT_EDEVICE;
    if (g->nx < 4 || (g->nx & 3u) || g->nx > 65536u || g->ny < 1 || g->ny > 65536u ||
        g->nz < 1 || g->nz > 4096u)
        return EMT_ERANGE;
    const unsigned long long plane = (unsigned long long)g->nx * g->ny;
    const unsigned long long npix = plane * g->nz;
    if (npix > (1ull << 31)) return EMT_ERANGE;
    if (!raw || !gain || !thr || !out) return EMT_EINVAL;
    const bool dev = (ctx->cfg.flags & EMT_F_DEVICE_PTRS) != 0;
    if (dev && (((uintptr_t)raw | (uintptr_t)gain | (uintptr_t)thr | (uintptr_t)out) & 15u))
        return EMT_EINVAL;
    if (hipSetDevice(ctx->cfg.device) != hipSuccess) {
        ctx->poisoned = true;
        return EMT_EDEVICE;
    }
    int rc;
    const uint8_t *d_raw = raw, *d_thr = thr;
    const uint16_t *d_gain = gain;
    uint8_t *d_out = out;
    hipStream_t s = ctx->stream;
    if (!dev) {
        const size_t bytes = 2 * bytes_of<uint8_t>((size_t)npix) + bytes_of<uint16_t>(plane) +
                             bytes_of<uint8_t>(plane);
        if ((rc = arena(ctx, ctx->stack_buf, bytes))) return rc;
        char *p = (char *)ctx->stack_buf.p;
        uint8_t *h_raw = carve<uint8_t>(p, (size_t)npix);
        d_out = carve<uint8_t>(p, (size_t)npix);
        uint16_t *h_gain = carve<uint16_t>(p, plane);
        uint8_t *h_thr = carve<uint8_t>(p, plane);
        HIP_OK(hipMemcpyAsync(h_raw, raw, (size_t)npix, hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(h_gain, gain, 2 * (size_t)plane, hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(h_thr, thr, (size_t)plane, hipMemcpyHostToDevice, s));
        d_raw = h_raw;
        d_gain = h_gain;
        d_thr = h_thr;
    }
    const bool stats = (ctx->cfg.flags & EMT_F_STATS) != 0;
    if (stats) HIP_OK(hipEventRecord(ctx->ev[0], s));
    if (!launch_filter(d_raw, d_gain, d_thr, d_out, g->nx, g->ny, g->nz, true, s))
        return EMT_ERANGE;
    HIP_OK(hipGetLastError());
    if (stats) HIP_OK(hipEventRecord(ctx->ev[1], s));
    if (!dev) HIP_OK(hipMemcpyAsync(out, d_out, (size_t)npix, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    ctx->last = emt_call_stats{};
    if (stats) (void)hipEventElapsedTime(&ctx->last.ms_total, ctx->ev[0], ctx->ev[1]);
    return EMT_OK;
}

int emt_filter_stack(emt_ctx *ctx, const uint8_t *raw, const emt_stack_geom *geom,
                     const uint16_t *gain, const uint8_t *thr, uint8_t *out) {
    const int rc = filter_impl(ctx, raw, geom, gain, thr, out);
    (void)hipGetLastError();
    return rc;
}

int emt_find_grains(emt_ctx *ctx, const uint8_t *stack, const emt_stack_geom *geom,
                    int32_t *xyz_out, uint32_t max_out, uint32_t *n_out) {
    const int rc = find_grains_impl(ctx, stack, geom, xyz_out, max_out, n_out);
    (void)hipGetLastError();
    return rc;
}

int emt_find_grains_noalloc(emt_ctx *ctx, const uint8_t *stack, const emt_stack_geom *geom,
                            int32_t *xyz_out, uint32_t max_out, uint32_t *n_out) {
    if (!ctx || !n_out) return EMT_EINVAL;
    void *buf = scratch_dev(ctx->cfg.device);
    if (!buf) {
        *n_out = 0;
        return EMT_EINVAL;
    }
    const int rc = find_grains_impl(ctx, stack, geom, xyz_out, max_out, n_out, buf);
    (void)hipGetLastError();
    return rc;
}

int emt_view_candidates(emt_ctx *ctx, uint32_t view, const uint32_t **ijn, uint32_t *n_cand) {
    if (!ctx || !ijn || !n_cand) return EMT_EINVAL;
    *ijn = nullptr;
    *n_cand = 0;
    if (!(ctx->cfg.flags & EMT_F_CANDIDATES) || view >= ctx->last_views) return EMT_EINVAL;
    const uint32_t a = ctx->cand_off[view], b = ctx->cand_off[view + 1];
    *ijn = ctx->h.cands + 3 * (size_t)a;
    *n_cand = b - a;
    return EMT_OK;
}

int emt_last_stats(emt_ctx *ctx, emt_call_stats *stats) {
    if (!ctx || !stats) return EMT_EINVAL;
    *stats = ctx->last;
    return EMT_OK;
}

void emt_destroy(emt_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->cfg.device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    drop_graphs(ctx);
    DevArena *arenas[] = {&ctx->grain_buf, &ctx->cell_buf, &ctx->seed_buf, &ctx->cand_buf,
                          &ctx->mem_buf, &ctx->view_buf, &ctx->misc_buf, &ctx->stack_buf};
    for (DevArena *a : arenas)
        if (a->p) (void)hipFree(a->p);
    void *hosts[] = {ctx->h_small, ctx->h_xyz, ctx->h_grids, ctx->h_desc, ctx->h.cnt, ctx->h.view_seeds,
                     ctx->h.view_cand, ctx->h.view_ntr, ctx->h.view_tr_off, ctx->h.view_err,
                     ctx->h.tracks, ctx->h.grains, ctx->h.cands};
    for (void *p : hosts)
        if (p) (void)hipHostFree(p);
    for (int i = 0; i <= EMT_N_STAGES; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    if (ctx->done) (void)hipEventDestroy(ctx->done);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    (void)hipGetLastError();
}

}  // extern "C"
