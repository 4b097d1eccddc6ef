// kernels.hip -- gfx950 kernels of the per-view 4pi track finder.
//
// Pipeline (paper Sec. 2, tracking paragraph; hash cells after the Sec. 3
// footnote), for a batch of views packed one after another:
//   bin      bounding box per view, counting sort of grains into cells
//   seeds    all pairs closer than R (one lane per anchor grain)
//   count    grains within r of each seed's infinite line (one lane per seed)
//   members  grain lists of the seeds that reach n_min
//   merge    exclusive association, rounds of deterministic reservations
//   fit      track order, grain order, least-squares direction
// Every geometric decision is exact integer arithmetic; floating point only
// chooses which cells to visit and carries a safety margin.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "emt_dev.h"

namespace emt {

namespace {

// Tuning constants; -D on the compiler line overrides them (the counting
// kernel's tiles come from tile_table.h, through emt_dev.h).
#ifndef EMT_DYN_MIN_SEEDS
#define EMT_DYN_MIN_SEEDS 8000000
#endif
constexpr float kMargin = 4.0f;  // units added to every cell window
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ unsigned long long lanes_below() {
    return (1ull << lane_id()) - 1ull;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ float wave_min(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// Make this lane's global writes visible to the other lanes of its wave.
__device__ __forceinline__ void wave_sync_mem() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Adds a workgroup's total of wave-uniform values v (one per wave) to one
// of the kPartSlots counters of total `which`: the waves' values are summed
// in LDS, then one atomic per workgroup, the workgroups spread over the
// counters. Every thread of the workgroup must call it (it synchronises the
// workgroup twice).
__device__ __forceinline__ void add_spread(unsigned long long *part64, int which,
                                           unsigned long long v) {
    __shared__ unsigned long long s_part[kBlock / 64];
    if (lane_id() == 0) s_part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (uint32_t w = 0; w < blockDim.x / 64; ++w) t += s_part[w];
        if (t)
            atomicAdd(&part64[(which * kPartSlots + (int)(blockIdx.x % kPartSlots)) * kPartStride], t);
    }
    __syncthreads();  // s_part is free again for the next call
}

__device__ __forceinline__ uint32_t grid_tid() { return blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ uint32_t grid_threads() { return gridDim.x * blockDim.x; }

// ------------------------------------------------------------------ scan

// Exclusive scan inside one block of kBlock threads.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wsum[kBlock / 64];
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int i = 0; i < kBlock / 64; ++i) {
        if (i < w) off += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

__device__ __forceinline__ uint32_t scan_len(const uint32_t *n_dev, uint32_t n_cap) {
    if (!n_dev) return n_cap;
    const uint32_t n = *n_dev;
    return n < n_cap ? n : n_cap;
}

template <bool kPopc>
__device__ __forceinline__ uint32_t scan_in(const uint32_t *in, uint32_t i) {
    const uint32_t v = in[i];
    return kPopc ? (uint32_t)__popc(v) : v;
}

template <bool kPopc>
__global__ void __launch_bounds__(kBlock) k_scan_part(const uint32_t *in, const uint32_t *n_dev,
                                                      uint32_t n_cap, uint32_t *part) {
    const uint32_t n = scan_len(n_dev, n_cap);
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += scan_in<kPopc>(in, base + i);
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_scan_part_scan(uint32_t *part, uint32_t n_part,
                                                           const uint32_t *n_dev, uint32_t n_cap,
                                                           uint32_t *out, uint32_t *total_out) {
    const uint32_t n = scan_len(n_dev, n_cap);
    const uint32_t nb = (n + kScanTile - 1) / kScanTile;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kBlock) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = (i < nb && i < n_part) ? part[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, &tot);
        if (i < nb && i < n_part) part[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[n] = carry;
        if (total_out) *total_out = carry;
    }
}

template <bool kPopc>
__global__ void __launch_bounds__(kBlock) k_scan_apply(const uint32_t *in, const uint32_t *n_dev,
                                                       uint32_t n_cap, const uint32_t *part,
                                                       uint32_t *out) {
    const uint32_t n = scan_len(n_dev, n_cap);
    if (blockIdx.x * kScanTile >= n) return;
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? scan_in<kPopc>(in, base + i) : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, &tot) + part[blockIdx.x];
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

// out[i] = sum of in[0..i) for i <= n, n = min(*n_dev, n_cap) (n_cap if no
// n_dev); *total_out = out[n]. With kPopc the summands are popcount(in[i]).
template <bool kPopc = false>
void scan_excl(const uint32_t *in, const uint32_t *n_dev, uint32_t n_cap, uint32_t *part,
               uint32_t *out, uint32_t *total_out, hipStream_t s) {
    const uint32_t nb = n_cap / kScanTile + 1;
    k_scan_part<kPopc><<<nb, kBlock, 0, s>>>(in, n_dev, n_cap, part);
    k_scan_part_scan<<<1, kBlock, 0, s>>>(part, nb, n_dev, n_cap, out, total_out);
    k_scan_apply<kPopc><<<nb, kBlock, 0, s>>>(in, n_dev, n_cap, part, out);
}

// ------------------------------------------------------------------- bin

__global__ void __launch_bounds__(kBlock) k_zero(Counters *cnt, unsigned long long *view_seeds,
                                                 uint32_t *view_cand, uint32_t *view_ntr,
                                                 uint32_t *view_cursor, uint32_t *view_tail,
                                                 uint32_t *cell_count, uint32_t *grab,
                                                 unsigned long long *part64,
                                                 const BatchDesc *desc) {
    const uint32_t tid = grid_tid();
    const uint32_t n_views = desc->n_views, n_cells = desc->n_cells;
    if (tid == 0) {
        Counters z = {};
        *cnt = z;
    }
    for (uint32_t i = tid; i < (uint32_t)kGrabWords; i += grid_threads()) grab[i] = 0;
    for (uint32_t i = tid; i < (uint32_t)kPartWords; i += grid_threads()) part64[i] = 0;
    for (uint32_t v = tid; v < n_views; v += grid_threads()) {
        view_seeds[v] = 0;
        view_cand[v] = 0;
        view_ntr[v] = 0;
        view_cursor[v] = 0;
        view_tail[v] = 0;
    }
    for (uint32_t i = tid; i < n_cells; i += grid_threads()) cell_count[i] = 0;
}

// Bounding box of every view (grid origin) and the view index of each grain.
__global__ void __launch_bounds__(kBlock) k_bbox(const int32_t *xyz, ViewGrid *grids,
                                                 uint32_t *view_of, const BatchDesc *desc) {
    const uint32_t v = blockIdx.y;
    if (v >= desc->n_views) return;
    const uint32_t off = grids[v].grain_off, n = grids[v].n;
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
    int hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const size_t g = (size_t)off + i;
        view_of[g] = v;
        for (int m = 0; m < 3; ++m) {
            const int x = xyz[3 * g + m];
            lo[m] = min(lo[m], x);
            hi[m] = max(hi[m], x);
        }
    }
    for (int m = 0; m < 3; ++m) {
        for (int o = 32; o > 0; o >>= 1) {
            lo[m] = min(lo[m], __shfl_xor(lo[m], o));
            hi[m] = max(hi[m], __shfl_xor(hi[m], o));
        }
    }
    // one atomic per workgroup and value: atomics on the six words of a
    // view serialise in L2, so they are reduced across the waves first
    __shared__ int s_box[kBlock / 64][6];
    const int wave = threadIdx.x >> 6;
    if (lane_id() == 0)
        for (int m = 0; m < 3; ++m) {
            s_box[wave][m] = lo[m];
            s_box[wave][3 + m] = hi[m];
        }
    __syncthreads();
    if (threadIdx.x < 6 && n > 0) {
        const int m = (int)threadIdx.x;
        int b = s_box[0][m];
        for (int w = 1; w < kBlock / 64; ++w)
            b = m < 3 ? min(b, s_box[w][m]) : max(b, s_box[w][m]);
        if (m < 3)
            atomicMin(&grids[v].lo[m], b);
        else
            atomicMax(&grids[v].hi[m - 3], b);
    }
}

// Cell geometry per view: the requested edges, doubled until the grid has at
// most cell_cap cells. A view whose span exceeds the limit is marked: its
// grains still go through the binning (into one cell, so every later view
// keeps its place in the sorted arrays) but it produces no seeds.
__global__ void k_grid(ViewGrid *grids, const BatchDesc *desc, Params P) {
    const uint32_t v = grid_tid();
    if (v >= desc->n_views) return;
    ViewGrid G = grids[v];
    long long span[3];
    for (int m = 0; m < 3; ++m) {
        if (G.n == 0) {
            G.lo[m] = 0;
            G.hi[m] = 0;
        }
        span[m] = (long long)G.hi[m] - (long long)G.lo[m];
        if (span[m] > kSpanMax) G.err = 1;
    }
    // cell edges: fixed, or by the view's grain density (bounding box)
    int b = 0;
    if (P.auto_cells) {
        const double vol_um3 = (double)(span[0] + 1) * (double)(span[1] + 1) *
                               (double)(span[2] + 1) * 1e-6;
        const double per_1000 = 1000.0 * (double)G.n / vol_um3;
        double edge = kCellEdge0;
        while (b < kCellBuckets - 1 && per_1000 >= edge) {
            ++b;
            edge *= 2.0;
        }
    }
    for (int m = 0; m < 3; ++m) G.cell[m] = P.auto_cells ? P.cell_tab[b][m] : P.cell_req[m];
    if (G.err) {
        for (int m = 0; m < 3; ++m) {
            G.cell[m] = 1;
            G.dims[m] = 1;
        }
        grids[v] = G;
        return;
    }
    for (;;) {
        long long tot = 1;
        for (int m = 0; m < 3; ++m) {
            G.dims[m] = (int)(span[m] / G.cell[m] + 1);
            tot *= G.dims[m];
        }
        if (tot <= (long long)G.cell_cap) break;
        for (int m = 0; m < 3; ++m) G.cell[m] *= 2;
    }
    grids[v] = G;
}

__device__ __forceinline__ int axis_cell(const ViewGrid &G, int m, int x) {
    const long long c = ((long long)x - (long long)G.lo[m]) / G.cell[m];
    return (int)(c < 0 ? 0 : (c >= G.dims[m] ? G.dims[m] - 1 : c));
}

__device__ __forceinline__ uint32_t cell_index(const ViewGrid &G, int x, int y, int z) {
    const int cx = axis_cell(G, 0, x), cy = axis_cell(G, 1, y), cz = axis_cell(G, 2, z);
    return G.cell_off + (uint32_t)((cz * G.dims[1] + cy) * G.dims[0] + cx);
}

__global__ void __launch_bounds__(kBlock) k_hist(const int32_t *xyz, const ViewGrid *grids,
                                                 uint32_t *cell_of, uint32_t *rank,
                                                 uint32_t *cell_count, const BatchDesc *desc) {
    const uint32_t v = blockIdx.y;
    if (v >= desc->n_views) return;
    const ViewGrid G = grids[v];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < G.n; i += gridDim.x * blockDim.x) {
        const size_t g = (size_t)G.grain_off + i;
        const uint32_t c = cell_index(G, xyz[3 * g], xyz[3 * g + 1], xyz[3 * g + 2]);
        cell_of[g] = c;
        rank[g] = atomicAdd(&cell_count[c], 1u);
    }
}

// Sorted grains: coordinates relative to the view origin (0 .. 2^18) and
// the input index within the view.
__global__ void __launch_bounds__(kBlock) k_scatter(const int32_t *xyz, const ViewGrid *grids,
                                                    const uint32_t *cell_of, const uint32_t *rank,
                                                    const uint32_t *cell_start, int4 *sg,
                                                    float4 *sgf, const BatchDesc *desc) {
    const uint32_t v = blockIdx.y;
    if (v >= desc->n_views) return;
    const ViewGrid G = grids[v];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < G.n; i += gridDim.x * blockDim.x) {
        const size_t g = (size_t)G.grain_off + i;
        const uint32_t pos = cell_start[cell_of[g]] + rank[g];
        const int x = xyz[3 * g] - G.lo[0], y = xyz[3 * g + 1] - G.lo[1], z = xyz[3 * g + 2] - G.lo[2];
        sg[pos] = make_int4(x, y, z, (int)i);
        sgf[pos] = make_float4((float)x, (float)y, (float)z, 0.0f);
    }
}

// ------------------------------------------------------------ line walk
//
// Which cells can hold a grain within r of the infinite line p(t) = g + t d?
// If |k - p(t*)| <= r then |k_m - p_m(t*)| <= r on every axis. Cells along x
// are contiguous in memory, so the walk enumerates (y, z) pencils: for each
// (y, z) cell that the projected line, widened by r on each axis, crosses,
// it takes the parameter interval during which p_y and p_z stay within r of
// that cell, and the x range p_x covers on it, widened by r. That x range is
// one contiguous run of sorted grains. The traversal steps along the larger
// of |d_y|, |d_z| (axis e), and for each e cell across the f cells the line
// can reach. FP32 values only choose cells: every bound is widened by
// kMargin units, more than the rounding of any coordinate below 2^20, and
// the exact integer predicate decides each grain.
struct Run {
    uint32_t k, e;
};

struct Pencil {
    // Per line, precomputed so a pencil costs few instructions: the line is
    // oriented so that x grows with t; e and f cell intervals in t are stored
    // low end first; x and f are kept in cell units (t * ds + gs) with the
    // widening folded in; rows advance by fixed strides.
    float tlo, thi;                  // t range within rr of the grid box
    float ue_lo0, ue_step, ue_w;     // e cell j: t in [ue_lo0 + j ue_step, + ue_w]
    float uf_lo0, uf_step, uf_w;     // f cell j likewise
    float dfs, gfs, rrf, fnf;        // f in cell units, its widening, nf
    float dxs, gxs_lo, gxs_hi, fnx;  // x in cell units minus / plus widening, nx
    int nx, nf, ie1;
    uint32_t off, se, sf;            // view's first cell, row strides of e and f
    // walk state: e cell ie of [.., ie1], f cells [jf, jf1] of it
    int ie, jf, jf1;
    uint32_t row_e;                  // off + ie * se
    float ta, tb;
    bool live;

    // part/nparts: this lane walks the part-th of nparts equal slices of the
    // e cells, so that several lanes can share one long line. No divisions:
    // reciprocals (within 1 ulp) are covered by the kMargin widening.
    // ext >= 0: a finite cylinder, whose grains project at most ext units
    // beyond the seed grains; the walk then covers only that stretch.
    __device__ __forceinline__ void init(const ViewGrid *__restrict__ Gp, int4 g, int idx, int idy,
                                         int idz, int r, bool valid, int part, int nparts,
                                         int ext = -1) {
        nx = Gp->dims[0];
        const int ny = Gp->dims[1];
        const int nz = Gp->dims[2];
        const int cxi = Gp->cell[0], cyi = Gp->cell[1], czi = Gp->cell[2];
        off = Gp->cell_off;
        const float rr = (float)r + kMargin;
        // the line is undirected: take the direction with d_x >= 0
        const bool flipped = idx < 0;
        if (idx < 0) {
            idx = -idx;
            idy = -idy;
            idz = -idz;
        }
        const float icx = __builtin_amdgcn_rcpf((float)cxi);
        const float gx = (float)g.x, dx = (float)idx;
        const float gy = (float)g.y, gz = (float)g.z, dy = (float)idy, dz = (float)idz;
        const float ix = idx ? __builtin_amdgcn_rcpf(dx) : 0.0f;
        const float iy = idy ? __builtin_amdgcn_rcpf(dy) : 0.0f;
        const float iz = idz ? __builtin_amdgcn_rcpf(dz) : 0.0f;
        // parameter range in which the line is within rr of the grid box
        constexpr float kBig = 1.0e38f;
        float t1, t2;
        tlo = -kBig;
        thi = kBig;
        if (idx) {
            t1 = (-rr - gx) * ix;
            t2 = ((float)(nx * cxi - 1) + rr - gx) * ix;
            tlo = fmaxf(tlo, fminf(t1, t2));
            thi = fminf(thi, fmaxf(t1, t2));
        }
        if (idy) {
            t1 = (-rr - gy) * iy;
            t2 = ((float)(ny * cyi - 1) + rr - gy) * iy;
            tlo = fmaxf(tlo, fminf(t1, t2));
            thi = fminf(thi, fmaxf(t1, t2));
        }
        if (idz) {
            t1 = (-rr - gz) * iz;
            t2 = ((float)(nz * czi - 1) + rr - gz) * iz;
            tlo = fmaxf(tlo, fminf(t1, t2));
            thi = fminf(thi, fmaxf(t1, t2));
        }
        if (ext >= 0) {
            // the seed grains sit at t = 0 and t = 1 (t = -1 once flipped);
            // grains of the cylinder project within (ext + rr) / |d| beyond
            // them (widened for the approximate reciprocal square root)
            const float reach = ((float)ext + rr) * 1.001f *
                                __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
            const float s0 = flipped ? -1.0f : 0.0f;
            tlo = fmaxf(tlo, s0 - reach);
            thi = fminf(thi, s0 + 1.0f + reach);
        }
        const bool e_is_y = abs(idy) >= abs(idz);
        const float ge = e_is_y ? gy : gz;
        const float de = e_is_y ? dy : dz;
        const float ie_ = e_is_y ? iy : iz;
        const float ce = (float)(e_is_y ? cyi : czi);
        const int ne = e_is_y ? ny : nz;
        const float gf = e_is_y ? gz : gy;
        const float df = e_is_y ? dz : dy;
        const float if_ = e_is_y ? iz : iy;
        const float cf = (float)(e_is_y ? czi : cyi);
        nf = e_is_y ? nz : ny;
        se = e_is_y ? (uint32_t)nx : (uint32_t)(nx * ny);
        sf = e_is_y ? (uint32_t)(nx * ny) : (uint32_t)nx;
        const float ice = __builtin_amdgcn_rcpf(ce);
        const float icf = __builtin_amdgcn_rcpf(cf);
        // cell j of an axis with direction d != 0 is met for parameters
        // between (j c - rr - g)/d and ((j+1) c - 1 + rr - g)/d, the first
        // the lower one when d > 0; with d == 0 every visited cell is met for
        // all parameters
        if (de != 0.0f) {
            const float a0 = (-rr - ge) * ie_, w = (ce - 1.0f + 2.0f * rr) * ie_;
            ue_step = ce * ie_;
            ue_lo0 = de > 0.0f ? a0 : a0 + w;
            ue_w = fabsf(w);
        } else {
            ue_lo0 = -kBig;
            ue_step = 0.0f;
            ue_w = 2.0f * kBig;
        }
        if (df != 0.0f) {
            const float a0 = (-rr - gf) * if_, w = (cf - 1.0f + 2.0f * rr) * if_;
            uf_step = cf * if_;
            uf_lo0 = df > 0.0f ? a0 : a0 + w;
            uf_w = fabsf(w);
        } else {
            uf_lo0 = -kBig;
            uf_step = 0.0f;
            uf_w = 2.0f * kBig;
        }
        dfs = df * icf;
        gfs = gf * icf;
        rrf = rr * icf;
        fnf = (float)nf;
        dxs = dx * icx;
        gxs_lo = (gx - rr) * icx;
        gxs_hi = (gx + rr) * icx;
        fnx = (float)nx;
        // e cells the widened projection touches
        const float ea = ge + tlo * de, eb = ge + thi * de;
        const float elo = (de != 0.0f ? fminf(ea, eb) : ge) - rr;
        const float ehi = (de != 0.0f ? fmaxf(ea, eb) : ge) + rr;
        int ie0 = max(0, (int)floorf(fmaxf(elo * ice, -1.0f)));
        ie1 = min(ne - 1, (int)floorf(fminf(ehi * ice, (float)ne)));
        if (nparts > 1 && ie0 <= ie1) {
            const int len = ie1 - ie0 + 1, per = (len + nparts - 1) / nparts;
            const int a0 = ie0 + part * per;
            ie1 = min(ie1, a0 + per - 1);
            ie0 = a0;
        }
        ie = ie0 - 1;
        jf = 1;
        jf1 = 0;
        row_e = 0;
        ta = tb = 0.0f;
        live = valid && ie0 <= ie1 && tlo <= thi;
    }

    // One move of the walk, straight-line: step to the next e cell when the
    // current one is used up, then take the next f cell of it. Fills out
    // with that pencil's run or an empty run; the two cell_start loads are
    // issued but not waited on. Truncation is the floor for lower bounds
    // (clamped at 0); for upper ones it can only add a cell, which costs
    // tests, not results.
    __device__ __forceinline__ void fetch(const uint32_t *__restrict__ cs, Run &out) {
        // set-up of e cell ie + 1, taken if the current one is used up
        const bool step_e = jf > jf1;
        const int ien = ie + 1;
        const float elo = fmaf((float)ien, ue_step, ue_lo0);
        const float tan_ = fmaxf(tlo, elo), tbn = fminf(thi, elo + ue_w);
        const float fa = fmaf(tan_, dfs, gfs), fb = fmaf(tbn, dfs, gfs);
        const int jf0n = (int)fmaxf(fminf(fa, fb) - rrf, 0.0f);
        const int jf1n = min(nf - 1, (int)fmaxf(fminf(fmaxf(fa, fb) + rrf, fnf), -1.0f));
        if (step_e) {
            ie = ien;
            ta = tan_;
            tb = tbn;
            jf = tan_ <= tbn ? jf0n : 1;
            jf1 = tan_ <= tbn ? jf1n : 0;
            row_e = off + (uint32_t)ien * se;
        }
        live = live && ie <= ie1;
        const int j = jf;
        const float flo = fmaf((float)j, uf_step, uf_lo0);
        const float tc = fmaxf(ta, flo), td = fminf(tb, flo + uf_w);
        // x grows with t, so [tc, td] maps to [x(tc), x(td)]
        const int x0 = (int)fmaxf(fmaf(tc, dxs, gxs_lo), 0.0f);
        const int x1 = min(nx - 1, (int)fmaxf(fminf(fmaf(td, dxs, gxs_hi), fnx), -1.0f));
        const bool ok = live && j <= jf1 && tc <= td && x0 <= x1;
        jf = j + 1;
        const uint32_t row = row_e + (uint32_t)j * sf;
        // 32-bit byte offsets from the table base (the table is far below
        // 4 GB), so the loads take a scalar base and one vector offset
        const char *base = reinterpret_cast<const char *>(cs);
        const uint32_t b0 = (row + (uint32_t)x0) * 4u, b1 = (row + (uint32_t)x1 + 1u) * 4u;
        out.k = ok ? *reinterpret_cast<const uint32_t *>(base + b0) : 0u;
        out.e = ok ? *reinterpret_cast<const uint32_t *>(base + b1) : 0u;
    }
};

// Acceptance variants.
//
// Finite cylinder: grain k also needs t = g_k.d in [lo, hi], lo = g_i.d - F,
// hi = g_i.d + |d|^2 + F, F = floor(cyl_ext |d|) = isqrt(cyl_ext^2 |d|^2):
// t is an integer, so t - g_i.d >= -cyl_ext |d| iff t >= g_i.d - F, and
// likewise above. Coordinates are in [0, 2^18] and |d| < 2^12, so |t| < 2^31
// and the 24-bit products are exact; the bounds are clamped to int32.
__device__ __forceinline__ int2 axial_bounds(int4 gi, int dx, int dy, int dz, int ext) {
    const long long D = (long long)dx * dx + (long long)dy * dy + (long long)dz * dz;
    const long long e2D = (long long)ext * ext * D;  // < 2^59
    long long F = (long long)sqrt((double)e2D);
    while (F > 0 && F * F > e2D) --F;
    while ((F + 1) * (F + 1) <= e2D) ++F;
    const long long gd = (long long)gi.x * dx + (long long)gi.y * dy + (long long)gi.z * dz;
    const long long lo = gd - F, hi = gd + D + F;
    return make_int2((int)max(lo, -2147483647ll - 1), (int)min(hi, 2147483647ll));
}

__device__ __forceinline__ bool axial_ok(int4 h, int4 A, int2 b) {
    const int t = __mul24(h.x, A.x) + __mul24(h.y, A.y) + __mul24(h.z, A.z);
    return t >= b.x && t <= b.y;
}

// Grain-count threshold of a seed with direction d: n_min + ceil(b tan(theta)),
// b = thr_num / thr_den, tan(theta) = sqrt(dx^2 + dy^2) / |dz|, capped at
// thr_max when set; dz = 0 needs the cap (no cap: unreachable). The ceiling
// m = ceil(sqrt(Q) / K), Q = thr_num^2 (dx^2 + dy^2), K = thr_den |dz|, is the
// smallest m >= 0 with (m K)^2 >= Q: a double estimate, corrected with exact
// integer squares (m K < 2^23).
__device__ __forceinline__ uint32_t seed_threshold(int dx, int dy, int dz, const Params &P) {
    if (P.thr_num == 0) return (uint32_t)P.n_min;
    const uint32_t cap = P.thr_max > 0 ? (uint32_t)P.thr_max : 0xffffffffu;
    const long long K = (long long)P.thr_den * (dz < 0 ? -dz : dz);
    if (K == 0) return cap;
    const long long Q =
        (long long)P.thr_num * P.thr_num * ((long long)dx * dx + (long long)dy * dy);
    long long m = (long long)ceil(sqrt((double)Q) / (double)K);
    while (m > 0 && (m - 1) * K * (m - 1) * K >= Q) --m;
    while (m * K * m * K < Q) ++m;
    const long long t = (long long)P.n_min + m;
    return t < (long long)cap ? (uint32_t)t : cap;
}

// Next grab of items for the calling wave: its own
// XCD's range first, then the others. grab[16 x] is range x's offset
// counter. Grabs are a quarter of a range's remainder per wave of the XCD,
// within [gmin, gmax] and a multiple of gmin. Returns false when every
// range is used up. Wave-uniform.
__device__ __forceinline__ bool xcd_grab(uint32_t *grab, uint32_t xcd, uint32_t per,
                                         uint32_t n_items, uint32_t wpx, uint32_t gmin,
                                         uint32_t gmax, uint32_t &next, uint32_t &end) {
    uint32_t s = 0xffffffffu, e = 0;
    if (lane_id() == 0) {
        for (uint32_t t = 0; t < 8; ++t) {
            const uint32_t x = (xcd + t) & 7u;
            const uint32_t lo = min(n_items, x * per), hi = min(n_items, x * per + per);
            uint32_t *ctr = grab + 16 * x;
            const uint32_t cur = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cur >= hi - lo) continue;
            uint32_t g = (hi - lo - cur) / (4u * wpx);
            g = min(gmax, max(gmin, (g + gmin - 1u) / gmin * gmin));
            const uint32_t at = atomicAdd(ctr, g);
            if (at >= hi - lo) continue;
            s = lo + at;
            e = min(hi, s + g);
            break;
        }
    }
    next = (uint32_t)__shfl((int)s, 0);
    end = (uint32_t)__shfl((int)e, 0);
    return next != 0xffffffffu;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum over the 64 lanes with DPP row shifts and row
// broadcasts (no LDS traffic).
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t x) {
    uint32_t v = x;
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// ----------------------------------------------------------------- seeds
//
// One wave per anchor grain p (a sorted position); lanes take the (y, z)
// rows of the cell box overlapping [g_p - (R-1), g_p + (R-1)]. Every grain q
// of those rows at a higher sorted position with 0 < |g_q - g_p|^2 < R^2
// makes a seed, stored with the lower input index first. A first pass counts
// the seeds of every anchor, a scan turns the counts into offsets, and a
// second pass writes them: no shared counter, and the seed list comes out in
// anchor order, so each view's seeds are contiguous.
template <bool kWrite>
__global__ void __launch_bounds__(kBlock) k_seeds(DevPtrs d, Caps c, Params P) {
    // per wave: the first flat element of each row, and sorted position
    // minus that (so that grain = dk[r] + element)
    __shared__ uint32_t s_rows[kBlock / 64][2][64];
    const int lane = lane_id();
    const uint32_t gw = grid_tid() >> 6, nw = grid_threads() >> 6;
    const int R1 = P.R - 1;
    const int R2 = P.R * P.R;
    const uint32_t n_total = d.desc->n_total;
    // the write pass has nothing to do when the seeds overflow their buffer
    if (kWrite && d.cnt->n_seeds_ok == 0) return;
    if constexpr (kWrite) {
        // the candidate bit mask starts clear; the counting kernel sets the
        // bits of the seeds that reach their threshold
        const uint32_t nwd = d.cnt->pass_words;
        for (uint32_t w = grid_tid(); w < nwd; w += grid_threads()) d.pass[w] = 0u;
    }
    unsigned long long wave_total = 0;  // count pass: seeds of this wave's anchors
    for (uint32_t p = gw; p < n_total; p += nw) {
        const uint32_t v = d.view_of[p];
        const ViewGrid *G = &d.grids[v];
        uint32_t base = kWrite ? d.seed_off[p] : 0u;
        uint32_t mine = 0;
        if (!G->err) {
            const int nx = G->dims[0], ny = G->dims[1], nz = G->dims[2];
            const int cx = G->cell[0], cy = G->cell[1], cz = G->cell[2];
            const uint32_t off = G->cell_off;
            const int4 g = d.sg[p];
            const int x0 = g.x - R1 < 0 ? 0 : (g.x - R1) / cx;
            const int y0 = g.y - R1 < 0 ? 0 : (g.y - R1) / cy;
            const int z0 = g.z - R1 < 0 ? 0 : (g.z - R1) / cz;
            const int x1 = min(nx - 1, (g.x + R1) / cx);
            const int y1 = min(ny - 1, (g.y + R1) / cy);
            const int z1 = min(nz - 1, (g.z + R1) / cz);
            // each unordered pair once, from the grain with the lower sorted
            // position: rows of the box that sort before the anchor's own row
            // hold only lower positions, and in its row the scan starts past it
            const int yp = min(ny - 1, g.y / cy), zp = min(nz - 1, g.z / cz);
            const int nyr = y1 - y0 + 1;
            const int nrows = nyr * (z1 - z0 + 1);
            const int row_p = (zp - z0) * nyr + (yp - y0);
            // the rows' grains are taken as one flat range: lane L tests
            // elements b + L and b + 64 + L of each trip, each found in row
            // r, the last row whose first element is at or below it (a
            // binary search over the rows' starts in LDS), so every lane has
            // grains whatever the row lengths
            uint32_t *ex_s = s_rows[threadIdx.x >> 6][0];
            uint32_t *dk_s = s_rows[threadIdx.x >> 6][1];
            for (int rb = row_p; rb < nrows; rb += 64) {
                const int rr = rb + lane;
                uint32_t k0 = 0, k1 = 0;
                if (rr < nrows) {
                    const int y = y0 + rr % nyr, z = z0 + rr / nyr;
                    const uint32_t row = off + (uint32_t)((z * ny + y) * nx);
                    k0 = max(d.cell_start[row + x0], p + 1);
                    k1 = d.cell_start[row + x1 + 1];
                }
                const uint32_t len = k1 > k0 ? k1 - k0 : 0u;
                const uint32_t incl = wave_incl_scan_dpp(len);
                const uint32_t T = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
                wave_lds_sync();  // the previous block's readers are done
                ex_s[lane] = incl - len;
                dk_s[lane] = k0 - (incl - len);
                wave_lds_sync();
                // the grain of flat element i (the anchor itself past the end)
                auto grain_of = [&](uint32_t i) -> uint32_t {
                    uint32_t r = 0;
#pragma unroll
                    for (uint32_t step = 32; step > 0; step >>= 1)
                        r = ex_s[r + step] <= i ? r + step : r;
                    return i < T ? dk_s[r] + i : p;
                };
                auto pairs = [&](const int4 &h, bool ok) {
                    const int ex = h.x - g.x, ey = h.y - g.y, ez = h.z - g.z;
                    ok = ok && abs(ex) <= R1 && abs(ey) <= R1 && abs(ez) <= R1;
                    const int D = ok ? ex * ex + ey * ey + ez * ez : 0;
                    return ok && D > 0 && D < R2;
                };
                auto write = [&](bool ok, const int4 &h, uint32_t q) {
                    const unsigned long long m = __ballot(ok);
                    if (ok) {
                        const unsigned long long slot =
                            (unsigned long long)base + (unsigned long long)__popcll(m & lanes_below());
                        // stored lower input index first: that grain is the
                        // seed's i (the fit's origin and key order)
                        if (slot < c.seed_cap)
                            d.seeds[slot] = h.w > g.w ? make_uint2(p, q) : make_uint2(q, p);
                    }
                    base += (uint32_t)__popcll(m);
                };
                // two elements a lane per trip: their row searches and grain
                // loads are in flight together
                for (uint32_t b = 0; b < T; b += 128) {
                    const uint32_t i0 = b + (uint32_t)lane, i1 = i0 + 64;
                    const uint32_t q0 = grain_of(i0), q1 = grain_of(i1);
                    const int4 h0 = d.sg[q0], h1 = d.sg[q1];
                    const bool ok0 = pairs(h0, i0 < T), ok1 = pairs(h1, i1 < T);
                    if (kWrite) {
                        write(ok0, h0, q0);
                        write(ok1, h1, q1);
                    } else {
                        mine += (ok0 ? 1u : 0u) + (ok1 ? 1u : 0u);
                    }
                }
            }
        }
        if (!kWrite) {
            mine = wave_sum(mine);
            if (lane == 0) d.seed_cnt[p] = mine;
            wave_total += mine;
        }
    }
    if constexpr (!kWrite) add_spread(d.part64, 0, wave_total);
}

// The seed total of the uint32 scan, replaced by the exact 64-bit count
// (saturated to 2^32 - 1), and the number of seeds the later stages take:
// none when they do not fit the seed buffer (the host then re-runs the call
// with a larger one, or fails if no buffer can hold them).
__global__ void k_seed_total(Counters *cnt, const unsigned long long *part64,
                             unsigned long long seed_cap) {
    // one wave: the spread partial sums (kPartSlots == 64, one per lane)
    const unsigned long long s = wave_sum(part64[lane_id() * kPartStride]);
    if (threadIdx.x != 0) return;
    cnt->seeds64 = s;
    const uint32_t n = s > 0xffffffffull ? 0xffffffffu : (uint32_t)s;
    cnt->n_seeds = n;
    cnt->n_seeds_ok = n <= seed_cap ? n : 0u;
    cnt->pass_words = (uint32_t)(((unsigned long long)cnt->n_seeds_ok + 31ull) / 32ull);
}

// Likewise for the member entries (the scan of candidate counts): a total
// that wrapped reads as an overflow, so no stage uses the wrapped offsets.
__global__ void k_member_total(Counters *cnt, const unsigned long long *part64) {
    const unsigned long long m = wave_sum(part64[(kPartSlots + lane_id()) * kPartStride]);
    // the counting kernel's tests and hits, summed here (it has finished)
    const unsigned long long t = wave_sum(part64[(2 * kPartSlots + lane_id()) * kPartStride]);
    const unsigned long long h = wave_sum(part64[(3 * kPartSlots + lane_id()) * kPartStride]);
    if (threadIdx.x != 0) return;
    cnt->tests = t;
    cnt->hits = h;
    cnt->members64 = m;
    cnt->n_members = m > 0xffffffffull ? 0xffffffffu : (uint32_t)m;
}


// ------------------------------------------------------- count / members

constexpr int kWaves = kBlock / 64;

// Counting with lane refill (one kernel counts the seeds and, as a second
// instance, lists the members of the candidates). A wave owns a chunk of
// seeds; each lane holds
// two seed slots in LDS. When a lane's walk ends it closes that slot and at
// once takes the next seed of the chunk into its other slot, so the wave's
// time is the sum of its lines' work rather than a multiple of the longest
// one. Hit counts of a closed slot are final after the next queue flush,
// which writes them out and frees the slot.
//
// The queue holds pieces: each run a lane queues is cut into pieces of at
// most kPiece consecutive grains, and the flush gives every lane one piece.
// The lane maps its piece to the run by one popcount, reads the seed's line
// constants once, issues the loads of all kPiece grains together and tests
// them against the one line, so the mapping and the line constants are paid
// once per piece and the grain loads of a piece are in flight together.
constexpr int kCountSlots = 128;
constexpr int kPiece = EMT_COUNT_PIECE;             // grains per queued piece
constexpr int kPieceCap = EMT_COUNT_PIECE_CAP;      // queued pieces per wave
constexpr int kLanePieces = EMT_COUNT_LANE_PIECES;  // pieces a lane queues per step
constexpr int kCountRunCap = EMT_COUNT_RUN_CAP;     // queued runs per wave
constexpr int kPieceWords = kPieceCap / 64;
constexpr int kChunkSeeds = EMT_CHUNK_SEEDS;
constexpr int kFetch = EMT_COUNT_FETCH;  // pencils a lane fetches per step
constexpr int kRefillMin = EMT_COUNT_REFILL;  // waiting lanes that start a refill
constexpr int kFlushUnroll = EMT_FLUSH_UNROLL;  // queue words a flush trip loads together
static_assert(kFlushUnroll >= 1 && kFlushUnroll <= 4, "flush unroll");
static_assert(64 * kFetch <= kCountRunCap, "a step's runs must fit the run queue");
static_assert(kRefillMin >= 1 && kRefillMin <= 64, "refill threshold is a lane count");
static_assert(64 * kLanePieces <= kPieceCap, "a step's pieces must fit the queue");
static_assert(kPieceWords <= 64 && kPieceCap % 64 == 0, "one mask word per lane");
static_assert(kPieceCap <= 4096 && kPiece * kLanePieces < 8192, "run record fields");
static_assert(kPiece >= 1 && (uint32_t)kPiece - 1u <= kSortedSpare, "piece size");

template <bool kFinite, bool kEmit = false>
struct CountLds {
    // line constants per seed slot (floats): d, -(g_i x d), the band
    // [tlo, thi] of the FP32 test, and the sorted position of g_i
    float4 la[kCountSlots];  // dx, dy, dz, tlo
    float4 lc[kCountSlots];  // -ex, -ey, -ez, thi
    uint32_t lp[kCountSlots];  // sorted position of g_i (the int64 test)
    int2 pc[kFinite ? kCountSlots : 1];  // finite cylinder: bounds of g_k.d
    uint32_t cnt[kCountSlots];
    // listing the members of candidates: where a slot's grains go, and how
    // many its list holds (its count)
    uint32_t out_off[kEmit ? kCountSlots : 1];
    uint32_t ncap[kEmit ? kCountSlots : 1];
    unsigned long long mask[kPieceWords];  // bit s: a run starts at piece s
    uint32_t before[kPieceWords];          // runs starting before word w
    uint2 run[kCountRunCap];  // first grain; first piece | seed slot << 12 | grains << 19
};

// The counting test in FP32, decided exactly. With coordinates in [0, 2^18]
// (exact floats) and |d| < 2^12, c = g_k x d - g_i x d is formed by two
// fused multiply-adds a component from d, -d and the rounded -(g_i x d).
// Each rounding is at most 2^-24 of a magnitude below 2^18 (1 + sqrt 2)|d|,
// so each component is within 0.06 |d| of the exact one and |c| within
// 0.104 |d|. A grain is certainly inside when the FP32 |c|^2 is at most
// tlo = (r - 1/8)^2 |d|^2 and certainly outside above thi = (r + 1/8)^2
// |d|^2, both widened by 2^-20 (tlo < 0 when r = 0); in between the test is
// redone in int64. The widening covers the rounding of the FP32 sum of
// squares (within 5 * 2^-24 relative) and of the FP32 products forming tlo
// and thi (|d|^2 < 2^26 rounded, a square, two products: within 4 * 2^-24).
__device__ __forceinline__ void line_consts(int4 gi, int dx, int dy, int dz, int r, float4 &A,
                                            float4 &C) {
    const float Df = (float)(dx * dx + dy * dy + dz * dz);  // |d| < 2^12: exact in int32
    const float rlo = (float)r - 0.125f, rhi = (float)r + 0.125f;  // exact
    const float tlo = r > 0 ? rlo * rlo * Df * (1.0f - 0x1p-20f) : -1.0f;
    const float thi = rhi * rhi * Df * (1.0f + 0x1p-20f);
    const long long ex = (long long)gi.y * dz - (long long)gi.z * dy;
    const long long ey = (long long)gi.z * dx - (long long)gi.x * dz;
    const long long ez = (long long)gi.x * dy - (long long)gi.y * dx;
    A = make_float4((float)dx, (float)dy, (float)dz, tlo);
    C = make_float4((float)-ex, (float)-ey, (float)-ez, thi);
}

// One queued piece for a flush lane: its run's grains k0 .. k0 + m - 1, the
// seed slot, the slot's line constants and the piece's grains, all loads
// issued and none waited on.
struct Piece {
    uint32_t k0, m, sl;
    float4 A, C;
    float4 h[kPiece];
};

// Loads piece (w, lane) of a queue holding qn pieces. A lane past the end
// (or past word nw - 1) reads run 0 and tests nothing (m = 0): every read
// stays inside the queue and the sorted grains, which carry kPiece - 1 spare
// entries past the last one.
template <bool kFinite, bool kEmit>
__device__ __forceinline__ void piece_load(const CountLds<kFinite, kEmit> &Q, uint32_t w, uint32_t nw,
                                           uint32_t qn, unsigned long long upto, int lane,
                                           const float4 *__restrict__ sgf, Piece &p) {
    const uint32_t wc = min(w, nw - 1u);
    const uint32_t s = (w << 6) + (uint32_t)lane;
    const bool valid = w < nw && s < qn;
    const unsigned long long word = Q.mask[wc];
    const uint32_t r = valid ? Q.before[wc] + (uint32_t)__popcll(word & upto) - 1u : 0u;
    const uint2 rec = Q.run[r];
    const uint32_t q = valid ? s - (rec.y & 0xfffu) : 0u;  // piece of the run
    p.sl = (rec.y >> 12) & 0x7fu;
    p.k0 = rec.x + (uint32_t)kPiece * q;
    p.m = valid ? min((rec.y >> 19) - (uint32_t)kPiece * q, (uint32_t)kPiece) : 0u;
    p.A = Q.la[p.sl];
    p.C = Q.lc[p.sl];
    const float4 *pp = sgf + p.k0;
#pragma unroll
    for (int t = 0; t < kPiece; ++t) p.h[t] = pp[t];
}

// The piece's hits as a bit mask over its grains: the FP32 test, the rare
// band case in int64.
template <bool kFinite, bool kEmit>
__device__ __forceinline__ uint32_t piece_test(const CountLds<kFinite, kEmit> &Q, const Piece &p,
                                               int tol_r, const int4 *__restrict__ sg) {
    uint32_t n = 0, amb = 0;
#pragma unroll
    for (int t = 0; t < kPiece; ++t) {
        const float4 &h = p.h[t];
        const float c0 = fmaf(h.y, p.A.z, fmaf(h.z, -p.A.y, p.C.x));
        const float c1 = fmaf(h.z, p.A.x, fmaf(h.x, -p.A.z, p.C.y));
        const float c2 = fmaf(h.x, p.A.y, fmaf(h.y, -p.A.x, p.C.z));
        const float fc = fmaf(c0, c0, fmaf(c1, c1, c2 * c2));
        bool ok = (uint32_t)t < p.m;
        if constexpr (kFinite) {
            const int4 hi = make_int4((int)h.x, (int)h.y, (int)h.z, 0);
            const int4 Ai = make_int4((int)p.A.x, (int)p.A.y, (int)p.A.z, 0);
            ok = ok && axial_ok(hi, Ai, Q.pc[p.sl]);
        }
        const bool in_lo = fc <= p.A.w, in_hi = fc <= p.C.w;
        n |= (ok && in_lo) ? (1u << t) : 0u;
        amb |= (ok && in_hi && !in_lo) ? (1u << t) : 0u;
    }
    if (amb) {
        // inside the band: decide in int64 from the integer grains (rare)
        const int dx = (int)p.A.x, dy = (int)p.A.y, dz = (int)p.A.z;
        const long long D = (long long)dx * dx + (long long)dy * dy + (long long)dz * dz;
        const long long thr = (long long)tol_r * tol_r * D;
        const int4 gi = sg[Q.lp[p.sl]];
#pragma unroll
        for (int t = 0; t < kPiece; ++t) {
            if (amb & (1u << t)) {
                const int4 g = sg[p.k0 + (uint32_t)t];
                const long long wx = g.x - gi.x, wy = g.y - gi.y, wz = g.z - gi.z;
                const long long e0 = wy * dz - wz * dy, e1 = wz * dx - wx * dz,
                                e2 = wx * dy - wy * dx;
                n |= e0 * e0 + e1 * e1 + e2 * e2 <= thr ? (1u << t) : 0u;
            }
        }
    }
    return n;
}

// Tests every queued piece, kFlushUnroll queue words per trip: the loads of
// all of a trip's pieces are issued before any is tested, so a lane has
// several chains of LDS and grain loads in flight instead of one.
// Counting adds a piece's hits to its seed's count with one LDS atomic;
// listing (kEmit) takes as many positions in the candidate's member list and
// writes the hit grains' sorted positions there (in any order: the merge
// treats a list as a set and the fit orders it).
template <bool kFinite, bool kEmit>
__device__ __forceinline__ void count_flush(CountLds<kFinite, kEmit> &Q, uint32_t qn, int tol_r,
                                            const int4 *__restrict__ sg,
                                            const float4 *__restrict__ sgf,
                                            uint32_t *__restrict__ members, int lane) {
    wave_lds_sync();
    const uint32_t nw = (qn + 63) >> 6;
    {
        const uint32_t c = (uint32_t)lane < nw ? (uint32_t)__popcll(Q.mask[lane]) : 0u;
        const uint32_t incl = wave_incl_scan_dpp(c);
        if ((uint32_t)lane < nw) Q.before[lane] = incl - c;
    }
    wave_lds_sync();
    const unsigned long long upto = (2ull << lane) - 1ull;
    for (uint32_t w = 0; w < nw; w += kFlushUnroll) {
        Piece p[kFlushUnroll];
#pragma unroll
        for (int u = 0; u < kFlushUnroll; ++u)
            piece_load(Q, w + (uint32_t)u, nw, qn, upto, lane, sgf, p[u]);
#pragma unroll
        for (int u = 0; u < kFlushUnroll; ++u) {
            const uint32_t bits = piece_test(Q, p[u], tol_r, sg);
            if (bits) {
                const uint32_t n = (uint32_t)__popc(bits);
                const uint32_t at = atomicAdd(&Q.cnt[p[u].sl], n);
                if constexpr (kEmit) {
                    const uint32_t cap = Q.ncap[p[u].sl], base = Q.out_off[p[u].sl];
                    uint32_t pos = at;
#pragma unroll
                    for (int t = 0; t < kPiece; ++t) {
                        if (bits & (1u << t)) {
                            if (pos < cap) members[base + pos] = p[u].k0 + (uint32_t)t;
                            ++pos;
                        }
                    }
                }
            }
        }
    }
    wave_lds_sync();
    if ((uint32_t)lane < nw) Q.mask[lane] = 0ull;
    wave_lds_sync();
}

// Waves per SIMD the counting kernel is compiled for: its test phase waits
// on grain loads, so more resident waves hide more of that latency (the
// compiler then keeps the kernel within 512 / kCountOccupancy VGPRs).
constexpr int kCountOccupancy = EMT_COUNT_OCCUPANCY;

// kEmit: the members stage. The same walk and test over the candidates
// instead of the seeds, listing each candidate's grains (its count is known:
// the list must come out exactly that long).
template <bool kFinite, bool kEmit>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kCountOccupancy)))
k_count(DevPtrs d, Caps c, Params P) {
    __shared__ CountLds<kFinite, kEmit> sQ[kWaves];
    const int lane = lane_id();
    CountLds<kFinite, kEmit> &Q = sQ[threadIdx.x >> 6];
    uint32_t n_items = d.cnt->n_seeds_ok;
    if constexpr (kEmit) {
        // nothing to list when the entries overflow their buffer (the call
        // is re-run)
        const bool skip = d.cnt->err || d.cnt->n_members > c.mem_cap;
        n_items = skip ? 0u : min(d.cnt->n_cand, c.cand_cap);
    }
    if (lane < kPieceWords) Q.mask[lane] = 0ull;
    wave_lds_sync();
    unsigned long long tests = 0, hits = 0;
    // Which seeds a wave counts. Few seeds (one view or so, whose grains fit
    // in L2): wave gw takes chunks gw, gw + nwv, gw + 2 nwv, ... of
    // kChunkSeeds seeds. Many seeds: they are split into eight ranges, one
    // per XCD (workgroups are dealt to the XCDs in turn); a wave takes grabs
    // from its own XCD's range, so that XCD's L2 holds the grains of those
    // views only, and moves on to the other ranges when its own is used up;
    // grabs shrink as a range empties, so the waves finish together. (Grabs
    // cost a device-scope atomic each, too many for a single view.) The
    // listing instance has range counters of its own: the counting one
    // leaves its counters used up.
    const bool dyn = n_items > (uint32_t)EMT_DYN_MIN_SEEDS;
    const uint32_t gw = grid_tid() >> 6, nwv = grid_threads() >> 6;
    const uint32_t xcd = blockIdx.x & 7u;
    const uint32_t per = ((n_items + 7u) / 8u + 63u) & ~63u;
    const uint32_t wpx = max(1u, (gridDim.x >> 3) * kWaves);
    // chunks shrink (to a quarter wave at least) when there are too few
    // items to give every wave a full one: a long walk per lane is better
    // than idle waves
    const uint32_t cs = min((uint32_t)kChunkSeeds, max(16u, (n_items + nwv - 1u) / nwv));
    uint32_t chunk = gw * cs;
    uint32_t next = dyn ? 0u : min(chunk, n_items);
    uint32_t end = dyn ? 0u : min(n_items, chunk + cs);
    bool more = true;
    bool have = false;
    bool pend0 = false, pend1 = false;  // slot closed, count not yet written
    uint32_t idx0 = 0, idx1 = 0;        // seed index held by each slot
    uint32_t th0 = 0, th1 = 0;          // grain-count threshold of each slot's seed
    int cur = lane;
    Pencil W;
    W.live = false;
    Run run[kFetch];
#pragma unroll
    for (int f = 0; f < kFetch; ++f) run[f] = Run{0, 0};
    uint32_t qn = 0, nr = 0;
    // counts of closed slots are final after a flush: write them, free slots
    auto close = [&](int sl, uint32_t idx, uint32_t th) {
        const uint32_t n = Q.cnt[sl];
        if constexpr (kEmit) {
            // the same walk and predicate as the count: a list of another
            // length is never expected; keep every entry a valid grain
            // index and flag an internal error
            const uint32_t cap = Q.ncap[sl];
            if (cap > 0 && n != cap) {
                const uint32_t p0 = d.cand[idx].p;
                for (uint32_t t = n; t < cap; ++t) d.members[Q.out_off[sl] + t] = p0;
                atomicOr(&d.cnt->err, 2u);
            }
        } else {
            // only counts that reach the threshold are written, with their
            // bit in the candidate mask (a few percent: scattered 4-byte
            // stores of every count would each cost a partial line write)
            hits += n;
            if (n >= th) {
                d.seed_n[idx] = n;
                atomicOr(&d.pass[idx >> 5], 1u << (idx & 31u));
            }
        }
    };
    auto finalize = [&]() {
        if (pend0) {
            close(lane, idx0, th0);
            pend0 = false;
        }
        if (pend1) {
            close(lane + 64, idx1, th1);
            pend1 = false;
        }
        wave_lds_sync();
    };
    for (;;) {
        {
            if (dyn) {
                if (next >= end && more)
                    more = xcd_grab(d.grab + (kEmit ? 8 * 16 : 0), xcd, per, n_items, wpx, 64u,
                                    4096u, next, end);
            } else {
                more = chunk + nwv * cs < n_items;
                if (next >= end && more) {
                    chunk += nwv * cs;
                    next = chunk;
                    end = min(n_items, chunk + cs);
                    more = chunk + nwv * cs < n_items;
                }
            }
            // take the next seeds into free slots. Setting up a seed (its
            // loads, line constants and walk) runs with whatever lanes take
            // one, so it is done in bulk: only once kRefillMin lanes wait, or
            // when no lane is walking. A lane may idle a few steps; the
            // set-up runs once per many seeds instead of almost every step.
            const bool want = !have && !(pend0 && pend1);
            const unsigned long long wm = __ballot(want);
            const uint32_t n_want = (uint32_t)__popcll(wm);
            const bool refill = n_want >= (uint32_t)kRefillMin || __ballot(have) == 0;
            const uint32_t rank = (uint32_t)__popcll(wm & lanes_below());
            const bool take = refill && want && next + rank < end;
            if (take) {
                const uint32_t idx = next + rank;
                cur = pend0 ? lane + 64 : lane;
                uint2 pq;
                uint32_t v;
                if constexpr (kEmit) {
                    const Cand cd = d.cand[idx];
                    pq = make_uint2(cd.p, cd.q);
                    v = cd.v;
                    const uint32_t off = d.mem_off[idx];
                    Q.out_off[cur] = off;
                    Q.ncap[cur] = ((unsigned long long)off + cd.n <= c.mem_cap) ? cd.n : 0u;
                } else {
                    pq = d.seeds[idx];
                    v = d.view_of[pq.x];
                }
                const int4 gi = d.sg[pq.x], gj = d.sg[pq.y];
                const int dx = gj.x - gi.x, dy = gj.y - gi.y, dz = gj.z - gi.z;
                const uint32_t th = seed_threshold(dx, dy, dz, P);
                if constexpr (kEmit) {
                    // the merge's priority key and threshold of the candidate
                    d.key[idx] = cand_key(d.cand[idx].n, (uint32_t)gi.w, (uint32_t)gj.w);
                    if (P.thr_num) d.cand_thr[idx] = th;
                }
                if (cur == lane) {
                    idx0 = idx;
                    th0 = th;
                } else {
                    idx1 = idx;
                    th1 = th;
                }
                if constexpr (kFinite) Q.pc[cur] = axial_bounds(gi, dx, dy, dz, P.cyl_ext);
                float4 A, C;
                line_consts(gi, dx, dy, dz, P.r, A, C);
                Q.la[cur] = A;
                Q.lc[cur] = C;
                Q.lp[cur] = pq.x;
                Q.cnt[cur] = 0;
                W.init(&d.grids[v], gi, dx, dy, dz, P.r, true, 0, 1, kFinite ? P.cyl_ext : -1);
                have = true;
            }
            if (refill) next = min(end, next + n_want);
            // fetch kFetch runs once the previous ones are queued
            bool drained = true;
#pragma unroll
            for (int f = 0; f < kFetch; ++f) drained = drained && run[f].k >= run[f].e;
            if (have && W.live && drained) {
#pragma unroll
                for (int f = 0; f < kFetch; ++f) W.fetch(d.cell_start, run[f]);
            }
            // queue up to kLanePieces pieces of the lane's runs
            uint32_t left = kLanePieces, mine = 0, nrun = 0, mtests = 0;
            uint32_t len[kFetch], np[kFetch];
#pragma unroll
            for (int f = 0; f < kFetch; ++f) {
                const uint32_t avail = run[f].e > run[f].k ? run[f].e - run[f].k : 0u;
                len[f] = min(avail, (uint32_t)kPiece * left);
                np[f] = (len[f] + (uint32_t)kPiece - 1u) / (uint32_t)kPiece;
                left -= np[f];
                mine += np[f];
                mtests += len[f];
                nrun += len[f] ? 1u : 0u;
            }
            const uint32_t pk = mine | (nrun << 16);
            const uint32_t incl = wave_incl_scan_dpp(pk);
            const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            // room first: test what is queued if this step's runs do not fit
            if (qn + (tot & 0xffffu) > (uint32_t)kPieceCap ||
                nr + (tot >> 16) > (uint32_t)kCountRunCap) {
                count_flush(Q, qn, P.r, d.sg, d.sgf, d.members, lane);
                qn = 0;
                nr = 0;
                finalize();
            }
            if (mine) {
                const uint32_t ex = incl - pk;
                uint32_t pos = qn + (ex & 0xffffu);
                uint32_t ri = nr + (ex >> 16);
                const uint32_t tag = (uint32_t)cur << 12;
#pragma unroll
                for (int f = 0; f < kFetch; ++f) {
                    if (len[f]) {
                        Q.run[ri++] = make_uint2(run[f].k, pos | tag | (len[f] << 19));
                        atomicOr(&Q.mask[pos >> 6], 1ull << (pos & 63));
                        pos += np[f];
                        run[f].k += len[f];
                    }
                }
            }
            qn += tot & 0xffffu;
            nr += tot >> 16;
            tests += mtests;
            // a seed whose walk ended and whose runs are all queued is closed
            bool queued = true;
#pragma unroll
            for (int f = 0; f < kFetch; ++f) queued = queued && run[f].k >= run[f].e;
            if (have && !W.live && queued) {
                have = false;
                if (cur == lane) pend0 = true; else pend1 = true;
            }
            const bool blocked = !have && pend0 && pend1;
            const uint32_t n_blocked = (uint32_t)__popcll(__ballot(blocked));
            const bool all_done = __ballot(have) == 0 && next >= end && !more;
            if (all_done || n_blocked > 16) {
                if (qn) count_flush(Q, qn, P.r, d.sg, d.sgf, d.members, lane);
                qn = 0;
                nr = 0;
                finalize();
                if (all_done) break;
            }
        }
    }
    if constexpr (!kEmit) {
        add_spread(d.part64, 2, wave_sum(tests));
        add_spread(d.part64, 3, wave_sum(hits));
    }
}

// Candidates among seeds [0, s), s <= n_seeds_ok: the scan of the mask's
// popcounts up to word s / 32, plus the set bits below s in that word.
__device__ __forceinline__ uint32_t cand_before(const DevPtrs &d, uint32_t s) {
    const uint32_t w = s >> 5, b = s & 31u;
    return d.pass_pos[w] + (b ? (uint32_t)__popc(d.pass[w] & ((1u << b) - 1u)) : 0u);
}

// Candidates in seed order, one mask word per thread: positions from the
// scan of the words' popcounts; their counts (for the member offsets); and
// the seeds and candidates of each view (views are contiguous in anchor
// order, so in seed and in candidate order too). Keys and thresholds are
// written by the member listing, which loads both seed grains anyway.
__global__ void __launch_bounds__(kBlock) k_cand_scatter(DevPtrs d, Caps c, Params P) {
    const uint32_t ns = d.cnt->n_seeds_ok;
    for (uint32_t v = grid_tid(); v < d.desc->n_views; v += grid_threads()) {
        const uint32_t g0 = d.grids[v].grain_off, g1 = g0 + d.grids[v].n;
        const uint32_t s0 = d.seed_off[g0], s1 = d.seed_off[g1];
        d.view_seeds[v] = s1 - s0;
        d.view_cand[v] = cand_before(d, min(s1, ns)) - cand_before(d, min(s0, ns));
    }
    unsigned long long listed = 0;  // member entries of the listed candidates
    const uint32_t nwd = d.cnt->pass_words;
    for (uint32_t w = grid_tid(); w < nwd; w += grid_threads()) {
        uint32_t bits = d.pass[w];
        for (uint32_t pos = d.pass_pos[w]; bits && pos < c.cand_cap; ++pos, bits &= bits - 1u) {
            const uint32_t s = (w << 5) | (uint32_t)(__ffs(bits) - 1);
            const uint32_t n = d.seed_n[s];
            listed += n;
            const uint2 pq = d.seeds[s];
            Cand cd;
            cd.p = pq.x;
            cd.q = pq.y;
            cd.n = n;
            cd.v = d.view_of[pq.x];
            d.cand[pos] = cd;
            d.cand_n[pos] = n;
        }
    }
    add_spread(d.part64, 1, wave_sum(listed));
}

// The threshold a candidate's unused grains must reach: n_min, or its own
// angle-dependent threshold when that variant is on.
__device__ __forceinline__ uint32_t cand_min(const DevPtrs &d, const Params &P, uint32_t ci) {
    return P.thr_num ? d.cand_thr[ci] : (uint32_t)P.n_min;
}

// ----------------------------------------------------------------- merge
//
// Exclusive association, identical to taking candidates one by one in key
// order: a candidate's outcome depends only on higher-priority candidates
// that share one of its still unused grains. Each round:
//   prune    a candidate left with fewer than n_min unused grains is
//            rejected (used grains never return); the others clear the
//            reservation of their unused grains;
//   reserve  every undecided candidate takes an atomic min of its key on
//            each of its unused grains;
//   decide   one holding every reservation of its unused grains has no
//            undecided predecessor on them, so its unused set is final: it
//            is accepted with that set if it still has n_min grains; one
//            holding at least n_min of them but not all is sure to be
//            accepted and takes the ones it holds at once (see decide).
// Candidates taking grains in one round own disjoint grains, so their
// updates do not interact, and a concurrent update can only hide grains
// taken by a higher-priority candidate. The grid-wide rounds fuse prune and
// reserve into one pass; the tail kernel keeps the three phases. A
// candidate sure to be accepted is never pruned.

constexpr int kMaxRounds = 256;
constexpr int kWideRounds = 16;  // most grid-wide rounds (distinct key tags) before the tail
// rounds a call runs grid-wide at most before the per-view tails take over
constexpr int kWideCap = EMT_MERGE_WIDE;
static_assert(kWideCap >= 1 && kWideCap <= kWideRounds, "grid-wide merge rounds");

__global__ void __launch_bounds__(kBlock) k_merge_init(DevPtrs d, Caps c) {
    const Counters *cn = d.cnt;
    const bool overflow = cn->n_seeds > c.seed_cap || cn->n_cand > c.cand_cap ||
                          cn->n_members > c.mem_cap;
    const uint32_t nc = overflow ? 0u : cn->n_cand;
    const uint32_t nm = overflow ? 0u : cn->n_members;
    for (uint32_t i = grid_tid(); i < nc; i += grid_threads()) {
        d.status[i] = kUndecided;
        d.mcount[i] = 0;
    }
    const uint32_t n_total = d.desc->n_total;
    for (uint32_t g = grid_tid(); g < n_total; g += grid_threads()) {
        d.owner[g] = ~0ull;
    }
    for (uint32_t e = grid_tid(); e < nm; e += grid_threads()) d.taken[e] = 0;
    for (uint32_t r = grid_tid(); r < kMaxRounds; r += grid_threads()) d.undecided[r] = 0;
    if (grid_tid() == 0) {
        d.cnt->n_act[0] = nc;  // candidates taking part in the merge
        d.cnt->err |= overflow ? 1u : 0u;
    }
}

// Grid-wide rounds. Eight lanes take one candidate and stride over its
// member entries; round r walks the list of candidates left undecided by
// round r-1 (all candidates for r = 0) and appends the ones it leaves
// undecided to the next list, whose length it counts in undecided[r]. A
// reservation carries its round in the top four bits of the key, counted
// down, so the keys of a newer round lie below every older value and no
// clearing pass is needed between rounds (keys use 60 bits: n, i and j are
// below 2^20 each).
// A grain's owner word is ~0 while nobody has reserved it, 0 once an
// accepted candidate has taken it (no key is 0: a seed's i and j differ),
// and otherwise the smallest key offered to it. So one load tells whether a
// grain is still unused and who holds it, and a reservation can never
// displace a taken grain.
// A reservation: the word only decreases during a round, so a value read at
// or below key means an equal or better reservation (or the grain's taking)
// is already there and the atomic would change nothing; most grains are
// offered to many candidates, and the read spares most of the atomics.
__device__ __forceinline__ void reserve(unsigned long long *owner, unsigned long long key) {
    if (*owner > key) atomicMin(owner, key);
}

constexpr int kMergeGroup = 8;
static_assert(kWideRounds <= 16, "round tags take four bits");

__device__ __forceinline__ uint32_t group_sum8(uint32_t v) {
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    return v;
}

__device__ __forceinline__ uint32_t *merge_list(const DevPtrs &d, int round) {
    return (round & 1) ? d.act2 : d.act;
}

// Candidates left undecided are staged in LDS and appended to the next list
// with one global atomic per flush: a single counter hit once per wave
// serialises at the L2.
constexpr uint32_t kListBuf = 2048;
constexpr uint32_t kGroupsPerBlock = kBlock / kMergeGroup;

__device__ __forceinline__ void flush_list(uint32_t *s_buf, uint32_t *s_cnt, uint32_t *s_base,
                                           uint32_t *counter, uint32_t *next) {
    __syncthreads();
    const uint32_t m = *s_cnt;
    if (threadIdx.x == 0 && m) *s_base = atomicAdd(counter, m);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) next[*s_base + i] = s_buf[i];
    __syncthreads();
    if (threadIdx.x == 0) *s_cnt = 0;
    __syncthreads();
}

// The decide phase for one candidate (its eight-lane group; every lane
// returns the same). Unused grains are those whose owner word is not 0; the
// candidate holds the ones whose word is its key. Fewer unused grains than
// its threshold: rejected. Holding every unused grain: accepted with them.
// Holding at least its threshold but not all: it is sure to be accepted,
// since no undecided candidate before it wants a grain it holds, so those
// grains are still unused when its turn comes in the one-by-one reading; it
// takes them now (kCertain) and waits for the others, taking each as it comes
// to hold it. A grain taken early is one a later candidate would have lost
// anyway, so nothing else changes. Returns whether it stays undecided.
__device__ __forceinline__ bool decide(const DevPtrs &d, const Params &P, uint32_t ci,
                                       unsigned long long key, uint32_t e0, uint32_t e1,
                                       int sub) {
    const bool certain = d.status[ci] == kCertain;
    uint32_t unused = 0, held = 0, lost = 0;
    for (uint32_t e = e0 + sub; e < e1; e += kMergeGroup) {
        const unsigned long long o = d.owner[d.members[e]];
        unused += o != 0ull ? 1u : 0u;
        held += o == key ? 1u : 0u;
        lost |= (o != 0ull && o != key) ? 1u : 0u;
    }
    unused = group_sum8(unused);
    held = group_sum8(held);
    lost = group_sum8(lost);
    const uint32_t need = cand_min(d, P, ci);
    if (!certain && unused < need) {
        if (sub == 0) d.status[ci] = kRejected;
        return false;
    }
    if (lost != 0 && !certain && held < need) return true;
    for (uint32_t e = e0 + sub; e < e1; e += kMergeGroup) {
        const uint32_t k = d.members[e];
        if (d.owner[k] == key) {
            d.owner[k] = 0ull;
            d.taken[e] = 1;
        }
    }
    if (sub == 0) {
        d.mcount[ci] += held;
        d.status[ci] = lost == 0 ? kAccepted : kCertain;
    }
    return lost != 0;
}

template <int kPhase>
__global__ void __launch_bounds__(kBlock) k_round(DevPtrs d, Params P, int round) {
    __shared__ uint32_t s_buf[kPhase == 1 ? kListBuf : 1];
    __shared__ uint32_t s_cnt, s_base;
    const uint32_t n = round == 0 ? d.cnt->n_act[0] : d.undecided[round - 1];
    if (n == 0) return;
    const uint32_t *list = merge_list(d, round);
    uint32_t *next = merge_list(d, round + 1);
    const unsigned long long tag = (unsigned long long)(kWideRounds - 1 - round) << 60;
    const int sub = threadIdx.x & (kMergeGroup - 1);
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    // block-uniform loop: the list flush below synchronises the workgroup
    for (uint32_t base = blockIdx.x * kGroupsPerBlock; base < n;
         base += gridDim.x * kGroupsPerBlock) {
        const uint32_t slot = base + threadIdx.x / kMergeGroup;
        uint32_t ci = 0;
        bool live = slot < n;
        if (live) {
            ci = round == 0 ? slot : list[slot];
            live = round == 0 || d.status[ci] == kUndecided || d.status[ci] == kCertain;
        }
        bool still = false;
        if (live) {
            const unsigned long long key = d.key[ci] | tag;
            const uint32_t e0 = d.mem_off[ci], e1 = e0 + d.cand[ci].n;
            if (kPhase == 0) {  // prune, then reserve
                // round 0: no grain is used yet and every candidate reached
                // its threshold, so nothing is pruned
                uint32_t unused = 0;
                if (round > 0) {
                    for (uint32_t e = e0 + sub; e < e1; e += kMergeGroup)
                        unused += d.owner[d.members[e]] != 0ull ? 1u : 0u;
                    unused = group_sum8(unused);
                }
                if (round > 0 && unused < cand_min(d, P, ci) && d.status[ci] != kCertain) {
                    if (sub == 0) d.status[ci] = kRejected;
                } else {
                    // a taken grain's word (0) is below every key: untouched
                    for (uint32_t e = e0 + sub; e < e1; e += kMergeGroup)
                        reserve(&d.owner[d.members[e]], key);
                }
            } else {  // decide
                still = decide(d, P, ci, key, e0, e1, sub) && sub == 0;
            }
        }
        if (kPhase == 1) {
            if (still) s_buf[atomicAdd(&s_cnt, 1u)] = ci;
            __syncthreads();
            const uint32_t held = s_cnt;
            __syncthreads();  // all have read it before the next iteration adds
            if (held + kGroupsPerBlock > kListBuf)
                flush_list(s_buf, &s_cnt, &s_base, &d.undecided[round], next);
        }
    }
    if (kPhase == 1) flush_list(s_buf, &s_cnt, &s_base, &d.undecided[round], next);
}

// First candidate of view v: candidates are listed in seed order, and a
// view's seeds are contiguous.
__device__ __forceinline__ uint32_t view_first_cand(const DevPtrs &d, uint32_t v, uint32_t ns) {
    return cand_before(d, min(d.seed_off[d.grids[v].grain_off], ns));
}

// Candidates of different views share no grain, so the rounds the grid-wide
// kernels leave are finished view by view, one workgroup each. First the
// undecided list is split by view: view v's go to its own stretch of the
// other list, starting at its first candidate (a view never has more
// undecided candidates than candidates). The order within a stretch does not
// matter: outcomes depend only on the keys.
__global__ void __launch_bounds__(kBlock) k_tail_split(DevPtrs d, int last_round) {
    const uint32_t n = d.undecided[last_round];
    const uint32_t *list = merge_list(d, last_round + 1);
    uint32_t *out = merge_list(d, last_round + 2);
    const uint32_t ns = d.cnt->n_seeds_ok;
    for (uint32_t i = grid_tid(); i < n; i += grid_threads()) {
        const uint32_t ci = list[i];
        const uint32_t v = d.cand[ci].v;
        out[view_first_cand(d, v, ns) + atomicAdd(&d.view_tail[v], 1u)] = ci;
    }
}

// The remaining rounds of one view in one workgroup, looping until none of
// its candidates is undecided (each round decides at least the highest-
// priority one, so it ends within as many rounds as there are candidates).
// Groups of eight lanes take candidates of the list; __syncthreads separates
// the phases, and the prune phase clears the reservations of the
// candidates' unused grains.
constexpr int kTailBlock = 1024;

__global__ void __launch_bounds__(kTailBlock) k_merge_tail(DevPtrs d, Params P, int last_round) {
    const uint32_t view = blockIdx.x;
    if (view >= d.desc->n_views) return;
    __shared__ uint32_t s_n[2];
    const int sub = threadIdx.x & (kMergeGroup - 1);
    const uint32_t group = threadIdx.x / kMergeGroup;
    constexpr uint32_t kTailGroups = kTailBlock / kMergeGroup;
    const uint32_t c0 = view_first_cand(d, view, d.cnt->n_seeds_ok);
    if (threadIdx.x == 0) {
        s_n[0] = d.view_tail[view];
        s_n[1] = 0;
    }
    __syncthreads();
    uint32_t *list[2] = {merge_list(d, last_round + 2) + c0, merge_list(d, last_round + 3) + c0};
    int cur = 0;
    uint32_t rounds = 0;
    const uint32_t limit = s_n[0] + 2;
    while (s_n[cur] > 0 && rounds < limit) {
        const uint32_t n = s_n[cur];
        // prune (groups are whole 8-lane slices of one wave, so the group
        // sums only read lanes that took the same branch)
        for (uint32_t i = group; i < n; i += kTailGroups) {
            const uint32_t ci = list[cur][i];
            const uint8_t st = d.status[ci];
            if (st != kUndecided && st != kCertain) continue;
            const uint32_t e0 = d.mem_off[ci], e1 = e0 + d.cand[ci].n;
            uint32_t unused = 0;
            for (uint32_t e = e0 + sub; e < e1; e += kMergeGroup) {
                const uint32_t k = d.members[e];
                if (d.owner[k] != 0ull) {
                    ++unused;
                    d.owner[k] = ~0ull;
                }
            }
            unused = group_sum8(unused);
            if (unused < cand_min(d, P, ci) && st != kCertain && sub == 0) d.status[ci] = kRejected;
        }
        __threadfence_block();
        __syncthreads();
        // reserve
        for (uint32_t i = group; i < n; i += kTailGroups) {
            const uint32_t ci = list[cur][i];
            if (d.status[ci] != kUndecided && d.status[ci] != kCertain) continue;
            const unsigned long long key = d.key[ci];
            const uint32_t e0 = d.mem_off[ci], e1 = e0 + d.cand[ci].n;
            for (uint32_t e = e0 + sub; e < e1; e += kMergeGroup)
                reserve(&d.owner[d.members[e]], key);
        }
        __threadfence_block();
        __syncthreads();
        // decide
        for (uint32_t i = group; i < n; i += kTailGroups) {
            const uint32_t ci = list[cur][i];
            if (d.status[ci] != kUndecided && d.status[ci] != kCertain) continue;
            const unsigned long long key = d.key[ci];
            const uint32_t e0 = d.mem_off[ci], e1 = e0 + d.cand[ci].n;
            if (decide(d, P, ci, key, e0, e1, sub) && sub == 0) {
                const uint32_t slot = atomicAdd(&s_n[cur ^ 1], 1u);
                list[cur ^ 1][slot] = ci;
            }
        }
        __threadfence_block();
        __syncthreads();
        if (threadIdx.x == 0) s_n[cur] = 0;
        cur ^= 1;
        ++rounds;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // grid-wide rounds that ran: round r runs while round r-1 left some
        uint32_t wide = d.cnt->n_act[0] ? 1u : 0u;
        while (wide >= 1 && wide <= (uint32_t)last_round && d.undecided[wide - 1]) ++wide;
        atomicMax(&d.cnt->rounds, wide + rounds);
        if (s_n[cur] > 0) atomicOr(&d.cnt->err, 4u);
    }
}

// ------------------------------------------------------------------- fit

// Accepted candidates into the list of tracks (any order: tracks are ranked
// by key afterwards) and the track count of each view. A thread takes four
// consecutive candidates with one 32-bit load of their status bytes (the
// array is padded to 256 bytes). A workgroup counts its accepted candidates
// first and reserves their slots with one atomic; a wave adds to a view's
// count once for its candidates of the view of its first accepted one (a
// wave's candidates are consecutive, so nearly always of one view).
__device__ __forceinline__ uint32_t accepted4(const DevPtrs &d, uint32_t q, uint32_t nc) {
    if (4ull * q >= nc) return 0u;
    const uint32_t w = reinterpret_cast<const uint32_t *>(d.status)[q];
    uint32_t bits = 0;
#pragma unroll
    for (uint32_t t = 0; t < 4; ++t)
        bits |= (((w >> (8 * t)) & 0xffu) == kAccepted && 4 * q + t < nc) ? (1u << t) : 0u;
    return bits;
}

__global__ void __launch_bounds__(kBlock) k_collect(DevPtrs d, Caps c) {
    __shared__ uint32_t s_cnt, s_base;
    const Counters *cn = d.cnt;
    const uint32_t nc = cn->err ? 0u : min(cn->n_cand, c.cand_cap);
    const uint32_t nq = (nc + 3u) / 4u;
    const int lane = lane_id();
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    // block-uniform loops: every lane of a wave takes part in its scans
    for (uint32_t b = blockIdx.x * blockDim.x; b < nq; b += grid_threads()) {
        const uint32_t n = wave_sum((uint32_t)__popc(accepted4(d, b + threadIdx.x, nc)));
        if (lane == 0 && n) atomicAdd(&s_cnt, n);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s_base = s_cnt ? atomicAdd(&d.cnt->n_acc, s_cnt) : 0u;
        s_cnt = 0;
    }
    __syncthreads();
    for (uint32_t b = blockIdx.x * blockDim.x; b < nq; b += grid_threads()) {
        const uint32_t q = b + threadIdx.x;
        uint32_t bits = accepted4(d, q, nc);
        const uint32_t k = (uint32_t)__popc(bits);
        const uint32_t incl = wave_incl_scan_dpp(k);
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        if (tot == 0) continue;
        uint32_t w = 0;
        if (lane == 0) w = atomicAdd(&s_cnt, tot);
        w = (uint32_t)__shfl((int)w, 0);
        const int first = __ffsll((long long)__ballot(bits != 0)) - 1;
        const uint32_t v_own = bits ? d.cand[4 * q + (uint32_t)(__ffs(bits) - 1)].v : 0u;
        const uint32_t v0 = (uint32_t)__shfl((int)v_own, first);
        uint32_t pos = s_base + w + incl - k, same = 0;
        while (bits) {
            const uint32_t i = 4 * q + (uint32_t)(__ffs(bits) - 1);
            bits &= bits - 1u;
            d.acc[pos++] = i;
            const uint32_t v = d.cand[i].v;
            if (v == v0)
                ++same;
            else
                atomicAdd(&d.view_ntr[v], 1u);
        }
        same = wave_sum(same);
        if (lane == first) atomicAdd(&d.view_ntr[v0], same);
    }
}

__global__ void __launch_bounds__(kBlock) k_view_offsets(DevPtrs d) {
    const uint32_t n_views = d.desc->n_views;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < n_views; base += kBlock) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < n_views ? d.view_ntr[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, &tot);
        if (i < n_views) d.view_tr_off[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) d.view_tr_off[n_views] = carry;
}

// Tracks grouped by view: a wave takes its slots of the view of its lane 0
// with one atomic on that view's cursor (a view's cursor hit once per track
// serialises in L2), other views one atomic per track.
__global__ void __launch_bounds__(kBlock) k_group(DevPtrs d, unsigned long long *gkey) {
    const uint32_t na = d.cnt->n_acc;
    const int lane = lane_id();
    for (uint32_t b = blockIdx.x * blockDim.x; b < na; b += grid_threads()) {
        const uint32_t a = b + threadIdx.x;
        const bool ok = a < na;  // false for lane 0 only if for the whole wave
        const uint32_t ci = ok ? d.acc[a] : 0u;
        const uint32_t v = ok ? d.cand[ci].v : 0u;
        const uint32_t v0 = (uint32_t)__shfl((int)v, 0);
        const unsigned long long same = __ballot(ok && v == v0);
        uint32_t base = 0;
        if (lane == 0 && same) base = atomicAdd(&d.view_cursor[v0], (uint32_t)__popcll(same));
        base = (uint32_t)__shfl((int)base, 0);
        if (ok) {
            const uint32_t at = v == v0 ? base + (uint32_t)__popcll(same & lanes_below())
                                        : atomicAdd(&d.view_cursor[v], 1u);
            const uint32_t pos = d.view_tr_off[v] + at;
            d.grouped[pos] = ci;
            gkey[pos] = d.key[ci];
        }
    }
}

// Track order within a view = key order (the order of acceptance in the
// one-by-one reading); rank by counting smaller keys of the same view.
__global__ void __launch_bounds__(kBlock) k_rank(DevPtrs d, const unsigned long long *gkey) {
    const uint32_t na = d.cnt->n_acc;
    for (uint32_t s = grid_tid(); s < na; s += grid_threads()) {
        const uint32_t ci = d.grouped[s];
        const uint32_t v = d.cand[ci].v;
        const uint32_t b = d.view_tr_off[v], e = b + d.view_ntr[v];
        const unsigned long long key = gkey[s];
        uint32_t rank = 0;
#pragma unroll 8
        for (uint32_t t = b; t < e; ++t) rank += gkey[t] < key ? 1u : 0u;
        d.track_cand[b + rank] = ci;
        d.tg_n[b + rank] = d.mcount[ci];
    }
}

// Convert an exact 128-bit integer to double/float without library calls.
__device__ __forceinline__ double i128_to_f64(__int128 x) {
    const bool neg = x < 0;
    const unsigned __int128 u = neg ? (unsigned __int128)(-x) : (unsigned __int128)x;
    const unsigned long long hi = (unsigned long long)(u >> 64);
    const unsigned long long lo = (unsigned long long)u;
    const double r = (double)hi * 0x1p64 + (double)lo;
    return neg ? -r : r;
}

__device__ __forceinline__ float i128_to_f32(__int128 x) {
    if (x >= -(((__int128)1) << 62) && x <= (((__int128)1) << 62)) return (float)(long long)x;
    return (float)i128_to_f64(x);
}

__device__ __forceinline__ int sign128(__int128 x) { return x > 0 ? 1 : (x < 0 ? -1 : 0); }

// One wave per track: gather the grains the track took, order them by
// (t, input index) with t = (g_k - g_i).d, and fit.
//
// Fit: exact integer moments about g_i, S1 = sum w, S2 = sum w w^T, give
// Q = n S2 - S1 S1^T = n^2 times the covariance. The fit axis a has the
// largest Q_aa (ties to the lower axis); slopes are Q_ab/Q_aa and Q_ac/Q_aa,
// divided in FP32, or in FP64 when a = z or the RMS spread along a is under
// 5 um (Q_aa < 250000 n^2) or when asked. The sign that puts the direction in
// the upper hemisphere comes from the integer Q entries.
__global__ void __launch_bounds__(kBlock) k_fit(DevPtrs d, Params P) {
    const uint32_t nt = d.cnt->n_acc;
    const int lane = lane_id();
    const uint32_t wave = grid_tid() >> 6;
    const uint32_t nwaves = grid_threads() >> 6;
    for (uint32_t t = wave; t < nt; t += nwaves) {
        const uint32_t ci = d.track_cand[t];
        const Cand cd = d.cand[ci];
        const ViewGrid *G = &d.grids[cd.v];
        const int4 gi = d.sg[cd.p], gj = d.sg[cd.q];
        const int dx = gj.x - gi.x, dy = gj.y - gi.y, dz = gj.z - gi.z;
        const uint32_t base = d.tg_off[t];
        const uint32_t m = d.mcount[ci];
        const uint32_t e0 = d.mem_off[ci];

        // 1. compact the taken entries
        uint32_t j = 0;
        for (uint32_t e = 0; e < cd.n; e += 64) {
            const uint32_t ee = e + lane;
            const bool tk = ee < cd.n && d.taken[e0 + ee];
            const unsigned long long mask = __ballot(tk);
            if (tk) {
                const uint32_t pos = j + (uint32_t)__popcll(mask & lanes_below());
                const uint32_t k = d.members[e0 + ee];
                const int4 h = d.sg[k];
                d.tord[base + pos] = k;
                d.tvals[base + pos] = (long long)(h.x - gi.x) * dx + (long long)(h.y - gi.y) * dy +
                                      (long long)(h.z - gi.z) * dz;
            }
            j += (uint32_t)__popcll(mask);
        }
        wave_sync_mem();

        // 2. exact moments
        long long s1[3] = {0, 0, 0}, s2[6] = {0, 0, 0, 0, 0, 0};
        for (uint32_t q = lane; q < m; q += 64) {
            const int4 h = d.sg[d.tord[base + q]];
            const long long w0 = h.x - gi.x, w1 = h.y - gi.y, w2 = h.z - gi.z;
            s1[0] += w0;
            s1[1] += w1;
            s1[2] += w2;
            s2[0] += w0 * w0;
            s2[1] += w0 * w1;
            s2[2] += w0 * w2;
            s2[3] += w1 * w1;
            s2[4] += w1 * w2;
            s2[5] += w2 * w2;
        }
        for (int u = 0; u < 3; ++u) s1[u] = wave_sum(s1[u]);
        for (int u = 0; u < 6; ++u) s2[u] = wave_sum(s2[u]);

        // 3. grain order by (t, input index), rank by counting: the wave
        // loads 64 entries at a time into registers and every lane compares
        // its own entry with each of them through readlane (input indices
        // are distinct, so no entry outranks itself)
        for (uint32_t q0 = 0; q0 < m; q0 += 64) {
            const uint32_t q = q0 + (uint32_t)lane;
            const bool vq = q < m;
            const long long tq = vq ? d.tvals[base + q] : 0;
            const int oq = vq ? d.sg[d.tord[base + q]].w : 0;
            uint32_t rank = 0;
            for (uint32_t o0 = 0; o0 < m; o0 += 64) {
                const uint32_t o = o0 + (uint32_t)lane;
                const long long tl = o < m ? d.tvals[base + o] : 0;
                const int ol = o < m ? d.sg[d.tord[base + o]].w : 0;
                const int t_lo = (int)(uint32_t)(unsigned long long)tl;
                const int t_hi = (int)(uint32_t)((unsigned long long)tl >> 32);
                const uint32_t cnt = min(64u, m - o0);
                for (uint32_t i = 0; i < cnt; ++i) {
                    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(t_lo, (int)i);
                    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(t_hi, (int)i);
                    const long long to = (long long)(((unsigned long long)hi << 32) | lo);
                    const int oo = __builtin_amdgcn_readlane(ol, (int)i);
                    rank += (to < tq || (to == tq && oo < oq)) ? 1u : 0u;
                }
            }
            if (vq) d.out_grains[base + rank] = (uint32_t)oq;
        }

        // 4. fit (every lane computes the same values)
        const long long n = (long long)m;
        __int128 Q[3][3];
        {
            const long long S2[3][3] = {{s2[0], s2[1], s2[2]}, {s2[1], s2[3], s2[4]},
                                        {s2[2], s2[4], s2[5]}};
            for (int u = 0; u < 3; ++u)
                for (int w = 0; w < 3; ++w)
                    Q[u][w] = (__int128)n * S2[u][w] - (__int128)s1[u] * s1[w];
        }
        int a = 0;
        if (Q[1][1] > Q[a][a]) a = 1;
        if (Q[2][2] > Q[a][a]) a = 2;
        int b = a == 0 ? 1 : 0;
        int cx = a == 2 ? 1 : 2;
        float dir[3];
        float slope[2];
        int comp_sign[3];
        uint32_t fp64 = 0, degen = 0;
        double s0d = 0.0, s1d = 0.0;  // slopes of the FP64 paths
        if (Q[a][a] == 0) {
            // every grain coincides: no spread to fit, the seed direction
            // stands in (its spread along any axis is 0, under the 5 um
            // rule, so the ratio is taken in FP64)
            degen = 1;
            fp64 = 1;
            const int ad[3] = {dx, dy, dz};
            a = 0;
            if (abs(ad[1]) > abs(ad[a])) a = 1;
            if (abs(ad[2]) > abs(ad[a])) a = 2;
            b = a == 0 ? 1 : 0;
            cx = a == 2 ? 1 : 2;
            s0d = (double)ad[b] / (double)ad[a];
            s1d = (double)ad[cx] / (double)ad[a];
            slope[0] = (float)s0d;
            slope[1] = (float)s1d;
            // (1, slope) on axes (a, b, c) is d / d_a: signs of d times that of d_a
            const int sa = ad[a] < 0 ? -1 : 1;
            for (int u = 0; u < 3; ++u) comp_sign[u] = sa * (ad[u] > 0 ? 1 : (ad[u] < 0 ? -1 : 0));
        } else {
            fp64 = (a == 2) || (Q[a][a] < (__int128)250000 * n * n) ||
                   (P.flags & EMT_F_FP64_FIT_ALWAYS) != 0;
            if (fp64) {
                const double qa = i128_to_f64(Q[a][a]);
                s0d = i128_to_f64(Q[a][b]) / qa;
                s1d = i128_to_f64(Q[a][cx]) / qa;
                slope[0] = (float)s0d;
                slope[1] = (float)s1d;
            } else {
                const float qa = i128_to_f32(Q[a][a]);
                slope[0] = i128_to_f32(Q[a][b]) / qa;
                slope[1] = i128_to_f32(Q[a][cx]) / qa;
            }
            comp_sign[a] = 1;
            comp_sign[b] = sign128(Q[a][b]);
            comp_sign[cx] = sign128(Q[a][cx]);
        }
        {
            if (fp64) {
                const double nrm = sqrt(1.0 + s0d * s0d + s1d * s1d);
                dir[a] = (float)(1.0 / nrm);
                dir[b] = (float)(s0d / nrm);
                dir[cx] = (float)(s1d / nrm);
            } else {
                const float nrm = sqrtf(1.0f + slope[0] * slope[0] + slope[1] * slope[1]);
                dir[a] = 1.0f / nrm;
                dir[b] = slope[0] / nrm;
                dir[cx] = slope[1] / nrm;
            }
            bool flip;
            if (comp_sign[2] != 0) flip = comp_sign[2] < 0;
            else if (comp_sign[1] != 0) flip = comp_sign[1] < 0;
            else flip = comp_sign[0] < 0;
            if (flip)
                for (int u = 0; u < 3; ++u) dir[u] = -dir[u];
        }

        // 5. centroid and extent along dir
        const long long g_abs[3] = {(long long)G->lo[0] + gi.x, (long long)G->lo[1] + gi.y,
                                    (long long)G->lo[2] + gi.z};
        float cen[3];
        for (int u = 0; u < 3; ++u) cen[u] = (float)(g_abs[u] * n + s1[u]) / (float)n * 0.01f;
        float tmin = 3.0e38f, tmax = -3.0e38f;
        for (uint32_t q = lane; q < m; q += 64) {
            const int4 h = d.sg[d.tord[base + q]];
            const long long w[3] = {h.x - gi.x, h.y - gi.y, h.z - gi.z};
            float pr = 0.0f;
            for (int u = 0; u < 3; ++u) pr = fmaf((float)(n * w[u] - s1[u]), dir[u], pr);
            pr = pr / (float)n * 0.01f;
            tmin = fminf(tmin, pr);
            tmax = fmaxf(tmax, pr);
        }
        tmin = wave_min(tmin);
        tmax = wave_max(tmax);
        if (lane == 0) {
            emt_track tr;
            tr.seed[0] = (uint32_t)gi.w;
            tr.seed[1] = (uint32_t)gj.w;
            tr.grain_offset = base;
            tr.n_grains = m;
            tr.axis = (uint32_t)a;
            tr.fit_fp64 = fp64;
            tr.degenerate = degen;
            tr.slope[0] = slope[0];
            tr.slope[1] = slope[1];
            for (int u = 0; u < 3; ++u) {
                tr.dir[u] = dir[u];
                tr.centroid[u] = cen[u];
            }
            tr.t_begin = tmin;
            tr.t_end = tmax;
            d.tracks[t] = tr;
            if (fp64) atomicAdd(&d.cnt->n_fp64, 1u);
        }
    }
}

// Results to the host: counters, per-view tables, tracks and grains, at the
// sizes the device knows, into mapped pinned host memory.
__global__ void __launch_bounds__(kBlock) k_copy_out(DevPtrs d, Caps c) {
    const uint32_t tid = grid_tid(), nt = grid_threads();
    const uint32_t nv = d.desc->n_views;
    const Counters cn = *d.cnt;
    if (tid == 0) *d.out.cnt = cn;
    for (uint32_t v = tid; v < nv; v += nt) {
        d.out.view_seeds[v] = d.view_seeds[v];
        d.out.view_cand[v] = d.view_cand[v];
        d.out.view_ntr[v] = d.view_ntr[v];
        d.out.view_err[v] = d.grids[v].err;
    }
    for (uint32_t v = tid; v <= nv; v += nt) d.out.view_tr_off[v] = d.view_tr_off[v];
    const uint32_t ntr = cn.n_acc <= c.cand_cap ? cn.n_acc : 0u;
    const uint32_t words = ntr * (uint32_t)(sizeof(emt_track) / 4);
    const uint32_t *src = reinterpret_cast<const uint32_t *>(d.tracks);
    uint32_t *dst = reinterpret_cast<uint32_t *>(d.out.tracks);
    for (uint32_t i = tid; i < words; i += nt) dst[i] = src[i];
    const uint32_t ng = cn.n_track_grains <= c.mem_cap ? cn.n_track_grains : 0u;
    for (uint32_t i = tid; i < ng; i += nt) d.out.grains[i] = d.out_grains[i];
    if (d.out.cands) {
        // candidates as input-index pairs with their counts, in list order
        const uint32_t nc = cn.n_cand <= c.cand_cap ? cn.n_cand : 0u;
        for (uint32_t i = tid; i < nc; i += nt) {
            const Cand cd = d.cand[i];
            d.out.cands[3 * i] = (uint32_t)d.sg[cd.p].w;
            d.out.cands[3 * i + 1] = (uint32_t)d.sg[cd.q].w;
            d.out.cands[3 * i + 2] = cd.n;
        }
    }
}

// ---------------------------------------------------- grain recognition
//
// 3D grain recognition on a filtered 8-bit stack (frames z, rows y, columns
// x, x fastest): a pixel above the threshold that no in-stack 3 x 3 x 3
// neighbour outranks (higher, or equal and earlier in frame, row, column
// order) defines a grain, placed at the pulse-height centre of mass of its
// block in 0.01 um units (pitch of each axis num/den units, rounded to the
// nearest unit, halves up, from exact integer sums).
//
// The stack is streamed once. A workgroup owns a tile of kTilePix
// consecutive pixels (the stack is one flat byte array, so a tile runs
// across row ends): each thread reads 32 of them as two 16-byte vectors and
// marks those above threshold; the workgroup lists its candidates in LDS in
// pixel order and tests them one per thread, which keeps the neighbourhood
// tests dense although few pixels pass the threshold. The grains' offsets in
// the tile go, in pixel order, to the tile's staging slots. Two pixels next
// to each other in a row cannot both be grains (one outranks the other), and
// tile and row boundaries fall on multiples of four pixels, so a tile holds
// at most kTilePix / 2 grains: the staging area is bounded. Tile counts are
// also summed per group of 64 tiles with one atomic add each. A second,
// small kernel (one workgroup per group of tiles) takes its place in the
// output from those sums, finds each staged grain's tile by a search over
// the group's tile offsets, and writes the centre of mass: grains come out
// in frame, row, column order without a separate scan or a second stream.

// q = n / d for n < 2^32, d >= 1: double-precision reciprocal, then an
// exact integer correction of the +-1 it may be off by.
__device__ __forceinline__ uint32_t div_rcp(uint32_t n, uint32_t d, double inv) {
    uint32_t q = (uint32_t)((double)n * inv);
    if ((unsigned long long)q * d > n) --q;
    if ((unsigned long long)(q + 1) * d <= n) ++q;
    return q;
}

#ifndef EMT_GRAIN_WORDS
#define EMT_GRAIN_WORDS 8
#endif
constexpr uint32_t kGrainWords = EMT_GRAIN_WORDS;           // four-pixel words a thread
constexpr uint32_t kCandMasks = kGrainWords / 8;            // 32-pixel candidate masks
static_assert(kGrainWords % 8 == 0, "candidate masks cover 32 pixels each");
constexpr uint32_t kTilePix = kBlock * kGrainWords * 4;     // pixels a workgroup streams
constexpr uint32_t kTileGrains = kTilePix / 2;              // staging slots per tile
constexpr uint32_t kTileGroup = 64;                         // tiles per atomic sum
constexpr uint32_t kCandCap = 2048;                         // candidates listed per round
static_assert(kTilePix <= 65536u, "tile offsets are staged as 16 bits");
static_assert(kTilePix == kGrainTilePix && kTileGrains == kGrainTileGrains &&
                  kTileGroup == kGrainTileGroup,
              "tile sizes the host sizes its buffers by");

__device__ __forceinline__ uint32_t block_excl_scan_small(uint32_t v, uint32_t *s_wave,
                                                          uint32_t *total) {
    const uint32_t incl = wave_incl_scan_dpp(v);
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        before += w < wave ? s_wave[w] : 0u;
        tot += s_wave[w];
    }
    __syncthreads();  // s_wave is reused by the next scan
    *total = tot;
    return before + incl - v;
}

// The 3 x 3 x 3 block around pixel p (flat index): pulse heights w[i]
// (0 outside the stack) with i = 9 (dz+1) + 3 (dy+1) + (dx+1), so
// neighbours 0..12 come before p in frame, row, column order.
struct Block27 {
    uint32_t x, y, z;
    uint32_t w[27];
    uint32_t inside;

    __device__ __forceinline__ void load(const uint8_t *__restrict__ img, const StackGeom &G,
                                         uint32_t p) {
        const uint32_t row = div_rcp(p, G.nx, G.inv_nx);
        x = p - row * G.nx;
        z = div_rcp(row, G.ny, G.inv_ny);
        y = row - z * G.ny;
        const uint32_t plane = G.nx * G.ny;  // at most 2^31 pixels: offsets fit 32 bits
        // bit d + 1: the frame / row / column at offset d exists
        const uint32_t zok = (z > 0 ? 1u : 0u) | 2u | (z + 1 < G.nz ? 4u : 0u);
        const uint32_t yok = (y > 0 ? 1u : 0u) | 2u | (y + 1 < G.ny ? 4u : 0u);
        const uint32_t xok = (x > 0 ? 1u : 0u) | 2u | (x + 1 < G.nx ? 4u : 0u);
        inside = 0;
        // all 27 loads are issued unconditionally (a missing neighbour reads
        // pixel p itself, so every address is inside the stack) and masked
        // afterwards: no branch or wait separates them
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int dz = i / 9 - 1, dy = (i / 3) % 3 - 1, dx = i % 3 - 1;
            const bool ok = ((zok >> (dz + 1)) & (yok >> (dy + 1)) & (xok >> (dx + 1)) & 1u) != 0;
            inside |= ok ? 1u << i : 0u;
            // unsigned arithmetic wraps modulo 2^32 to the exact offset
            const uint32_t q =
                ok ? p + (uint32_t)dz * plane + (uint32_t)dy * G.nx + (uint32_t)dx : p;
            // the mask is opaque to the compiler, which would otherwise
            // turn "ok ? load : 0" back into a branch around the load
            uint32_t mask = ok ? 0xffu : 0u;
            asm("" : "+v"(mask));
            w[i] = (uint32_t)img[q] & mask;
        }
    }
    // No neighbour outranks the centre: higher, or equal and earlier. A
    // missing neighbour reads 0 and the centre is above the threshold, so it
    // never outranks. Bitwise, without short-circuits, so that every load is
    // needed and none is moved into a branch.
    __device__ __forceinline__ bool is_top() const {
        const uint32_t v = w[13];
        uint32_t beaten = 0;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            if (i < 13) beaten |= (uint32_t)(w[i] >= v);
            if (i > 13) beaten |= (uint32_t)(w[i] > v);
        }
        return beaten == 0;
    }
    __device__ __forceinline__ void centre(const StackGeom &G, int32_t *out) const {
        int sw = 0, sx = 0, sy = 0, sz = 0;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int wi = (int)w[i];
            sw += wi;
            sx += wi * ((int)x + i % 3 - 1);
            sy += wi * ((int)y + (i / 3) % 3 - 1);
            sz += wi * ((int)z + i / 9 - 1);
        }
        const int sums[3] = {sx, sy, sz};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            // floor(num / den), num < 2^47 and 0 < den < 2^31: a double
            // quotient is within one of it, and integer products fix that
            const long long num = 2ll * sums[m] * G.pnum[m] + (long long)sw * G.pden[m];
            const long long den = 2ll * sw * G.pden[m];
            long long q = (long long)((double)num / (double)den);
            if (q * den > num) --q;
            if ((q + 1) * den <= num) ++q;
            out[m] = (int32_t)q;
        }
    }
};

__global__ void __launch_bounds__(kBlock) k_grain_find(const uint8_t *__restrict__ img,
                                                       StackGeom G, uint32_t *tile_cnt,
                                                       uint32_t *group_cnt, uint16_t *stage) {
    __shared__ uint32_t s_wave[kBlock / 64];
    __shared__ uint32_t s_cand[kCandCap];
    const uint32_t n_groups = (G.nx >> 2) * G.ny * G.nz;  // four-pixel words
    const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) * kGrainWords;
    uint32_t words[kGrainWords];
    if (g0 + kGrainWords <= n_groups) {
        const uint4 *p = reinterpret_cast<const uint4 *>(img + 4ull * g0);
#pragma unroll
        for (int h = 0; h < (int)kGrainWords / 4; ++h) {
            const uint4 q = p[h];
            words[4 * h] = q.x;
            words[4 * h + 1] = q.y;
            words[4 * h + 2] = q.z;
            words[4 * h + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < (int)kGrainWords; ++k)
            words[k] = g0 + k < n_groups
                           ? *reinterpret_cast<const uint32_t *>(img + 4ull * (g0 + k))
                           : 0u;
    }
    uint32_t cand[kCandMasks], n_cand = 0;
#pragma unroll
    for (int j = 0; j < (int)kCandMasks; ++j) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                c |= ((words[8 * j + k] >> (8 * b)) & 0xffu) > G.thr ? 1u << (4 * k + b) : 0u;
        cand[j] = c;
        n_cand += (uint32_t)__popc(c);
    }
    uint32_t c_total;
    const uint32_t c_before = block_excl_scan_small(n_cand, s_wave, &c_total);
    const uint32_t tile0 = blockIdx.x * kTilePix;
    uint16_t *st = stage + (size_t)blockIdx.x * kTileGrains;
    uint32_t found = 0;
    for (uint32_t base = 0; base < c_total; base += kCandCap) {  // uniform
        // list this round's candidates, in pixel order
        uint32_t idx = c_before;
#pragma unroll
        for (int j = 0; j < (int)kCandMasks; ++j) {
            uint32_t bits = cand[j];
            while (bits) {
                const int i = __ffs((int)bits) - 1;
                bits &= bits - 1;
                if (idx >= base && idx < base + kCandCap)
                    s_cand[idx - base] = 4u * g0 + 32u * (uint32_t)j + (uint32_t)i;
                ++idx;
            }
        }
        __syncthreads();
        const uint32_t m = min(kCandCap, c_total - base);
        for (uint32_t c0 = 0; c0 < m; c0 += kBlock) {  // uniform
            const uint32_t c = c0 + threadIdx.x;
            bool top = false;
            if (c < m) {
                Block27 B;
                B.load(img, G, s_cand[c]);
                top = B.is_top();
            }
            uint32_t n_top;
            const uint32_t before = block_excl_scan_small(top ? 1u : 0u, s_wave, &n_top);
            if (top && found + before < kTileGrains)  // always true: see the bound above
                st[found + before] = (uint16_t)(s_cand[c] - tile0);
            found += n_top;
        }
        __syncthreads();  // s_cand is rewritten by the next round
    }
    if (threadIdx.x == 0) {
        tile_cnt[blockIdx.x] = found;
        if (found) atomicAdd(group_cnt + blockIdx.x / kTileGroup, found);
    }
}

// One workgroup per group of kTileGroup tiles: its grains' place in the
// output is the sum of the earlier groups' counts plus the offset of the
// tile within the group.
__global__ void __launch_bounds__(kBlock) k_grain_place(
    const uint8_t *__restrict__ img, StackGeom G, const uint32_t *__restrict__ tile_cnt,
    const uint32_t *__restrict__ group_cnt, uint32_t n_tiles,
    const uint16_t *__restrict__ stage, int32_t *out, uint32_t max_out, uint32_t *total) {
    static_assert(kTileGroup == 64, "tile offsets are scanned by one wave");
    __shared__ uint32_t s_wave[kBlock / 64];
    __shared__ uint32_t s_off[kTileGroup + 1];
    const uint32_t grp = blockIdx.x;
    uint32_t acc = 0;
    for (uint32_t i = threadIdx.x; i < grp; i += kBlock) acc += group_cnt[i];
    uint32_t prefix;
    (void)block_excl_scan_small(acc, s_wave, &prefix);
    const uint32_t t0 = grp * kTileGroup;
    if (threadIdx.x < 64) {
        const uint32_t t = t0 + threadIdx.x;
        const uint32_t c = t < n_tiles ? min(tile_cnt[t], kTileGrains) : 0u;
        s_off[threadIdx.x + 1] = wave_incl_scan_dpp(c);
        if (threadIdx.x == 0) s_off[0] = 0;
    }
    __syncthreads();
    const uint32_t n_here = s_off[kTileGroup];
    if (grp + 1 == gridDim.x && threadIdx.x == 0) *total = prefix + n_here;
    for (uint32_t g = threadIdx.x; g < n_here; g += kBlock) {
        // the tile holding grain g: s_off[lo] <= g < s_off[lo + 1]
        uint32_t lo = 0, hi = kTileGroup;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_off[mid] <= g) lo = mid;
            else hi = mid;
        }
        const uint32_t t = t0 + lo;
        const uint32_t p = t * kTilePix + stage[(size_t)t * kTileGrains + (g - s_off[lo])];
        const uint32_t q = prefix + g;
        if (q < max_out) {
            Block27 B;
            B.load(img, G, p);
            B.centre(G, out + 3ull * q);
        }
    }
}

__global__ void k_clear_words(uint32_t *p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

size_t grain_tile_count(const StackGeom &G) {
    const unsigned long long pix = (unsigned long long)G.nx * G.ny * G.nz;
    return (size_t)((pix + kTilePix - 1) / kTilePix);
}

size_t grain_group_count(const StackGeom &G) {
    return (grain_tile_count(G) + kTileGroup - 1) / kTileGroup;
}

size_t grain_stage_slots(const StackGeom &G) { return grain_tile_count(G) * kTileGrains; }

void launch_find_grains(const uint8_t *img, const StackGeom &G, const GrainBufs &b,
                        hipStream_t s) {
    const uint32_t nt = (uint32_t)grain_tile_count(G), ng = (uint32_t)grain_group_count(G);
    k_clear_words<<<(ng + kBlock - 1) / kBlock, kBlock, 0, s>>>(b.group_cnt, ng);
    k_grain_find<<<nt, kBlock, 0, s>>>(img, G, b.tile_cnt, b.group_cnt, b.stage);
    k_grain_place<<<ng, kBlock, 0, s>>>(img, G, b.tile_cnt, b.group_cnt, nt, b.stage, b.out,
                                        b.max_out, b.total);
}

// ---------------------------------------------------------- filtering
//
// Image filtering: every camera pixel (x, y) has its own gain correction
// (unsigned, 1/256 units) and its own threshold, the same in every frame.
// Per pixel: t = min(255, raw * gain / 256 rounded half up); u = 255 - t
// (inversion: grains become bright); out = u - thr if u > thr, else 0.
// A thread owns kPix consecutive pixels of the frame, keeps their gains and
// thresholds in registers and walks kFilterFrames frames, loading all of
// them before it computes, so the maps are read once per frame group and
// raw and filtered pixels stream through once.

namespace {

constexpr uint32_t kFilterFrames = 8;

__device__ __forceinline__ uint32_t filter_word(uint32_t r, uint32_t g01, uint32_t g23,
                                                uint32_t t) {
    uint32_t o = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t rb = (r >> (8 * b)) & 0xffu;
        const uint32_t gb = ((b < 2 ? g01 : g23) >> (16 * (b & 1))) & 0xffffu;
        const uint32_t tb = (t >> (8 * b)) & 0xffu;
        const uint32_t tuned = min(255u, (__umul24(rb, gb) + 128u) >> 8);
        const uint32_t inv = 255u - tuned;
        o |= (inv > tb ? inv - tb : 0u) << (8 * b);
    }
    return o;
}

template <int kPix>  // pixels a thread owns in each frame: 4 or 16
__global__ void __launch_bounds__(kBlock) k_filter(const uint8_t *__restrict__ raw,
                                                   const uint16_t *__restrict__ gain,
                                                   const uint8_t *__restrict__ thr,
                                                   uint8_t *__restrict__ out, uint32_t chunks,
                                                   uint32_t plane, uint32_t nz) {
    static_assert(kPix == 4 || kPix == 16, "one or four words a frame");
    constexpr int kW = kPix / 4;  // four-pixel words
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= chunks) return;
    const uint32_t z0 = blockIdx.y * kFilterFrames;
    const uint32_t nf = min(kFilterFrames, nz - z0);  // uniform
    uint32_t g[2 * kW], t[kW];
    if constexpr (kPix == 16) {
        const uint4 ga = reinterpret_cast<const uint4 *>(gain)[2 * c];
        const uint4 gb = reinterpret_cast<const uint4 *>(gain)[2 * c + 1];
        const uint4 ta = reinterpret_cast<const uint4 *>(thr)[c];
        g[0] = ga.x; g[1] = ga.y; g[2] = ga.z; g[3] = ga.w;
        g[4] = gb.x; g[5] = gb.y; g[6] = gb.z; g[7] = gb.w;
        t[0] = ta.x; t[1] = ta.y; t[2] = ta.z; t[3] = ta.w;
    } else {
        const uint2 ga = reinterpret_cast<const uint2 *>(gain)[c];
        g[0] = ga.x;
        g[1] = ga.y;
        t[0] = reinterpret_cast<const uint32_t *>(thr)[c];
    }
    uint32_t r[kFilterFrames][kW];
#pragma unroll
    for (int f = 0; f < (int)kFilterFrames; ++f) {
        if ((uint32_t)f >= nf) break;
        const size_t off = (size_t)(z0 + f) * plane + (size_t)c * kPix;
        if constexpr (kPix == 16) {
            const uint4 v = *reinterpret_cast<const uint4 *>(raw + off);
            r[f][0] = v.x; r[f][1] = v.y; r[f][2] = v.z; r[f][3] = v.w;
        } else {
            r[f][0] = *reinterpret_cast<const uint32_t *>(raw + off);
        }
    }
#pragma unroll
    for (int f = 0; f < (int)kFilterFrames; ++f) {
        if ((uint32_t)f >= nf) break;
        uint32_t o[kW];
#pragma unroll
        for (int k = 0; k < kW; ++k) o[k] = filter_word(r[f][k], g[2 * k], g[2 * k + 1], t[k]);
        const size_t off = (size_t)(z0 + f) * plane + (size_t)c * kPix;
        if constexpr (kPix == 16)
            *reinterpret_cast<uint4 *>(out + off) = make_uint4(o[0], o[1], o[2], o[3]);
        else
            *reinterpret_cast<uint32_t *>(out + off) = o[0];
    }
}

}  // namespace

bool launch_filter(const uint8_t *raw, const uint16_t *gain, const uint8_t *thr, uint8_t *out,
                   uint32_t nx, uint32_t ny, uint32_t nz, bool vec16, hipStream_t s) {
    const uint32_t plane = nx * ny;
    if (plane % 4u) return false;
    if (vec16 && plane % 16u) vec16 = false;
    const uint32_t pix = vec16 ? 16u : 4u, chunks = plane / pix;
    const dim3 grid((chunks + kBlock - 1) / kBlock, (nz + kFilterFrames - 1) / kFilterFrames);
    if (vec16)
        k_filter<16><<<grid, kBlock, 0, s>>>(raw, gain, thr, out, chunks, plane, nz);
    else
        k_filter<4><<<grid, kBlock, 0, s>>>(raw, gain, thr, out, chunks, plane, nz);
    return true;
}

namespace {

uint32_t blocks_for(unsigned long long n, uint32_t max_blocks) {
    unsigned long long b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (uint32_t)(b < max_blocks ? b : max_blocks);
}

#ifndef EMT_PERSISTENT_BLOCKS
#define EMT_PERSISTENT_BLOCKS 2048
#endif
constexpr uint32_t kPersistentBlocks = EMT_PERSISTENT_BLOCKS;  // 8 blocks of 4 waves per CU
// the counting kernel's grid: one resident generation (4 workgroups per CU,
// bound by its LDS and registers), so no workgroup waits for another's slot
constexpr uint32_t kCountBlocks = EMT_COUNT_BLOCKS;
static_assert(kCountBlocks % 8 == 0, "whole workgroups per XCD");

}  // namespace

size_t scan_scratch_words(uint32_t n_cap) { return (size_t)n_cap / kScanTile + 2; }

void launch_prepare(const DevPtrs &d, const Caps &c, const Params &, hipStream_t s) {
    k_zero<<<blocks_for(c.n_cells, 1024), kBlock, 0, s>>>(d.cnt, d.view_seeds, d.view_cand,
                                                          d.view_ntr, d.view_cursor, d.view_tail,
                                                          d.cell_count, d.grab, d.part64, d.desc);
}

void launch_bin(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    const uint32_t bx = blocks_for(c.max_view_n, 64);
    dim3 grid(bx, c.n_views);
    k_bbox<<<grid, kBlock, 0, s>>>(d.xyz, d.grids, d.view_of, d.desc);
    k_grid<<<(c.n_views + 63) / 64, 64, 0, s>>>(d.grids, d.desc, P);
    k_hist<<<grid, kBlock, 0, s>>>(d.xyz, d.grids, d.cell_of, d.rank, d.cell_count, d.desc);
    scan_excl(d.cell_count, &d.desc->n_cells_m1, c.n_cells, d.scan_part, d.cell_start, nullptr, s);
    k_scatter<<<grid, kBlock, 0, s>>>(d.xyz, d.grids, d.cell_of, d.rank, d.cell_start, d.sg, d.sgf,
                                      d.desc);
}

void launch_seeds(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    const uint32_t nb = blocks_for(64ull * c.n_total, 4 * kPersistentBlocks);
    k_seeds<false><<<nb, kBlock, 0, s>>>(d, c, P);
    // the scan total counts every seed (it wraps only above 2^32 - 1 a call)
    // offsets in uint32: exact whenever the total fits, which k_seed_total checks
    scan_excl(d.seed_cnt, &d.desc->n_total, c.n_total, d.scan_part, d.seed_off, &d.cnt->n_seeds, s);
    k_seed_total<<<1, 64, 0, s>>>(d.cnt, d.part64, c.seed_cap);
    k_seeds<true><<<nb, kBlock, 0, s>>>(d, c, P);
}

void launch_count(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    if (P.cyl_ext >= 0)
        k_count<true, false><<<kCountBlocks, kBlock, 0, s>>>(d, c, P);
    else
        k_count<false, false><<<kCountBlocks, kBlock, 0, s>>>(d, c, P);
}

void launch_candidates(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    const uint32_t words = (uint32_t)(c.seed_cap / 32 + 1);
    scan_excl<true>(d.pass, &d.cnt->pass_words, words, d.scan_part, d.pass_pos, &d.cnt->n_cand, s);
    k_cand_scatter<<<blocks_for(words, kPersistentBlocks), kBlock, 0, s>>>(d, c, P);
}

void launch_members(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    scan_excl(d.cand_n, &d.cnt->n_cand, c.cand_cap, d.scan_part, d.mem_off, &d.cnt->n_members, s);
    k_member_total<<<1, 64, 0, s>>>(d.cnt, d.part64);
    // the counting kernel's walk and test, listing the grains of each candidate
    if (P.cyl_ext >= 0)
        k_count<true, true><<<kCountBlocks, kBlock, 0, s>>>(d, c, P);
    else
        k_count<false, true><<<kCountBlocks, kBlock, 0, s>>>(d, c, P);
}

void launch_merge_init(const DevPtrs &d, const Caps &c, const Params &, hipStream_t s) {
    unsigned long long n = c.cand_cap;
    if (c.n_total > n) n = c.n_total;
    if (c.mem_cap > n) n = c.mem_cap;
    k_merge_init<<<blocks_for(n, kPersistentBlocks), kBlock, 0, s>>>(d, c);
}

void launch_merge(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    // Later rounds see a fraction of the candidates: their grids shrink by
    // half per round down to a floor (the loops stride, so any grid is correct).
    // The number of grid-wide rounds comes with the capacities (the host
    // sizes it from the rounds earlier calls needed); the tail finishes
    // whatever they leave.
    const int wide = c.wide_rounds < 1 ? 1 : (c.wide_rounds > kWideRounds ? kWideRounds : c.wide_rounds);
    uint32_t nb = blocks_for((unsigned long long)kMergeGroup * c.cand_cap, 2 * kPersistentBlocks);
    for (int round = 0; round < wide; ++round) {
        k_round<0><<<nb, kBlock, 0, s>>>(d, P, round);
        k_round<1><<<nb, kBlock, 0, s>>>(d, P, round);
        if (round >= 1 && nb > 1024) nb = nb / 2 > 1024 ? nb / 2 : 1024;
    }
    k_tail_split<<<64, kBlock, 0, s>>>(d, wide - 1);
    k_merge_tail<<<c.n_views, kTailBlock, 0, s>>>(d, P, wide - 1);
}

int max_merge_rounds() { return kMaxRounds; }
int max_wide_rounds() { return kWideCap; }

void launch_copy_out(const DevPtrs &d, const Caps &c, const Params &, hipStream_t s) {
    k_copy_out<<<64, kBlock, 0, s>>>(d, c);
}

void launch_fit(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    const uint32_t nb = blocks_for(c.cand_cap, kPersistentBlocks);
    k_collect<<<nb, kBlock, 0, s>>>(d, c);
    k_view_offsets<<<1, kBlock, 0, s>>>(d);
    // keys of the grouped tracks reuse the owner array (merge is over)
    unsigned long long *gkey = d.owner;
    k_group<<<nb, kBlock, 0, s>>>(d, gkey);
    k_rank<<<nb, kBlock, 0, s>>>(d, gkey);
    scan_excl(d.tg_n, &d.cnt->n_acc, c.cand_cap, d.scan_part, d.tg_off, &d.cnt->n_track_grains, s);
    k_fit<<<nb, kBlock, 0, s>>>(d, P);
}

}  // namespace emt
