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

constexpr float kMargin = 4.0f;  // units added to every cell window
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ unsigned long long lanes_below() {
    return (1ull << lane_id()) - 1ull;
}

// Reserve one slot per lane with pred among the active lanes of the wave;
// a single atomic per wave.
__device__ __forceinline__ unsigned long long wave_append(
    bool pred, unsigned long long *counter) {
    const unsigned long long mask = __ballot(pred);
    if (mask == 0) return 0;
    const int leader = __ffsll((long long)mask) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
    return base + (unsigned long long)__popcll(mask & lanes_below());
}

__device__ __forceinline__ uint32_t wave_append32(bool pred, uint32_t *counter) {
    const unsigned long long mask = __ballot(pred);
    if (mask == 0) return 0;
    const int leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    return base + (uint32_t)__popcll(mask & lanes_below());
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

__global__ void __launch_bounds__(kBlock) k_scan_part(const uint32_t *in, const uint32_t *n_dev,
                                                      uint32_t n_cap, uint32_t *part) {
    const uint32_t n = scan_len(n_dev, n_cap);
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
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

__global__ void __launch_bounds__(kBlock) k_scan_apply(const uint32_t *in, const uint32_t *n_dev,
                                                       uint32_t n_cap, const uint32_t *part,
                                                       uint32_t *out) {
    const uint32_t n = scan_len(n_dev, n_cap);
    if (blockIdx.x * kScanTile >= n) return;
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
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
// n_dev); *total_out = out[n].
void scan_excl(const uint32_t *in, const uint32_t *n_dev, uint32_t n_cap, uint32_t *part,
               uint32_t *out, uint32_t *total_out, hipStream_t s) {
    const uint32_t nb = n_cap / kScanTile + 1;
    k_scan_part<<<nb, kBlock, 0, s>>>(in, n_dev, n_cap, part);
    k_scan_part_scan<<<1, kBlock, 0, s>>>(part, nb, n_dev, n_cap, out, total_out);
    k_scan_apply<<<nb, kBlock, 0, s>>>(in, n_dev, n_cap, part, out);
}

// ------------------------------------------------------------------- bin

__global__ void __launch_bounds__(kBlock) k_zero(Counters *cnt, unsigned long long *view_seeds,
                                                 uint32_t *view_cand, uint32_t *view_ntr,
                                                 uint32_t *view_cursor, uint32_t n_views,
                                                 uint32_t *cell_count, uint32_t n_cells) {
    const uint32_t tid = grid_tid();
    if (tid == 0) {
        Counters z = {};
        *cnt = z;
    }
    for (uint32_t v = tid; v < n_views; v += grid_threads()) {
        view_seeds[v] = 0;
        view_cand[v] = 0;
        view_ntr[v] = 0;
        view_cursor[v] = 0;
    }
    for (uint32_t i = tid; i < n_cells; i += grid_threads()) cell_count[i] = 0;
}

// Bounding box of every view (grid origin) and the view index of each grain.
__global__ void __launch_bounds__(kBlock) k_bbox(const int32_t *xyz, ViewGrid *grids,
                                                 uint32_t *view_of) {
    const uint32_t v = blockIdx.y;
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
    if (lane_id() == 0 && n > 0) {
        for (int m = 0; m < 3; ++m) {
            atomicMin(&grids[v].lo[m], lo[m]);
            atomicMax(&grids[v].hi[m], hi[m]);
        }
    }
}

// Cell geometry per view: the requested edges, doubled until the grid has at
// most cell_cap cells. A view whose span exceeds the limit is marked: its
// grains still go through the binning (into one cell, so every later view
// keeps its place in the sorted arrays) but it produces no seeds.
__global__ void k_grid(ViewGrid *grids, uint32_t n_views, Params P) {
    const uint32_t v = grid_tid();
    if (v >= n_views) return;
    ViewGrid G = grids[v];
    long long span[3];
    for (int m = 0; m < 3; ++m) {
        if (G.n == 0) {
            G.lo[m] = 0;
            G.hi[m] = 0;
        }
        span[m] = (long long)G.hi[m] - (long long)G.lo[m];
        if (span[m] > kSpanMax) G.err = 1;
        G.cell[m] = P.cell_req[m];
    }
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
                                                 uint32_t *cell_count) {
    const uint32_t v = blockIdx.y;
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
                                                    const uint32_t *cell_start, int4 *sg) {
    const uint32_t v = blockIdx.y;
    const ViewGrid G = grids[v];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < G.n; i += gridDim.x * blockDim.x) {
        const size_t g = (size_t)G.grain_off + i;
        const uint32_t pos = cell_start[cell_of[g]] + rank[g];
        sg[pos] = make_int4(xyz[3 * g] - G.lo[0], xyz[3 * g + 1] - G.lo[1], xyz[3 * g + 2] - G.lo[2],
                            (int)i);
    }
}

// ------------------------------------------------------------ line walk

// Visit every grain that can lie within r of the infinite line through g
// with direction d (any view grain closer than r is visited; the caller's
// exact predicate decides).
//
// With a the axis of largest |d_a| and b, c the others: a grain k in the cell
// layers [A0, A1] along a and within r of the line satisfies
// |k_b - p_b(k_a)| <= r|d|/|d_a| (p = line point with the same a), because
// for v = k - p(k_a), v_a = 0 and |v x d| >= |v| |d_a|. p_b is linear in a,
// so the b range of the layer is [min(p_b(A0), p_b(A1)) - rho,
// max(...) + rho]; same for c. Cells along x are contiguous in memory, so each
// (y, z) row of the window is one run of grains.
template <class F>
__device__ __forceinline__ void walk_line(const int4 *__restrict__ sg,
                                          const uint32_t *__restrict__ cs,
                                          const ViewGrid *__restrict__ Gp, int slab_x, int gx,
                                          int gy, int gz, int dx, int dy, int dz, int r, F &on) {
    const int nx = Gp->dims[0], ny = Gp->dims[1], nz = Gp->dims[2];
    const int cx = Gp->cell[0], cy = Gp->cell[1], cz = Gp->cell[2];
    const uint32_t off = Gp->cell_off;
    const int adx = abs(dx), ady = abs(dy), adz = abs(dz);
    const int a = (adx >= ady && adx >= adz) ? 0 : (ady >= adz ? 1 : 2);
    const int ga = a == 0 ? gx : (a == 1 ? gy : gz);
    const int gb = a == 0 ? gy : gx;
    const int gc = a == 2 ? gy : gz;
    const int da = a == 0 ? dx : (a == 1 ? dy : dz);
    const int db = a == 0 ? dy : dx;
    const int dc = a == 2 ? dy : dz;
    const int ca = a == 0 ? cx : (a == 1 ? cy : cz);
    const int cb = a == 0 ? cy : cx;
    const int cc = a == 2 ? cy : cz;
    const int na = a == 0 ? nx : (a == 1 ? ny : nz);
    const int nb = a == 0 ? ny : nx;
    const int nc = a == 2 ? ny : nz;
    const float inv = 1.0f / (float)da;
    const float sb = (float)db * inv, sc = (float)dc * inv;
    const float rho = (float)r * sqrtf((float)(dx * dx + dy * dy + dz * dz)) * fabsf(inv) + kMargin;
    const float ica = 1.0f / (float)ca, icb = 1.0f / (float)cb, icc = 1.0f / (float)cc;

    // Layers along a where the widened line meets the grid in b and c.
    float alo = 0.0f, ahi = (float)(na * ca - 1);
    if (db != 0) {
        const float t1 = (float)ga + (-rho - (float)gb) / sb;
        const float t2 = (float)ga + ((float)(nb * cb - 1) + rho - (float)gb) / sb;
        alo = fmaxf(alo, fminf(t1, t2));
        ahi = fminf(ahi, fmaxf(t1, t2));
    }
    if (dc != 0) {
        const float t1 = (float)ga + (-rho - (float)gc) / sc;
        const float t2 = (float)ga + ((float)(nc * cc - 1) + rho - (float)gc) / sc;
        alo = fmaxf(alo, fminf(t1, t2));
        ahi = fminf(ahi, fmaxf(t1, t2));
    }
    const int ia0 = (int)floorf(fminf(fmaxf(alo * ica - 1.0f, 0.0f), (float)na));
    const int ia1 = (int)floorf(fmaxf(fminf(ahi * ica + 1.0f, (float)(na - 1)), -1.0f));
    const int T = a == 0 ? slab_x : 1;

    for (int ia = ia0; ia <= ia1; ia += T) {
        const int ie = min(ia + T - 1, na - 1);
        const float u0 = (float)(ia * ca - ga);
        const float u1 = (float)((ie + 1) * ca - 1 - ga);
        const float pb0 = (float)gb + u0 * sb, pb1 = (float)gb + u1 * sb;
        const float pc0 = (float)gc + u0 * sc, pc1 = (float)gc + u1 * sc;
        const int ib0 = max(0, (int)floorf(fmaxf((fminf(pb0, pb1) - rho) * icb, -1.0f)));
        const int ib1 = min(nb - 1, (int)floorf(fminf((fmaxf(pb0, pb1) + rho) * icb, (float)nb)));
        const int ic0 = max(0, (int)floorf(fmaxf((fminf(pc0, pc1) - rho) * icc, -1.0f)));
        const int ic1 = min(nc - 1, (int)floorf(fminf((fmaxf(pc0, pc1) + rho) * icc, (float)nc)));
        if (ib0 > ib1 || ic0 > ic1) continue;
        const int x0 = a == 0 ? ia : ib0;
        const int x1 = a == 0 ? ie : ib1;
        const int y0 = a == 1 ? ia : (a == 0 ? ib0 : ic0);
        const int y1 = a == 1 ? ia : (a == 0 ? ib1 : ic1);
        const int z0 = a == 2 ? ia : ic0;
        const int z1 = a == 2 ? ia : ic1;
        for (int z = z0; z <= z1; ++z) {
            for (int y = y0; y <= y1; ++y) {
                const uint32_t row = off + (uint32_t)((z * ny + y) * nx);
                const uint32_t k0 = cs[row + x0], k1 = cs[row + x1 + 1];
                for (uint32_t k = k0; k < k1; ++k) on(k, sg[k]);
            }
        }
    }
}

// The cylinder predicate |(g_k - g_i) x d|^2 <= r^2 |d|^2, exact.
// c = g_k x d - g_i x d is formed with 24-bit multiplies in wrapping 32-bit
// arithmetic: coordinates are < 2^18 + 1 and |d_m| < 2^12, so every true
// component of c is below 2^31 and the wrapped result equals it. |c|^2 is
// compared in FP32 with a relative guard band of 2^-20 (the FP32 sum of
// squares is within 5 * 2^-24 of exact); inside the band the test is redone
// in int64.
struct LineTest {
    int dx, dy, dz;
    uint32_t ex, ey, ez;
    float tlo, thi;
    long long T;

    __device__ __forceinline__ void init(int4 gi, int dx_, int dy_, int dz_, int r) {
        dx = dx_;
        dy = dy_;
        dz = dz_;
        ex = (uint32_t)__mul24(gi.y, dz) - (uint32_t)__mul24(gi.z, dy);
        ey = (uint32_t)__mul24(gi.z, dx) - (uint32_t)__mul24(gi.x, dz);
        ez = (uint32_t)__mul24(gi.x, dy) - (uint32_t)__mul24(gi.y, dx);
        const long long D = (long long)dx * dx + (long long)dy * dy + (long long)dz * dz;
        T = (long long)r * r * D;
        const float tf = (float)T;
        tlo = tf * (1.0f - 0x1p-20f);
        thi = tf * (1.0f + 0x1p-20f);
    }

    __device__ __forceinline__ bool hit(int4 h) const {
        const int c0 = (int)((uint32_t)__mul24(h.y, dz) - (uint32_t)__mul24(h.z, dy) - ex);
        const int c1 = (int)((uint32_t)__mul24(h.z, dx) - (uint32_t)__mul24(h.x, dz) - ey);
        const int c2 = (int)((uint32_t)__mul24(h.x, dy) - (uint32_t)__mul24(h.y, dx) - ez);
        const float f0 = (float)c0, f1 = (float)c1, f2 = (float)c2;
        const float fc = fmaf(f0, f0, fmaf(f1, f1, f2 * f2));
        if (fc <= tlo) return true;
        if (fc > thi) return false;
        const long long cc = (long long)c0 * c0 + (long long)c1 * c1 + (long long)c2 * c2;
        return cc <= T;
    }
};

struct CountOp {
    LineTest L;
    uint32_t n;
    uint32_t tests;
    __device__ __forceinline__ void operator()(uint32_t, int4 h) {
        ++tests;
        n += L.hit(h) ? 1u : 0u;
    }
};

struct MemberOp {
    LineTest L;
    uint32_t *out;
    uint32_t n, cap;
    __device__ __forceinline__ void operator()(uint32_t k, int4 h) {
        if (L.hit(h)) {
            if (n < cap) out[n] = k;
            ++n;
        }
    }
};

// ----------------------------------------------------------------- seeds

// One lane per anchor grain p: every grain q of the cells overlapping the
// box [g_p - (R-1), g_p + (R-1)] with a higher input index and
// 0 < |g_q - g_p|^2 < R^2 is a seed (p, q).
__global__ void __launch_bounds__(kBlock) k_seeds(DevPtrs d, Caps c, Params P) {
    const int R1 = P.R - 1;
    const int R2 = P.R * P.R;
    for (uint32_t p = grid_tid(); p < c.n_total; p += grid_threads()) {
        const uint32_t v = d.view_of[p];
        const ViewGrid *G = &d.grids[v];
        if (G->err) continue;
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
        unsigned long long mine = 0;
        for (int z = z0; z <= z1; ++z) {
            for (int y = y0; y <= y1; ++y) {
                const uint32_t row = off + (uint32_t)((z * ny + y) * nx);
                const uint32_t k0 = d.cell_start[row + x0], k1 = d.cell_start[row + x1 + 1];
                for (uint32_t q = k0; q < k1; ++q) {
                    const int4 h = d.sg[q];
                    const int ex = h.x - g.x, ey = h.y - g.y, ez = h.z - g.z;
                    bool ok = h.w > g.w && abs(ex) <= R1 && abs(ey) <= R1 && abs(ez) <= R1;
                    const int D = ok ? ex * ex + ey * ey + ez * ez : 0;
                    ok = ok && D > 0 && D < R2;
                    const unsigned long long slot = wave_append(ok, &d.cnt->n_seeds);
                    if (ok) {
                        ++mine;
                        if (slot < c.seed_cap) d.seeds[slot] = make_uint2(p, q);
                    }
                }
            }
        }
        if (mine) atomicAdd(&d.view_seeds[v], mine);
    }
}

// ----------------------------------------------------------------- count

// One lane per seed: count the grains on its line; seeds reaching n_min are
// appended to the candidate list with their priority key.
__global__ void __launch_bounds__(kBlock) k_count(DevPtrs d, Caps c, Params P) {
    const unsigned long long ns_all = d.cnt->n_seeds;
    const unsigned long long ns = ns_all < c.seed_cap ? ns_all : c.seed_cap;
    unsigned long long tests = 0, hits = 0;
    for (unsigned long long s = grid_tid(); s < ns; s += grid_threads()) {
        const uint2 pq = d.seeds[s];
        const int4 gi = d.sg[pq.x], gj = d.sg[pq.y];
        const uint32_t v = d.view_of[pq.x];
        const int dx = gj.x - gi.x, dy = gj.y - gi.y, dz = gj.z - gi.z;
        CountOp op;
        op.L.init(gi, dx, dy, dz, P.r);
        op.n = 0;
        op.tests = 0;
        walk_line(d.sg, d.cell_start, &d.grids[v], P.slab_x, gi.x, gi.y, gi.z, dx, dy, dz, P.r, op);
        tests += op.tests;
        hits += op.n;
        const bool pred = op.n >= (uint32_t)P.n_min;
        const uint32_t slot = wave_append32(pred, &d.cnt->n_cand);
        if (pred) {
            if (slot < c.cand_cap) {
                Cand cd;
                cd.p = pq.x;
                cd.q = pq.y;
                cd.n = op.n;
                cd.v = v;
                d.cand[slot] = cd;
                d.key[slot] = cand_key(op.n, (uint32_t)gi.w, (uint32_t)gj.w);
            }
            atomicAdd(&d.view_cand[v], 1u);
        }
    }
    tests = wave_sum(tests);
    hits = wave_sum(hits);
    if (lane_id() == 0) {
        atomicAdd(&d.cnt->tests, tests);
        atomicAdd(&d.cnt->hits, hits);
    }
}

// --------------------------------------------------------------- members

__global__ void __launch_bounds__(kBlock) k_cand_n(DevPtrs d, Caps c) {
    const uint32_t nc = min(d.cnt->n_cand, c.cand_cap);
    for (uint32_t i = grid_tid(); i < nc; i += grid_threads()) d.cand_n[i] = d.cand[i].n;
}

__global__ void __launch_bounds__(kBlock) k_members(DevPtrs d, Caps c, Params P) {
    const uint32_t nc = min(d.cnt->n_cand, c.cand_cap);
    for (uint32_t i = grid_tid(); i < nc; i += grid_threads()) {
        const Cand cd = d.cand[i];
        const uint32_t off = d.mem_off[i];
        if ((unsigned long long)off + cd.n > c.mem_cap) continue;
        const int4 gi = d.sg[cd.p], gj = d.sg[cd.q];
        const int dx = gj.x - gi.x, dy = gj.y - gi.y, dz = gj.z - gi.z;
        MemberOp op;
        op.L.init(gi, dx, dy, dz, P.r);
        op.out = d.members + off;
        op.n = 0;
        op.cap = cd.n;
        walk_line(d.sg, d.cell_start, &d.grids[cd.v], P.slab_x, gi.x, gi.y, gi.z, dx, dy, dz, P.r,
                  op);
        if (op.n != cd.n) {
            // the same walk and predicate as the count: never expected; keep
            // every entry a valid grain index and report an internal error
            for (uint32_t t = op.n; t < cd.n; ++t) op.out[t] = cd.p;
            atomicOr(&d.cnt->err, 2u);
        }
    }
}

// ----------------------------------------------------------------- merge
//
// Exclusive association, identical to taking candidates one by one in key
// order: a candidate's outcome depends only on higher-priority candidates
// that share one of its still unused grains. Each round, every undecided
// candidate reserves its unused grains with an atomic min of its key. One
// that holds every reservation has no undecided predecessor on its grains,
// so its unused set is final: it is accepted if that set still has n_min
// grains and takes them. A candidate left with fewer than n_min unused
// grains is rejected at once (used grains never return). Accepted ones in
// the same round own disjoint grains, so their updates do not interact.

__global__ void __launch_bounds__(kBlock) k_merge_init(DevPtrs d, Caps c) {
    const Counters *cn = d.cnt;
    const bool overflow = cn->n_seeds > c.seed_cap || cn->n_cand > c.cand_cap ||
                          cn->n_members > c.mem_cap;
    const uint32_t nc = overflow ? 0u : cn->n_cand;
    const uint32_t nm = overflow ? 0u : cn->n_members;
    for (uint32_t i = grid_tid(); i < nc; i += grid_threads()) {
        d.act[0][i] = i;
        d.status[i] = kUndecided;
        d.mcount[i] = 0;
    }
    for (uint32_t g = grid_tid(); g < c.n_total; g += grid_threads()) {
        d.used[g] = 0;
        d.owner[g] = ~0ull;
    }
    for (uint32_t e = grid_tid(); e < nm; e += grid_threads()) d.taken[e] = 0;
    if (grid_tid() == 0) {
        d.cnt->n_act[0] = nc;
        d.cnt->n_act[1] = 0;
        d.cnt->err |= overflow ? 1u : 0u;
    }
}

__global__ void __launch_bounds__(kBlock) k_round_reset(DevPtrs d, int cur) {
    const uint32_t n = d.cnt->n_act[cur];
    if (grid_tid() == 0) d.cnt->n_act[cur ^ 1] = 0;
    for (uint32_t i = grid_tid(); i < n; i += grid_threads()) {
        const uint32_t ci = d.act[cur][i];
        const uint32_t e0 = d.mem_off[ci], e1 = e0 + d.cand[ci].n;
        for (uint32_t e = e0; e < e1; ++e) d.owner[d.members[e]] = ~0ull;
    }
}

__global__ void __launch_bounds__(kBlock) k_round_reserve(DevPtrs d, int cur) {
    const uint32_t n = d.cnt->n_act[cur];
    for (uint32_t i = grid_tid(); i < n; i += grid_threads()) {
        const uint32_t ci = d.act[cur][i];
        const unsigned long long key = d.key[ci];
        const uint32_t e0 = d.mem_off[ci], e1 = e0 + d.cand[ci].n;
        for (uint32_t e = e0; e < e1; ++e) {
            const uint32_t k = d.members[e];
            if (!d.used[k]) atomicMin(&d.owner[k], key);
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_round_decide(DevPtrs d, Params P, int cur) {
    const uint32_t n = d.cnt->n_act[cur];
    if (grid_tid() == 0 && n > 0) d.cnt->rounds += 1;
    for (uint32_t i = grid_tid(); i < n; i += grid_threads()) {
        const uint32_t ci = d.act[cur][i];
        const unsigned long long key = d.key[ci];
        const uint32_t e0 = d.mem_off[ci], e1 = e0 + d.cand[ci].n;
        uint32_t unused = 0;
        bool owns = true;
        for (uint32_t e = e0; e < e1; ++e) {
            const uint32_t k = d.members[e];
            if (!d.used[k]) {
                ++unused;
                owns = owns && d.owner[k] == key;
            }
        }
        if (unused < (uint32_t)P.n_min) {
            d.status[ci] = kRejected;
        } else if (owns) {
            d.status[ci] = kAccepted;
            d.mcount[ci] = unused;
            for (uint32_t e = e0; e < e1; ++e) {
                const uint32_t k = d.members[e];
                if (!d.used[k]) {
                    d.used[k] = 1;
                    d.taken[e] = 1;
                }
            }
        } else {
            const uint32_t slot = atomicAdd(&d.cnt->n_act[cur ^ 1], 1u);
            d.act[cur ^ 1][slot] = ci;
        }
    }
}

// ------------------------------------------------------------------- fit

__global__ void __launch_bounds__(kBlock) k_collect(DevPtrs d, Caps c) {
    const Counters *cn = d.cnt;
    const uint32_t nc = cn->err ? 0u : min(cn->n_cand, c.cand_cap);
    for (uint32_t i = grid_tid(); i < nc; i += grid_threads()) {
        if (d.status[i] == kAccepted) {
            const uint32_t slot = atomicAdd(&d.cnt->n_acc, 1u);
            d.acc[slot] = i;
            atomicAdd(&d.view_ntr[d.cand[i].v], 1u);
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_view_offsets(DevPtrs d, uint32_t n_views) {
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

__global__ void __launch_bounds__(kBlock) k_group(DevPtrs d, unsigned long long *gkey) {
    const uint32_t na = d.cnt->n_acc;
    for (uint32_t a = grid_tid(); a < na; a += grid_threads()) {
        const uint32_t ci = d.acc[a];
        const uint32_t v = d.cand[ci].v;
        const uint32_t pos = d.view_tr_off[v] + atomicAdd(&d.view_cursor[v], 1u);
        d.grouped[pos] = ci;
        gkey[pos] = d.key[ci];
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

        // 3. grain order by (t, input index), rank by counting
        for (uint32_t q = lane; q < m; q += 64) {
            const long long tq = d.tvals[base + q];
            const uint32_t kq = d.tord[base + q];
            const int oq = d.sg[kq].w;
            uint32_t rank = 0;
            for (uint32_t o = 0; o < m; ++o) {
                const long long to = d.tvals[base + o];
                if (to < tq) {
                    ++rank;
                } else if (to == tq && o != q) {
                    rank += d.sg[d.tord[base + o]].w < oq ? 1u : 0u;
                }
            }
            d.out_grains[base + rank] = (uint32_t)oq;
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
        if (Q[a][a] == 0) {
            degen = 1;
            const int ad[3] = {dx, dy, dz};
            a = 0;
            if (abs(ad[1]) > abs(ad[a])) a = 1;
            if (abs(ad[2]) > abs(ad[a])) a = 2;
            b = a == 0 ? 1 : 0;
            cx = a == 2 ? 1 : 2;
            slope[0] = (float)ad[b] / (float)ad[a];
            slope[1] = (float)ad[cx] / (float)ad[a];
            for (int u = 0; u < 3; ++u) comp_sign[u] = ad[u] > 0 ? 1 : (ad[u] < 0 ? -1 : 0);
        } else {
            fp64 = (a == 2) || (Q[a][a] < (__int128)250000 * n * n) ||
                   (P.flags & EMT_F_FP64_FIT_ALWAYS) != 0;
            if (fp64) {
                const double qa = i128_to_f64(Q[a][a]);
                slope[0] = (float)(i128_to_f64(Q[a][b]) / qa);
                slope[1] = (float)(i128_to_f64(Q[a][cx]) / qa);
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
                // fp64 is only set for a non-degenerate fit
                const double qa = i128_to_f64(Q[a][a]);
                const double s0d = i128_to_f64(Q[a][b]) / qa;
                const double s1d = i128_to_f64(Q[a][cx]) / qa;
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

uint32_t blocks_for(unsigned long long n, uint32_t max_blocks) {
    unsigned long long b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (uint32_t)(b < max_blocks ? b : max_blocks);
}

constexpr uint32_t kPersistentBlocks = 2048;  // 8 blocks of 4 waves per CU on 256 CUs

}  // namespace

size_t scan_scratch_words(uint32_t n_cap) { return (size_t)n_cap / kScanTile + 2; }

void launch_prepare(const DevPtrs &d, const Caps &c, const Params &, hipStream_t s) {
    k_zero<<<blocks_for(c.n_cells, 1024), kBlock, 0, s>>>(d.cnt, d.view_seeds, d.view_cand,
                                                          d.view_ntr, d.view_cursor, c.n_views,
                                                          d.cell_count, c.n_cells);
}

void launch_bin(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    const uint32_t bx = blocks_for(c.max_view_n, 64);
    dim3 grid(bx, c.n_views);
    k_bbox<<<grid, kBlock, 0, s>>>(d.xyz, d.grids, d.view_of);
    k_grid<<<(c.n_views + 63) / 64, 64, 0, s>>>(d.grids, c.n_views, P);
    k_hist<<<grid, kBlock, 0, s>>>(d.xyz, d.grids, d.cell_of, d.rank, d.cell_count);
    scan_excl(d.cell_count, nullptr, c.n_cells - 1, d.scan_part, d.cell_start, nullptr, s);
    k_scatter<<<grid, kBlock, 0, s>>>(d.xyz, d.grids, d.cell_of, d.rank, d.cell_start, d.sg);
}

void launch_seeds(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    k_seeds<<<blocks_for(c.n_total, kPersistentBlocks), kBlock, 0, s>>>(d, c, P);
}

void launch_count(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    k_count<<<blocks_for(c.seed_cap, kPersistentBlocks), kBlock, 0, s>>>(d, c, P);
}

void launch_members(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    k_cand_n<<<blocks_for(c.cand_cap, 1024), kBlock, 0, s>>>(d, c);
    scan_excl(d.cand_n, &d.cnt->n_cand, c.cand_cap, d.scan_part, d.mem_off, &d.cnt->n_members, s);
    k_members<<<blocks_for(c.cand_cap, kPersistentBlocks), kBlock, 0, s>>>(d, c, P);
}

void launch_merge_init(const DevPtrs &d, const Caps &c, const Params &, hipStream_t s) {
    unsigned long long n = c.cand_cap;
    if (c.n_total > n) n = c.n_total;
    if (c.mem_cap > n) n = c.mem_cap;
    k_merge_init<<<blocks_for(n, kPersistentBlocks), kBlock, 0, s>>>(d, c);
}

void launch_merge_round(const DevPtrs &d, const Caps &c, const Params &P, int round,
                        hipStream_t s) {
    const int cur = round & 1;
    const uint32_t nb = blocks_for(c.cand_cap, kPersistentBlocks);
    k_round_reset<<<nb, kBlock, 0, s>>>(d, cur);
    k_round_reserve<<<nb, kBlock, 0, s>>>(d, cur);
    k_round_decide<<<nb, kBlock, 0, s>>>(d, P, cur);
}

void launch_fit(const DevPtrs &d, const Caps &c, const Params &P, hipStream_t s) {
    const uint32_t nb = blocks_for(c.cand_cap, kPersistentBlocks);
    k_collect<<<nb, kBlock, 0, s>>>(d, c);
    k_view_offsets<<<1, kBlock, 0, s>>>(d, c.n_views);
    // keys of the grouped tracks reuse the owner array (merge is over)
    unsigned long long *gkey = d.owner;
    k_group<<<nb, kBlock, 0, s>>>(d, gkey);
    k_rank<<<nb, kBlock, 0, s>>>(d, gkey);
    scan_excl(d.tg_n, &d.cnt->n_acc, c.cand_cap, d.scan_part, d.tg_off, &d.cnt->n_track_grains, s);
    k_fit<<<nb, kBlock, 0, s>>>(d, P);
}

}  // namespace emt
