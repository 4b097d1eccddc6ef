/*
 * emt_oracle.c -- CPU oracle of the per-view 4pi track finding.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path. Plain C, one
 * thread, written for reading, not speed.
 *
 * Every step follows the tracking paragraph of paper Sec. 2 (and Fig. 4):
 *   (1) a seed is any grain pair closer than 25 um, at any angle;
 *   (2) the line through the two seed grains is formed and the grains along
 *       it are counted;
 *   (3) a seed whose count passes a preset threshold is a track candidate;
 *   (4) each grain is then associated with one track only and the threshold
 *       is applied once more, which suppresses duplicate tracks.
 * Sec. 3 (footnote) adds that grains are first put into 3D cells so that
 * later steps look only at relevant cells; mode scan_all=0 does that, mode
 * scan_all=1 looks at every grain, and both give the same answer.
 * The least-squares fit of step (5) is not in the paper; it gives each
 * accepted track a direction (the paper reports directions as unit-vector
 * components in Sec. 3) and its start and end along it.
 */
#include "emt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define SPAN_MAX (1 << 18)  /* largest per-axis coordinate span (units) */
#define N_MAX (1u << 20)    /* grains per view must stay below this     */
#define R_MAX 4096          /* largest seed distance (units)            */

typedef struct {
    int64_t org[3];
    int64_t cell[3];
    int64_t dims[3];
    uint32_t *start; /* dims0*dims1*dims2 + 1 offsets */
    uint32_t *item;  /* input indices, increasing within a cell */
} grid_t;

static int64_t floordiv(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

static int64_t cell_id(const grid_t *G, int64_t cx, int64_t cy, int64_t cz) {
    return (cz * G->dims[1] + cy) * G->dims[0] + cx;
}

static int64_t axis_cell(const grid_t *G, int m, int64_t v) {
    return floordiv(v - G->org[m], G->cell[m]);
}

/* Hash cells (Sec. 3 footnote): a uniform grid over the bounding box of the
 * view, each grain in exactly one cell; a cell lists its grains in input
 * order (a stable counting sort). */
static int grid_build(grid_t *G, const int32_t *xyz, uint32_t n,
                      const int32_t cell[3]) {
    int64_t lo[3], hi[3];
    for (int m = 0; m < 3; m++) {
        lo[m] = n ? xyz[m] : 0;
        hi[m] = lo[m];
    }
    for (uint32_t k = 0; k < n; k++)
        for (int m = 0; m < 3; m++) {
            int64_t v = xyz[3 * (size_t)k + m];
            if (v < lo[m]) lo[m] = v;
            if (v > hi[m]) hi[m] = v;
        }
    for (int m = 0; m < 3; m++) {
        G->org[m] = lo[m];
        G->cell[m] = cell[m] > 0 ? cell[m] : 750;
    }
    /* Keep the table modest: widen cells until it has at most 4N+4096 of
     * them. Cell size never changes a result, only the work. */
    for (;;) {
        int64_t tot = 1;
        for (int m = 0; m < 3; m++) {
            G->dims[m] = (hi[m] - lo[m]) / G->cell[m] + 1;
            tot *= G->dims[m];
        }
        if (tot <= 4 * (int64_t)n + 4096) break;
        for (int m = 0; m < 3; m++) G->cell[m] *= 2;
    }
    int64_t nc = G->dims[0] * G->dims[1] * G->dims[2];
    G->start = (uint32_t *)calloc((size_t)nc + 1, sizeof(uint32_t));
    G->item = (uint32_t *)malloc(((size_t)n + 1) * sizeof(uint32_t));
    if (!G->start || !G->item) return EMTO_ENOMEM;
    for (uint32_t k = 0; k < n; k++) {
        const int32_t *g = xyz + 3 * (size_t)k;
        int64_t c = cell_id(G, axis_cell(G, 0, g[0]), axis_cell(G, 1, g[1]),
                            axis_cell(G, 2, g[2]));
        G->start[c + 1]++;
    }
    for (int64_t c = 0; c < nc; c++) G->start[c + 1] += G->start[c];
    uint32_t *fill = (uint32_t *)malloc((size_t)(nc + 1) * sizeof(uint32_t));
    if (!fill) return EMTO_ENOMEM;
    memcpy(fill, G->start, (size_t)(nc + 1) * sizeof(uint32_t));
    for (uint32_t k = 0; k < n; k++) {
        const int32_t *g = xyz + 3 * (size_t)k;
        int64_t c = cell_id(G, axis_cell(G, 0, g[0]), axis_cell(G, 1, g[1]),
                            axis_cell(G, 2, g[2]));
        G->item[fill[c]++] = k;
    }
    free(fill);
    return EMTO_OK;
}

static void grid_free(grid_t *G) {
    free(G->start);
    free(G->item);
}

/* The cylinder predicate of step (2): with d = g_j - g_i and w = g_k - g_i,
 * grain k lies within r of the (infinite) line iff |w x d|^2 <= r^2 |d|^2.
 * The radius is inclusive. Exact in int64 under the span and R limits.
 *
 * Acceptance variant (finite cylinder), ext >= 0: grain k must also project
 * onto the line no further than ext beyond either seed grain, i.e. with
 * t = w.d, -ext |d| <= t <= |d|^2 + ext |d|. Both sides are compared
 * squared where they are negative: t >= -ext |d| holds if t >= 0, else iff
 * t^2 <= ext^2 |d|^2; likewise for t - |d|^2 <= ext |d|. (|t| < 2^31 and
 * ext^2 |d|^2 < 2^59, so int64 is exact.) */
static int on_line(const int32_t *xyz, uint32_t i, const int64_t d[3],
                   int64_t r2D, int64_t ext, uint32_t k) {
    const int32_t *gi = xyz + 3 * (size_t)i, *gk = xyz + 3 * (size_t)k;
    int64_t w0 = (int64_t)gk[0] - gi[0];
    int64_t w1 = (int64_t)gk[1] - gi[1];
    int64_t w2 = (int64_t)gk[2] - gi[2];
    int64_t c0 = w1 * d[2] - w2 * d[1];
    int64_t c1 = w2 * d[0] - w0 * d[2];
    int64_t c2 = w0 * d[1] - w1 * d[0];
    if (c0 * c0 + c1 * c1 + c2 * c2 > r2D) return 0;
    if (ext < 0) return 1;
    int64_t D = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    int64_t t = w0 * d[0] + w1 * d[1] + w2 * d[2];
    int64_t e2D = ext * ext * D;
    if (t < 0 && t * t > e2D) return 0;
    if (t > D && (t - D) * (t - D) > e2D) return 0;
    return 1;
}

/* Acceptance variant (grain-count threshold rising with the angle; paper
 * Sec. 3: a cut on the number of grains along a line in the plane of grain
 * count against track angle, Fig. 8c). For seed direction d, with
 * tan(theta) = sqrt(d_x^2 + d_y^2) / |d_z| and b = thr_num / thr_den, the
 * threshold is the smallest integer m >= n_min with m - n_min >= b tan(theta),
 * capped at thr_max (if set). Tested exactly, squared in 128-bit integers:
 * ((m - n_min) |d_z| thr_den)^2 >= thr_num^2 (d_x^2 + d_y^2); the smallest
 * such m is found by bisection (the test is monotone in m). A seed with
 * d_z = 0 gets the cap (no cap: no count suffices). */
static uint32_t seed_threshold(const int64_t d[3], const emto_params *p) {
    const uint32_t n_min = (uint32_t)p->min_grains;
    if (p->thr_num == 0) return n_min;
    const uint32_t cap = p->thr_max > 0 ? (uint32_t)p->thr_max : UINT32_MAX;
    const int64_t adz = d[2] < 0 ? -d[2] : d[2];
    if (adz == 0) return cap;
    const unsigned __int128 rhs = (unsigned __int128)((int64_t)p->thr_num * p->thr_num) *
                                  (unsigned __int128)(d[0] * d[0] + d[1] * d[1]);
    /* m - n_min never needs more than thr_num * |d| < 2^24 */
    uint64_t lo = 0, hi = (uint64_t)1 << 24;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        unsigned __int128 l = (unsigned __int128)(mid * (uint64_t)adz * (uint64_t)p->thr_den);
        if (l * l >= rhs)
            hi = mid;
        else
            lo = mid + 1;
    }
    uint64_t m = (uint64_t)n_min + lo;
    return m < cap ? (uint32_t)m : cap;
}

/* Count (and optionally list) the grains on the line of seed (i, j).
 *
 * scan_all: test every grain of the view -- the definition itself.
 *
 * Cells: let a be the axis of largest |d_a| and b, c the other two. Walk the
 * cell layers along a. A grain k in a layer has a_k in [A0, A1]. Let p(a_k)
 * be the line point with the same a coordinate; v = g_k - p(a_k) has v_a = 0,
 * so |v x d|^2 = |v|^2 |d|^2 - (v.d)^2 >= |v|^2 d_a^2 (Cauchy-Schwarz on the
 * b, c parts). A grain within r of the line therefore has
 * |v_b|, |v_c| <= r |d| / |d_a|. Since p is linear in a, p_b over [A0, A1]
 * lies between p_b(A0) and p_b(A1). So every such grain sits in a cell whose
 * b (and c) range meets [min p_b - rho, max p_b + rho], rho = r|d|/|d_a|.
 * Those cells are visited and the exact predicate decides; the double
 * arithmetic here only chooses cells and gets a 1-unit safety margin. */
static uint32_t count_seed(const grid_t *G, const int32_t *xyz, uint32_t n,
                           uint32_t i, uint32_t j, int64_t r, int64_t ext,
                           int scan_all, uint64_t *tests, uint32_t *list) {
    const int32_t *gi = xyz + 3 * (size_t)i, *gj = xyz + 3 * (size_t)j;
    int64_t d[3] = {(int64_t)gj[0] - gi[0], (int64_t)gj[1] - gi[1],
                    (int64_t)gj[2] - gi[2]};
    int64_t D = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    int64_t r2D = r * r * D;
    uint32_t cnt = 0;
    if (scan_all || !G) {
        for (uint32_t k = 0; k < n; k++) {
            if (on_line(xyz, i, d, r2D, ext, k)) {
                if (list) list[cnt] = k;
                cnt++;
            }
        }
        if (tests) *tests += n;
        return cnt;
    }
    int a = 0;
    for (int m = 1; m < 3; m++)
        if (llabs(d[m]) > llabs(d[a])) a = m;
    int ax[2], q = 0;
    for (int m = 0; m < 3; m++)
        if (m != a) ax[q++] = m;
    double rho = (double)r * sqrt((double)D) / fabs((double)d[a]) + 1.0;
    for (int64_t ia = 0; ia < G->dims[a]; ia++) {
        int64_t A0 = G->org[a] + ia * G->cell[a];
        int64_t A1 = A0 + G->cell[a] - 1;
        int64_t lo_c[2], hi_c[2];
        int empty = 0;
        for (int e = 0; e < 2; e++) {
            int b = ax[e];
            double s = (double)d[b] / (double)d[a];
            double p0 = (double)gi[b] + (double)(A0 - gi[a]) * s;
            double p1 = (double)gi[b] + (double)(A1 - gi[a]) * s;
            double lo = (p0 < p1 ? p0 : p1) - rho;
            double hi = (p0 < p1 ? p1 : p0) + rho;
            double clo = floor((lo - (double)G->org[b]) / (double)G->cell[b]);
            double chi = floor((hi - (double)G->org[b]) / (double)G->cell[b]);
            if (chi < 0.0 || clo > (double)(G->dims[b] - 1)) {
                empty = 1;
                break;
            }
            lo_c[e] = clo < 0.0 ? 0 : (int64_t)clo;
            hi_c[e] = chi > (double)(G->dims[b] - 1) ? G->dims[b] - 1
                                                     : (int64_t)chi;
        }
        if (empty) continue;
        for (int64_t u = lo_c[0]; u <= hi_c[0]; u++) {
            for (int64_t v = lo_c[1]; v <= hi_c[1]; v++) {
                int64_t c3[3];
                c3[a] = ia;
                c3[ax[0]] = u;
                c3[ax[1]] = v;
                int64_t cid = cell_id(G, c3[0], c3[1], c3[2]);
                for (uint32_t t = G->start[cid]; t < G->start[cid + 1]; t++) {
                    uint32_t k = G->item[t];
                    if (tests) (*tests)++;
                    if (on_line(xyz, i, d, r2D, ext, k)) {
                        if (list) list[cnt] = k;
                        cnt++;
                    }
                }
            }
        }
    }
    return cnt;
}

uint32_t emto_count_seed(const int32_t *xyz, uint32_t n, uint32_t i,
                         uint32_t j, int64_t r) {
    if (!xyz || i >= n || j >= n) return 0;
    const int32_t *gi = xyz + 3 * (size_t)i, *gj = xyz + 3 * (size_t)j;
    if (gi[0] == gj[0] && gi[1] == gj[1] && gi[2] == gj[2]) return 0;
    return count_seed(NULL, xyz, n, i, j, r, -1, 1, NULL, NULL);
}

/* Priority of step (4): the paper fixes no order for the exclusive
 * association. Reading: best first, by grain count (descending), ties by the
 * seed's input indices i then j (ascending). */
static int cand_cmp(const void *pa, const void *pb) {
    const emto_cand *a = (const emto_cand *)pa, *b = (const emto_cand *)pb;
    if (a->n != b->n) return a->n > b->n ? -1 : 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    return 0;
}

typedef struct {
    int64_t t;
    uint32_t k;
} tk_t;

static int tk_cmp(const void *pa, const void *pb) {
    const tk_t *a = (const tk_t *)pa, *b = (const tk_t *)pb;
    if (a->t != b->t) return a->t < b->t ? -1 : 1;
    if (a->k != b->k) return a->k < b->k ? -1 : 1;
    return 0;
}

typedef __int128 i128;

/* Step (5), least squares in FP64 over the associated grains M:
 * the fit axis a is the one of largest spread, decided on exact integer
 * second moments Q_mm' = n sum(w_m w_m') - sum(w_m) sum(w_m') with
 * w = g_k - g_i (ties to the lower axis); the two slopes are the regression
 * coefficients of the other coordinates on a, Q_ab/Q_aa and Q_ac/Q_aa,
 * computed here from two-pass centred sums in double. The direction
 * (1, s_b, s_c) placed on axes (a, b, c) is normalised and turned into the
 * upper hemisphere (z > 0, else y > 0, else x > 0); the sign test uses the
 * exact integers. */
static void fit_track(const int32_t *xyz, uint32_t i, uint32_t j,
                      const uint32_t *m, uint32_t nm, emto_track *T) {
    const int32_t *gi = xyz + 3 * (size_t)i;
    i128 S1[3] = {0, 0, 0}, S2[3][3];
    memset(S2, 0, sizeof(S2));
    double mean[3] = {0, 0, 0};
    for (uint32_t q = 0; q < nm; q++) {
        const int32_t *g = xyz + 3 * (size_t)m[q];
        int64_t w[3] = {(int64_t)g[0] - gi[0], (int64_t)g[1] - gi[1],
                        (int64_t)g[2] - gi[2]};
        for (int u = 0; u < 3; u++) {
            S1[u] += w[u];
            mean[u] += (double)g[u];
            for (int v = 0; v < 3; v++) S2[u][v] += (i128)w[u] * w[v];
        }
    }
    for (int u = 0; u < 3; u++) mean[u] /= (double)nm;
    i128 Q[3][3];
    for (int u = 0; u < 3; u++)
        for (int v = 0; v < 3; v++) Q[u][v] = (i128)nm * S2[u][v] - S1[u] * S1[v];
    double C[3][3];
    for (int u = 0; u < 3; u++)
        for (int v = 0; v < 3; v++) C[u][v] = 0.0;
    for (uint32_t q = 0; q < nm; q++) {
        const int32_t *g = xyz + 3 * (size_t)m[q];
        double e[3] = {(double)g[0] - mean[0], (double)g[1] - mean[1],
                       (double)g[2] - mean[2]};
        for (int u = 0; u < 3; u++)
            for (int v = 0; v < 3; v++) C[u][v] += e[u] * e[v];
    }
    int a = 0;
    for (int u = 1; u < 3; u++)
        if (Q[u][u] > Q[a][a]) a = u;
    int b = (a == 0) ? 1 : 0;
    int c = (a == 2) ? 1 : 2;
    double dir[3];
    i128 comp[3];
    T->degenerate = 0;
    if (Q[a][a] == 0) {
        /* All associated grains coincide: no spread to fit, so take the
         * seed direction. */
        const int32_t *gj = xyz + 3 * (size_t)j;
        int64_t d[3] = {(int64_t)gj[0] - gi[0], (int64_t)gj[1] - gi[1],
                        (int64_t)gj[2] - gi[2]};
        a = 0;
        for (int u = 1; u < 3; u++)
            if (llabs(d[u]) > llabs(d[a])) a = u;
        b = (a == 0) ? 1 : 0;
        c = (a == 2) ? 1 : 2;
        T->slope[0] = (double)d[b] / (double)d[a];
        T->slope[1] = (double)d[c] / (double)d[a];
        /* (1, slope0, slope1) on axes (a, b, c) is d / d_a: its signs are
         * those of d times the sign of d_a */
        for (int u = 0; u < 3; u++) comp[u] = d[a] < 0 ? -d[u] : d[u];
        T->degenerate = 1;
    } else {
        T->slope[0] = C[a][b] / C[a][a];
        T->slope[1] = C[a][c] / C[a][a];
        comp[a] = Q[a][a];
        comp[b] = Q[a][b];
        comp[c] = Q[a][c];
    }
    dir[a] = 1.0;
    dir[b] = T->slope[0];
    dir[c] = T->slope[1];
    double nrm = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    int flip;
    if (comp[2] != 0) flip = comp[2] < 0;
    else if (comp[1] != 0) flip = comp[1] < 0;
    else flip = comp[0] < 0;
    for (int u = 0; u < 3; u++) T->dir[u] = (flip ? -dir[u] : dir[u]) / nrm;
    T->axis = (uint32_t)a;
    /* FP64 on the device: near-vertical fits (a = z) and short tracks whose
     * RMS spread along a is under 5 um, i.e. Q_aa < (500 units)^2 n^2. */
    T->fit_fp64 = (a == 2) || (Q[a][a] < (i128)250000 * nm * nm);
    double tmin = 0.0, tmax = 0.0;
    for (uint32_t q = 0; q < nm; q++) {
        const int32_t *g = xyz + 3 * (size_t)m[q];
        double t = 0.0;
        for (int u = 0; u < 3; u++) t += ((double)g[u] - mean[u]) * T->dir[u];
        if (q == 0 || t < tmin) tmin = t;
        if (q == 0 || t > tmax) tmax = t;
    }
    for (int u = 0; u < 3; u++) T->centroid[u] = mean[u] / 100.0;
    T->t_begin = tmin / 100.0;
    T->t_end = tmax / 100.0;
}

int emto_track_view(const int32_t *xyz, uint32_t n, const emto_params *p,
                    emto_result *out) {
    if (!p || !out || (n && !xyz)) return EMTO_EINVAL;
    memset(out, 0, sizeof(*out));
    if (p->seed_dist < 1 || p->seed_dist > R_MAX || p->tol_radius < 0 ||
        p->tol_radius >= p->seed_dist || p->min_grains < 2 ||
        (uint32_t)p->min_grains >= N_MAX)
        return EMTO_ERANGE;
    if (p->cyl_ext < -1 || p->cyl_ext > SPAN_MAX || p->thr_num < 0 || p->thr_num > 1024 ||
        p->thr_den < 1 || p->thr_den > 1024 || p->thr_max < 0 ||
        (p->thr_max > 0 && (p->thr_max < p->min_grains || (uint32_t)p->thr_max >= N_MAX)))
        return EMTO_ERANGE;
    if (n >= N_MAX) return EMTO_ERANGE;
    if (n) {
        for (int m = 0; m < 3; m++) {
            int64_t lo = xyz[m], hi = xyz[m];
            for (uint32_t k = 1; k < n; k++) {
                int64_t v = xyz[3 * (size_t)k + m];
                if (v < lo) lo = v;
                if (v > hi) hi = v;
            }
            if (hi - lo > SPAN_MAX) return EMTO_ERANGE;
        }
    }
    const int64_t R = p->seed_dist, r = p->tol_radius;
    const int64_t R2 = R * R;
    grid_t G;
    memset(&G, 0, sizeof(G));
    int rc = grid_build(&G, xyz, n, p->cell);
    if (rc) {
        grid_free(&G);
        return rc;
    }

    /* Steps (1)-(3): every pair i < j with 0 < D < R^2 (strict: the paper
     * says closer than 25 um; coincident grains define no line) is a seed;
     * count its line and keep it if the count reaches n_min. The pair box
     * [g_i - (R-1), g_i + (R-1)] holds every partner closer than R. */
    size_t cap = 1024;
    emto_cand *cand = (emto_cand *)malloc(cap * sizeof(emto_cand));
    if (!cand) {
        grid_free(&G);
        return EMTO_ENOMEM;
    }
    uint32_t ncand = 0;
    uint64_t nseeds = 0, ntests = 0;
    for (uint32_t i = 0; i < n; i++) {
        const int32_t *gi = xyz + 3 * (size_t)i;
        int64_t lo[3], hi[3];
        for (int m = 0; m < 3; m++) {
            lo[m] = axis_cell(&G, m, gi[m] - (R - 1));
            hi[m] = axis_cell(&G, m, gi[m] + (R - 1));
            if (lo[m] < 0) lo[m] = 0;
            if (hi[m] > G.dims[m] - 1) hi[m] = G.dims[m] - 1;
        }
        for (int64_t cz = lo[2]; cz <= hi[2]; cz++)
            for (int64_t cy = lo[1]; cy <= hi[1]; cy++)
                for (int64_t cx = lo[0]; cx <= hi[0]; cx++) {
                    int64_t cid = cell_id(&G, cx, cy, cz);
                    for (uint32_t t = G.start[cid]; t < G.start[cid + 1]; t++) {
                        uint32_t j = G.item[t];
                        if (j <= i) continue;
                        const int32_t *gj = xyz + 3 * (size_t)j;
                        int64_t d0 = (int64_t)gj[0] - gi[0];
                        int64_t d1 = (int64_t)gj[1] - gi[1];
                        int64_t d2 = (int64_t)gj[2] - gi[2];
                        int64_t D = d0 * d0 + d1 * d1 + d2 * d2;
                        if (D <= 0 || D >= R2) continue;
                        nseeds++;
                        uint32_t cnt = count_seed(&G, xyz, n, i, j, r, p->cyl_ext,
                                                  p->scan_all, &ntests, NULL);
                        const int64_t dd[3] = {d0, d1, d2};
                        if (cnt >= seed_threshold(dd, p)) {
                            if (ncand == cap) {
                                cap *= 2;
                                emto_cand *nc = (emto_cand *)realloc(
                                    cand, cap * sizeof(emto_cand));
                                if (!nc) {
                                    free(cand);
                                    grid_free(&G);
                                    return EMTO_ENOMEM;
                                }
                                cand = nc;
                            }
                            cand[ncand].i = i;
                            cand[ncand].j = j;
                            cand[ncand].n = cnt;
                            ncand++;
                        }
                    }
                }
    }
    qsort(cand, ncand, sizeof(emto_cand), cand_cmp);

    /* Step (4): exclusive association in priority order. A candidate keeps
     * the grains of its line not yet taken by an earlier track; with at
     * least n_min of them it becomes a track and takes them. A candidate
     * whose own seed grains were taken stays eligible. */
    unsigned char *used = (unsigned char *)calloc((size_t)n + 1, 1);
    uint32_t *members = (uint32_t *)malloc(((size_t)n + 1) * sizeof(uint32_t));
    tk_t *tk = (tk_t *)malloc(((size_t)n + 1) * sizeof(tk_t));
    size_t tcap = 64, gcap = 1024;
    emto_track *tracks = (emto_track *)malloc(tcap * sizeof(emto_track));
    uint32_t *grains = (uint32_t *)malloc(gcap * sizeof(uint32_t));
    if (!used || !members || !tk || !tracks || !grains) {
        free(used); free(members); free(tk); free(tracks); free(grains);
        free(cand);
        grid_free(&G);
        return EMTO_ENOMEM;
    }
    uint32_t ntr = 0, ngr = 0;
    for (uint32_t s = 0; s < ncand; s++) {
        uint32_t i = cand[s].i, j = cand[s].j;
        uint32_t cnt = count_seed(&G, xyz, n, i, j, r, p->cyl_ext, p->scan_all,
                                  NULL, members);
        uint32_t m = 0;
        for (uint32_t q = 0; q < cnt; q++)
            if (!used[members[q]]) members[m++] = members[q];
        {
            const int32_t *si = xyz + 3 * (size_t)i, *sj = xyz + 3 * (size_t)j;
            const int64_t sd[3] = {(int64_t)sj[0] - si[0], (int64_t)sj[1] - si[1],
                                   (int64_t)sj[2] - si[2]};
            if (m < seed_threshold(sd, p)) continue;
        }
        for (uint32_t q = 0; q < m; q++) used[members[q]] = 1;
        /* Track record: grains ordered along the seed direction by
         * t = (g_k - g_i).d, ties by input index. */
        const int32_t *gi = xyz + 3 * (size_t)i, *gj = xyz + 3 * (size_t)j;
        int64_t d[3] = {(int64_t)gj[0] - gi[0], (int64_t)gj[1] - gi[1],
                        (int64_t)gj[2] - gi[2]};
        for (uint32_t q = 0; q < m; q++) {
            const int32_t *g = xyz + 3 * (size_t)members[q];
            tk[q].t = ((int64_t)g[0] - gi[0]) * d[0] +
                      ((int64_t)g[1] - gi[1]) * d[1] +
                      ((int64_t)g[2] - gi[2]) * d[2];
            tk[q].k = members[q];
        }
        qsort(tk, m, sizeof(tk_t), tk_cmp);
        if (ntr == tcap) {
            tcap *= 2;
            emto_track *nt = (emto_track *)realloc(tracks, tcap * sizeof(emto_track));
            if (!nt) { rc = EMTO_ENOMEM; break; }
            tracks = nt;
        }
        while ((size_t)ngr + m > gcap) {
            gcap *= 2;
            uint32_t *ng = (uint32_t *)realloc(grains, gcap * sizeof(uint32_t));
            if (!ng) { rc = EMTO_ENOMEM; break; }
            grains = ng;
        }
        if (rc) break;
        for (uint32_t q = 0; q < m; q++) {
            members[q] = tk[q].k;
            grains[ngr + q] = tk[q].k;
        }
        emto_track *T = &tracks[ntr];
        memset(T, 0, sizeof(*T));
        T->i = i;
        T->j = j;
        T->grain_offset = ngr;
        T->n_grains = m;
        fit_track(xyz, i, j, members, m, T);
        ntr++;
        ngr += m;
    }
    free(used);
    free(members);
    free(tk);
    grid_free(&G);
    if (rc) {
        free(cand); free(tracks); free(grains);
        return rc;
    }
    out->n_seeds = nseeds;
    out->n_tests = ntests;
    out->n_cand = ncand;
    out->cand = cand;
    out->n_tracks = ntr;
    out->tracks = tracks;
    out->n_track_grains = ngr;
    out->grains = grains;
    return EMTO_OK;
}

void emto_free(emto_result *r) {
    if (!r) return;
    free(r->cand);
    free(r->tracks);
    free(r->grains);
    memset(r, 0, sizeof(*r));
}
