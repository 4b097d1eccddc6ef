/*
 * emt_oracle.h -- CPU oracle of the per-view 4pi track finding.
 *
 * TEST INFRASTRUCTURE ONLY. This is the slow, single-threaded reference
 * against which the GPU library is checked. Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never calls it and shares no code, header or table with it.
 *
 * Method (paper Sec. 2, tracking paragraph and Fig. 4; hash cells from the
 * Sec. 3 footnote):
 *   seeds      every grain pair closer than R, any direction (Fig. 4a)
 *   count      grains within r of the infinite line through the pair (Fig. 4b)
 *              (variant: of a finite cylinder around the pair)
 *   threshold  keep seeds with at least n_min grains (variant: a threshold
 *              rising with the seed's angle to the z axis, Sec. 3, Fig. 8c)
 *   associate  each grain used by one track only, then the threshold again
 *   fit        least-squares direction of each accepted track (FP64)
 *
 * All geometry is exact integer arithmetic on int32 coordinates in 0.01 um
 * units. Readings of points the paper leaves open (infinite line, inclusive
 * radius, strict seed distance, greedy order by grain count then input
 * indices, ...) are stated next to the code that takes them.
 */
#ifndef EMT_ORACLE_H
#define EMT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EMTO_OK 0
#define EMTO_EINVAL (-1)
#define EMTO_ERANGE (-2)
#define EMTO_ENOMEM (-3)

typedef struct {
    int64_t seed_dist;  /* R: a seed needs 0 < |g_j - g_i|^2 < R^2 (units)        */
    int64_t tol_radius; /* r: grain on the line iff |w x d|^2 <= r^2 |d|^2 (units) */
    int32_t min_grains; /* n_min: threshold on the grain count (also re-applied)   */
    int32_t scan_all;   /* 1: count every seed over all N grains (the definition);
                           0: visit only the hash cells the cylinder can reach     */
    int32_t cell[3];    /* hash cell edge per axis in units (acceleration only)    */
    int32_t thr_num;    /* acceptance variant: a seed needs n_min + ceil(b tan th)  */
    int32_t thr_den;    /*   grains, b = thr_num / thr_den (thr_num 0: n_min)       */
    int32_t thr_max;    /*   that threshold capped at thr_max (0: no cap)          */
    int64_t cyl_ext;    /* -1: infinite line; >= 0: finite cylinder, grains whose
                           projection lies at most cyl_ext units beyond a seed
                           grain along the line                                   */
} emto_params;

typedef struct {
    uint32_t i, j; /* seed grains as input indices, i < j */
    uint32_t n;    /* number of grains within r of the seed line */
} emto_cand;

typedef struct {
    uint32_t i, j;          /* seed of the accepted candidate               */
    uint32_t grain_offset;  /* into emto_result.grains                      */
    uint32_t n_grains;      /* grains exclusively associated to this track  */
    uint32_t axis;          /* 0,1,2 = x,y,z: axis of largest spread        */
    uint32_t fit_fp64;      /* 1 if axis == z or RMS spread along it < 5 um */
    uint32_t degenerate;    /* 1 if all associated grains coincide          */
    double slope[2];        /* d(b)/d(a), d(c)/d(a); b < c the other axes   */
    double dir[3];          /* unit direction, upper hemisphere             */
    double centroid[3];     /* um                                           */
    double t_begin, t_end;  /* um, extent along dir about the centroid      */
} emto_track;

typedef struct {
    uint64_t n_seeds;
    uint64_t n_tests;        /* grains examined while counting (diagnostic) */
    uint32_t n_cand;
    emto_cand *cand;         /* priority order: n desc, i asc, j asc       */
    uint32_t n_tracks;
    emto_track *tracks;      /* acceptance order                           */
    uint32_t n_track_grains;
    uint32_t *grains;        /* input indices, per track ordered by (t, k) */
} emto_result;

int emto_track_view(const int32_t *xyz, uint32_t n, const emto_params *p,
                    emto_result *out);
void emto_free(emto_result *r);

/* Number of grains within r of the line through grains i and j, over all N
 * grains (the counting definition, no cells). Returns 0 if g_i == g_j. */
uint32_t emto_count_seed(const int32_t *xyz, uint32_t n, uint32_t i,
                         uint32_t j, int64_t r);

#ifdef __cplusplus
}
#endif
#endif
