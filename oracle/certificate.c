/* Max-distortion certificate by direct differences (oracle, FP64, plain C).
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * benchmark's CPU baseline, never by the product library.
 *
 * Paper: eq. (2) defines the distortion of a pair as | ||f(x)-f(y)|| / ||x-y|| - 1 |
 * and eq. (3) the distortion of the embedding as its maximum over the cloud.
 * Readings: the maximum runs over unordered pairs i < j; pairs with x_i == x_j
 * (0/0 in eq. 2) are skipped and counted, since any linear map keeps them at
 * distance 0.  Ties are broken towards the smallest (i, j).
 *
 * Every pair is evaluated from the coordinates themselves:
 *   D^2 = sum_l (x_il - x_jl)^2,  E^2 = sum_m (y_im - y_jm)^2,
 *   distortion = | sqrt(E^2) / sqrt(D^2) - 1 |.
 * No Gram identity, blocking or reordering is used.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>

typedef struct {
    double best;          /* largest distortion                          */
    double second;        /* largest distortion over the other pairs     */
    int64_t bi, bj;       /* argmax pair, bi < bj (-1 when none)         */
    int64_t si, sj;       /* runner-up pair (-1 when none)               */
    int32_t bside;        /* +1 expansion, -1 contraction, 0 equal       */
    int32_t sside;
    int64_t nzero;        /* pairs skipped because x_i == x_j            */
    int64_t npairs;       /* pairs visited                               */
} oracle_cert;

typedef struct { double v; int64_t i, j; int32_t side; } rec;

static int better(const rec *a, const rec *b) {
    if (a->v != b->v) return a->v > b->v;
    if (a->i != b->i) return a->i < b->i;
    return a->j < b->j;
}

static void push(rec top[2], const rec *c) {
    if (better(c, &top[0])) { top[1] = top[0]; top[0] = *c; }
    else if (better(c, &top[1])) { top[1] = *c; }
}

static double pair_distortion(const double *X, const double *Y, int64_t d, int64_t r,
                              int64_t i, int64_t j, int32_t *side, int *zero) {
    const double *xi = X + i * d, *xj = X + j * d;
    const double *yi = Y + i * r, *yj = Y + j * r;
    double D2 = 0.0, E2 = 0.0;
    for (int64_t l = 0; l < d; ++l) { double t = xi[l] - xj[l]; D2 += t * t; }
    for (int64_t m = 0; m < r; ++m) { double t = yi[m] - yj[m]; E2 += t * t; }
    if (D2 == 0.0) { *zero = 1; *side = 0; return 0.0; }
    *zero = 0;
    double ratio = sqrt(E2) / sqrt(D2);
    *side = ratio > 1.0 ? 1 : (ratio < 1.0 ? -1 : 0);
    return fabs(ratio - 1.0);
}

/* Pairs (i, j) with i0 <= i < i1 and i < j < n.  X is n x d, Y is n x r,
 * both row-major FP64. */
void oracle_certificate(const double *X, const double *Y, int64_t n, int64_t d, int64_t r,
                        int64_t i0, int64_t i1, oracle_cert *out) {
    rec top[2] = {{-1.0, -1, -1, 0}, {-1.0, -1, -1, 0}};
    int64_t nzero = 0, npairs = 0;
    if (i1 > n) i1 = n;
#pragma omp parallel
    {
        rec loc[2] = {{-1.0, -1, -1, 0}, {-1.0, -1, -1, 0}};
        int64_t lz = 0, lp = 0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = i0; i < i1; ++i) {
            for (int64_t j = i + 1; j < n; ++j) {
                int32_t side; int zero;
                double v = pair_distortion(X, Y, d, r, i, j, &side, &zero);
                ++lp;
                if (zero) { ++lz; continue; }
                rec c = {v, i, j, side};
                push(loc, &c);
            }
        }
#pragma omp critical
        {
            push(top, &loc[0]);
            if (loc[1].i >= 0) push(top, &loc[1]);
            nzero += lz; npairs += lp;
        }
    }
    out->best = top[0].i >= 0 ? top[0].v : 0.0;
    out->bi = top[0].i; out->bj = top[0].j; out->bside = top[0].side;
    out->second = top[1].i >= 0 ? top[1].v : 0.0;
    out->si = top[1].i; out->sj = top[1].j; out->sside = top[1].side;
    out->nzero = nzero; out->npairs = npairs;
}

/* Pairs (IA[a], IB[b]) of two lists of row indices, counted when
 * IA[a] < IB[b] (a sample of the unordered pairs of eq. (3): row blocks
 * against row blocks, or one row against every other).  X and Y hold every
 * row of the cloud, as in oracle_certificate. */
void oracle_cross_certificate(const double *X, const double *Y, int64_t d, int64_t r,
                              const int64_t *IA, int64_t na, const int64_t *IB, int64_t nb,
                              oracle_cert *out) {
    rec top[2] = {{-1.0, -1, -1, 0}, {-1.0, -1, -1, 0}};
    int64_t nzero = 0, npairs = 0;
#pragma omp parallel
    {
        rec loc[2] = {{-1.0, -1, -1, 0}, {-1.0, -1, -1, 0}};
        int64_t lz = 0, lp = 0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t a = 0; a < na; ++a) {
            for (int64_t b = 0; b < nb; ++b) {
                int64_t i = IA[a], j = IB[b];
                if (i >= j) continue;
                int32_t side; int zero;
                double v = pair_distortion(X, Y, d, r, i, j, &side, &zero);
                ++lp;
                if (zero) { ++lz; continue; }
                rec c = {v, i, j, side};
                push(loc, &c);
            }
        }
#pragma omp critical
        {
            push(top, &loc[0]);
            if (loc[1].i >= 0) push(top, &loc[1]);
            nzero += lz; npairs += lp;
        }
    }
    out->best = top[0].i >= 0 ? top[0].v : 0.0;
    out->bi = top[0].i; out->bj = top[0].j; out->bside = top[0].side;
    out->second = top[1].i >= 0 ? top[1].v : 0.0;
    out->si = top[1].i; out->sj = top[1].j; out->sside = top[1].side;
    out->nzero = nzero; out->npairs = npairs;
}

/* Distortion of an explicit list of pairs (sampled checks at full size).
 * out[t] = -1 marks a skipped pair with x_i == x_j. */
void oracle_pair_list(const double *X, const double *Y, int64_t d, int64_t r,
                      const int64_t *I, const int64_t *J, int64_t m,
                      double *out, int32_t *side) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < m; ++t) {
        int zero;
        double v = pair_distortion(X, Y, d, r, I[t], J[t], &side[t], &zero);
        out[t] = zero ? -1.0 : v;
    }
}

/* Threads the OpenMP loops above use (for reporting the CPU baseline), and
 * a way to change it (a 1-thread reference run). */
int oracle_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
