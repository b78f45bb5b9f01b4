/* Test driver for the oracle's C certificate under AddressSanitizer and
 * UndefinedBehaviorSanitizer (CPU only): every entry point on small clouds,
 * with the edge cases the certificate has (two points, identical points, a
 * row block, pair lists), each result checked against a brute force written
 * here.  Exit status 0 when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    double best, second;
    int64_t bi, bj, si, sj;
    int32_t bside, sside;
    int64_t nzero, npairs;
} oracle_cert;

void oracle_certificate(const double *X, const double *Y, int64_t n, int64_t d, int64_t r,
                        int64_t i0, int64_t i1, oracle_cert *out);
void oracle_cross_certificate(const double *X, const double *Y, int64_t d, int64_t r,
                              const int64_t *IA, int64_t na, const int64_t *IB, int64_t nb,
                              oracle_cert *out);
void oracle_pair_list(const double *X, const double *Y, int64_t d, int64_t r,
                      const int64_t *I, const int64_t *J, int64_t m, double *out, int32_t *side);
int oracle_threads(void);
void oracle_set_threads(int t);

static uint64_t state = 88172645463325252ull;
static double uniform(void) {
    state ^= state << 13; state ^= state >> 7; state ^= state << 17;
    return (double)(state >> 11) * 0x1.0p-53 - 0.5;
}

static double brute(const double *X, const double *Y, int64_t n, int64_t d, int64_t r, int64_t i0, int64_t i1,
                    int64_t *bi, int64_t *bj) {
    double best = -1.0;
    *bi = *bj = -1;
    for (int64_t i = i0; i < i1; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double D = 0.0, E = 0.0;
            for (int64_t l = 0; l < d; ++l) D += (X[i * d + l] - X[j * d + l]) * (X[i * d + l] - X[j * d + l]);
            for (int64_t m = 0; m < r; ++m) E += (Y[i * r + m] - Y[j * r + m]) * (Y[i * r + m] - Y[j * r + m]);
            if (D == 0.0) continue;
            const double v = fabs(sqrt(E) / sqrt(D) - 1.0);
            if (v > best) { best = v; *bi = i; *bj = j; }
        }
    return best < 0.0 ? 0.0 : best;
}

static int fails = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); ++fails; } } while (0)

int main(void) {
    const int64_t sizes[][3] = {{2, 3, 2}, {17, 5, 3}, {64, 9, 4}, {130, 7, 7}};
    for (int t = 0; t < 2; ++t) {
        oracle_set_threads(t == 0 ? 1 : 4);
        CHECK(oracle_threads() == (t == 0 ? 1 : 4));
        for (unsigned c = 0; c < sizeof(sizes) / sizeof(sizes[0]); ++c) {
            const int64_t n = sizes[c][0], d = sizes[c][1], r = sizes[c][2];
            double *X = malloc(sizeof(double) * n * d), *Y = malloc(sizeof(double) * n * r);
            for (int64_t e = 0; e < n * d; ++e) X[e] = uniform();
            for (int64_t e = 0; e < n * r; ++e) Y[e] = uniform();
            if (n > 3) {   /* two identical points (and images): a skipped pair */
                for (int64_t l = 0; l < d; ++l) X[3 * d + l] = X[1 * d + l];
                for (int64_t m = 0; m < r; ++m) Y[3 * r + m] = Y[1 * r + m];
            }
            oracle_cert o;
            int64_t bi, bj;
            oracle_certificate(X, Y, n, d, r, 0, n, &o);
            const double want = brute(X, Y, n, d, r, 0, n, &bi, &bj);
            CHECK(o.best == want && o.bi == bi && o.bj == bj);
            CHECK(o.npairs == n * (n - 1) / 2);
            CHECK(o.nzero == (n > 3 ? 1 : 0));
            /* a row block, clipped at n */
            oracle_certificate(X, Y, n, d, r, n / 2, n + 5, &o);
            const double wb = brute(X, Y, n, d, r, n / 2, n, &bi, &bj);
            CHECK(o.best == wb && o.bi == bi && o.bj == bj);
            /* every row against every row as lists: the full certificate again */
            int64_t *I = malloc(sizeof(int64_t) * n);
            for (int64_t i = 0; i < n; ++i) I[i] = i;
            oracle_cross_certificate(X, Y, d, r, I, n, I, n, &o);
            CHECK(o.best == want && o.npairs == n * (n - 1) / 2);
            /* the argmax pair as a list of one */
            double v;
            int32_t side;
            const int64_t pi = bi >= 0 ? bi : 0, pj = bj >= 0 ? bj : 1;
            oracle_pair_list(X, Y, d, r, &pi, &pj, 1, &v, &side);
            CHECK(bi < 0 || fabs(v - wb) == 0.0);
            free(I);
            free(X);
            free(Y);
        }
    }
    if (fails) return 1;
    printf("oracle driver: all checks passed\n");
    return 0;
}
