/* Runs the CPU oracle's entry points on small inputs -- empty, single,
 * duplicate and random objects of every kind, tiles at zooms 0 to 30,
 * binary, anti-aliased and fill output, and rejected arguments -- so that a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer can report any
 * out-of-bounds access, leak or undefined operation in it.  Exit 0: every
 * call behaved as documented (the sanitizers abort on their own findings). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void *oracle_build(const double *objects, int kind, int64_t n);
void oracle_free(void *h);
int oracle_render(const void *h, const int32_t *tiles, int64_t ntiles, const double *r, uint8_t *tri,
                  uint8_t *bit, double *dist, int64_t *counters, int nthreads);
int oracle_render_aa(const void *h, const int32_t *tiles, int64_t ntiles, const double *r, int mode,
                     uint8_t *val, uint8_t *amb, uint8_t *sure, int nthreads);
void *oracle_build_polygons(const double *edges, int64_t n, const int64_t *first, int64_t npoly, int merc01);
void oracle_free_polygons(void *h);
int oracle_render_fill(const void *h, const int32_t *tiles, int64_t ntiles, uint8_t *tri, uint8_t *bit,
                       int nthreads);
int oracle_project(const double *lonlat, int64_t n, double *X, double *Y);

static int fails = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); ++fails; } } while (0)

static uint64_t rng = 88172645463325252ull;
static double urand(void) { rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17; return (rng >> 11) * (1.0 / 9007199254740992.0); }

int main(void) {
    enum { NT = 6 };
    const int32_t tiles[NT * 3] = {0, 0, 0, 3, 4, 2, 12, 2000, 1500, 22, 3000000, 2000000, 30, 5, 7, 1, 1, 0};
    const double r[NT] = {0.5, 1.0, 2.5, 64.0, 3.0, 0.7};
    uint8_t *tri = malloc(NT * 65536), *bit = malloc(NT * 65536), *amb = malloc(NT * 65536), *sure = malloc(NT * 65536);
    double *dist = malloc(NT * 65536 * sizeof(double));
    int64_t cnt[NT * 5];
    for (int kind = 0; kind < 3; ++kind) {
        const int w = kind == 0 ? 2 : 4;
        for (int64_t n = 0; n <= 3000; n = n ? n * 10 : 1) {
            double *o = malloc((size_t)(n > 0 ? n : 1) * w * sizeof(double));
            for (int64_t k = 0; k < n * w; k += 2) {
                o[k] = -180.0 + 360.0 * urand();
                o[k + 1] = -89.0 + 178.0 * urand();
            }
            if (n >= 3) memcpy(o + w, o, (size_t)w * sizeof(double));   /* a duplicate */
            void *h = oracle_build(o, kind, n);
            CHECK(h != NULL);
            CHECK(oracle_render(h, tiles, NT, r, tri, bit, dist, cnt, 3) == 0);
            CHECK(oracle_render_aa(h, tiles, NT - 1, r, 0, tri, amb, sure, 2) == 0);
            CHECK(oracle_render_aa(h, tiles, NT - 1, r, 1, tri, amb, NULL, 2) == 0);
            for (int t = 0; t < NT * 65536; ++t) CHECK(tri[t] <= 4 && bit[t] <= 1);
            oracle_free(h);
            /* normalised input and rejected arguments */
            for (int64_t k = 0; k < n * w; ++k) o[k] = urand();
            h = oracle_build(o, kind | 0x100, n);
            CHECK(h != NULL);
            CHECK(oracle_render(h, tiles, NT, r, tri, NULL, NULL, NULL, 1) == 0);
            const int32_t bad[3] = {3, 8, 0};
            const double rneg = -1.0;
            CHECK(oracle_render(h, bad, 1, r, tri, NULL, NULL, NULL, 1) == -1);
            CHECK(oracle_render(h, tiles, 1, &rneg, tri, NULL, NULL, NULL, 1) == -1);
            oracle_free(h);
            free(o);
        }
    }
    CHECK(oracle_build(NULL, 9, 0) == NULL);
    oracle_free(NULL);
    /* polygons: a square with a hole, a triangle, and a star of many edges */
    {
        const int64_t nv = 64;
        double e[(4 + 4 + 3 + 64) * 4];
        int64_t first[5] = {0, 8, 11, 11 + nv, 0};
        const double sq[4][2] = {{0.2, 0.2}, {0.6, 0.2}, {0.6, 0.6}, {0.2, 0.6}}, hole[4][2] = {{0.3, 0.3}, {0.3, 0.4}, {0.4, 0.4}, {0.4, 0.3}};
        int q = 0;
        for (int k = 0; k < 4; ++k, ++q) { e[4*q] = sq[k][0]; e[4*q+1] = sq[k][1]; e[4*q+2] = sq[(k+1)%4][0]; e[4*q+3] = sq[(k+1)%4][1]; }
        for (int k = 0; k < 4; ++k, ++q) { e[4*q] = hole[k][0]; e[4*q+1] = hole[k][1]; e[4*q+2] = hole[(k+1)%4][0]; e[4*q+3] = hole[(k+1)%4][1]; }
        const double tr[3][2] = {{0.7, 0.1}, {0.9, 0.1}, {0.8, 0.3}};
        for (int k = 0; k < 3; ++k, ++q) { e[4*q] = tr[k][0]; e[4*q+1] = tr[k][1]; e[4*q+2] = tr[(k+1)%3][0]; e[4*q+3] = tr[(k+1)%3][1]; }
        for (int k = 0; k < nv; ++k, ++q) {
            const double a0 = 6.283185307179586 * k / nv, a1 = 6.283185307179586 * (k + 1) / nv;
            const double r0 = 0.05 + 0.03 * (k & 1), r1 = 0.05 + 0.03 * ((k + 1) & 1);
            e[4*q] = 0.5 + r0 * __builtin_cos(a0); e[4*q+1] = 0.8 + r0 * __builtin_sin(a0);
            e[4*q+2] = 0.5 + r1 * __builtin_cos(a1); e[4*q+3] = 0.8 + r1 * __builtin_sin(a1);
        }
        first[4] = q;
        first[3] = q;
        void *P = oracle_build_polygons(e, q, first, 3, 1);
        CHECK(P != NULL);
        CHECK(oracle_render_fill(P, tiles, NT, tri, bit, 3) == 0);
        oracle_free_polygons(P);
        const int64_t badfirst[3] = {0, 2, 4};
        CHECK(oracle_build_polygons(e, 4, badfirst, 2, 1) == NULL);
    }
    {
        double ll[8] = {-180, 0, 180, 85.0511287798066, 0, -90, 12.5, 47.25}, X[4], Y[4];
        CHECK(oracle_project(ll, 4, X, Y) == 0);
    }
    free(tri); free(bit); free(amb); free(sure); free(dist);
    if (fails) { fprintf(stderr, "%d checks failed\n", fails); return 1; }
    printf("oracle driver ok\n");
    return 0;
}
