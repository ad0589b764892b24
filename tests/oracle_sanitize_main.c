/*
 * Driver for the sanitizer build of the oracle (tests/test_oracle_sanitize.py):
 * reads one input file, runs every exported oracle routine on it, and writes
 * their results, so that an AddressSanitizer / UndefinedBehaviorSanitizer build
 * of oracle.c exercises the same code paths as the ctypes-loaded library.
 *
 * Input  (little endian): int64 n, int32 dim, float eps, int32 min_pts,
 *                         then n*dim float32 coordinates (row-major).
 * Output (little endian): for mode 0 (brute) then mode 1 (grid):
 *                         int64 K, int32 labels[n], uint8 is_core[n],
 *                         int32 counts[n], int64 border violations;
 *                         then int64 neighbours of point 0 (brute force).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_neighbor_counts(const float *pts, int64_t n, int dim, float eps, int mode, int threads,
                           int32_t *counts);
int64_t oracle_dbscan(const float *pts, int64_t n, int dim, float eps, int32_t min_pts, int mode, int threads,
                      int32_t *labels, uint8_t *is_core);
int64_t oracle_check_border(const float *pts, int64_t n, int dim, float eps, const uint8_t *is_core,
                            const int32_t *labels, int mode, int threads);
int64_t oracle_neighbors_of(const float *pts, int64_t n, int dim, float eps, int64_t i, int64_t *out,
                            int64_t cap);

static int rd(void *p, size_t sz, size_t k, FILE *f) { return fread(p, sz, k, f) == k ? 0 : 1; }

int main(int argc, char **argv)
{
    if (argc != 4) {
        fprintf(stderr, "usage: %s input output threads\n", argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 3;
    int64_t n;
    int32_t dim, min_pts;
    float eps;
    if (rd(&n, 8, 1, f) || rd(&dim, 4, 1, f) || rd(&eps, 4, 1, f) || rd(&min_pts, 4, 1, f) || n < 0) return 4;
    float *pts = (float *)malloc((size_t)(n > 0 ? n : 1) * (size_t)dim * sizeof(float));
    if (!pts || (n > 0 && rd(pts, sizeof(float), (size_t)n * (size_t)dim, f))) return 5;
    fclose(f);
    const int threads = atoi(argv[3]);
    const size_t N = (size_t)(n > 0 ? n : 1);
    int32_t *labels = (int32_t *)malloc(N * 4);
    int32_t *counts = (int32_t *)malloc(N * 4);
    uint8_t *core = (uint8_t *)malloc(N);
    int64_t *nb = (int64_t *)malloc(N * 8);
    FILE *o = fopen(argv[2], "wb");
    if (!labels || !counts || !core || !nb || !o) return 6;
    for (int mode = 0; mode < 2; ++mode) {
        int64_t k = oracle_dbscan(pts, n, dim, eps, min_pts, mode, threads, labels, core);
        if (k < 0) return 7;
        if (oracle_neighbor_counts(pts, n, dim, eps, mode, threads, counts) != 0) return 8;
        int64_t bad = oracle_check_border(pts, n, dim, eps, core, labels, mode, threads);
        if (bad < 0) return 9;
        fwrite(&k, 8, 1, o);
        fwrite(labels, 4, (size_t)n, o);
        fwrite(core, 1, (size_t)n, o);
        fwrite(counts, 4, (size_t)n, o);
        fwrite(&bad, 8, 1, o);
    }
    int64_t cnt = n > 0 ? oracle_neighbors_of(pts, n, dim, eps, 0, nb, n) : 0;
    fwrite(&cnt, 8, 1, o);
    fclose(o);
    free(pts);
    free(labels);
    free(counts);
    free(core);
    free(nb);
    return 0;
}
