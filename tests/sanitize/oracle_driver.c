/*
 * Drives the oracle's entry points on small seeded inputs so that a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer can check its memory
 * accesses and arithmetic (test infrastructure; built by
 * tests/test_sanitizers.py with gcc, host code only).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

long fsro_reconstruct(const double *img, const uint8_t *mask, double *out, int H, int W, long stride,
                      int B, int L, int iters, double rho, double gamma, int tie_larger,
                      uint16_t *log_idx, double *log_sep, int threads);
long fsro_reconstruct_blocks(const double *img, const uint8_t *mask, int H, int W, long stride, int B,
                             int L, int iters, double rho, double gamma, int tie_larger,
                             const int64_t *block_ids, long n, double *out_targets, uint16_t *log_idx,
                             double *log_p, double *log_sep, int threads);
long fsro_reconstruct_reuse(const double *img, const uint8_t *mask, double *out, int H, int W,
                            long stride, int B, int L, int iters, double rho, double gamma, double delta,
                            int tie_larger, uint16_t *log_idx);

static uint32_t state = 12345u;
static uint32_t next(void) { state = state * 1664525u + 1013904223u; return state >> 8; }

static int run(int H, int W, long stride, int B, int L, int iters)
{
    const int nb = ((H + B - 1) / B) * ((W + B - 1) / B);
    double *img = malloc(sizeof(double) * H * stride), *out = malloc(sizeof(double) * H * stride);
    uint8_t *mask = malloc((size_t)H * stride);
    /* the log serves the whole image (nb blocks) and the two listed blocks */
    uint16_t *log = malloc(sizeof(uint16_t) * (nb > 2 ? nb : 2) * (iters > 0 ? iters : 1));
    double *tg = malloc(sizeof(double) * 2 * B * B), *lp = malloc(sizeof(double) * 2 * 2 * (iters > 0 ? iters : 1));
    double *ls = malloc(sizeof(double) * 2 * (nb > 2 ? nb : 2) * (iters > 0 ? iters : 1));
    for (long i = 0; i < (long)H * stride; ++i) {
        img[i] = (double)(next() % 256);
        mask[i] = (uint8_t)(next() % 4 == 0);
    }
    long e = fsro_reconstruct(img, mask, out, H, W, stride, B, L, iters, 0.7, 0.5, 0, log, ls, 2);
    e += fsro_reconstruct_reuse(img, mask, out, H, W, stride, B, L, iters, 0.7, 0.5, 0.5, 0, log);
    int64_t ids[2] = {0, nb - 1};
    e += fsro_reconstruct_blocks(img, mask, H, W, stride, B, L, iters, 0.7, 0.5, 0, ids, 2, tg, log, lp, ls, 2);
    printf("%dx%d stride %ld B=%d L=%d I=%d: %ld empty\n", H, W, stride, B, L, iters, e);
    free(img); free(out); free(mask); free(log); free(tg); free(lp); free(ls);
    return 0;
}

int main(void)
{
    run(13, 11, 16, 4, 14, 20);   /* ragged, strided, S = 32 */
    run(9, 20, 20, 2, 3, 10);     /* S = 8 */
    run(1, 1, 1, 4, 6, 5);        /* one pixel */
    run(16, 16, 16, 8, 4, 0);     /* no iteration */
    return 0;
}
