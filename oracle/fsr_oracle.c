/*
 * fsr_oracle.c -- plain FP64 reference of block-independent Frequency
 * Selective Reconstruction (FSR), written from Regensky et al., "Real-Time
 * Frequency Selective Reconstruction through Register-Based Argmax
 * Calculation" (MMSP 2020), Sec. II.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * implementation that the HIP library is checked against.  Only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Everything is double precision and follows the paper's steps in order:
 *   O1  support block: target B x B plus an L-pixel border, S = B + 2L;
 *       pixels outside the image count as unknown                 (Sec. II)
 *   O2  spatial weight w = rho^dist on known pixels, else 0       (Eq. 5)
 *   O3  frequency weight w_f                                      (Eq. 9)
 *   O4  R_w = DFT2(f~ w), W = DFT2(w), unnormalised, e^{-j}       (Eq. 7)
 *   O5  G = 0                                                     (Sec. II)
 *   O6  I times: argmax of w_f |R_w|^2, p = R_w[u,v] / W[0,0],
 *       G[u,v] += gamma p S^2, R_w -= gamma p W[k-u, l-v]  (Eqs. 8, 10-12,
 *       cyclic indices as in Eqs. 14-15)
 *   O7  g = inverse DFT2 of G (1/S^2, e^{+j}) on the target pixels
 *   O8  output = f~ on known pixels, Re g on unknown ones         (Sec. II)
 *   O9  the sequential variant that reuses reconstructed pixels, the
 *       original FSR that the paper departs from (Sec. II): blocks in
 *       raster order, and a missing support pixel in the target of an
 *       earlier block counts as known with its reconstructed value and the
 *       weight delta rho^dist (fsro_reconstruct_reuse); and each of its
 *       blocks on its own, given the frame the reused pixels come from
 *       (fsro_reconstruct_reuse_given)
 *
 * Readings of points the paper leaves open (each is listed with its reason
 * in the design notes):
 *   - DFT convention: forward unnormalised with e^{-j2pi(km+ln)/S}, k pairs
 *     with the row index m.  This is the convention under which Eq. 10 is
 *     the weighted least-squares coefficient and Eq. 12 holds exactly.
 *   - Argmax (Eq. 8): the FP64 objectives are compared as they are; the
 *     larger wins, equal objectives go to the smaller linear index k*S + l
 *     (tie_larger = 1 flips this, for tests only).
 *   - The twiddle table is exactly conjugate-symmetric so that the spectra of
 *     real inputs are bitwise Hermitian.
 *   - A support with no known pixel (W[0,0] == 0) runs no iteration; its
 *     unknown target pixels are 0 and its log entries are 0xFFFF.
 *   - Unknown pixels take Re g; outputs are not clipped.
 *   - O9: "earlier" is raster order of the blocks (block row, then block
 *     column); delta is a parameter in [0, 1] (the tests use 0.25 to 1);
 *     delta = 0 reuses nothing, so the variant then equals the
 *     block-independent method.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off
 * (no fast-math: the symmetry arguments above rely on IEEE rounding).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define FSRO_API __attribute__((visibility("default")))

/* t[q] = exp(-j 2 pi q / S), q in [0, S), with t[S-q] = conj(t[q]) exactly
 * and the quarter points set exactly when S is a multiple of 4. */
FSRO_API void fsro_twiddles(int S, double *tr, double *ti)
{
    const double pi = 3.14159265358979323846264338327950288;
    tr[0] = 1.0;
    ti[0] = 0.0;
    for (int q = 1; q < S; ++q) {
        if (2 * q < S) {
            tr[q] = cos(2.0 * pi * (double)q / (double)S);
            ti[q] = -sin(2.0 * pi * (double)q / (double)S);
        } else if (2 * q == S) {
            tr[q] = -1.0;
            ti[q] = 0.0;
        } else {
            tr[q] = tr[S - q];
            ti[q] = -ti[S - q];
        }
    }
    if (S % 4 == 0) {
        tr[S / 4] = 0.0;
        ti[S / 4] = -1.0;
        tr[3 * S / 4] = 0.0;
        ti[3 * S / 4] = 1.0;
    }
}

/* Eq. 5: w[m,n] = rho^sqrt((m-(S-1)/2)^2 + (n-(S-1)/2)^2) on known pixels. */
FSRO_API void fsro_spatial_weight(int S, double rho, const uint8_t *known, double *w)
{
    const double c = 0.5 * (double)(S - 1);
    for (int m = 0; m < S; ++m)
        for (int n = 0; n < S; ++n) {
            double dm = (double)m - c, dn = (double)n - c;
            w[m * S + n] = known[m * S + n] ? pow(rho, sqrt(dm * dm + dn * dn)) : 0.0;
        }
}

/* Eq. 9: w_f[k,l] = (1 - sqrt(2) sqrt(kt^2/S^2 + lt^2/S^2))^2,
 * kt = S/2 - |k - S/2|, lt likewise. */
FSRO_API void fsro_freq_weight(int S, double *wf)
{
    const double h = 0.5 * (double)S;
    for (int k = 0; k < S; ++k)
        for (int l = 0; l < S; ++l) {
            double kt = h - fabs((double)k - h);
            double lt = h - fabs((double)l - h);
            double r = sqrt(kt * kt / ((double)S * S) + lt * lt / ((double)S * S));
            double a = 1.0 - sqrt(2.0) * r;
            wf[k * S + l] = a * a;
        }
}

/* Forward 2D DFT of a real S x S array, unnormalised:
 *   X[k,l] = sum_m sum_n x[m,n] t[(k m) mod S] t[(l n) mod S]
 * computed as direct sums, first over n for every (m, l), then over m. */
FSRO_API void fsro_dft2_real(int S, const double *x, double *Xr, double *Xi)
{
    double *tr = malloc(sizeof(double) * S), *ti = malloc(sizeof(double) * S);
    double *Yr = malloc(sizeof(double) * S * S), *Yi = malloc(sizeof(double) * S * S);
    fsro_twiddles(S, tr, ti);
    for (int m = 0; m < S; ++m)
        for (int l = 0; l < S; ++l) {
            double sr = 0.0, si = 0.0;
            for (int n = 0; n < S; ++n) {
                int q = (l * n) % S;
                sr += x[m * S + n] * tr[q];
                si += x[m * S + n] * ti[q];
            }
            Yr[m * S + l] = sr;
            Yi[m * S + l] = si;
        }
    for (int k = 0; k < S; ++k)
        for (int l = 0; l < S; ++l) {
            double sr = 0.0, si = 0.0;
            for (int m = 0; m < S; ++m) {
                int q = (k * m) % S;
                double a = Yr[m * S + l], b = Yi[m * S + l];
                sr += a * tr[q] - b * ti[q];
                si += a * ti[q] + b * tr[q];
            }
            Xr[k * S + l] = sr;
            Xi[k * S + l] = si;
        }
    free(tr); free(ti); free(Yr); free(Yi);
}

/*
 * One support block, steps O2-O6.
 *   ft      S x S sampled signal f~ (0 on unknown pixels)
 *   known   S x S, nonzero = known
 * Outputs (each may be NULL):
 *   Gr, Gi  S x S final model spectrum G
 *   Rr, Ri  S x S final weighted residual spectrum R_w
 *   log_idx I entries: selected bin u*S + v per iteration (0xFFFF if skipped)
 *   log_p   2I entries: projection coefficient p (re, im) per iteration
 *   log_sep 2I entries per iteration: the winning objective w_f |R_w|^2 and
 *           its relative separation (obj - next) / obj from the largest
 *           objective of any other bin, where the winner's conjugate bin
 *           (-u, -v) is passed over when its objective is exactly equal (a
 *           tie Eq. 8 settles by the index rule); 0 when obj is 0
 * Returns 1 when the support holds no known pixel (no iteration ran), else 0.
 */
FSRO_API int fsro_block_weighted(int S, int iters, double gamma, int tie_larger,
                                 const double *ft, const double *w,
                                 double *Gr_out, double *Gi_out, double *Rr_out, double *Ri_out,
                                 uint16_t *log_idx, double *log_p, double *log_sep);

FSRO_API int fsro_block(int S, int iters, double rho, double gamma, int tie_larger,
                        const double *ft, const uint8_t *known,
                        double *Gr_out, double *Gi_out, double *Rr_out, double *Ri_out,
                        uint16_t *log_idx, double *log_p, double *log_sep)
{
    double *w = malloc(sizeof(double) * S * S);
    fsro_spatial_weight(S, rho, known, w);                /* O2 */
    int empty = fsro_block_weighted(S, iters, gamma, tie_larger, ft, w, Gr_out, Gi_out,
                                    Rr_out, Ri_out, log_idx, log_p, log_sep);
    free(w);
    return empty;
}

/*
 * Steps O3-O6 for a support whose spatial weight w (S x S, zero on pixels
 * that do not take part) is given; fsro_block passes the weight of Eq. 5,
 * the reuse variant (O9) one with a third class of pixels.  Outputs as for
 * fsro_block; returns 1 when W[0,0] is not positive (no iteration ran).
 */
FSRO_API int fsro_block_weighted(int S, int iters, double gamma, int tie_larger,
                                 const double *ft, const double *w,
                                 double *Gr_out, double *Gi_out, double *Rr_out, double *Ri_out,
                                 uint16_t *log_idx, double *log_p, double *log_sep)
{
    const int n2 = S * S;
    double *x = malloc(sizeof(double) * n2);
    double *wf = malloc(sizeof(double) * n2);
    double *Rr = malloc(sizeof(double) * n2), *Ri = malloc(sizeof(double) * n2);
    double *Wr = malloc(sizeof(double) * n2), *Wi = malloc(sizeof(double) * n2);
    double *Gr = calloc(n2, sizeof(double)), *Gi = calloc(n2, sizeof(double));

    fsro_freq_weight(S, wf);                              /* O3 */
    for (int i = 0; i < n2; ++i) x[i] = ft[i] * w[i];
    fsro_dft2_real(S, x, Rr, Ri);                         /* O4 */
    fsro_dft2_real(S, w, Wr, Wi);

    const double w00 = Wr[0];
    int empty = !(w00 > 0.0);
    for (int it = 0; it < iters; ++it) {                  /* O6 */
        if (empty) {
            if (log_idx) log_idx[it] = 0xFFFF;
            if (log_p) { log_p[2 * it] = 0.0; log_p[2 * it + 1] = 0.0; }
            if (log_sep) { log_sep[2 * it] = 0.0; log_sep[2 * it + 1] = 0.0; }
            continue;
        }
        /* (u,v) = argmax_{k,l} w_f |R_w|^2 (Eq. 8), scanned in linear order */
        int best = 0;
        double best_obj = -1.0;
        for (int b = 0; b < n2; ++b) {
            double obj = wf[b] * (Rr[b] * Rr[b] + Ri[b] * Ri[b]);
            if (tie_larger ? (obj >= best_obj) : (obj > best_obj)) {
                best_obj = obj;
                best = b;
            }
        }
        const int u = best / S, v = best % S;
        if (log_sep) {
            /* the largest objective of the other bins, the conjugate of the
             * winner left out when it ties exactly */
            const int conj = ((S - u) % S) * S + (S - v) % S;
            double next = 0.0;
            for (int b = 0; b < n2; ++b) {
                if (b == best) continue;
                const double ob = wf[b] * (Rr[b] * Rr[b] + Ri[b] * Ri[b]);
                if (b == conj && ob == best_obj) continue;
                if (ob > next) next = ob;
            }
            log_sep[2 * it] = best_obj;
            log_sep[2 * it + 1] = best_obj > 0.0 ? (best_obj - next) / best_obj : 0.0;
        }
        const double p_re = Rr[best] / w00, p_im = Ri[best] / w00;  /* Eq. 10 */
        Gr[best] += gamma * p_re * (double)n2;                      /* Eq. 11 */
        Gi[best] += gamma * p_im * (double)n2;
        const double cr = gamma * p_re, ci = gamma * p_im;
        for (int k = 0; k < S; ++k)                                 /* Eq. 12 */
            for (int l = 0; l < S; ++l) {
                int i = (k - u >= 0) ? k - u : S + k - u;           /* Eq. 14 */
                int j = (l - v >= 0) ? l - v : S + l - v;           /* Eq. 15 */
                double ar = Wr[i * S + j], ai = Wi[i * S + j];
                Rr[k * S + l] -= cr * ar - ci * ai;
                Ri[k * S + l] -= cr * ai + ci * ar;
            }
        if (log_idx) log_idx[it] = (uint16_t)best;
        if (log_p) { log_p[2 * it] = p_re; log_p[2 * it + 1] = p_im; }
    }

    if (Gr_out) memcpy(Gr_out, Gr, sizeof(double) * n2);
    if (Gi_out) memcpy(Gi_out, Gi, sizeof(double) * n2);
    if (Rr_out) memcpy(Rr_out, Rr, sizeof(double) * n2);
    if (Ri_out) memcpy(Ri_out, Ri, sizeof(double) * n2);
    free(x); free(wf); free(Rr); free(Ri); free(Wr); free(Wi); free(Gr); free(Gi);
    return empty;
}

/* O7: Re g[m,n] = S^-2 sum_{k,l} Re(G[k,l] exp(+j 2 pi (k m + l n) / S)). */
FSRO_API double fsro_model_pixel(int S, const double *Gr, const double *Gi, int m, int n)
{
    double *tr = malloc(sizeof(double) * S), *ti = malloc(sizeof(double) * S);
    fsro_twiddles(S, tr, ti);
    double acc = 0.0;
    for (int k = 0; k < S; ++k)
        for (int l = 0; l < S; ++l) {
            int q = (k * m + l * n) % S;
            /* exp(+j 2 pi q / S) = conj(t[q]) */
            acc += Gr[k * S + l] * tr[q] + Gi[k * S + l] * ti[q];
        }
    free(tr); free(ti);
    return acc / ((double)S * S);
}

/* O1 for block id (by * nbx + bx): sampled support signal and known flags. */
static void gather_support(const double *img, const uint8_t *mask, int H, int W, long stride,
                           int B, int L, int by, int bx, double *ft, uint8_t *known)
{
    const int S = B + 2 * L;
    const int y0 = by * B - L, x0 = bx * B - L;
    for (int m = 0; m < S; ++m)
        for (int n = 0; n < S; ++n) {
            int y = y0 + m, x = x0 + n;
            int in = (y >= 0 && y < H && x >= 0 && x < W);
            int k = in && mask[(long)y * stride + x] != 0;
            known[m * S + n] = (uint8_t)k;
            ft[m * S + n] = k ? img[(long)y * stride + x] : 0.0;
        }
}

/* O1-O8 for one block; writes the in-image target pixels of out_target
 * (row-major B x B; entries of out-of-image pixels are left untouched). */
static int reconstruct_one(const double *img, const uint8_t *mask, int H, int W, long stride,
                           int B, int L, int iters, double rho, double gamma, int tie_larger,
                           long block_id, double *out_target, uint16_t *log_idx, double *log_p,
                           double *log_sep)
{
    const int S = B + 2 * L, n2 = S * S;
    const int nbx = (W + B - 1) / B;
    const int by = (int)(block_id / nbx), bx = (int)(block_id % nbx);
    double *ft = malloc(sizeof(double) * n2);
    uint8_t *known = malloc(n2);
    double *Gr = malloc(sizeof(double) * n2), *Gi = malloc(sizeof(double) * n2);
    gather_support(img, mask, H, W, stride, B, L, by, bx, ft, known);
    int empty = fsro_block(S, iters, rho, gamma, tie_larger, ft, known, Gr, Gi,
                           NULL, NULL, log_idx, log_p, log_sep);
    for (int i = 0; i < B; ++i)
        for (int j = 0; j < B; ++j) {
            int m = L + i, n = L + j;
            int y = by * B + i, x = bx * B + j;
            if (y >= H || x >= W) continue;                 /* partial target */
            out_target[i * B + j] = known[m * S + n] ? ft[m * S + n]
                                                     : fsro_model_pixel(S, Gr, Gi, m, n);
        }
    free(ft); free(known); free(Gr); free(Gi);
    return empty;
}

/*
 * Whole-image reconstruction.  Blocks are independent; OpenMP runs them in
 * parallel over `threads` threads (<= 0: the OpenMP default).
 *   img, mask  H x W, row stride `stride` elements; mask != 0 means known
 *   out        H x W, row stride `stride`; every pixel is written
 *   log_idx    optional, N x I (N = ceil(H/B) * ceil(W/B), block-major)
 *   log_sep    optional, N x I x 2: winning objective and its separation
 *              (see fsro_block_weighted)
 * Returns the number of blocks whose support held no known pixel.
 */
FSRO_API long fsro_reconstruct(const double *img, const uint8_t *mask, double *out,
                               int H, int W, long stride, int B, int L, int iters,
                               double rho, double gamma, int tie_larger,
                               uint16_t *log_idx, double *log_sep, int threads)
{
    const int nby = (H + B - 1) / B, nbx = (W + B - 1) / B;
    const long N = (long)nby * nbx;
    long empty = 0;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(threads) reduction(+ : empty)
#endif
    for (long b = 0; b < N; ++b) {
        double tgt[32 * 32];
        double *t = (B * B <= 32 * 32) ? tgt : malloc(sizeof(double) * B * B);
        empty += reconstruct_one(img, mask, H, W, stride, B, L, iters, rho, gamma, tie_larger,
                                 b, t, log_idx ? log_idx + b * (long)iters : NULL,
                                 NULL, log_sep ? log_sep + 2 * b * (long)iters : NULL);
        const int by = (int)(b / nbx), bx = (int)(b % nbx);
        for (int i = 0; i < B; ++i)
            for (int j = 0; j < B; ++j) {
                int y = by * B + i, x = bx * B + j;
                if (y < H && x < W) out[(long)y * stride + x] = t[i * B + j];
            }
        if (t != tgt) free(t);
    }
    return empty;
}

/*
 * A chosen subset of blocks (for checks of large frames on sampled outputs).
 *   block_ids   n entries, each in [0, N)
 *   out_targets n x B x B (row-major target of each block; out-of-image
 *               entries are set to NaN)
 *   log_idx     optional, n x I
 *   log_p       optional, n x I x 2
 *   log_sep     optional, n x I x 2 (see fsro_block_weighted)
 * Returns the number of listed blocks whose support held no known pixel.
 */
FSRO_API long fsro_reconstruct_blocks(const double *img, const uint8_t *mask,
                                      int H, int W, long stride, int B, int L, int iters,
                                      double rho, double gamma, int tie_larger,
                                      const int64_t *block_ids, long n, double *out_targets,
                                      uint16_t *log_idx, double *log_p, double *log_sep,
                                      int threads)
{
    long empty = 0;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) reduction(+ : empty)
#endif
    for (long i = 0; i < n; ++i) {
        double *t = out_targets + i * (long)B * B;
        for (int q = 0; q < B * B; ++q) t[q] = NAN;
        empty += reconstruct_one(img, mask, H, W, stride, B, L, iters, rho, gamma, tie_larger,
                                 (long)block_ids[i], t,
                                 log_idx ? log_idx + i * (long)iters : NULL,
                                 log_p ? log_p + 2 * i * (long)iters : NULL,
                                 log_sep ? log_sep + 2 * i * (long)iters : NULL);
    }
    return empty;
}

/*
 * One block of the sequential variant (O9).  In the support of block
 * (by, bx) a pixel takes part
 *   - as known, weight rho^dist, value from img, where mask marks it;
 *   - as reused, weight delta rho^dist, value from src, where it is missing
 *     but lies in the target of an earlier block in raster order (only when
 *     delta > 0);
 *   - not at all otherwise (missing pixels of this or later blocks, pixels
 *     outside the image).
 * The block then runs O3-O8 as in the block-independent method and writes
 * its in-image target pixels to dst.  rp is rho^dist on the whole support.
 * Returns 1 when no support pixel has a positive weight.
 */
static int reuse_block(const double *img, const uint8_t *mask, const double *src, double *dst,
                       int H, int W, long stride, int B, int L, int iters, const double *rp,
                       double gamma, double delta, int tie_larger, int by, int bx,
                       uint16_t *log_idx)
{
    const int S = B + 2 * L, n2 = S * S;
    double *ft = malloc(sizeof(double) * n2), *w = malloc(sizeof(double) * n2);
    double *Gr = malloc(sizeof(double) * n2), *Gi = malloc(sizeof(double) * n2);
    uint8_t *known = malloc(n2);
    const int y0 = by * B - L, x0 = bx * B - L;
    for (int m = 0; m < S; ++m)
        for (int n = 0; n < S; ++n) {
            const int y = y0 + m, x = x0 + n, i = m * S + n;
            const int in = (y >= 0 && y < H && x >= 0 && x < W);
            const int k = in && mask[(long)y * stride + x] != 0;
            const int earlier = y < by * B || (y < (by + 1) * B && x < bx * B);
            const int reused = in && !k && earlier && delta > 0.0;
            known[i] = (uint8_t)k;
            ft[i] = k ? img[(long)y * stride + x] : reused ? src[(long)y * stride + x] : 0.0;
            w[i] = k ? rp[i] : reused ? delta * rp[i] : 0.0;
        }
    const int empty = fsro_block_weighted(S, iters, gamma, tie_larger, ft, w, Gr, Gi, NULL, NULL,
                                          log_idx, NULL, NULL);
    for (int i = 0; i < B; ++i)                           /* O8 on the target */
        for (int j = 0; j < B; ++j) {
            const int y = by * B + i, x = bx * B + j, m = L + i, n = L + j;
            if (y >= H || x >= W) continue;
            dst[(long)y * stride + x] = known[m * S + n]
                ? ft[m * S + n] : fsro_model_pixel(S, Gr, Gi, m, n);
        }
    free(ft); free(w); free(Gr); free(Gi); free(known);
    return empty;
}

/*
 * O9: the sequential variant.  Blocks run one after another in raster order
 * (block row, then block column), each reading its reused pixels from out,
 * where the earlier blocks have already written their reconstructions.
 * Arguments as for fsro_reconstruct plus delta; out is read as well as
 * written and must not alias img.  Returns the number of blocks whose
 * support held no pixel with positive weight.
 */
FSRO_API long fsro_reconstruct_reuse(const double *img, const uint8_t *mask, double *out,
                                     int H, int W, long stride, int B, int L, int iters,
                                     double rho, double gamma, double delta, int tie_larger,
                                     uint16_t *log_idx)
{
    const int S = B + 2 * L, n2 = S * S;
    const int nby = (H + B - 1) / B, nbx = (W + B - 1) / B;
    double *rp = malloc(sizeof(double) * n2);
    uint8_t *all = malloc(n2);
    memset(all, 1, n2);
    fsro_spatial_weight(S, rho, all, rp);                 /* rho^dist everywhere */
    long empty = 0;
    for (int by = 0; by < nby; ++by)
        for (int bx = 0; bx < nbx; ++bx) {
            const long b = (long)by * nbx + bx;
            empty += reuse_block(img, mask, out, out, H, W, stride, B, L, iters, rp, gamma, delta,
                                 tie_larger, by, bx, log_idx ? log_idx + b * (long)iters : NULL);
        }
    free(rp); free(all);
    return empty;
}

/*
 * Every block of the sequential variant (O9) taken on its own: the reused
 * pixels of each support take their values from the frame `reused` (for
 * example another implementation's output) instead of from this function's
 * own earlier blocks.  Blocks are then independent and run in parallel.
 * Given O9's own output as `reused`, each block sees exactly the inputs it
 * saw inside O9, so `out` and the log equal O9's.  `out` must alias neither
 * img nor reused; every in-image pixel of it is written.
 */
FSRO_API long fsro_reconstruct_reuse_given(const double *img, const uint8_t *mask,
                                           const double *reused, double *out, int H, int W,
                                           long stride, int B, int L, int iters, double rho,
                                           double gamma, double delta, int tie_larger,
                                           uint16_t *log_idx, int threads)
{
    const int S = B + 2 * L, n2 = S * S;
    const int nby = (H + B - 1) / B, nbx = (W + B - 1) / B;
    const long N = (long)nby * nbx;
    double *rp = malloc(sizeof(double) * n2);
    uint8_t *all = malloc(n2);
    memset(all, 1, n2);
    fsro_spatial_weight(S, rho, all, rp);
    long empty = 0;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(threads) reduction(+ : empty)
#endif
    for (long b = 0; b < N; ++b)
        empty += reuse_block(img, mask, reused, out, H, W, stride, B, L, iters, rp, gamma, delta,
                             tie_larger, (int)(b / nbx), (int)(b % nbx),
                             log_idx ? log_idx + b * (long)iters : NULL);
    free(rp); free(all);
    return empty;
}

FSRO_API int fsro_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
