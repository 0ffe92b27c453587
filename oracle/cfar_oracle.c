/*
 * FP64 CPU oracle for integral-image 2D cell-averaging CFAR.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this file.  The product path
 * (the HIP library) shares no code with it and never calls it.
 *
 * Paper: Rohman, Andra, Nishimoto, "Optimized 2D CA-CFAR for Drone-Mounted
 * Radar Signal Processing Using Integral Image Algorithm" (arXiv 2012.11077).
 *
 * Everything is plain, sequential IEEE double arithmetic, compiled with
 * -O2 -ffp-contract=off (no fused multiply-add), so that a reader can check it
 * against the paper by eye:
 *
 *   Sec. II.B, eq. (3): integral image  s(x,y) = i(x,y) + s(x-1,y) + s(x,y-1) - s(x-1,y-1)
 *   Sec. II.B, eq. (4): rectangle sum   A = L1 + L4 - (L2 + L3)
 *   Sec. II.B, eq. (2): threshold       T = alpha * A,  A = mean of the N training cells
 *   Sec. II.B, eq. (1): decision        H1 if CUT > T, H0 if CUT < T
 *
 * Readings of the paper taken here (each one is listed with its reason in the
 * design notes of the repository):
 *   - eq. (2) is printed as alpha = N (Pfa^(1/N) - 1), which is negative for
 *     0 < Pfa < 1.  The oracle uses the square-law CA-CFAR factor
 *     alpha = N (Pfa^(-1/N) - 1), evaluated as N * expm1(-log(Pfa) / N).
 *   - "guard" and "background" (Table I) are half-widths per side; the training
 *     band lies outside the guard band, so the outer half-width is guard+train.
 *   - windows are clipped at the map border; N counts the training cells that
 *     are inside the map; N == 0 means no decision (H0).
 *   - CUT == T is H0 (only the strict test CUT > T declares a target).
 *   - the four corners of eq. (4): L1 = outside top-left, L4 = inclusive
 *     bottom-right, L2 / L3 = the two off-diagonal outside corners.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* eq. (3), with the implied zero boundary s(-1,.) = s(.,-1) = 0 held as a
 * leading zero row and column: S has (R+1) x (F+1) entries, row-major, and
 * S[(i+1)*(F+1) + (j+1)] is the sum of x over rows 0..i and columns 0..j. */
void oracle_sat(const double *x, int64_t R, int64_t F, int64_t ld, double *S)
{
    const int64_t W = F + 1;
    for (int64_t j = 0; j <= F; ++j)
        S[j] = 0.0;
    for (int64_t i = 0; i < R; ++i) {
        S[(i + 1) * W] = 0.0;
        for (int64_t j = 0; j < F; ++j) {
            /* s(x,y) = i(x,y) + s(x-1,y) + s(x,y-1) - s(x-1,y-1) */
            S[(i + 1) * W + (j + 1)] =
                x[i * ld + j] + S[i * W + (j + 1)] + S[(i + 1) * W + j] - S[i * W + j];
        }
    }
}

/* eq. (4): sum of x over rows r0..r1 and columns c0..c1 (inclusive) from the
 * padded integral image. */
static double rect_sum(const double *S, int64_t W, int64_t r0, int64_t r1, int64_t c0, int64_t c1)
{
    const double L1 = S[r0 * W + c0];             /* outside, top-left      */
    const double L2 = S[r0 * W + (c1 + 1)];       /* outside, top-right     */
    const double L3 = S[(r1 + 1) * W + c0];       /* outside, bottom-left   */
    const double L4 = S[(r1 + 1) * W + (c1 + 1)]; /* inclusive bottom-right */
    return L1 + L4 - (L2 + L3);
}

/* eq. (2), scale factor for N training cells (sign of the exponent read as
 * -1/N; see the header). */
double oracle_alpha(int64_t n, double pfa)
{
    const double nn = (double)n;
    return nn * expm1(-log(pfa) / nn);
}

static int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }
static int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }

/* One cell under test from training sum st and count nt: T = alpha * A with
 * A = st / nt (eq. 2), decision CUT > T (eq. 1).  Returns the decision and
 * writes T (infinity when there are no training cells). */
static int decide(double cut, double st, int64_t nt, double pfa, double *thr)
{
    if (nt <= 0) {
        *thr = INFINITY;
        return 0;
    }
    const double A = st / (double)nt;
    const double T = oracle_alpha(nt, pfa) * A;
    *thr = T;
    return cut > T;
}

/* Integral-image CA-CFAR over the whole map (the paper's "II CA-CFAR").
 * x: R x F row-major with leading dimension ld.  Window: guard half-widths
 * gr (rows) / gf (cols), training half-widths tr / tf.  Outputs (any may be
 * NULL except mask): mask R x F (0/1), training sum, training count and
 * threshold per cell, all with leading dimension F.  nthreads > 1 splits the
 * rows of the per-cell loop over that many OpenMP threads; every cell runs
 * the same code on the same integral image, so the outputs do not depend on
 * it.  Returns 0, or -1 when the SAT could not be allocated. */
int oracle_cfar2d(const double *x, int64_t R, int64_t F, int64_t ld,
                  int64_t gr, int64_t gf, int64_t tr, int64_t tf, double pfa,
                  uint8_t *mask, double *train_sum, int64_t *n_train, double *thresh, int nthreads)
{
    const int64_t W = F + 1;
    double *S = (double *)malloc(sizeof(double) * (size_t)(R + 1) * (size_t)W);
    if (!S)
        return -1;
    oracle_sat(x, R, F, ld, S);
    const int64_t hr = gr + tr, hf = gf + tf;
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t i = 0; i < R; ++i) {
        for (int64_t j = 0; j < F; ++j) {
            /* outer (guard + training) and inner (guard, holds the CUT) rectangles, clipped */
            const int64_t ro0 = imax(0, i - hr), ro1 = imin(R - 1, i + hr);
            const int64_t co0 = imax(0, j - hf), co1 = imin(F - 1, j + hf);
            const int64_t ri0 = imax(0, i - gr), ri1 = imin(R - 1, i + gr);
            const int64_t ci0 = imax(0, j - gf), ci1 = imin(F - 1, j + gf);
            const double outer = rect_sum(S, W, ro0, ro1, co0, co1);
            const double inner = rect_sum(S, W, ri0, ri1, ci0, ci1);
            const double st = outer - inner;
            const int64_t nt = (ro1 - ro0 + 1) * (co1 - co0 + 1) - (ri1 - ri0 + 1) * (ci1 - ci0 + 1);
            double thr;
            const int d = decide(x[i * ld + j], st, nt, pfa, &thr);
            mask[i * F + j] = (uint8_t)d;
            if (train_sum)
                train_sum[i * F + j] = st;
            if (n_train)
                n_train[i * F + j] = nt;
            if (thresh)
                thresh[i * F + j] = thr;
        }
    }
    free(S);
    return 0;
}

/* Direct CA-CFAR (no integral image; the comparison column of Table I) on a
 * list of cells: the training sum is the plain sum over every cell of the
 * clipped outer rectangle that is not in the clipped inner rectangle, in
 * row-major order.  Used on sampled cells of maps too large for the full SAT. */
void oracle_cfar2d_cells(const double *x, int64_t R, int64_t F, int64_t ld,
                         int64_t gr, int64_t gf, int64_t tr, int64_t tf, double pfa,
                         const int64_t *rows, const int64_t *cols, int64_t n,
                         uint8_t *mask, double *train_sum, int64_t *n_train, double *thresh)
{
    const int64_t hr = gr + tr, hf = gf + tf;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t i = rows[k], j = cols[k];
        double st = 0.0;
        int64_t nt = 0;
        for (int64_t a = imax(0, i - hr); a <= imin(R - 1, i + hr); ++a) {
            for (int64_t b = imax(0, j - hf); b <= imin(F - 1, j + hf); ++b) {
                const int in_guard = (a >= i - gr) && (a <= i + gr) && (b >= j - gf) && (b <= j + gf);
                if (!in_guard) {
                    st += x[a * ld + b];
                    nt += 1;
                }
            }
        }
        double thr;
        const int d = decide(x[i * ld + j], st, nt, pfa, &thr);
        mask[k] = (uint8_t)d;
        if (train_sum)
            train_sum[k] = st;
        if (n_train)
            n_train[k] = nt;
        if (thresh)
            thresh[k] = thr;
    }
}
