/*
 * Plain FP64 direct sum of one wavenumber's Nystrom operator (test infrastructure).
 *
 * For every requested target row alpha and every source beta in a different
 * triangle:
 *   y_alpha += w_beta [ n_beta (grad'g . a_beta) - (n_beta . grad'g) a_beta
 *                       - grad'g (n_beta . a_beta) + g b_beta ]
 * with g = exp(i k R)/(4 pi R) (eq. 2.4), grad'g = (i k R - 1) exp(i k R)
 * (s_beta - s_alpha)/(4 pi R^3) the gradient at the source, and the Nystrom
 * rule of eq. 2.8 replacing the boundary integral of eq. 2.5 / 2.12.
 *
 * One plain double loop, OpenMP over target rows.  Compiled with gcc; it
 * shares nothing with the GPU library.
 *
 * Complex arrays are interleaved (re, im) doubles:
 *   a, b : [nrhs][n][3] complex      y : [nrhs][nrows][3] complex
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>

void oracle_point_sum(int64_t n, const double *pts, const double *nrm, const double *w,
                      const int32_t *tri, double k_re, double k_im, int32_t nrhs,
                      const double *a, const double *b, int64_t nrows, const int64_t *rows,
                      double *y)
{
    const double complex k = k_re + I * k_im;
    const double inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t al = rows[r];
        const double tx = pts[3 * al], ty = pts[3 * al + 1], tz = pts[3 * al + 2];
        for (int32_t q = 0; q < nrhs; ++q) {
            double complex acc[3] = {0, 0, 0};
            const double complex *A = (const double complex *)a + (int64_t)q * n * 3;
            const double complex *B = (const double complex *)b + (int64_t)q * n * 3;
            for (int64_t be = 0; be < n; ++be) {
                if (tri[be] == tri[al])
                    continue;
                const double dx = pts[3 * be] - tx, dy = pts[3 * be + 1] - ty, dz = pts[3 * be + 2] - tz;
                const double R = sqrt(dx * dx + dy * dy + dz * dz);
                const double complex e = cexp(I * k * R);
                const double complex g = e * inv4pi / R;
                const double complex f = (I * k * R - 1.0) * e * inv4pi / (R * R * R);
                const double complex G[3] = {f * dx, f * dy, f * dz};
                const double nx = nrm[3 * be], ny = nrm[3 * be + 1], nz = nrm[3 * be + 2];
                const double wb = w[be];
                const double complex a0 = A[3 * be], a1 = A[3 * be + 1], a2 = A[3 * be + 2];
                const double complex Ga = G[0] * a0 + G[1] * a1 + G[2] * a2;
                const double complex nG = nx * G[0] + ny * G[1] + nz * G[2];
                const double complex na = nx * a0 + ny * a1 + nz * a2;
                acc[0] += wb * (nx * Ga - nG * a0 - G[0] * na + g * B[3 * be]);
                acc[1] += wb * (ny * Ga - nG * a1 - G[1] * na + g * B[3 * be + 1]);
                acc[2] += wb * (nz * Ga - nG * a2 - G[2] * na + g * B[3 * be + 2]);
            }
            double complex *Y = (double complex *)y + ((int64_t)q * nrows + r) * 3;
            Y[0] = acc[0];
            Y[1] = acc[1];
            Y[2] = acc[2];
        }
    }
}
