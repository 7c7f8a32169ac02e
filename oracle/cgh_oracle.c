/*
 * FP64 CPU oracle for the point-cloud hologram sum.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library, and the GPU library never
 * calls it.
 *
 * What it computes (Section 2.1, "Direct calculation"):
 *
 *   Eq. (2), the Fresnel approximation of the spherical wave of N point
 *   sources,  O(x_h, y_h) = sum_j A_j exp( i (2 pi / lambda)
 *                            (z_j + ((x_h - x_j)^2 + (y_h - y_j)^2) / (2 z_j)) ),
 *   read with the imaginary unit in the exponent (the printed equation drops
 *   it), and Eq. (5), the amplitude hologram I = sum_j A_j cos(phase_j + phi_r)
 *   with the constant 2 A_r dropped.  The hot path takes phi_r = 0 and drops
 *   the per-point constant 2 pi z_j / lambda (as the paper's own programs do,
 *   List 1 to List 3), which leaves
 *
 *     I(x_h, y_h) = sum_j A_j cos( pi / (lambda z_j) ((x_h - x_j)^2 + (y_h - y_j)^2) ).
 *
 *   cgh_oracle_fresnel returns that real part and, on request, the imaginary
 *   part sum_j A_j sin(...) of the same complex sum, which Eq. (3) needs for a
 *   phase-only hologram.
 *
 * Reading of the coordinates: pixel (ix, iy) of a W x H hologram with pitch p
 * sits at x_h = (ix - (W-1)/2) p, y_h = (iy - (H-1)/2) p, i.e. the point
 * coordinates are measured from the hologram centre (the paper's programs put
 * pixel 0 at the origin; a centred grid is what makes clouds of +-mm extent in
 * front of a mm-sized hologram meaningful, and it makes x/y mirror symmetry
 * exact).  Output is row-major, x fastest, as in the paper's programs.
 *
 * It is a plain triple loop: rows x columns x points, FP64, libm cos/sin, a
 * sequential sum over the points in index order, no separability, no
 * tables, no fast-math.  Rows of the evaluation set are split over threads.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    /* evaluation set: all (row, column) pairs of rows[] x cols[] */
    const int32_t *cols, *rows;
    int64_t n_cols, n_rows;
    int32_t width, height;
    double pitch, wavelength;
    const double *x, *y, *z, *a;
    int64_t n_points;
    double *out_re, *out_im;     /* [n_rows][n_cols]; out_im may be NULL */
    int64_t row_begin, row_end;  /* this worker's share of rows[] */
    int spherical;               /* 0: Eq. (2) Fresnel form; 1: Eq. (1) exact distance */
} job_t;

static void *worker(void *arg)
{
    const job_t *jb = (const job_t *)arg;
    const double pi = 3.14159265358979323846;
    const double half_w = 0.5 * (double)(jb->width - 1);
    const double half_h = 0.5 * (double)(jb->height - 1);
    for (int64_t r = jb->row_begin; r < jb->row_end; ++r) {
        const double yh = ((double)jb->rows[r] - half_h) * jb->pitch;
        for (int64_t c = 0; c < jb->n_cols; ++c) {
            const double xh = ((double)jb->cols[c] - half_w) * jb->pitch;
            double re = 0.0, im = 0.0;
            for (int64_t j = 0; j < jb->n_points; ++j) {
                const double dx = xh - jb->x[j];
                const double dy = yh - jb->y[j];
                double theta;
                if (jb->spherical) {
                    /* Eq. (1): 2 pi / lambda * sqrt(dx^2 + dy^2 + z^2) */
                    theta = 2.0 * pi / jb->wavelength *
                            sqrt(dx * dx + dy * dy + jb->z[j] * jb->z[j]);
                } else {
                    /* Eq. (2) without the per-point z_j term:
                     * (2 pi / lambda) (dx^2 + dy^2) / (2 z_j) */
                    theta = pi * (dx * dx + dy * dy) / (jb->wavelength * jb->z[j]);
                }
                re += jb->a[j] * cos(theta);
                if (jb->out_im)
                    im += jb->a[j] * sin(theta);
            }
            jb->out_re[r * jb->n_cols + c] = re;
            if (jb->out_im)
                jb->out_im[r * jb->n_cols + c] = im;
        }
    }
    return NULL;
}

static int run(int32_t width, int32_t height, double pitch, double wavelength,
               int64_t n_points, const double *x, const double *y, const double *z,
               const double *a, int64_t n_cols, const int32_t *cols, int64_t n_rows,
               const int32_t *rows, double *out_re, double *out_im, int32_t n_threads,
               int spherical)
{
    if (width <= 0 || height <= 0 || n_points < 0 || n_cols < 0 || n_rows < 0)
        return 1;
    if (!(pitch > 0.0) || !(wavelength > 0.0) || !out_re)
        return 1;
    if (n_points > 0 && (!x || !y || !z || !a))
        return 1;
    if ((n_cols > 0 && !cols) || (n_rows > 0 && !rows))
        return 1;
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > n_rows)
        n_threads = n_rows > 0 ? (int32_t)n_rows : 1;

    job_t *jobs = (job_t *)calloc((size_t)n_threads, sizeof(job_t));
    pthread_t *tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return 2;
    }
    for (int32_t t = 0; t < n_threads; ++t) {
        job_t *jb = &jobs[t];
        jb->cols = cols; jb->rows = rows; jb->n_cols = n_cols; jb->n_rows = n_rows;
        jb->width = width; jb->height = height; jb->pitch = pitch; jb->wavelength = wavelength;
        jb->x = x; jb->y = y; jb->z = z; jb->a = a; jb->n_points = n_points;
        jb->out_re = out_re; jb->out_im = out_im; jb->spherical = spherical;
        jb->row_begin = n_rows * t / n_threads;
        jb->row_end = n_rows * (t + 1) / n_threads;
    }
    int rc = 0;
    int32_t started = 0;
    for (int32_t t = 1; t < n_threads; ++t) {
        if (pthread_create(&tids[t], NULL, worker, &jobs[t]) != 0) {
            rc = 3;
            break;
        }
        started = t;
    }
    if (rc == 0)
        worker(&jobs[0]);
    for (int32_t t = 1; t <= started; ++t)
        pthread_join(tids[t], NULL);
    free(jobs);
    free(tids);
    return rc;
}

/* Fresnel form, Eq. (2)/(5) as described above.  Returns 0 on success. */
int cgh_oracle_fresnel(int32_t width, int32_t height, double pitch, double wavelength,
                       int64_t n_points, const double *x, const double *y, const double *z,
                       const double *a, int64_t n_cols, const int32_t *cols, int64_t n_rows,
                       const int32_t *rows, double *out_re, double *out_im, int32_t n_threads)
{
    return run(width, height, pitch, wavelength, n_points, x, y, z, a, n_cols, cols, n_rows,
               rows, out_re, out_im, n_threads, 0);
}

/* Exact spherical wave, Eq. (1): phase (2 pi / lambda) * distance, including
 * the z_j part of the distance.  Returns 0 on success. */
int cgh_oracle_spherical(int32_t width, int32_t height, double pitch, double wavelength,
                         int64_t n_points, const double *x, const double *y, const double *z,
                         const double *a, int64_t n_cols, const int32_t *cols, int64_t n_rows,
                         const int32_t *rows, double *out_re, double *out_im, int32_t n_threads)
{
    return run(width, height, pitch, wavelength, n_points, x, y, z, a, n_cols, cols, n_rows,
               rows, out_re, out_im, n_threads, 1);
}


/* ------------------------------------------------------------------------
 * Fresnel diffraction of a sampled field, Eq. (10) (Section 2.3, the second
 * step of the wavefront-recording method): the field u on an n x n grid of
 * pitch p at distance z from the hologram plane propagates to
 *
 *   O(x_h, y_h) = exp(i 2 pi z / lambda) / (i lambda z)
 *                 * integral u(x_w, y_w) exp(i pi / (lambda z) ((x_h - x_w)^2 + (y_h - y_w)^2)) dx_w dy_w,
 *
 * read on the same n x n grid, the integral taken as the sum over the samples
 * times the sample area p^2:
 *
 *   O[m][c] = exp(i 2 pi z / lambda) / (i lambda z) * p^2
 *             * sum_k sum_l u[k][l] exp(i pi p^2 ((m - k)^2 + (c - l)^2) / (lambda z)).
 *
 * A plain quadruple loop (output rows of the evaluation set x columns x
 * input rows x input columns), FP64, libm cos/sin, sequential sums.  The
 * phase is evaluated in revolutions, ((m-k)^2 + (c-l)^2) p^2 / (2 lambda z),
 * and z / lambda likewise (one FP64 rounding each, relative 1e-16), and
 * reduced with fmod (exact) before the trigonometric call.
 */
typedef struct {
    int32_t n;
    double pitch, wavelength, z;
    const double *u_re, *u_im;
    const int32_t *rows;
    double *out_re, *out_im;
    int64_t row_begin, row_end;
} diff_job_t;

static void *diff_worker(void *arg)
{
    const diff_job_t *jb = (const diff_job_t *)arg;
    const double two_pi = 6.28318530717958647692;
    const int32_t n = jb->n;
    const double q = jb->pitch * jb->pitch / (2.0 * jb->wavelength * jb->z);   /* rev per px^2 */
    for (int64_t r = jb->row_begin; r < jb->row_end; ++r) {
        const int32_t m = jb->rows[r];
        for (int32_t c = 0; c < n; ++c) {
            double re = 0.0, im = 0.0;
            for (int32_t k = 0; k < n; ++k) {
                const double dm = (double)(m - k);
                for (int32_t l = 0; l < n; ++l) {
                    const double dc = (double)(c - l);
                    const double rev = fmod(q * (dm * dm + dc * dc), 1.0);
                    const double hr = cos(two_pi * rev), hi = sin(two_pi * rev);
                    const double ur = jb->u_re[(int64_t)k * n + l];
                    const double ui = jb->u_im[(int64_t)k * n + l];
                    re += ur * hr - ui * hi;
                    im += ur * hi + ui * hr;
                }
            }
            /* prefactor exp(i 2 pi z / lambda) / (i lambda z) * p^2 */
            const double zrev = fmod(jb->z / jb->wavelength, 1.0);
            const double er = cos(two_pi * zrev), ei = sin(two_pi * zrev);
            const double s = jb->pitch * jb->pitch / (jb->wavelength * jb->z);
            /* (er + i ei) * (-i) * s = s (ei - i er) */
            const double pr = s * ei, pi_ = -s * er;
            jb->out_re[r * n + c] = re * pr - im * pi_;
            jb->out_im[r * n + c] = re * pi_ + im * pr;
        }
    }
    return NULL;
}

/* Eq. (10) by direct summation for output rows rows[0 .. n_rows) (all n
 * columns each).  u_re, u_im: n x n row-major; out_re, out_im: n_rows x n.
 * Returns 0 on success. */
int cgh_oracle_diffraction(int32_t n, double pitch, double wavelength, double z,
                           const double *u_re, const double *u_im, int64_t n_rows,
                           const int32_t *rows, double *out_re, double *out_im,
                           int32_t n_threads)
{
    if (n <= 0 || n_rows < 0 || !(pitch > 0.0) || !(wavelength > 0.0) || !(z != 0.0))
        return 1;
    if (!u_re || !u_im || !out_re || !out_im || (n_rows > 0 && !rows))
        return 1;
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > n_rows)
        n_threads = n_rows > 0 ? (int32_t)n_rows : 1;
    diff_job_t *jobs = (diff_job_t *)calloc((size_t)n_threads, sizeof(diff_job_t));
    pthread_t *tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return 2;
    }
    for (int32_t t = 0; t < n_threads; ++t) {
        diff_job_t *jb = &jobs[t];
        jb->n = n; jb->pitch = pitch; jb->wavelength = wavelength; jb->z = z;
        jb->u_re = u_re; jb->u_im = u_im; jb->rows = rows;
        jb->out_re = out_re; jb->out_im = out_im;
        jb->row_begin = n_rows * t / n_threads;
        jb->row_end = n_rows * (t + 1) / n_threads;
    }
    int rc = 0;
    int32_t started = 0;
    for (int32_t t = 1; t < n_threads; ++t) {
        if (pthread_create(&tids[t], NULL, diff_worker, &jobs[t]) != 0) {
            rc = 3;
            break;
        }
        started = t;
    }
    if (rc == 0)
        diff_worker(&jobs[0]);
    for (int32_t t = 1; t <= started; ++t)
        pthread_join(tids[t], NULL);
    free(jobs);
    free(tids);
    return rc;
}


/* ------------------------------------------------------------------------
 * Wavefront-recording method, first step (Section 2.3): the object wave of
 * the cloud recorded on a virtual plane placed at distance zw from the
 * hologram, between the hologram and the points, with each point's wave
 * written only over the small region of the plane its light crosses.
 *
 * The plane is an n x n grid of pitch p centred like the hologram: sample
 * (m, c) sits at x_w = (c - (n-1)/2) p, y_w = (m - (n-1)/2) p.  Point j lies
 * d_j = z_j - zw beyond the plane.  Its wave on the plane is Eq. (2) with
 * z_j replaced by d_j, without the per-point constant phase 2 pi d_j / lambda
 * (dropped as in the direct calculation):
 *
 *   u_w(x_w, y_w) = sum_{j : d_j > 0, (x_w - x_j)^2 + (y_w - y_j)^2 <= r_j^2}
 *                   A_j exp( i pi ((x_w - x_j)^2 + (y_w - y_j)^2) / (lambda d_j) ),
 *
 * over the disc of radius r_j = lambda d_j / (2 p) around (x_j, y_j): the
 * local frequency of the chirp, r / (lambda d_j) cycles per metre, reaches
 * the grid's limit 1 / (2 p) at r = r_j, so a larger region would alias.
 * Points at or in front of the plane (d_j <= 0) are not recorded.
 *
 * A plain loop over samples and points, FP64, libm cos/sin.  The region test
 * is evaluated exactly as written above (differences in metres, squared and
 * summed, against r_j squared), in FP64 without contraction.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    double pitch, wavelength, zw;
    const double *x, *y, *z, *a;
    int64_t n_points;
    const int32_t *rows;
    double *out_re, *out_im;
    int64_t row_begin, row_end;
} wrm_job_t;

static void *wrm_worker(void *arg)
{
    const wrm_job_t *jb = (const wrm_job_t *)arg;
    const double pi = 3.14159265358979323846;
    const double half = 0.5 * (double)(jb->n - 1);
    for (int64_t r = jb->row_begin; r < jb->row_end; ++r) {
        const double yw = ((double)jb->rows[r] - half) * jb->pitch;
        for (int32_t c = 0; c < jb->n; ++c) {
            const double xw = ((double)c - half) * jb->pitch;
            double sum_re = 0.0, sum_im = 0.0;
            for (int64_t i = 0; i < jb->n_points; ++i) {
                const double d = jb->z[i] - jb->zw;          /* beyond the plane */
                if (!(d > 0.0))
                    continue;
                const double dx = xw - jb->x[i];
                const double dy = yw - jb->y[i];
                const double rr = dx * dx + dy * dy;
                const double rj = jb->wavelength * d / (2.0 * jb->pitch);
                if (rr > rj * rj)
                    continue;                                  /* outside the region */
                const double theta = pi * rr / (jb->wavelength * d);
                sum_re += jb->a[i] * cos(theta);
                sum_im += jb->a[i] * sin(theta);
            }
            jb->out_re[r * jb->n + c] = sum_re;
            jb->out_im[r * jb->n + c] = sum_im;
        }
    }
    return NULL;
}

/* The recorded plane for rows rows[0 .. n_rows) (all n columns each);
 * out_re, out_im: n_rows x n.  Returns 0 on success. */
int cgh_oracle_wrm_record(int32_t n, double pitch, double wavelength, double zw,
                          int64_t n_points, const double *x, const double *y, const double *z,
                          const double *a, int64_t n_rows, const int32_t *rows, double *out_re,
                          double *out_im, int32_t n_threads)
{
    if (n <= 0 || n_points < 0 || n_rows < 0 || !(pitch > 0.0) || !(wavelength > 0.0))
        return 1;
    if (!out_re || !out_im || (n_rows > 0 && !rows))
        return 1;
    if (n_points > 0 && (!x || !y || !z || !a))
        return 1;
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > n_rows)
        n_threads = n_rows > 0 ? (int32_t)n_rows : 1;
    wrm_job_t *jobs = (wrm_job_t *)calloc((size_t)n_threads, sizeof(wrm_job_t));
    pthread_t *tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return 2;
    }
    for (int32_t t = 0; t < n_threads; ++t) {
        wrm_job_t *jb = &jobs[t];
        jb->n = n; jb->pitch = pitch; jb->wavelength = wavelength; jb->zw = zw;
        jb->x = x; jb->y = y; jb->z = z; jb->a = a; jb->n_points = n_points;
        jb->rows = rows; jb->out_re = out_re; jb->out_im = out_im;
        jb->row_begin = n_rows * t / n_threads;
        jb->row_end = n_rows * (t + 1) / n_threads;
    }
    int rc = 0;
    int32_t started = 0;
    for (int32_t t = 1; t < n_threads; ++t) {
        if (pthread_create(&tids[t], NULL, wrm_worker, &jobs[t]) != 0) {
            rc = 3;
            break;
        }
        started = t;
    }
    if (rc == 0)
        wrm_worker(&jobs[0]);
    for (int32_t t = 1; t <= started; ++t)
        pthread_join(tids[t], NULL);
    free(jobs);
    free(tids);
    return rc;
}
