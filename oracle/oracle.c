/*
 * CPU oracle for homogeneous diffusion inpainting -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library. The product path never calls it and shares
 * no code with it.
 *
 * What it computes (Sec. 2, eqs. 5-6): the exact solution of
 *     A u = b,   A = C - (I - C) L,   b = C f,
 * per channel, in double precision. L is the 5-point Laplacian with
 * reflecting (homogeneous Neumann, eq. 3) boundary conditions, read as
 * half-sample mirroring: a neighbour outside the image equals the border
 * pixel itself, so it contributes nothing and the diagonal counts only the
 * in-image neighbours (2, 3 or 4). C is the 0/1 diagonal of the mask.
 *
 * Rows of known pixels say u_p = f_p. Moving them to the right-hand side
 * leaves, for every unknown pixel p,
 *     sum_{q in N(p)} (u_p - u_q) = 0,
 * i.e. K u_U = g with K symmetric, diagonally dominant and positive definite
 * as soon as one pixel is known. That reduced system is solved by plain
 * conjugate gradients (Hestenes-Stiefel) from u_U = 0 until the recursively
 * updated residual satisfies ||g - K u_U||_2 <= tol * ||g||_2; then u_K = f_K
 * is copied bit for bit.
 *
 * Everything is matrix-free on the full H x W grid: vectors hold 0 at known
 * pixels. Reductions are summed per row and then over rows in a fixed
 * order, so the result does not depend on the number of OpenMP threads.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Threads only pay off on large images; tiny ones run serially. */
#define PAR(h, w) ((long)(h) * (long)(w) >= 65536L)

/* (K x)_p for unknown p; 0 at known pixels. x must be 0 at known pixels. */
static void apply_k(int h, int w, const unsigned char *c, const double *x,
                    double *y)
{
#pragma omp parallel for schedule(static) if (PAR(h, w))
    for (int i = 0; i < h; ++i) {
        for (int j = 0; j < w; ++j) {
            long p = (long)i * w + j;
            if (c[p]) { y[p] = 0.0; continue; }
            double deg = 0.0, s = 0.0;
            if (i > 0)     { deg += 1.0; s += x[p - w]; }
            if (i < h - 1) { deg += 1.0; s += x[p + w]; }
            if (j > 0)     { deg += 1.0; s += x[p - 1]; }
            if (j < w - 1) { deg += 1.0; s += x[p + 1]; }
            y[p] = deg * x[p] - s;
        }
    }
}

/* Fixed-order dot product: per-row partial sums, then rows in order. */
static double dot(int h, int w, const double *a, const double *b, double *rowbuf)
{
#pragma omp parallel for schedule(static) if (PAR(h, w))
    for (int i = 0; i < h; ++i) {
        double s = 0.0;
        const double *pa = a + (long)i * w, *pb = b + (long)i * w;
        for (int j = 0; j < w; ++j) s += pa[j] * pb[j];
        rowbuf[i] = s;
    }
    double s = 0.0;
    for (int i = 0; i < h; ++i) s += rowbuf[i];
    return s;
}

/*
 * Solve one channel. f, u: h*w doubles, row-major. c: h*w bytes, 0 or 1.
 * Returns 0 on success, 1 if the mask is empty (A singular), 2 if max_iter
 * was reached, -1 on bad arguments or allocation failure. *iters and
 * *relres report the CG iteration count and the final relative residual
 * of the reduced system (true residual, recomputed at the end).
 */
int oracle_solve(int h, int w, const double *f, const unsigned char *c,
                 double *u, double tol, int max_iter, int *iters,
                 double *relres)
{
    if (h <= 0 || w <= 0 || !f || !c || !u) return -1;
    long n = (long)h * w;
    long nknown = 0;
    for (long p = 0; p < n; ++p) {
        if (c[p] > 1) return -1;
        nknown += c[p];
    }
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    if (nknown == 0) return 1;

    double *g = calloc(n, sizeof(double));
    double *x = calloc(n, sizeof(double));
    double *r = calloc(n, sizeof(double));
    double *p = calloc(n, sizeof(double));
    double *q = calloc(n, sizeof(double));
    double *rowbuf = calloc(h, sizeof(double));
    if (!g || !x || !r || !p || !q || !rowbuf) {
        free(g); free(x); free(r); free(p); free(q); free(rowbuf);
        return -1;
    }

    /* g_p = sum of f over the known neighbours of unknown p. */
#pragma omp parallel for schedule(static) if (PAR(h, w))
    for (int i = 0; i < h; ++i) {
        for (int j = 0; j < w; ++j) {
            long k = (long)i * w + j;
            if (c[k]) continue;
            double s = 0.0;
            if (i > 0 && c[k - w])     s += f[k - w];
            if (i < h - 1 && c[k + w]) s += f[k + w];
            if (j > 0 && c[k - 1])     s += f[k - 1];
            if (j < w - 1 && c[k + 1]) s += f[k + 1];
            g[k] = s;
        }
    }

    double gnorm = sqrt(dot(h, w, g, g, rowbuf));
    int it = 0, status = 0;
    if (gnorm > 0.0) {
        memcpy(r, g, n * sizeof(double));      /* x = 0, r = g */
        memcpy(p, r, n * sizeof(double));
        double rho = dot(h, w, r, r, rowbuf);
        while (sqrt(rho) > tol * gnorm) {
            if (it >= max_iter) { status = 2; break; }
            apply_k(h, w, c, p, q);
            double alpha = rho / dot(h, w, p, q, rowbuf);
#pragma omp parallel for schedule(static) if (PAR(h, w))
            for (long k = 0; k < n; ++k) {
                x[k] += alpha * p[k];
                r[k] -= alpha * q[k];
            }
            double rho_new = dot(h, w, r, r, rowbuf);
            double beta = rho_new / rho;
#pragma omp parallel for schedule(static) if (PAR(h, w))
            for (long k = 0; k < n; ++k) p[k] = r[k] + beta * p[k];
            rho = rho_new;
            ++it;
        }
        /* true residual of the reduced system */
        apply_k(h, w, c, x, q);
#pragma omp parallel for schedule(static) if (PAR(h, w))
        for (long k = 0; k < n; ++k) r[k] = g[k] - q[k];
        if (relres) *relres = sqrt(dot(h, w, r, r, rowbuf)) / gnorm;
    }

#pragma omp parallel for schedule(static) if (PAR(h, w))
    for (long k = 0; k < n; ++k) u[k] = c[k] ? f[k] : x[k];

    if (iters) *iters = it;
    free(g); free(x); free(r); free(p); free(q); free(rowbuf);
    return status;
}

/* Number of OpenMP threads a parallel region of this library uses. */
int oracle_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
