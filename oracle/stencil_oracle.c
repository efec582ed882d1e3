/*
 * FP64 CPU oracle for iterated 1-D / 2-D / 3-D stencils with a fixed zero halo.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the GPU
 * path.
 *
 * What it computes (SPIDER, Sec. 2.2 "Stencil Computation" and Sec. 1): every
 * interior point is replaced by a weighted linear combination of the points in
 * its radius-r neighbourhood, one coefficient per neighbour, and the update is
 * repeated for `steps` time steps, each step reading only the result of the
 * previous one (Jacobi).  The paper's matrix formulation Y = K X of Sec. 3.1.1
 * is stated to be exactly this update, and the strided swap of Sec. 3.1.2 /
 * the row swap of Sec. 3.2 are stated to preserve it, so the oracle is the plain
 * definition written out:
 *
 *     y[p] = sum over offsets o in [-r, r]^d with w[o] != 0 of  w[o] * x[p + o]
 *
 * with x[p + o] = 0 when p + o lies outside the grid (fixed zero Dirichlet
 * halo), offsets visited in lexicographic order (dz, dy, dx), each product
 * rounded to fp64 and added to an fp64 accumulator in that order (the file is
 * compiled with -ffp-contract=off so no fused multiply-add changes a rounding).
 * The coefficient array is correlation-ordered: w[o] multiplies x[p + o]; no
 * flip.  Layout: row-major, x fastest: 1-D x[x], 2-D x[y][x], 3-D x[z][y][x];
 * coefficients w[dz][dy][dx] with each index running 0..2r (offset + r).
 *
 * Parallelism: OpenMP over the outermost grid axis only (1-D: over points;
 * each output point is still computed by one thread in the order above, so
 * results do not depend on the thread count).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* One step in 1-D (the paper's d = 1 case, Sec. 2.2). */
static void step1d(int64_t nx, int r, const double* w, const double* x, double* y) {
#pragma omp parallel for schedule(static)
    for (int64_t ix = 0; ix < nx; ++ix) {
        double acc = 0.0;
        for (int64_t dx = -r; dx <= r; ++dx) {
            const double c = w[dx + r];
            if (c == 0.0) continue;
            const int64_t sx = ix + dx;
            const double v = (sx >= 0 && sx < nx) ? x[sx] : 0.0;
            acc += c * v;
        }
        y[ix] = acc;
    }
}

/* One step in 2-D.  Returns nothing; all sizes are validated by the caller. */
static void step2d(int64_t ny, int64_t nx, int r, const double* w, const double* x, double* y) {
    const int64_t kw = 2 * r + 1;
#pragma omp parallel for schedule(static)
    for (int64_t iy = 0; iy < ny; ++iy) {
        for (int64_t ix = 0; ix < nx; ++ix) {
            double acc = 0.0;
            for (int64_t dy = -r; dy <= r; ++dy) {
                for (int64_t dx = -r; dx <= r; ++dx) {
                    const double c = w[(dy + r) * kw + (dx + r)];
                    if (c == 0.0) continue;
                    const int64_t sy = iy + dy, sx = ix + dx;
                    const double v = (sy >= 0 && sy < ny && sx >= 0 && sx < nx) ? x[sy * nx + sx] : 0.0;
                    acc += c * v;
                }
            }
            y[iy * nx + ix] = acc;
        }
    }
}

/* One step in 3-D. */
static void step3d(int64_t nz, int64_t ny, int64_t nx, int r, const double* w, const double* x, double* y) {
    const int64_t kw = 2 * r + 1;
#pragma omp parallel for schedule(static)
    for (int64_t iz = 0; iz < nz; ++iz) {
        for (int64_t iy = 0; iy < ny; ++iy) {
            for (int64_t ix = 0; ix < nx; ++ix) {
                double acc = 0.0;
                for (int64_t dz = -r; dz <= r; ++dz) {
                    for (int64_t dy = -r; dy <= r; ++dy) {
                        for (int64_t dx = -r; dx <= r; ++dx) {
                            const double c = w[((dz + r) * kw + (dy + r)) * kw + (dx + r)];
                            if (c == 0.0) continue;
                            const int64_t sz = iz + dz, sy = iy + dy, sx = ix + dx;
                            const int inside = sz >= 0 && sz < nz && sy >= 0 && sy < ny && sx >= 0 && sx < nx;
                            const double v = inside ? x[(sz * ny + sy) * nx + sx] : 0.0;
                            acc += c * v;
                        }
                    }
                }
                y[(iz * ny + iy) * nx + ix] = acc;
            }
        }
    }
}

/*
 * oracle_stencil: apply `steps` Jacobi steps.
 *   ndim    1, 2 or 3
 *   shape   ndim extents, slowest first ([nx], [ny, nx] or [nz, ny, nx]), each >= 1
 *   radius  r >= 0
 *   coeffs  (2r+1)^ndim fp64 coefficients, layout described above
 *   in      input grid (not modified unless in == out)
 *   out     output grid (may alias in)
 *   steps   >= 0 (0 copies in to out)
 *   nthreads  > 0 sets the OpenMP thread count for this call, <= 0 keeps the default
 * Returns 0 on success, -1 on invalid arguments, -2 if scratch allocation fails.
 */
int oracle_stencil(int ndim, const int64_t* shape, int radius, const double* coeffs,
                   const double* in, double* out, int steps, int nthreads) {
    if (ndim < 1 || ndim > 3 || !shape || radius < 0 || !coeffs || !in || !out || steps < 0) return -1;
    int64_t n = 1;
    for (int i = 0; i < ndim; ++i) {
        if (shape[i] < 1) return -1;
        n *= shape[i];
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    double* a = (double*)malloc((size_t)n * sizeof(double));
    double* b = (double*)malloc((size_t)n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -2; }
    memcpy(a, in, (size_t)n * sizeof(double));
    for (int s = 0; s < steps; ++s) {
        if (ndim == 1) step1d(shape[0], radius, coeffs, a, b);
        else if (ndim == 2) step2d(shape[0], shape[1], radius, coeffs, a, b);
        else step3d(shape[0], shape[1], shape[2], radius, coeffs, a, b);
        double* t = a; a = b; b = t;
    }
    memcpy(out, a, (size_t)n * sizeof(double));
    free(a);
    free(b);
    return 0;
}

/* Thread count OpenMP would use for a parallel region in this library. */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
