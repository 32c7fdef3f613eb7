/* Lattice Green's function by conjugate gradients (test infrastructure of the
 * CPU oracle; nothing outside tests/ and the benchmark's CPU baseline uses
 * it).
 *
 * The free-field action of the paper (Sec. 2, the discretised action and its
 * propagator) has the Hessian A = -Delta_L: 6 on the diagonal and -1 to each
 * of the 6 nearest neighbours, the field being 0 outside the box (Dirichlet
 * boundary).  The propagator is G = A^{-1}; a column G(., n) is the solution
 * u of A u = e_n.  This file solves A u = b in FP64 by plain conjugate
 * gradients (no preconditioner, no transform: independent of the DST-I
 * solution in exact.py).  Natural layout, x fastest: i = x + lx (y + ly z).
 * Dot products are summed per z plane and the planes in order, so the result
 * does not depend on the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static void apply_a(const double *p, double *q, int64_t lx, int64_t ly, int64_t lz) {
    const int64_t plane = lx * ly;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < lz; ++z)
        for (int64_t y = 0; y < ly; ++y) {
            const int64_t row = lx * (y + ly * z);
            for (int64_t x = 0; x < lx; ++x) {
                const int64_t i = row + x;
                double s = 0.0;
                if (x > 0) s += p[i - 1];
                if (x + 1 < lx) s += p[i + 1];
                if (y > 0) s += p[i - lx];
                if (y + 1 < ly) s += p[i + lx];
                if (z > 0) s += p[i - plane];
                if (z + 1 < lz) s += p[i + plane];
                q[i] = 6.0 * p[i] - s;
            }
        }
}

static double dot(const double *a, const double *b, int64_t lz, int64_t plane, double *part) {
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < lz; ++z) {
        double s = 0.0;
        for (int64_t i = z * plane; i < (z + 1) * plane; ++i) s += a[i] * b[i];
        part[z] = s;
    }
    double s = 0.0;
    for (int64_t z = 0; z < lz; ++z) s += part[z];
    return s;
}

/* u = A^{-1} b to ||b - A u|| <= rtol ||b|| (u need not be initialised).
 * Returns the number of iterations, -1 if maxit was reached, -2 on an
 * allocation failure. */
int64_t orc_cg_laplacian(int64_t lx, int64_t ly, int64_t lz, const double *b, double *u, double rtol,
                         int64_t maxit) {
    const int64_t plane = lx * ly, n = plane * lz;
    double *r = malloc(sizeof(double) * (size_t)n), *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n), *part = malloc(sizeof(double) * (size_t)lz);
    if (!r || !p || !q || !part) {
        free(r), free(p), free(q), free(part);
        return -2;
    }
    memset(u, 0, sizeof(double) * (size_t)n);
    memcpy(r, b, sizeof(double) * (size_t)n);
    memcpy(p, b, sizeof(double) * (size_t)n);
    double rs = dot(r, r, lz, plane, part);
    const double stop = rtol * rtol * rs;
    int64_t it = 0;
    while (rs > stop) {
        if (it == maxit) {
            it = -1;
            break;
        }
        apply_a(p, q, lx, ly, lz);
        const double alpha = rs / dot(p, q, lz, plane, part);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            u[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        const double rs1 = dot(r, r, lz, plane, part);
        const double beta = rs1 / rs;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rs = rs1;
        ++it;
    }
    free(r), free(p), free(q), free(part);
    return it;
}
