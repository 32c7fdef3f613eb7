/*
 * CPU oracle of the heat-bath estimator of the lattice N-body Coulomb energy.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the HIP library: it has its
 * own Philox, its own inverse normal CDF and its own storage rounding, all
 * written from their published definitions, in plain loops with no blocking,
 * fusion or reordering.
 *
 * What it computes (the paper's equations, restated):
 *   - Lattice action H_L = 1/2 sum over nearest-neighbour pairs of
 *     (phi_m - phi_n)^2 (the discretised free-field action, Eq. proplat).
 *     Sites outside the box hold phi = 0 (open boundary read as Dirichlet
 *     ghosts), so every site keeps 6 neighbours.
 *   - Heat-bath update (Eq. hb1 inverted as Eq. phi): the new value of a
 *     site is the mean of its 6 neighbours plus a Gaussian of variance 1/6,
 *     drawn by inverting the conditional CDF at a uniform r:
 *       phi_n = (1/6) sum_m phi_m - erfc^{-1}(2r)/sqrt(3)
 *             = (1/6) sum_m phi_m + Phi^{-1}(r)/sqrt(6).
 *   - Sites are visited in red-black order (colour c = (x+y+z) & 1; all
 *     colour-0 sites, then all colour-1 sites).  Same-colour sites are not
 *     neighbours, so this order has the same stationary law e^{-H_L} as the
 *     paper's sequential order.
 *   - Measurement (Eq. nsum2): X = sum_i q_i phi(n_i), Y = sum_i q_i^2
 *     phi(n_i)^2, sample O = X^2 - Y; E_N is the mean of O.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11).  Site with linear index
 * i = x + lx*(y + ly*z) and compact index j = i >> 1, in half-sweep h, uses
 * word (j & 3) of Philox(counter = (j >> 2, h, chain, 0), key = (lo32(seed),
 * hi32(seed))).  Uniform: k = word >> 8, r = (k + 1/2) * 2^-24.
 *
 * Arithmetic is FP64; each stored value is rounded to the storage format:
 * 0 = FP32, 1 = BF16, 2 = FP16 (round-to-nearest-even), 3 = BF16, 4 = FP16
 * (stochastic rounding with the 8 low bits of the site's Philox word, which
 * the uniform does not use; ties broken by the parity of those bits).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10                                                       */
/* ------------------------------------------------------------------ */
/* Multipliers and Weyl key increments of Philox4x32 (Salmon et al. 2011). */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { /* key schedule: add the Weyl constants before rounds 2..10 */
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------ */
/* Standard normal CDF and its inverse (FP64)                          */
/* ------------------------------------------------------------------ */
static const double ORC_INV_SQRT2 = 0.70710678118654752440;
static const double ORC_INV_SQRT2PI = 0.39894228040143267794;

/* Phi(z) = erfc(-z / sqrt 2) / 2, from libm. */
double orc_norm_cdf(double z) { return 0.5 * erfc(-z * ORC_INV_SQRT2); }

/*
 * Phi^{-1}(r) for 0 < r < 1: the root of Phi(z) = r, found by Newton's method
 * on the libm CDF.  Start: Abramowitz & Stegun 26.2.23 (|error| < 4.5e-4).
 * Near the centre the residual is formed as erf(z/sqrt2)/2 - (r - 1/2) to
 * avoid cancellation; in the tails by erfc.  Upper half by symmetry.
 */
double orc_inv_norm_cdf(double r) {
    if (!(r > 0.0 && r < 1.0)) return NAN;
    if (r == 0.5) return 0.0;
    if (r > 0.5) return -orc_inv_norm_cdf(1.0 - r);
    /* lower half: z < 0 */
    double t = sqrt(-2.0 * log(r));
    double z = -(t - (2.515517 + t * (0.802853 + t * 0.010328)) /
                         (1.0 + t * (1.432788 + t * (0.189269 + t * 0.001308))));
    double dr = r - 0.5; /* exact for r on a dyadic grid */
    for (int it = 0; it < 50; ++it) {
        double f;
        if (r > 0.25)
            f = 0.5 * erf(z * ORC_INV_SQRT2) - dr;
        else
            f = 0.5 * erfc(-z * ORC_INV_SQRT2) - r;
        double dens = ORC_INV_SQRT2PI * exp(-0.5 * z * z);
        double step = f / dens;
        z -= step;
        if (fabs(step) <= 4e-17 * fabs(z) || step == 0.0) break;
    }
    return z;
}

/* ------------------------------------------------------------------ */
/* Storage rounding                                                     */
/* ------------------------------------------------------------------ */
/* Round v to p significant bits, round-to-nearest-even, with the smallest
 * normal exponent emin (below it the spacing stays 2^(emin-p+1), i.e. the
 * subnormal grid).  Overflow is not handled: field values stay far below it. */
static double orc_round_sig(double v, int p, int emin) {
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    (void)frexp(v, &e); /* |v| = m 2^e, 1/2 <= m < 1: leading bit has weight 2^(e-1) */
    int lead = e - 1;
    if (lead < emin) lead = emin;
    double ulp = ldexp(1.0, lead - p + 1);
    return nearbyint(v / ulp) * ulp; /* division by a power of two is exact */
}

double orc_round_storage(double v, int storage) {
    switch (storage) {
        case 0: return (double)(float)v;                 /* FP32, RNE        */
        case 1: return orc_round_sig(v, 8, -126);        /* BF16: 8-bit sig  */
        case 2: return orc_round_sig(v, 11, -14);        /* FP16: 11-bit sig */
        default: return NAN;
    }
}

/* Stochastic rounding to p significant bits (smallest normal exponent emin,
 * the subnormal grid below it).  lo is |v| rounded toward zero to the grid,
 * ulp the grid spacing there and f = (|v| - lo) / ulp in [0, 1).  With u8
 * the 8 random bits (0 .. 255) and t = 256 f + u8, the magnitude becomes
 * lo + ulp when t > 255.5, or when t = 255.5 and u8 is even, else lo.  Over
 * the 256 values of u8 it rounds up in the nearest whole number of cases to
 * 256 f, so the mean result is |v| up to ulp / 512.  The tie t = 255.5 needs
 * 256 f to end in exactly one half, which values with few bits below the
 * grid (FP32 values: 13 bits below FP16's, 16 below BF16's) reach for 1/32
 * and 1/256 of values: sending every tie up would move magnitudes away from
 * zero on average, so ties go up for even u8 (u8 = 255.5 - 256 f: the parity
 * of the value's own digit) and down for odd.  The sign is kept. */
static double orc_round_sig_sr(double v, int p, int emin, uint32_t u8) {
    if (v == 0.0 || !isfinite(v)) return v;
    const double a = fabs(v);
    int e;
    (void)frexp(a, &e);
    int lead = e - 1;
    if (lead < emin) lead = emin;
    const double ulp = ldexp(1.0, lead - p + 1);
    const double lo = floor(a / ulp) * ulp;  /* exact: division by a power of two */
    const double f = (a - lo) / ulp;          /* exact */
    const double t = 256.0 * f + (double)(u8 & 0xFFu);  /* exact: below 512, 53 bits */
    const int up = t > 255.5 || (t == 255.5 && (u8 & 1u) == 0u);
    const double m = up ? lo + ulp : lo;
    return v < 0.0 ? -m : m;
}

double orc_round_storage_sr(double v, int storage, uint32_t u8) {
    switch (storage) {
        case 3: return orc_round_sig_sr(v, 8, -126, u8);  /* BF16 */
        case 4: return orc_round_sig_sr(v, 11, -14, u8);  /* FP16 */
        default: return NAN;
    }
}

/* The mean over the 256 values of u8 of the stochastic rounding of each of
 * v[0 .. n-1] (tests of the rounding's bias). */
void orc_round_storage_sr_mean(const double *v, int64_t n, int storage, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (uint32_t u = 0; u < 256u; ++u) s += orc_round_storage_sr(v[i], storage, u);
        out[i] = s / 256.0;
    }
}

/* ------------------------------------------------------------------ */
/* Heat bath                                                            */
/* ------------------------------------------------------------------ */
static inline double orc_at(const double *phi, int64_t lx, int64_t ly, int64_t lz,
                            int64_t x, int64_t y, int64_t z) {
    if (x < 0 || x >= lx || y < 0 || y >= ly || z < 0 || z >= lz) return 0.0; /* ghost */
    return phi[x + lx * (y + ly * z)];
}

/* The Philox word of site (x,y,z) in half-sweep h. */
uint32_t orc_site_word(int64_t lx, int64_t ly, int64_t x, int64_t y, int64_t z,
                       uint64_t seed, uint32_t chain, uint32_t h) {
    int64_t i = x + lx * (y + ly * z);
    int64_t j = i >> 1;
    uint32_t ctr[4] = {(uint32_t)(j >> 2), h, chain, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    return w[j & 3];
}

/* Uniform r in (0,1) used by site (x,y,z) in half-sweep h. */
double orc_site_uniform(int64_t lx, int64_t ly, int64_t x, int64_t y, int64_t z,
                        uint64_t seed, uint32_t chain, uint32_t h) {
    uint32_t k = orc_site_word(lx, ly, x, y, z, seed, chain, h) >> 8;
    return ((double)k + 0.5) * 0x1p-24;
}

/* The heat-bath value of site (x,y,z) in half-sweep h, before rounding. */
double orc_site_value(const double *phi, int64_t lx, int64_t ly, int64_t lz,
                      int64_t x, int64_t y, int64_t z, uint64_t seed, uint32_t chain, uint32_t h) {
    double s = orc_at(phi, lx, ly, lz, x - 1, y, z) + orc_at(phi, lx, ly, lz, x + 1, y, z) +
               orc_at(phi, lx, ly, lz, x, y - 1, z) + orc_at(phi, lx, ly, lz, x, y + 1, z) +
               orc_at(phi, lx, ly, lz, x, y, z - 1) + orc_at(phi, lx, ly, lz, x, y, z + 1);
    double r = orc_site_uniform(lx, ly, x, y, z, seed, chain, h);
    return s / 6.0 + orc_inv_norm_cdf(r) / sqrt(6.0);
}

/* One half-sweep: every site of colour (h & 1) takes its heat-bath value. */
void orc_halfsweep(double *phi, int64_t lx, int64_t ly, int64_t lz, int storage,
                   uint64_t seed, uint32_t chain, uint32_t h) {
    int c = (int)(h & 1u);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < lz; ++z)
        for (int64_t y = 0; y < ly; ++y)
            for (int64_t x = 0; x < lx; ++x) {
                if ((int)((x + y + z) & 1) != c) continue;
                double v = orc_site_value(phi, lx, ly, lz, x, y, z, seed, chain, h);
                phi[x + lx * (y + ly * z)] =
                    storage >= 3 ? orc_round_storage_sr(v, storage, orc_site_word(lx, ly, x, y, z, seed, chain, h) & 0xFFu)
                                 : orc_round_storage(v, storage);
            }
}

/* X = sum q_i phi(n_i) and Y = sum q_i^2 phi(n_i)^2 over the raw charge list. */
void orc_gather(const double *phi, int64_t lx, int64_t ly, int64_t lz, int64_t n,
                const int32_t *xyz, const double *q, double out[2]) {
    double X = 0.0, Y = 0.0;
    (void)lz;
    for (int64_t i = 0; i < n; ++i) {
        double v = phi[xyz[3 * i] + lx * (xyz[3 * i + 1] + ly * (int64_t)xyz[3 * i + 2])];
        X += q[i] * v;
        Y += (q[i] * v) * (q[i] * v);
    }
    out[0] = X;
    out[1] = Y;
}

/*
 * Off-lattice charges (the paper's closing remark: an arbitrary position can
 * be modelled by its nearest eight lattice sites, and forces evaluated by
 * interpolation in the same way).  Site (x, y, z) sits at position (x, y, z)
 * (lattice units).  A charge at r with 0 <= r_d <= L_d - 1 (L_d >= 2) lies in
 * the cell with origin b_d = min(floor(r_d), L_d - 2) and fraction
 * f_d = r_d - b_d in [0, 1]; corner b + e (e in {0, 1}^3) carries the
 * trilinear weight w = prod_d (e_d ? f_d : 1 - f_d).  The field at the charge
 * is the interpolant phi~(r) = sum over corners of w phi(corner); its
 * gradient in r within the cell is, for x, sum over corners of
 * (e_x ? 1 : -1) * (y and z weight factors) * phi(corner), and likewise for y
 * and z.  Samples: X = sum_i q_i phi~(r_i), Y = sum_i (q_i phi~(r_i))^2.
 * phit (n values) and grad (3n values) receive phi~ and its gradient when
 * not NULL.
 */
void orc_gather_offlattice(const double *phi, int64_t lx, int64_t ly, int64_t lz, int64_t n,
                           const double *r, const double *q, double out[2], double *phit, double *grad) {
    const int64_t L[3] = {lx, ly, lz};
    double X = 0.0, Y = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t b[3];
        double f[3];
        for (int d = 0; d < 3; ++d) {
            double fl = floor(r[3 * i + d]);
            if (fl > (double)(L[d] - 2)) fl = (double)(L[d] - 2);
            b[d] = (int64_t)fl;
            f[d] = r[3 * i + d] - fl;
        }
        double v = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int ez = 0; ez < 2; ++ez)
            for (int ey = 0; ey < 2; ++ey)
                for (int ex = 0; ex < 2; ++ex) {
                    const double wx = ex ? f[0] : 1.0 - f[0];
                    const double wy = ey ? f[1] : 1.0 - f[1];
                    const double wz = ez ? f[2] : 1.0 - f[2];
                    const double p = phi[(b[0] + ex) + lx * ((b[1] + ey) + ly * (b[2] + ez))];
                    v += wx * wy * wz * p;
                    g[0] += (ex ? 1.0 : -1.0) * wy * wz * p;
                    g[1] += wx * (ey ? 1.0 : -1.0) * wz * p;
                    g[2] += wx * wy * (ez ? 1.0 : -1.0) * p;
                }
        X += q[i] * v;
        Y += (q[i] * v) * (q[i] * v);
        if (phit) phit[i] = v;
        if (grad)
            for (int d = 0; d < 3; ++d) grad[3 * i + d] = g[d];
    }
    out[0] = X;
    out[1] = Y;
}

/*
 * n_sweeps full sweeps starting at sweep counter t0 (sweep t = half-sweeps
 * 2t then 2t+1).  After every sweep whose 1-based position in this call is a
 * multiple of measure_every (0 = never), one sample is written:
 * samples[3m+0..2] = (X, Y, X^2 - Y).  Returns the number of samples.
 */
int64_t orc_run(double *phi, int64_t lx, int64_t ly, int64_t lz, int storage, uint64_t seed,
                uint32_t chain, int64_t t0, int64_t n_sweeps, int64_t measure_every, int64_t n,
                const int32_t *xyz, const double *q, double *samples) {
    int64_t m = 0;
    for (int64_t s = 0; s < n_sweeps; ++s) {
        int64_t t = t0 + s;
        orc_halfsweep(phi, lx, ly, lz, storage, seed, chain, (uint32_t)(2 * t));
        orc_halfsweep(phi, lx, ly, lz, storage, seed, chain, (uint32_t)(2 * t + 1));
        if (measure_every > 0 && (s + 1) % measure_every == 0) {
            double xy[2];
            orc_gather(phi, lx, ly, lz, n, xyz, q, xy);
            samples[3 * m + 0] = xy[0];
            samples[3 * m + 1] = xy[1];
            samples[3 * m + 2] = xy[0] * xy[0] - xy[1];
            ++m;
        }
    }
    return m;
}

/*
 * Heat-bath values (before rounding) at a list of sites, all of colour
 * (h & 1), read from an FP32 field in natural order: used to check sampled
 * sites of a large lattice one by one.
 */
void orc_site_values_f32(const float *phi, int64_t lx, int64_t ly, int64_t lz, int64_t n,
                         const int64_t *xyz, uint64_t seed, uint32_t chain, uint32_t h,
                         double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        int64_t x = xyz[3 * k], y = xyz[3 * k + 1], z = xyz[3 * k + 2];
        double s = 0.0;
        const int64_t dx[6] = {-1, 1, 0, 0, 0, 0}, dy[6] = {0, 0, -1, 1, 0, 0},
                      dz[6] = {0, 0, 0, 0, -1, 1};
        for (int d = 0; d < 6; ++d) {
            int64_t a = x + dx[d], b = y + dy[d], c = z + dz[d];
            if (a < 0 || a >= lx || b < 0 || b >= ly || c < 0 || c >= lz) continue;
            s += (double)phi[a + lx * (b + ly * c)];
        }
        double r = orc_site_uniform(lx, ly, x, y, z, seed, chain, h);
        out[k] = s / 6.0 + orc_inv_norm_cdf(r) / sqrt(6.0);
    }
}

/*
 * The heat-bath noise Phi^{-1}(r)/sqrt(6) of Eq. (phi) at the grid points
 * k = k_first .. k_first + n - 1 of the uniform r = (k + 1/2) 2^-24.
 */
void orc_noise_grid(int64_t k_first, int64_t n, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = orc_inv_norm_cdf(((double)(k_first + i) + 0.5) * 0x1p-24) / sqrt(6.0);
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
