/*
 * lattice_coulomb.h -- C ABI of the MI355X heat-bath estimator of the
 * lattice N-body Coulomb energy.
 *
 * The method (Sugihara, Higo, Nakamura, "Local Representation of N-body
 * Coulomb Energy with Path Integrals"):
 *   - The Coulomb energy of charges q_i at sites r_i, summed over ordered
 *     pairs, E_N = (1/4pi) sum_{i != j} q_i q_j / |r_i - r_j| (Eq. s1), is a
 *     sum of Green's functions of -Laplacian, and each Green's function is a
 *     two-point average of a free scalar field (Eq. path).
 *   - On a cubic lattice with unit spacing and action
 *     H_L = 1/2 sum_<m,n> (phi_m - phi_n)^2 (Eq. proplat), the field average
 *     E_N ~ < (sum_i q_i phi_{n_i})^2 - sum_i (q_i phi_{n_i})^2 > (Eq. nsum)
 *     is estimated by the mean over M Monte-Carlo samples (Eq. nsum2).
 *   - Samples come from a Gaussian heat bath: a site takes the mean of its 6
 *     neighbours plus a Gaussian of variance 1/6, drawn by inverting the
 *     conditional CDF at a uniform r (Eqs. hb1 and phi).
 *
 * What this library computes, exactly:
 *   - Box lx * ly * lz, sites (x, y, z) 0-based, x fastest.  The paper's open
 *     boundary is read as Dirichlet ghosts: phi = 0 outside the box, so every
 *     site keeps 6 neighbours and the update is unchanged at the boundary.
 *   - Red-black order: colour c = (x + y + z) & 1; sweep t updates colour 0
 *     (half-sweep h = 2t) then colour 1 (h = 2t + 1).  t counts every sweep
 *     since lattice_create (thermalisation included).
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11).  Site
 *     i = x + lx (y + ly z), compact index j = i >> 1, half-sweep h, uses word
 *     (j & 3) of Philox(counter = (j >> 2, h, chain_id, 0),
 *     key = (lo32(seed), hi32(seed))); k = word >> 8; r = (k + 1/2) 2^-24.
 *   - Update: phi = (1/6) sum of the 6 neighbours + erfinv(2r - 1)/sqrt(3)
 *     (= Eq. phi's -erfc^{-1}(2r)/sqrt(3)), in FP32 arithmetic, stored
 *     rounded in the storage format (to nearest even, or stochastically
 *     with the word's low 8 bits: LAT_BF16_SR, LAT_FP16_SR).
 *   - A measured sweep adds O = X^2 - Y, X = sum_i q_i phi(n_i),
 *     Y = sum_i q_i^2 phi(n_i)^2 (FP64), into bins of bin_size consecutive
 *     samples with compensated (Kahan) FP64 sums.
 *
 * Conventions for every call:
 *   - Sizes are int64_t; host arrays are read during the call and copied
 *     (the caller keeps ownership).  Device memory belongs to the handle.
 *   - Work is enqueued on the HIP stream given at creation (NULL = the null
 *     stream).  Calls that return data to the host synchronise that stream.
 *   - Every call returns LAT_OK or an error code; nothing is thrown across
 *     the ABI.  A failed validation leaves the handle unchanged.  The message
 *     of the last error on the calling thread is lattice_last_error().
 *   - A handle is not thread-safe: calls on one handle must not overlap.
 */
#ifndef LATTICE_COULOMB_H
#define LATTICE_COULOMB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lattice lattice_t;
typedef struct lattice_batch lattice_batch_t;

/* Device-memory provider.  alloc returns device memory of `bytes` bytes on
 * the current device (NULL on failure); release frees it.  A NULL provider
 * means hipMalloc / hipFree.  The provider must outlive the handle. */
typedef struct {
    void *ctx;
    void *(*alloc)(void *ctx, size_t bytes);
    void (*release)(void *ctx, void *ptr);
} lat_allocator;

enum {
    LAT_OK = 0,
    LAT_ERR_ARG = 1,    /* invalid argument                                   */
    LAT_ERR_STATE = 2,  /* call not valid in the handle's state               */
    LAT_ERR_ALLOC = 3,  /* the allocator returned NULL                         */
    LAT_ERR_DEVICE = 4  /* a HIP call failed                                   */
};

/* Field storage format.  Arithmetic is FP32 in every format; an updated
 * value is stored rounded to nearest even (FP32, BF16, FP16) or, in the SR
 * formats, stochastically rounded to BF16 or FP16 with the 8 low bits u8 of
 * the site's Philox word (which the uniform does not use): with f the
 * value's distance past the grid point below its magnitude in grid
 * spacings, the magnitude goes up to the next grid point when
 * 256 f + u8 >= 255.5.  Over the 256 values of u8 the mean stored value is
 * the FP32 value to 1/512 of a spacing.  Rounding to nearest even instead
 * shrinks values toward zero on average (at each power of two its cell
 * reaches half the smaller spacing below and half the larger one above),
 * a weak mass term that lowers E_N on large boxes.  An SR format's arrays
 * are those of the round-to-nearest format of the same width (field
 * uploads round to nearest even). */
enum { LAT_FP32 = 0, LAT_BF16 = 1, LAT_FP16 = 2, LAT_BF16_SR = 3, LAT_FP16_SR = 4 };

/* Sweep kernel selection for lattice_set_variant. */
enum {
    LAT_SWEEP_AUTO = 0,    /* library choice: resident (<= 16,384 sites, one on-lattice
                              set), generic (lx % 8 != 0), stream (fields >= 256 MB),
                              zslab (FP32/BF16 from 2^23 sites), else quad             */
    LAT_SWEEP_QUAD = 1,    /* 4 sites per thread, one pass per half-sweep (lx % 8 == 0) */
    LAT_SWEEP_GENERIC = 2, /* 1 site per thread, any even lx                        */
    LAT_SWEEP_ZSLAB = 3,   /* z-marching slabs, plane staged in LDS (lx % 8 == 0)   */
    LAT_SWEEP_FUSED = 4,   /* both half-sweeps in one pass (lx % 8 == 0)             */
    LAT_SWEEP_RESIDENT = 5, /* small boxes: one workgroup runs every sweep of a call in one launch */
    LAT_SWEEP_STREAM = 6,   /* z-marching slabs fed by a producer wave through an LDS ring
                               (lx % 8 == 0, each colour array below 2 GiB)         */
    LAT_SWEEP_BLOCKED = 7   /* both half-sweeps per pass over memory, colour 0 kept in LDS:
                               full-row tiles walking z-slabs (lx % 8 == 0; 16-bit storage
                               lx % 16 == 0; rows of at most ~2300 sites at FP32) */
};

/* ------------------------------------------------------------------ */
/* Single lattice                                                      */
/* ------------------------------------------------------------------ */

/* Create a chain on an lx*ly*lz box with field phi = 0 and sweep counter 0.
 * lx must be even and >= 2, ly, lz >= 1, lx*ly*lz < 2^31.  storage is a
 * LAT_FP32/BF16/FP16/BF16_SR/FP16_SR value.  seed keys Philox; chain_id is counter word 2
 * (independent chains of one seed use distinct chain_ids).  hip_stream is a
 * hipStream_t (NULL = null stream), borrowed, never destroyed.
 * Paper: the lattice L^3 and spacing a = 1 of the discretisation (Eq.
 * proplat), the open boundary of the paper's tests. */
int lattice_create(int64_t lx, int64_t ly, int64_t lz, int storage, uint64_t seed,
                   uint32_t chain_id, const lat_allocator *alloc, void *hip_stream,
                   lattice_t **out);

/* Place n charges: xyz = 3n int32 (x, y, z) host array, q = n doubles (host).
 * Charges on one site are summed per site keeping the ordered-pair sum of
 * Eq. (nsum) exact (co-located i != j pairs included).  n = 0 is allowed
 * (E = 0).  Errors: LAT_ERR_ARG for a site outside the box or a non-finite q.
 * Resets the measurement bins (samples of a different charge set do not
 * mix); the field and the sweep counter are kept (the samples of the field
 * do not depend on the charges, as the paper notes). */
int set_charges(lattice_t *lat, int64_t n, const int32_t *xyz, const double *q);

/* Several charge sets measured on one field chain: every measured sweep
 * takes one sample per set, each into its own bins.  The paper notes that a
 * stored set of field samples can serve any charge configuration; here the
 * sets share the sweeps as they are made, so the sweep cost is paid once for
 * all of them.  n_sets in [1, 65535]; counts = n_sets int64 (charges per
 * set); xyz (3 int32 per charge) and q (one double per charge) hold the sets
 * one after the other.  Each set is aggregated per site as in set_charges.
 * Resets the bins of every set; the field and sweep counter are kept.
 * Up to four sets are gathered inside the blocked sweep (one walk over
 * lists holding every set's sites); more sets, or other kernels, gather
 * each sample from memory.
 * set_charges is the case n_sets = 1.  Errors as set_charges; LAT_ERR_ARG
 * also for n_sets out of range, a negative count, or n_sets > 1 with the
 * variant LAT_SWEEP_RESIDENT (which measures one set). */
int lattice_set_charge_sets(lattice_t *lat, int64_t n_sets, const int64_t *counts,
                            const int32_t *xyz, const double *q);

/* Charges at arbitrary positions (the paper's closing remark: model each
 * position by its nearest eight lattice sites, and evaluate forces by
 * interpolation the same way).  Site (x, y, z) sits at position (x, y, z)
 * in lattice units; r = 3n doubles (host), each coordinate in
 * [0, L_d - 1]; q = n doubles (host).  A charge at r lies in the cell with
 * origin b_d = min(floor(r_d), L_d - 2) and spreads over its 8 corners with
 * trilinear weights w; the field at the charge is phi~ = sum w phi.  A
 * sample is O = X^2 - Y with X = sum_i q_i phi~_i and Y = sum_i
 * (q_i phi~_i)^2, whose mean is sum_{i != j} q_i q_j w_i^T G w_j (equal to
 * the on-lattice energy at integer positions).  forces != 0 also
 * accumulates, at every sample, dO/dr_i = 2 q_i grad phi~_i (X - q_i phi~_i)
 * (the gradient of the interpolant within the cell), whose mean is dE/dr_i
 * (read with lattice_force_estimate; E sums ordered pairs, so the physical
 * force on charge i is -(1/2) dE/dr_i).  The library keeps the charges
 * sorted by cell (nearby charges then read shared cache lines close in
 * time); lattice_force_estimate returns them in the caller's order, and only
 * the order of the FP64 sums X and Y follows the sorted one.  Replaces all
 * charge sets; resets the bins and force sums; the field and sweep counter
 * are kept.  Errors:
 * LAT_ERR_ARG for a position outside the box, a box edge below 2, a
 * non-finite q or the variant LAT_SWEEP_RESIDENT (on-lattice charges only);
 * LAT_ERR_ALLOC. */
int lattice_set_offlattice_charges(lattice_t *lat, int64_t n, const double *r, const double *q,
                                   int forces);

/* Synchronise and read the force estimate of off-lattice charges set with
 * forces: dE_dr (3n doubles, x y z per charge) = mean of the samples of
 * dE/dr_i since the charges were set (or since lattice_set_state); stderr
 * (3n, may be NULL) = their standard error computed as if the samples were
 * independent (the chain's samples are correlated: bin the energy samples
 * to see by how much).  LAT_ERR_STATE without such charges or with fewer
 * than 2 samples. */
int lattice_force_estimate(lattice_t *lat, double *dE_dr, double *stderr_naive, int64_t *n_samples);

/* Enqueue n_sweeps sweeps without measurement (thermalisation). n_sweeps >= 0. */
int thermalise(lattice_t *lat, int64_t n_sweeps);

/* Enqueue n_sweeps sweeps; after every measure_every-th one (counted within
 * this call) take one sample O = X^2 - Y into the bins (Eq. nsum2).
 * bin_size >= 1 must equal the value used by earlier calls since the last
 * set_charges.  Samples fill consecutive bins of bin_size across calls, so
 * bin_size need not divide the number of samples: the last bin may be
 * partial, and energy_estimate counts it in the mean only.  Errors:
 * LAT_ERR_ARG for n_sweeps < 0, measure_every < 1, bin_size < 1 or a changed
 * bin_size. */
int sweep_and_measure(lattice_t *lat, int64_t n_sweeps, int64_t measure_every,
                      int64_t bin_size);

/* Synchronise and form the estimate (Eq. nsum2): mean = (sum of all samples)
 * / M; stderr_binned = sqrt(sum_b (m_b - m)^2 / (n_b (n_b - 1))) over the
 * n_b full bins (m_b bin means, m their mean); a partial last bin enters the
 * mean only.  Any output pointer may be NULL.  Errors: LAT_ERR_STATE with
 * fewer than 2 full bins (outputs still written, stderr = NaN) or when a
 * bin holds a non-finite sum.  Only the samples are checked, not the field:
 * a non-finite field value reaches the estimate through the samples taken
 * after it appeared (lattice_get_field reads the field itself). */
int energy_estimate(lattice_t *lat, double *mean, double *stderr_binned, int64_t *n_samples,
                    int64_t *n_bins);

/* sweep_and_measure for callers that cannot allocate device memory: code
 * under HIP stream capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, same samples and field as sweep_and_measure
 * (bit for bit; sample sums up to FP64 summation order); no hipMalloc,
 * hipFree, allocator callback or graph capture happens in the call.  The
 * partial sums of the sample gather live in a static device array of 1 MiB
 * per GPU (held until the process ends) instead of the lattice's buffers;
 * sweeps are launched one by one.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (several host threads, or several
 * streams) race on it.
 * Needs: charges placed; bins with room for every sample of the call (bins
 * grow only in sweep_and_measure, to at least 64 bins, doubling); the sample
 * lists of the current tiling built (set_charges builds them; a change of
 * kernel or tiling needs a sweep_and_measure to rebuild them).
 * Errors: as sweep_and_measure; LAT_ERR_STATE when one of the needs is not
 * met; LAT_ERR_ARG when this lattice's partial sums exceed the 1 MiB array. */
int sweep_and_measure_noalloc(lattice_t *lat, int64_t n_sweeps, int64_t measure_every,
                              int64_t bin_size);

/* The estimate of charge set `set` (as energy_estimate; energy_estimate is
 * set 0).  LAT_ERR_ARG for a set that does not exist. */
int lattice_energy_estimate_set(lattice_t *lat, int64_t set, double *mean, double *stderr_binned,
                                int64_t *n_samples, int64_t *n_bins);

/* Release all device memory of the handle (NULL is ignored). */
void lattice_destroy(lattice_t *lat);

/* Message of the last error on the calling thread ("" if none). */
const char *lattice_last_error(void);

/* Number of sweeps done since creation. */
int lattice_sweep_count(const lattice_t *lat, int64_t *sweeps);

/* Choose the sweep kernel (LAT_SWEEP_*).  Every variant draws the same
 * random numbers and computes the same update; LAT_ERR_ARG if the variant
 * cannot handle this box. */
int lattice_set_variant(lattice_t *lat, int variant);

/* Tuning of the slab kernels (LAT_SWEEP_ZSLAB, LAT_SWEEP_STREAM, and the
 * planes of LAT_SWEEP_FUSED): planes of the box one workgroup walks along z
 * (0 = library default: 24 for the streaming kernel's full-row FP32 tile 9,
 * 8 for the z-slab kernel when the library chose it (LAT_SWEEP_AUTO), else
 * 16 at FP32 and 32 at 16-bit storage; at most lz); tile configuration
 * (-1 = library default: for LAT_SWEEP_STREAM 96-quad tiles at FP32 where
 * they divide the rows, else 32-quad tiles, with non-temporal stores where a
 * colour array is at least 256 MiB: tiles 9 / 6 / 0 / 3; tile 7 for the
 * z-slab kernel the library chose; tile 0 for the other kernels): 0..7 for LAT_SWEEP_ZSLAB (workgroup tile width x rows and
 * register budget), 0..10 for LAT_SWEEP_STREAM (tile width 128..512 sites,
 * or 64 for tile 10, rows, depth of the LDS plane ring, non-temporal
 * stores); xcd_order, the
 * order of workgroups over the chip's 8 XCDs: 0 the hardware's round-robin
 * order, 1 a contiguous run of tiles per XCD, 2 (streaming kernel; 1 for
 * the others) a band of each slab's tiles per XCD with all XCDs moving
 * through the slabs together, -1 = library default (2 for the streaming
 * kernel's tile 9 at FP32, else 1).  Defaults are resolved for the kernel
 * each sweep runs.
 * LAT_ERR_ARG for a tile the selected variant does not have (and
 * lattice_set_variant(LAT_SWEEP_STREAM) with a tile above 10).  Results do
 * not depend on any of them. */
int lattice_set_tuning(lattice_t *lat, int64_t planes, int tile, int xcd_order);

/* The configuration the next sweep runs (any output may be NULL): the
 * variant (LAT_SWEEP_AUTO resolved to the library's choice for the box), the
 * planes per workgroup, the tile (the library default resolved) and the XCD
 * order. */
int lattice_get_tuning(const lattice_t *lat, int *variant, int64_t *planes, int *tile, int *xcd_order);

/* How the samples of the most recent sweep_and_measure were gathered:
 * *fused = 1 if the sweep kernel summed X and Y of each sample from its LDS
 * rings: the streaming sweep (LAT_SWEEP_STREAM) the charged colour-0 sites
 * while it updated colour 1 of the measured sweep and the colour-1 sites
 * while it updated colour 0 of the next sweep; the blocked sweep
 * (LAT_SWEEP_BLOCKED) the colour-0 sites in the measured sweep's launch and
 * the colour-1 sites in the next launch.  This needs one on-lattice charge
 * set and per-tile charge lists that can be staged in LDS (streaming: short
 * enough not to lower the kernel's occupancy; blocked: in at most 8 parts);
 * *fused = 0 if a separate gather kernel read the field after each measured
 * sweep.  The two give the same samples up to the order of the FP64 partial
 * sums. */
int lattice_get_sample_path(const lattice_t *lat, int *fused);

/* Staging of the blocked sweep's fused gather: each tile's charge lists are
 * staged into LDS in *parts parts of at most *part_entries entries each (the
 * fewest parts that leave room for the deepest plane ring; the environment
 * variable LATCOUL_GATHER_PART_CAP, read when the lists are built, bounds
 * the entries of a part further).  Both 0 when the current kernel does not
 * gather inside the blocked sweep.  Either pointer may be NULL. */
int lattice_get_gather_parts(const lattice_t *lat, int *parts, int *part_entries);

/* Graph capture of the multi-launch sweep path: runs of sweeps (with their
 * samples) are recorded once as a hipGraph of K-sweep chunks whose kernels
 * read the sweep and sample counters from device memory, then replayed.
 * mode 0: never; 1 (default): boxes of at most 2^24 sites, whose sweeps are
 * short enough for launch overhead to matter; 2: every box.  Results do not
 * depend on the mode. */
int lattice_use_graphs(lattice_t *lat, int mode);

/* Autotuner: time every sweep kernel and tuning that can handle this box
 * (reps sweeps each, after one warm-up sweep) on scratch memory of the
 * handle's size, so the chain itself is not advanced; select the fastest on
 * the handle and cache it per (device architecture, box, storage, whether
 * the single-workgroup kernel may run: one on-lattice charge set) for the
 * process.  If the environment variable LATCOUL_TUNE_CACHE names a file, the
 * choices it holds are used too (read once per process; a choice that names
 * a kernel or tuning this library lacks for the box is ignored) and new
 * choices are appended to it, one line "arch lx ly lz storage single variant
 * planes tile xcd_order ms" each; a file that cannot be read or written is
 * ignored.  Outputs (any may be NULL): the chosen variant, planes, tile, XCD
 * order and the measured
 * ms per sweep.  Synchronises the stream.  Errors: LAT_ERR_ARG for reps
 * outside [1, 1000]; LAT_ERR_ALLOC if the scratch cannot be allocated. */
int lattice_autotune(lattice_t *lat, int64_t reps, int *variant, int64_t *planes, int *tile,
                     int *xcd_order, double *ms_per_sweep);

/* ---- test / checkpoint hooks (all synchronise the stream) ---------- */

/* Copy the field to host_out: lx*ly*lz floats, natural order x fastest. */
int lattice_get_field(lattice_t *lat, float *host_out);

/* Replace the field from host_in (natural order), rounded to the storage
 * format.  Errors: LAT_ERR_ARG for non-finite values. */
int lattice_set_field(lattice_t *lat, const float *host_in);

/* The heat-bath noise of the device for the grid points k = k_first ..
 * k_first + n - 1 of the uniform r = (k + 1/2) 2^-24: dev_out (device memory
 * of n floats, the caller's) receives erfinv(2r - 1)/sqrt(3) as every sweep
 * kernel computes it (the Gaussian term of Eq. phi).  Enqueued on hip_stream
 * (NULL = null stream), not synchronised.  Errors: LAT_ERR_ARG unless
 * 0 <= k_first and k_first + n <= 2^24, or for a NULL dev_out with n > 0.
 * Paper: Eq. (hb1) inverted as Eq. (phi). */
int lattice_noise_values(int64_t k_first, int64_t n, float *dev_out, void *hip_stream);

/* The (X, Y) of the most recent sample (charge set 0). */
int lattice_last_measure(lattice_t *lat, double *X, double *Y);

/* Checkpoint: sweep counter, number of samples and the bins (2 doubles per
 * bin: compensated sum, compensation); *n_bins = bins in use per charge set.
 * bins_host (may be NULL) receives the n_bins bins of set 0, then those of
 * set 1, ...: at most cap bins in all. */
int lattice_get_state(lattice_t *lat, int64_t *sweep_counter, int64_t *n_samples,
                      double *bins_host, int64_t cap, int64_t *n_bins);

/* Restore a checkpoint taken by lattice_get_state (field restored separately
 * with lattice_set_field; the charge sets placed first): bins_host holds
 * n_bins bins per charge set, set after set.  bin_size as used when it was
 * taken.  Force sums of off-lattice charges are not part of a checkpoint:
 * they restart from zero. */
int lattice_set_state(lattice_t *lat, int64_t sweep_counter, int64_t n_samples, int64_t bin_size,
                      const double *bins_host, int64_t n_bins);

/* ------------------------------------------------------------------ */
/* Batch of independent chains on boxes of uneven size                 */
/* ------------------------------------------------------------------ */

/* n_chains chains; edges = 3 int64 per chain (lx, ly, lz; lx even, each box
 * below 2^31 sites); chain_ids = n_chains uint32 (NULL: 0 .. n_chains-1).
 * All chains share storage, seed and stream.  Chain k draws the same random
 * numbers as a single lattice with chain_id = chain_ids[k]. */
int batch_create(int64_t n_chains, const int64_t *edges, const uint32_t *chain_ids, int storage,
                 uint64_t seed, const lat_allocator *alloc, void *hip_stream,
                 lattice_batch_t **out);

/* Charges of one chain (as set_charges).  Resets that chain's bins. */
int batch_set_charges(lattice_batch_t *b, int64_t chain, int64_t n, const int32_t *xyz,
                      const double *q);

/* Enqueue n_therm sweeps then n_meas measured sweeps (one sample per sweep,
 * bins of bin_size) for every chain, in one persistent launch.  Batches whose
 * fields fill the 256 MiB last-level cache sweep chains of at most 3072 quads
 * (4 compact sites) per plane through an LDS ring, each value loaded from
 * memory once per half-sweep (after batch_autotune: the form it chose for
 * each box); chains of at most 8192 sites (lx / 8 * ly * lz quads <= 1024)
 * keep their whole field in LDS in any batch.  The chains' fields are the
 * same either way. */
int batch_run(lattice_batch_t *b, int64_t n_therm, int64_t n_meas, int64_t bin_size);

/* Choose the half-sweep form (LDS ring or memory) per box of the batch: for
 * each box the ring applies to, a scratch batch of as many chains of that box
 * as this batch holds is timed over reps sweeps (1 <= reps <= 1000) each way,
 * and the ring kept only where it is more than 3% faster.  Choices are cached
 * per (device architecture, box, storage, number of chains) for the process.
 * The chains' fields and samples do not change.  *n_ring (may be NULL): the
 * chains that will use the ring.  Synchronises; allocates scratch fields. */
int batch_autotune(lattice_batch_t *b, int64_t reps, int64_t *n_ring);

/* Estimate of one chain (as energy_estimate). */
int batch_energy_estimate(lattice_batch_t *b, int64_t chain, double *mean,
                          double *stderr_binned, int64_t *n_samples, int64_t *n_bins);

/* Field of one chain, natural order (synchronises). */
int batch_get_field(lattice_batch_t *b, int64_t chain, float *host_out);

void batch_destroy(lattice_batch_t *b);

#ifdef __cplusplus
}
#endif

#endif /* LATTICE_COULOMB_H */
