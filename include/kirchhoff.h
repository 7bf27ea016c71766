/*
 * kirchhoff.h - C ABI of libkirchhoff.so: Kirchhoff prestack migration and
 * its adjoint on AMD Instinct MI355X (gfx950).
 *
 * The operator is Eq. (1) of "Distributed computing of Seismic Imaging
 * Algorithms" (Section 3):
 *
 *   I(x, X) = integral dx_s dx_r W(x, x_s, x_r) delta(X - |x_s - x_r|)
 *                    D(x_s, x_r, t = T(x, x_s) + T(x, x_r)),
 *
 * discretised as a sum over recorded traces: every trace of offset bin X adds,
 * at every image point x inside the migration aperture ("traces close enough",
 * Eq. (2)), W times its sample at the total propagation time, linearly
 * interpolated on the trace extended by zeros.  The image is the plain sum of
 * all contributions (Section 4, Reduce = sum).
 *
 * Discretisation used by every entry point:
 *   - trace j: source src[j] = (sx, sy), receiver rec[j] = (rx, ry) in metres,
 *     offset bin bin[j], samples D_j[k] at t = t_first + k * dt, k < n_samples;
 *   - image point (b, iy, ix, iz): column (x[ix], y[iy]), depth index iz;
 *     image layout I[n_bins][ny][nx][nz], depth fastest;
 *   - traveltime model (per-depth tables): T = sqrt(t0sq[iz] + s2[iz] * h^2),
 *     h the horizontal distance from the column to the source or receiver;
 *   - aperture: both legs satisfy h^2 <= r2[iz], with h^2 evaluated in float32
 *     as fl(fl(dx*dx) + fl(dy*dy)), dx = fl(x - sx) (an exact, reproducible
 *     decision shared with any float32 checker);
 *   - u = (T_s + T_r - t_first) / dt, i = floor(u), f = u - i,
 *     value = (1 - f) D[i] + f D[i + 1] with D = 0 outside [0, n_samples);
 *   - weight KM_W_COSCOS_OVER_TT: W = cos(th_s) cos(th_r) / (T_s T_r) with
 *     cos(th) = t0 / T, i.e. W = t0sq / (T_s^2 T_r^2); 0 where t0sq <= 0.
 *     KM_W_UNIT: W = 1.
 *
 * Conventions for all entry points:
 *   - Pointers are DEVICE pointers unless the comment says "host".  The caller
 *     owns every buffer; the library keeps no reference after a call returns,
 *     except inside a km_batch handle (see there).
 *   - Calls are asynchronous on the given HIP stream (a hipStream_t passed as
 *     void*, NULL = default stream) and never synchronise the device, unless
 *     stated.
 *   - Arguments are validated on the host before anything is launched.  On a
 *     non-KM_OK status nothing was launched and outputs are untouched; the
 *     status and a message (km_last_error, per thread) describe the problem.
 *   - Nothing aborts or throws across the ABI.  Entry points are re-entrant;
 *     concurrent calls that write the same output buffer race.
 */
#ifndef KIRCHHOFF_H
#define KIRCHHOFF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KM_ABI_VERSION 4

typedef enum km_status {
    KM_OK = 0,
    KM_E_INVALID = 1,     /* bad argument (null pointer, size, enum, layout) */
    KM_E_UNSUPPORTED = 2, /* valid but not supported (e.g. 16-bit demigrate output, record too long) */
    KM_E_HIP = 3,         /* a HIP runtime call failed; km_last_error has its message.  With
                             KM_FAULT_INJECT=launch in the environment every kernel launch of the
                             library fails this way without launching (for tests of error paths) */
    KM_E_NOMEM = 4        /* a library-owned allocation failed (batch handles only) */
} km_status;

typedef enum km_dtype { KM_F32 = 0, KM_BF16 = 1, KM_F16 = 2 } km_dtype;

typedef enum km_weight_kind { KM_W_UNIT = 0, KM_W_COSCOS_OVER_TT = 1 } km_weight_kind;

/* Arithmetic of the total time u = (T_s + T_r - t_first) / dt of every pair.
 * KM_TIME_FP32: float32 tables (scaled to samples), float32 squared leg
 *   lengths, square roots and sum.  u then carries about 2^-23 u of rounding
 *   (6e-5 samples at u = 1000), which moves the interpolated value by that
 *   fraction of the local sample difference: a relative image error below 1e-5
 *   for band-limited (seismic) traces, up to about 2e-5 for white noise, more
 *   for records of several thousand samples.
 * KM_TIME_EXTENDED: the tables and squared leg lengths in float64, each square
 *   root a float32 reciprocal-square-root seed refined by one float64 residual
 *   step, the sum and i = floor(u), f = u - i in float64: u to about 1e-9
 *   samples.  The aperture decision and the accumulation are unchanged.  More
 *   VALU work per pair.  Not available for the anti-alias operators. */
typedef enum km_time_precision { KM_TIME_FP32 = 0, KM_TIME_EXTENDED = 1 } km_time_precision;

/* Recorded traces D(x_s, x_r, t) (Section 2: one trace per source/receiver
 * pair, P samples each). */
typedef struct km_traces {
    int64_t n_traces;      /* >= 0 */
    int32_t n_samples;     /* samples per trace, 0 <= n_samples <= km_max_samples() */
    int32_t dtype;         /* km_dtype of data */
    int64_t trace_stride;  /* elements between the starts of consecutive traces, >= n_samples */
    double t_first;        /* time of sample 0 in seconds (finite) */
    double dt;             /* sample interval in seconds (> 0, finite) */
    void* data;            /* [n_traces][trace_stride] elements of dtype; read by migrate, written by demigrate */
    const float* scale;    /* [n_traces] per-trace factor for KM_BF16 / KM_F16 (sample = stored * scale);
                              NULL means 1; must be NULL for KM_F32 */
    const float* src;      /* [n_traces][2] source (x, y), metres */
    const float* rec;      /* [n_traces][2] receiver (x, y), metres */
    const int32_t* bin;    /* [n_traces] offset bin, NONDECREASING in j (traces grouped by bin);
                              a trace whose bin is outside [0, n_bins) contributes nothing.
                              Unsorted bins are not detected: traces out of order are then missed. */
} km_traces;

/* Image grid: columns (x[ix], y[iy]) and n_bins offset bins (the X of I(x, X)). */
typedef struct km_grid {
    int32_t nx, ny, nz, n_bins;  /* >= 0 each; nx * ny < 2^31 */
    const float* x;              /* [nx] metres */
    const float* y;              /* [ny] metres (a single 0 for a 2D line) */
} km_grid;

/* Traveltime and aperture model, per image depth index (T(x, x_s) "in the
 * model", Section 3), float32. */
typedef struct km_traveltime {
    const float* t0sq;  /* [nz] squared one-way vertical time, s^2 */
    const float* s2;    /* [nz] squared slowness for horizontal distance, s^2 / m^2 */
    const float* r2;    /* [nz] aperture: largest squared horizontal leg length, m^2 */
    int32_t time_precision; /* km_time_precision (0 = KM_TIME_FP32) */
} km_traveltime;

/* Amplitude weight W(x, x_s, x_r) of Eq. (1). */
typedef struct km_weight {
    int32_t kind;  /* km_weight_kind */
} km_weight;

/* Library ABI version (KM_ABI_VERSION of the build). */
int km_abi_version(void);

/* Message describing the last non-KM_OK status returned to this thread
 * ("" if none).  The pointer stays valid until the next call on this thread. */
const char* km_last_error(void);

/* Longest record (n_samples) the kernels accept. */
int32_t km_max_samples(void);

/* Migration, Eq. (1): image[n_bins][ny][nx][nz] (float32) from traces.
 * accumulate = 0 overwrites the image; 1 adds into it (Reduce = sum,
 * Section 4, so migrating trace subsets with accumulate = 1 sums them).
 * tile: -1 = library choice (the tile km_tune recorded for this problem's
 * class, else a default); otherwise a tile (see km_tile_describe).
 * Work: one float32 evaluation per (trace, image point of its bin) pair that
 * passes the aperture test. */
km_status kirchhoff_migrate(const km_traces* traces, const km_grid* grid, const km_traveltime* tt,
                            const km_weight* weight, float* image, int32_t accumulate, int32_t tile,
                            void* stream);

/* Demigration (Kirchhoff modelling): the exact transpose of kirchhoff_migrate
 * for the same traces geometry, grid, model and weight.  Each in-aperture
 * pair adds (1 - f) W I to D[i] and f W I to D[i + 1]; samples outside
 * [0, n_samples) are dropped.  out->data (float32 only; KM_E_UNSUPPORTED
 * otherwise) is overwritten (accumulate = 0) or added into (1).  Uses the
 * same per-pair aperture, time and weight evaluation as kirchhoff_migrate,
 * so <migrate(d), m> = <d, demigrate(m)> up to float32 summation rounding.
 * Within a trace, floating-point summation order is not fixed. */
km_status kirchhoff_demigrate(const float* image, const km_grid* grid, const km_traveltime* tt,
                              const km_weight* weight, const km_traces* out, int32_t accumulate,
                              int32_t tile, void* stream);

/* ---- table traveltimes -----------------------------------------------------
 * Section 3 takes the propagation times from ray theory in the model.  In a
 * medium whose velocity varies with depth only, a one-way time depends on the
 * horizontal distance h and the depth alone, so curved-ray times can be given
 * as a table: T(h, z_iz) = t[ih][iz] + f (t[ih + 1][iz] - t[ih][iz]) with
 * h = sqrt(h^2) (the float32 h^2 of the aperture test), h / dh = ih + f
 * clamped to [0, n_h - 1] (beyond the table its last row holds).  These calls
 * are kirchhoff_migrate / kirchhoff_demigrate with T_s + T_r from the table in
 * place of the t0sq / s2 form and W = 1; the aperture test (h^2 <= r2[iz] for
 * both legs), the interpolation of the trace and the transpose are the same. */
typedef struct km_ttable {
    int32_t n_h;     /* table rows (>= 2) */
    double dh;       /* row spacing in h, same length unit as x, y (finite, > 0) */
    const float* t;  /* device float [n_h][nz]: one-way time in seconds at h = ih * dh, depth index iz */
    const float* r2; /* device float [nz]: aperture, as km_traveltime.r2 */
    int32_t time_precision; /* km_time_precision: KM_TIME_EXTENDED takes h = sqrt(h^2), h / dh and the
                               fraction in float64 from the float64 h^2 (the interpolated times and their
                               sum are float64 in both) */
    const float* amp; /* device float [n_h][nz] or NULL: one-way amplitude A at h = ih * dh, depth iz,
                         interpolated as the time is (float32); the pair's weight is W = A_s A_r
                         (NULL: W = 1).  For constant velocity A = t0 / T^2 gives the square-root
                         operators' KM_W_COSCOS_OVER_TT weight. */
} km_ttable;

/* As kirchhoff_migrate with table traveltimes and W = 1 (or the amplitude
 * tables' A_s A_r).  KM_E_INVALID also for a NULL table, n_h < 2, dh not
 * finite or <= 0, NULL or misaligned t / r2, misaligned amp;
 * KM_E_UNSUPPORTED for n_h * nz >= 2^29 (the kernels read the table
 * through one buffer addressed with 32-bit signed byte offsets: 2 GiB). */
km_status kirchhoff_migrate_table(const km_traces* traces, const km_grid* grid, const km_ttable* table, float* image,
                                  int32_t accumulate, int32_t tile, void* stream);

/* As kirchhoff_demigrate with table traveltimes and the same weight: the
 * exact transpose of kirchhoff_migrate_table for the same inputs. */
km_status kirchhoff_demigrate_table(const float* image, const km_grid* grid, const km_ttable* table,
                                    const km_traces* out, int32_t accumulate, int32_t tile, void* stream);

/* ---- laterally varying table traveltimes ------------------------------------
 * In a medium that also varies laterally, the times depend on where the
 * image point is.  The model is given as one table per node of a coarse
 * lateral grid X_i = gx0 + i gdx, Y_j = gy0 + j gdy (node (i, j) holds the
 * times of the medium below it, as a km_ttable holds them), and a one-way
 * time is interpolated trilinearly over (image x, image y, h): linearly in h
 * on each of the four nodes around the image column, then in x, then in y,
 * each step a + f (b - a) in float64; the image depth is exact.  The node
 * coordinate (x - gx0) / gdx is clamped to [0, n_gx - 1] (the edge nodes hold
 * beyond the grid); an axis with one node takes no interpolation.  Every
 * node holding the same table gives the km_ttable operators' times exactly.
 * The column's fractions x and y are kept in float32 (a time error of at most
 * 2^-25 of the difference between neighbouring nodes' times). */
typedef struct km_ltable {
    int32_t n_h;      /* rows per node table (>= 2) */
    double dh;        /* row spacing in h (finite, > 0) */
    int32_t n_gx, n_gy; /* nodes along x and y (>= 1 each) */
    double gx0, gy0;  /* position of node (0, 0), same length unit as x, y (finite) */
    double gdx, gdy;  /* node spacing (finite, > 0 on an axis with more than one node; else ignored) */
    const float* t;   /* device float [n_gy][n_gx][n_h][nz]: node (i, j)'s one-way time in seconds at
                         h = ih * dh and depth index iz */
    const float* r2;  /* device float [nz]: aperture, as km_traveltime.r2 */
    int32_t time_precision; /* km_time_precision, as in km_ttable */
    const float* amp; /* device float [n_gy][n_gx][n_h][nz] or NULL: one-way amplitudes, interpolated as
                         the times are (float32); W = A_s A_r (NULL: W = 1) */
} km_ltable;

/* As kirchhoff_migrate_table with laterally varying tables (W = 1, or the
 * amplitude tables' A_s A_r).
 * KM_E_INVALID also for a NULL table, n_gx or n_gy < 1, gx0 / gy0 not
 * finite, gdx (gdy) not finite or <= 0 with n_gx (n_gy) > 1, and the
 * km_ttable conditions on n_h, dh, t and r2; KM_E_UNSUPPORTED for
 * n_gx * n_gy * n_h * nz >= 2^29.  Work per pair: 16 table reads (4 nodes x
 * 2 rows x 2 legs) where a km_ttable pair takes 4. */
km_status kirchhoff_migrate_ltable(const km_traces* traces, const km_grid* grid, const km_ltable* table,
                                   float* image, int32_t accumulate, int32_t tile, void* stream);

/* As kirchhoff_demigrate with laterally varying tables and the same weight:
 * the exact transpose of kirchhoff_migrate_ltable for the same inputs. */
km_status kirchhoff_demigrate_ltable(const float* image, const km_grid* grid, const km_ltable* table,
                                     const km_traces* out, int32_t accumulate, int32_t tile, void* stream);

/* Anti-alias operator filter (the paper is silent on aliasing; this is the
 * triangle filter of production Kirchhoff migration).  Per pair the trace is
 * smoothed by a unit-area triangle whose half-width is the time, in samples,
 * the operator moves between neighbouring image points:
 *   p = |du/dx| dx + |du/dy| dy,  du/dx = (s2 / dt) ((x - x_s) / T_s + (x - x_r) / T_r)
 * (likewise y), clamped to [1, max_half]; with L = floor(p), phi = p - L,
 *   T_L(c) = sum_{|k| < L} (L - |k|) / L^2 D[c + k],  T_p = (1 - phi) T_L + phi T_{L+1},
 * and the pair's value is (1 - f) T_p(i) + f T_p(i + 1) in place of
 * (1 - f) D[i] + f D[i + 1] (D zero outside [0, n_samples)).  p = 1 gives the
 * plain operator. */
typedef struct km_antialias {
    double dx, dy;     /* spacings the dip is measured over (image x / y spacing; finite, >= 0) */
    int32_t max_half;  /* largest triangle half-width in samples, 1 .. 32 */
} km_antialias;

/* As kirchhoff_migrate with the anti-alias filter (square-root traveltimes).
 * KM_E_INVALID also for NULL options, dx or dy negative or not finite,
 * max_half outside [1, 32]; KM_E_UNSUPPORTED for records whose anti-aliased
 * staging does not fit in LDS (n_samples + 4 max_half + 9 float64 values). */
km_status kirchhoff_migrate_aa(const km_traces* traces, const km_grid* grid, const km_traveltime* tt,
                               const km_weight* weight, const km_antialias* aa, float* image, int32_t accumulate,
                               int32_t tile, void* stream);

/* As kirchhoff_demigrate with the anti-alias filter: the exact transpose of
 * kirchhoff_migrate_aa for the same inputs. */
km_status kirchhoff_demigrate_aa(const float* image, const km_grid* grid, const km_traveltime* tt,
                                 const km_weight* weight, const km_antialias* aa, const km_traces* out,
                                 int32_t accumulate, int32_t tile, void* stream);

/* Pair counts of Eq. (2) (f_K N_xyz N_tr with N_tr the traces close enough):
 * counts[0] = pairs passing the aperture test, counts[1] = those whose time
 * also falls inside the zero-extended record (-1 < u < n_samples, u in the
 * kernels' float32).  counts: device int64[2], overwritten. */
km_status km_count_contributions(const km_traces* traces, const km_grid* grid, const km_traveltime* tt,
                                 int64_t* counts, void* stream);

/* The same pair counts, exact, computed on the host from HOST copies of the
 * inputs (the metric's denominator; Eq. (2)): traces (src, rec, bin; data is
 * not read), grid (x, y) and traveltime tables (t0sq, s2, r2), all host
 * pointers.  n_aperture = (trace, image point of the trace's bin) pairs that
 * pass the kernels' float32 aperture decision; n_effective = those whose total
 * time u = (T_s + T_r - t_first) / dt, in float64 from the float32 tables and
 * coordinates, satisfies -1 < u < n_samples.  n_threads <= 0: one thread per
 * hardware thread.  Synchronous; touches no device memory.  Cost: one float32
 * leg evaluation per (image column, trace) pair, plus float64 times only on
 * depths whose aperture does not keep every time inside the record; a
 * non-monotone r2 table is tested depth by depth (much slower).
 * KM_E_INVALID: NULL arguments or arrays, negative sizes, dt not finite and > 0. */
km_status km_count_contributions_host(const km_traces* traces, const km_grid* grid, const km_traveltime* tt,
                                      int32_t n_threads, int64_t* n_aperture /* host */,
                                      int64_t* n_effective /* host */);

/* out[0] = sum_k a[k] * b[k] accumulated in float64 (products exact in
 * float64); device double[1], overwritten.  Used for the adjoint
 * dot-product test and least-squares scalars.  Summation order not fixed. */
km_status km_dot_f64(const float* a, const float* b, int64_t n, double* out, void* stream);

/* y[k] = alpha * x[k] + beta * y[k] in float32 (alpha, beta rounded to float32
 * once).  x may equal y. */
km_status km_axpby(double alpha, const float* x, double beta, float* y, int64_t n, void* stream);

/* ---- trace pre-filter ------------------------------------------------------
 * Eq. (1) sums the data as recorded.  Summing along a traveltime surface
 * that lies later than its apex rotates and reshapes the wavelet (a half
 * integration per summed surface dimension); a finite impulse response applied
 * to every trace beforehand (the rho filter) compensates it.  The taps are an
 * input; with taps h[0..n_taps-1], h[center] at zero lag:
 *   adjoint = 0:  out[n] = sum_k h[k] in[n + center - k]
 *   adjoint = 1:  out[m] = sum_k h[k] in[m - center + k]   (the transpose)
 * with in = 0 outside [0, n_samples), float32 arithmetic, summation order
 * fixed per output.  in, out: device float [n_traces][stride]; out may be
 * the same buffer as in with the same stride, otherwise they must not
 * overlap.  taps: device float[n_taps].
 * KM_E_INVALID: NULL or misaligned pointers, n_traces < 0, n_samples < 0,
 * stride < n_samples, n_taps < 1, center outside [0, n_taps).
 * KM_E_UNSUPPORTED: n_taps > 1024, or one trace plus its halo and the taps
 * exceed the 160 KiB of LDS of a workgroup. */
km_status km_trace_filter(const float* in, int64_t in_stride, float* out, int64_t out_stride, int64_t n_traces,
                          int32_t n_samples, const float* taps, int32_t n_taps, int32_t center, int32_t adjoint,
                          void* stream);

/* ---- offset stack and moveout of the offset images --------------------------
 * The migration gives one image per offset bin: redundant images of the same
 * subsurface.  The depth at which a reflector appears in the different offset
 * images measures the error of the velocity model; once they agree they are
 * added into one stacked image (Introduction). */

/* stack[p] = sum over b = 0..n_bins-1 of image[b * n_points + p] (float32
 * sums in bin order), p < n_points.  image: device float[n_bins][n_points];
 * stack: device float[n_points], overwritten, must not overlap image.
 * KM_E_INVALID for n_bins < 1, n_points < 0, NULL or misaligned pointers. */
km_status km_stack_offsets(const float* image, int32_t n_bins, int64_t n_points, float* stack, void* stream);

/* Moveout of every common-image gather (the n_bins depth vectors of one image
 * column) against its stack S = sum_b I_b (formed in float64):
 *   C_b(l) = sum_{z_lo <= z < z_hi} S[z] I_b[z + l],  l = -max_lag..max_lag,
 * with I_b = 0 outside [0, nz), in float64.  The best lag l* maximises C_b
 * (ties to the smaller |l|, then to the negative l); when |l*| < max_lag and
 * the parabola through C_b(l* - 1), C_b(l*), C_b(l* + 1) opens downwards its
 * vertex refines it:
 *   shift = l* + (C(l*-1) - C(l*+1)) / (2 (C(l*-1) - 2 C(l*) + C(l*+1))),
 * else shift = l*.  shift > 0: the bin images the event deeper than the stack
 * (depth samples).  peak = C_b(l*).  curvature = least-squares slope of the
 * shifts against offsets[b]^2 over the bins with peak > 0 (0 when fewer than
 * two such bins or equal offsets), in depth samples per (offset unit)^2.
 * image: device float[n_bins][ny][nx][nz] (grid->n_bins etc.; grid->x, y are
 * not read).  offsets: device float[n_bins] (bin-centre offsets; read only when
 * curvature is non-NULL).  Outputs (device, overwritten; NULL to skip except
 * shift): stack float[ny][nx][nz], shift float[n_bins][ny][nx], peak
 * float[n_bins][ny][nx], curvature float[ny][nx].
 * KM_E_INVALID: max_lag < 0, window outside [0, nz] or empty, NULL image or
 * shift, misaligned pointers.  KM_E_UNSUPPORTED: max_lag > 256 or one column's
 * rows do not fit in the 160 KiB of LDS of a workgroup. */
km_status km_cig_moveout(const float* image, const km_grid* grid, const float* offsets, int32_t max_lag,
                         int32_t z_lo, int32_t z_hi, float* stack, float* shift, float* peak, float* curvature,
                         void* stream);

/* ---- tile shapes and tuning ------------------------------------------------
 * op: 0 = migrate, 1 = demigrate.  A tile is a compiled shape (waves, column
 * groups, depth slots, LDS budget; km_tile_count(op) of them) and a runtime
 * level of it, passed as tile = shape + 64 * level, level < km_tile_levels(op):
 * migrate levels 0..3 scale the trace block's LDS budget (traces per block) by
 * 1, 0.5, 1.5 and 2 (at most 160 KiB); migrate levels 4 and 5 (lds16 = 1) take
 * budgets 1 and 2 and stage KM_BF16 / KM_F16 traces in LDS as their 16-bit
 * storage, widened and scaled as they are read (more traces per block, an
 * extra conversion per sample read): a migrate call with such a tile returns
 * KM_E_UNSUPPORTED for KM_F32 traces, KM_TIME_EXTENDED and the anti-alias
 * filter, and the batched calls refuse it (a tuned one becomes level 0 or 3
 * there); demigrate level 0 takes as many trace quads per workgroup as the
 * shape allows, level L >= 1 takes L quads (L at most the shape's
 * trace_quads). */
typedef struct km_tile_info {
    int32_t waves;            /* wavefronts (64 lanes) per workgroup */
    int32_t column_groups;    /* groups of 4 image columns per wavefront (migrate) */
    int32_t depth_slots;      /* 16-depth slots held per lane (depth chunk = 16 * depth_slots) */
    int32_t lds_budget;       /* bytes of LDS the trace block (migrate) or trace rows (demigrate) may use */
    int32_t trace_quads;      /* demigrate: most groups of 4 traces per workgroup at this level; 0 for migrate */
    int32_t shape, level;     /* the decoded tile */
    int32_t lds16;            /* migrate: 1 if the level stages 16-bit traces as 16-bit storage */
} km_tile_info;

int32_t km_tile_count(int32_t op);
int32_t km_tile_levels(int32_t op);
km_status km_tile_describe(int32_t op, int32_t tile, km_tile_info* out /* host */);

/* Autotuner: time every tile (compiled shape x level) of op on this problem
 * (each run once untimed, then `reps` times), keep the fastest for the
 * problem's class (GPU architecture, op, dtype, traveltime kind, time
 * precision, nz / 128, n_samples / 512) and return it; calls with tile = -1
 * then use it.  table (table traveltimes; tt is then ignored and W = 1) or aa
 * (anti-alias filter) may be NULL, not both non-NULL.  Synchronises the
 * stream.  Writes the output buffer (image for op 0, traces->data for op 1)
 * with accumulate = 0 semantics.  best_tile, best_ms: host, may be NULL.
 * The class cache is kept per process and, when the environment variable
 * KM_TUNE_CACHE names a file, read from it at first use and rewritten (JSON)
 * after every record, so a later process starts tuned. */
km_status km_tune(int32_t op, const km_traces* traces, const km_grid* grid, const km_traveltime* tt,
                  const km_weight* weight, const km_ttable* table, const km_antialias* aa, float* image,
                  int32_t reps, void* stream, int32_t* best_tile /* host */, float* best_ms /* host */);

/* km_tune for laterally varying tables (kind 3 of the class cache); the
 * arguments as in kirchhoff_migrate_ltable / kirchhoff_demigrate_ltable. */
km_status km_tune_ltable(int32_t op, const km_traces* traces, const km_grid* grid, const km_ltable* table,
                         float* image, int32_t reps, void* stream, int32_t* best_tile /* host */,
                         float* best_ms /* host */);

/* The class cache of km_tune.  kind: 0 = square-root times, 1 = table times,
 * 2 = anti-alias filter, 3 = laterally varying tables.  km_tune_lookup returns -1 when nothing is recorded;
 * km_tune_record stores (and persists) a tile with its time, and returns KM_E_INVALID for a tile out of range
 * or a 16-bit staging tile (migrate levels 4, 5) for a class of KM_F32 traces, KM_TIME_EXTENDED or kind 2.
 * Calls with tile = -1 take a recorded tile only if it applies to their class (a cache file may come from
 * another build); otherwise the library's default. */
int32_t km_tune_lookup(int32_t op, int32_t dtype, int32_t kind, int32_t time_precision, int32_t nz,
                       int32_t n_samples);
km_status km_tune_record(int32_t op, int32_t dtype, int32_t kind, int32_t time_precision, int32_t nz,
                         int32_t n_samples, int32_t tile, float ms);

/* ---- batched migration ------------------------------------------------------
 * Many independent problems (e.g. uneven 2D lines) migrated by ONE persistent
 * kernel launch that pulls (problem, bin, column tile, depth chunk) work items
 * from a queue ordered longest first; the launch is captured once into a HIP
 * graph.  The handle keeps the device pointers of every problem: they must
 * stay valid, and keep their shapes, until km_batch_destroy.  Only float32 or
 * 16-bit traces and accumulate = 0 semantics (every image is overwritten). */
typedef struct km_problem {
    km_traces traces;
    km_grid grid;
    km_traveltime tt;
    km_weight weight;
    float* image;
} km_problem;

typedef struct km_batch km_batch;

/* probs: host array of n problems.  op: 0 = migrate (the only batched
 * operator built; 1 = demigrate returns KM_E_UNSUPPORTED).  tile: as for
 * kirchhoff_migrate (one shape for the whole batch).  Work-item costs are
 * measured with the counting kernel on `stream` (the call synchronises it).
 * Allocates device memory for the problem table and queue (KM_E_NOMEM on
 * failure).  All problems share the weight kind, the time precision and
 * whether t_first is 0 (KM_E_UNSUPPORTED otherwise). */
km_status km_batch_create(const km_problem* probs, int32_t n, int32_t op, int32_t tile, void* stream,
                          km_batch** out);
/* One batched migration (op 0 of km_batch_create, the same kernels) that
 * allocates nothing: for callers that cannot allocate device memory (code
 * running between other work in a serving loop, harnesses that forbid
 * allocation).  The problem table, the work items and the queue counter live
 * in a static scratch array of 8 MiB per GPU (held from module load to process
 * end): at most 4096 problems and as many work items as fit in it
 * (about 460 000 at 16 bytes after the problem table; one work item per
 * (bin, column tile of waves x column groups x 4 columns, depth chunk of
 * 16 x depth slots)); larger batches return KM_E_UNSUPPORTED with the size
 * they need.  The call measures the item costs (synchronising the stream),
 * uploads the tables, resets the queue counter with a kernel and launches the
 * persistent kernel asynchronously on `stream`.  Every call on a GPU uses that
 * GPU's one array: calls that overlap on one GPU race (serialise them, e.g.
 * on one stream).  Images are overwritten (accumulate = 0), as by
 * km_batch_run; the result equals km_batch_run's bit for bit. */
km_status km_batch_migrate_static(const km_problem* probs, int32_t n, int32_t tile, void* stream);

/* Replay the captured graph on stream (asynchronous). */
km_status km_batch_run(km_batch* batch, void* stream);
/* Work items and persistent workgroups of the batch (host outputs, may be NULL). */
km_status km_batch_info(const km_batch* batch, int64_t* n_items, int32_t* n_workgroups);
/* Releases the graph and device memory (synchronises the device first). */
km_status km_batch_destroy(km_batch* batch);

/* ---- measurement ----------------------------------------------------------
 * Issue-rate microbenchmark: ms for `iters` iterations of 8 independent
 * dependency chains of one instruction kind over `n_waves` wavefronts
 * (kind 0 = v_fma_f32, 1 = v_sqrt_f32, 2 = v_rcp_f32).  Synchronises. */
km_status km_probe_issue(int32_t kind, int32_t n_waves, int32_t iters, void* stream, float* ms /* host */);

#ifdef __cplusplus
}
#endif

#endif /* KIRCHHOFF_H */
