/*
 * Plain FP64 CPU evaluation of the Kirchhoff prestack migration integral.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It shares no code, header or table with the library:
 * only tests, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * What it computes (Section 3, Eq. (1) of "Distributed computing of Seismic
 * Imaging Algorithms"):
 *
 *   I(x, X) = sum over traces j with offset bin X of
 *             W(x, x_s, x_r) * D_j(t = T(x, x_s) + T(x, x_r)),
 *
 * i.e. every trace whose offset |x_s - x_r| falls in bin X contributes, at
 * every image point x that is close enough (the aperture of Eq. (2)), its
 * sample at the total propagation time, weighted by W; the image is the sum
 * of all such contributions (the Reduce step of Section 4 is a plain sum).
 *
 * Discretisation (the paper leaves these open; the readings are stated here):
 *  - T(x, x_s) = sqrt(t0sq[iz] + s2[iz] * h_s^2), h_s the horizontal distance
 *    between image column and source; t0sq, s2 are per-depth model tables.
 *  - Aperture: both legs satisfy h^2 <= r2[iz].  The decision is taken in
 *    float32 with the operation order dx = fl(x - sx), h2 = fl(fl(dx*dx) +
 *    fl(dy*dy)), so that any float32 implementation can take the identical
 *    decision; r2 is itself a float32 input.
 *  - Everything continuous is FP64 (coordinates widened from float32).
 *  - u = (T_s + T_r - t_first) / dt, i = floor(u), f = u - i and the data value
 *    is (1 - f) * D[i] + f * D[i + 1] on the trace extended by zeros outside
 *    [0, n_t).
 *  - Weight kind 1: W = cos(th_s) cos(th_r) / (T_s T_r) with cos(th) = t0 / T,
 *    i.e. W = t0sq / (a_s * a_r) where a = T^2; W = 0 when t0sq = 0.
 *    Weight kind 0: W = 1.
 *  - The adjoint (demigration) is the exact transpose: each in-aperture pair
 *    adds (1 - f) W I to D[i] and f W I to D[i + 1] (samples outside [0, n_t)
 *    are dropped).
 *  - Anti-aliasing (aa_max > 0; the operator anti-alias filter of production
 *    Kirchhoff migration, which the paper does not discuss): the trace is
 *    smoothed, per pair, by a triangle whose half-width is the time the
 *    operator moves between neighbouring image points.  In samples,
 *        p = |du/dx| aa_dx + |du/dy| aa_dy,
 *        du/dx = (s2 / dt) ((x - x_s) / T_s + (x - x_r) / T_r)   (likewise y),
 *    clamped to [1, aa_max]; with L = floor(p), phi = p - L,
 *        T_L(c) = sum_{|k| < L} (L - |k|) / L^2 D(c + k)   (unit area; T_1 = D),
 *        T_p(c) = (1 - phi) T_L(c) + phi T_{L+1}(c)        (continuous in p),
 *    and the data value is (1 - f) T_p(i) + f T_p(i + 1).  Square-root times
 *    only.  The adjoint spreads each pair the same way.
 *  - Table traveltimes (ttab != NULL; curved rays in a laterally invariant
 *    medium, where a one-way time depends only on the horizontal distance h
 *    and the depth): T(h, z[iz]) is the linear interpolation in h of
 *    ttab[ih][iz], the time at h = ih * dh, with h = sqrt(h^2) in FP64 and
 *    h / dh clamped to [0, n_h - 1] (beyond the table the last value holds).
 *    The aperture test is unchanged; W = 1 (weight kind 0 only).
 *  - Laterally varying tables (ttab != NULL and n_gx >= 1; the medium below
 *    each node of a coarse lateral grid X_i = gx0 + i gdx, Y_j = gy0 + j gdy
 *    has its own table ttab[j][i][ih][iz]): the one-way time from a surface
 *    point to image point (x, y, z[iz]) is the trilinear interpolation over
 *    (x, y, h), taken as nested linear interpolations a + f (b - a): in h on
 *    each of the four nodes around the image column (as above), then in x,
 *    then in y.  The node coordinate (x - gx0) / gdx is clamped to
 *    [0, n_gx - 1] (beyond the grid the edge nodes hold); a single node along
 *    an axis takes no interpolation there.  With every node holding the same
 *    table this is the laterally invariant table exactly (b - a = 0).
 *  - Amplitudes for table traveltimes (tamp != NULL, same layout as ttab): a
 *    one-way amplitude A per leg, interpolated exactly as the time is, and
 *    W = A_s A_r in place of W = 1.  (For constant velocity A = t0 / T^2 gives
 *    the cos cos / (T_s T_r) weight of the square-root form.)
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#if !defined(FLT_EVAL_METHOD) || FLT_EVAL_METHOD != 0
#error "float arithmetic must be evaluated in float precision for the aperture decision"
#endif

typedef struct {
    int64_t n_traces;
    int32_t n_t;
    double t_first, dt;
    const double* data;    /* [n_traces][n_t]; may be NULL for count / adjoint */
    const float* src;      /* [n_traces][2] (x, y) */
    const float* rec;      /* [n_traces][2] */
    const int32_t* bin;    /* [n_traces]; outside [0, n_bins) = trace unused */
    int32_t nx, ny, nz, n_bins;
    const float* x;        /* [nx] */
    const float* y;        /* [ny] */
    const double* t0sq;    /* [nz] */
    const double* s2;      /* [nz] */
    const float* r2;       /* [nz] */
    int32_t weight;        /* 0: W = 1; 1: W = t0sq / (a_s a_r) */
    int32_t n_h;           /* table traveltimes: rows of ttab (>= 2) */
    double dh;             /* table spacing in h (> 0) */
    const float* ttab;     /* [n_h][nz] one-way seconds, or NULL for the t0sq / s2 form */
    double aa_dx, aa_dy;   /* anti-aliasing: image spacings the dip is measured over */
    int32_t aa_max;        /* anti-aliasing: largest triangle half-width (samples); 0 = off */
    int32_t n_gx, n_gy;    /* lateral table nodes (0: one table for every column) */
    double gx0, gy0;       /* position of node (0, 0) */
    double gdx, gdy;       /* node spacing (> 0 along an axis with more than one node) */
    const float* tamp;     /* table traveltimes: one-way amplitudes, same layout as ttab, or NULL (W = 1) */
} ko_problem;

/* Linear interpolation in h of the one-way time table at depth iz. */
static double ko_table_time(const ko_problem* P, double h, int iz)
{
    double hf = h / P->dh;
    const double top = (double)(P->n_h - 1);
    if (!(hf < top)) hf = top;
    int64_t ih = (int64_t)floor(hf);
    if (ih > P->n_h - 2) ih = P->n_h - 2;
    const double f = hf - (double)ih;
    const double t0 = P->ttab[ih * (int64_t)P->nz + iz], t1 = P->ttab[(ih + 1) * (int64_t)P->nz + iz];
    return t0 + f * (t1 - t0);
}

/* Position of coordinate c on a node axis of n nodes (origin c0, spacing g):
 * lower node *i and fraction *f with c clamped to the axis (see header). */
static void ko_node_axis(double c, double c0, double g, int32_t n, int64_t* i, double* f)
{
    if (n <= 1) {
        *i = 0;
        *f = 0.0;
        return;
    }
    double a = (c - c0) / g;
    if (!(a > 0.0)) a = 0.0;
    if (a > (double)(n - 1)) a = (double)(n - 1);
    int64_t k = (int64_t)floor(a);
    if (k > n - 2) k = n - 2;
    *i = k;
    *f = a - (double)k;
}

/* One-way time at horizontal distance h from the image column (px, py),
 * depth iz, on the laterally varying tables (see header). */
static double ko_lateral_time(const ko_problem* P, double px, double py, double h, int iz)
{
    int64_t i, j;
    double fx, fy;
    ko_node_axis(px, P->gx0, P->gdx, P->n_gx, &i, &fx);
    ko_node_axis(py, P->gy0, P->gdy, P->n_gy, &j, &fy);
    const int64_t i1 = P->n_gx > 1 ? i + 1 : i, j1 = P->n_gy > 1 ? j + 1 : j;
    /* node (a, b) as a table of its own: ko_table_time on a shifted copy */
    ko_problem Q = *P;
    const int64_t node = (int64_t)P->n_h * P->nz;
    Q.ttab = P->ttab + (j * P->n_gx + i) * node;
    const double t00 = ko_table_time(&Q, h, iz);
    Q.ttab = P->ttab + (j * P->n_gx + i1) * node;
    const double t10 = ko_table_time(&Q, h, iz);
    Q.ttab = P->ttab + (j1 * P->n_gx + i) * node;
    const double t01 = ko_table_time(&Q, h, iz);
    Q.ttab = P->ttab + (j1 * P->n_gx + i1) * node;
    const double t11 = ko_table_time(&Q, h, iz);
    const double t0 = t00 + fx * (t10 - t00), t1 = t01 + fx * (t11 - t01);
    return t0 + fy * (t1 - t0);
}

/* Aperture decision in float32 (see header). */
static int ko_in_aperture(float px, float py, float sx, float sy, float rx, float ry, float r2)
{
    float dxs = px - sx, dys = py - sy;
    float dxr = px - rx, dyr = py - ry;
    float hs2 = dxs * dxs + dys * dys;
    float hr2 = dxr * dxr + dyr * dyr;
    return hs2 <= r2 && hr2 <= r2;
}

/* One (trace, image point) pair.  Returns 0 when the pair is outside the
 * aperture; otherwise sets *u (fractional sample index), *w (weight) and,
 * with anti-aliasing, *p (triangle half-width in samples, in [1, aa_max]). */
static int ko_pair_p(const ko_problem* P, int64_t j, int ix, int iy, int iz, double* u, double* w, double* p)
{
    const float px = P->x[ix], py = P->y[iy];
    const float sx = P->src[2 * j], sy = P->src[2 * j + 1];
    const float rx = P->rec[2 * j], ry = P->rec[2 * j + 1];
    if (!ko_in_aperture(px, py, sx, sy, rx, ry, P->r2[iz])) return 0;
    double hs2 = ((double)px - sx) * ((double)px - sx) + ((double)py - sy) * ((double)py - sy);
    double hr2 = ((double)px - rx) * ((double)px - rx) + ((double)py - ry) * ((double)py - ry);
    if (P->ttab) {
        const double hs = sqrt(hs2), hr = sqrt(hr2);
        const int lat = P->n_gx > 0;
        const double T = lat ? ko_lateral_time(P, px, py, hs, iz) + ko_lateral_time(P, px, py, hr, iz)
                             : ko_table_time(P, hs, iz) + ko_table_time(P, hr, iz);
        *u = (T - P->t_first) / P->dt;
        *w = 1.0;
        if (P->tamp) {
            /* the amplitude tables, interpolated as the time tables are */
            ko_problem A = *P;
            A.ttab = P->tamp;
            *w = lat ? ko_lateral_time(&A, px, py, hs, iz) * ko_lateral_time(&A, px, py, hr, iz)
                     : ko_table_time(&A, hs, iz) * ko_table_time(&A, hr, iz);
        }
        return 1;
    }
    double a_s = P->t0sq[iz] + P->s2[iz] * hs2;
    double a_r = P->t0sq[iz] + P->s2[iz] * hr2;
    double T = sqrt(a_s) + sqrt(a_r);
    *u = (T - P->t_first) / P->dt;
    if (P->weight == 1)
        *w = P->t0sq[iz] > 0.0 ? P->t0sq[iz] / (a_s * a_r) : 0.0;
    else
        *w = 1.0;
    if (P->aa_max > 0 && p) {
        const double g = P->s2[iz] / P->dt;
        const double ux = g * (((double)px - sx) / sqrt(a_s) + ((double)px - rx) / sqrt(a_r));
        const double uy = g * (((double)py - sy) / sqrt(a_s) + ((double)py - ry) / sqrt(a_r));
        double q = fabs(ux) * P->aa_dx + fabs(uy) * P->aa_dy;
        if (!(q >= 1.0)) q = 1.0;
        if (q > (double)P->aa_max) q = (double)P->aa_max;
        *p = q;
    }
    return 1;
}

static int ko_pair(const ko_problem* P, int64_t j, int ix, int iy, int iz, double* u, double* w)
{
    return ko_pair_p(P, j, ix, iy, iz, u, w, NULL);
}

/* Weight of sample c + k in the triangle-smoothed value at c, half-width p
 * (see header): (1 - phi) (L - |k|)+ / L^2 + phi (L + 1 - |k|)+ / (L + 1)^2. */
static double ko_tri_weight(double p, int64_t k)
{
    const double L = floor(p), phi = p - L;
    const double a = fabs((double)k);
    double wt = 0.0;
    if (a < L) wt += (1.0 - phi) * (L - a) / (L * L);
    if (a < L + 1.0) wt += phi * (L + 1.0 - a) / ((L + 1.0) * (L + 1.0));
    return wt;
}

/* Triangle-smoothed sample of row d at integer index c (zero outside [0, n_t)). */
static double ko_tri_sample(const double* d, int32_t n_t, int64_t c, double p)
{
    const int64_t r = (int64_t)floor(p) + 1;
    double acc = 0.0;
    for (int64_t k = -r; k <= r; ++k) {
        const int64_t n = c + k;
        if (n >= 0 && n < n_t) acc += ko_tri_weight(p, k) * d[n];
    }
    return acc;
}

/* Anti-aliased data value: (1 - f) T_p(i) + f T_p(i + 1), u = i + f. */
static double ko_sample_aa(const double* d, int32_t n_t, double u, double p)
{
    const double fl = floor(u), reach = floor(p) + 2.0;
    if (!(fl > -reach && fl < (double)n_t + reach)) return 0.0;  /* no overlap with the record */
    const int64_t i = (int64_t)fl;
    const double f = u - fl;
    return (1.0 - f) * ko_tri_sample(d, n_t, i, p) + f * ko_tri_sample(d, n_t, i + 1, p);
}

/* Zero-extended linear interpolation of trace row d at fractional index u. */
static double ko_sample(const double* d, int32_t n_t, double u)
{
    if (!(u > -1.0 && u < (double)n_t)) return 0.0;
    double fl = floor(u);
    int64_t i = (int64_t)fl;
    double f = u - fl;
    double d0 = (i >= 0 && i < n_t) ? d[i] : 0.0;
    double d1 = (i + 1 >= 0 && i + 1 < n_t) ? d[i + 1] : 0.0;
    return (1.0 - f) * d0 + f * d1;
}

/* Pair value of trace row d: the interpolated sample, anti-aliased when enabled. */
static double ko_value(const ko_problem* P, const double* d, double u, double p)
{
    return P->aa_max > 0 ? ko_sample_aa(d, P->n_t, u, p) : ko_sample(d, P->n_t, u);
}

/* Adjoint of ko_value: adds val times the weight of each sample to row d. */
static void ko_spread(const ko_problem* P, double* d, double u, double p, double val)
{
    const int32_t nt = P->n_t;
    if (P->aa_max <= 0) {
        if (!(u > -1.0 && u < (double)nt)) return;
        const double fl = floor(u);
        const int64_t i = (int64_t)fl;
        const double f = u - fl;
        if (i >= 0) d[i] += (1.0 - f) * val;
        if (i + 1 < nt) d[i + 1] += f * val;
        return;
    }
    const double fl = floor(u), reach = floor(p) + 2.0;
    if (!(fl > -reach && fl < (double)nt + reach)) return;
    const int64_t i = (int64_t)fl;
    const double f = u - fl;
    const int64_t r = (int64_t)floor(p) + 1;
    for (int64_t k = -r; k <= r; ++k) {
        const double wt = ko_tri_weight(p, k);
        if (i + k >= 0 && i + k < nt) d[i + k] += (1.0 - f) * wt * val;
        if (i + 1 + k >= 0 && i + 1 + k < nt) d[i + 1 + k] += f * wt * val;
    }
}

static int ko_check(const ko_problem* P)
{
    if (!P || P->n_traces < 0 || P->n_t < 0 || P->nx < 0 || P->ny < 0 || P->nz < 0 || P->n_bins < 0) return 1;
    if (!(P->dt > 0.0)) return 1;
    if (P->ttab && (P->n_h < 2 || !(P->dh > 0.0) || P->weight != 0)) return 1;
    if (P->n_gx < 0 || P->n_gy < 0 || (P->n_gx > 0) != (P->n_gy > 0)) return 1;
    if (P->tamp && !P->ttab) return 1;
    if (P->n_gx > 0 && (!P->ttab || (P->n_gx > 1 && !(P->gdx > 0.0)) || (P->n_gy > 1 && !(P->gdy > 0.0))))
        return 1;
    if (P->aa_max < 0 || (P->aa_max > 0 && (P->ttab || !(P->aa_dx >= 0.0) || !(P->aa_dy >= 0.0)))) return 1;
    return 0;
}

/* Image columns (b, iy, ix) listed in cols[3*c .. 3*c+2]; out[c][iz], nz values each. */
int oracle_migrate_columns(const ko_problem* P, int64_t n_cols, const int32_t* cols, double* out)
{
    if (ko_check(P) || !P->data) return 1;
    const int32_t nz = P->nz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < n_cols; ++c) {
        const int b = cols[3 * c], iy = cols[3 * c + 1], ix = cols[3 * c + 2];
        double* o = out + c * (int64_t)nz;
        for (int iz = 0; iz < nz; ++iz) o[iz] = 0.0;
        for (int64_t j = 0; j < P->n_traces; ++j) {
            if (P->bin[j] != b) continue;
            const double* d = P->data + j * (int64_t)P->n_t;
            for (int iz = 0; iz < nz; ++iz) {
                double u, w, p = 1.0;
                if (!ko_pair_p(P, j, ix, iy, iz, &u, &w, &p)) continue;
                o[iz] += w * ko_value(P, d, u, p);
            }
        }
    }
    return 0;
}

/* Depths z_lo <= iz < z_hi of image columns cols[3*c .. 3*c+2] = (b, iy, ix);
 * out[c][iz - z_lo] (z_hi - z_lo values each): the same sums as
 * oracle_migrate_columns over a window of depths (a sub-volume). */
int oracle_migrate_window(const ko_problem* P, int64_t n_cols, const int32_t* cols, int32_t z_lo, int32_t z_hi,
                          double* out)
{
    if (ko_check(P) || !P->data || z_lo < 0 || z_hi > P->nz || z_lo > z_hi) return 1;
    const int32_t nw = z_hi - z_lo;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < n_cols; ++c) {
        const int b = cols[3 * c], iy = cols[3 * c + 1], ix = cols[3 * c + 2];
        double* o = out + c * (int64_t)nw;
        for (int k = 0; k < nw; ++k) o[k] = 0.0;
        for (int64_t j = 0; j < P->n_traces; ++j) {
            if (P->bin[j] != b) continue;
            const double* d = P->data + j * (int64_t)P->n_t;
            for (int iz = z_lo; iz < z_hi; ++iz) {
                double u, w, p = 1.0;
                if (!ko_pair_p(P, j, ix, iy, iz, &u, &w, &p)) continue;
                o[iz - z_lo] += w * ko_value(P, d, u, p);
            }
        }
    }
    return 0;
}

/* Full image I[n_bins][ny][nx][nz] (overwritten). */
int oracle_migrate(const ko_problem* P, double* image)
{
    if (ko_check(P) || !P->data) return 1;
    int64_t n_cols = (int64_t)P->n_bins * P->ny * P->nx;
    int32_t* cols = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)(n_cols > 0 ? n_cols : 1));
    if (!cols) return 2;
    int64_t c = 0;
    for (int b = 0; b < P->n_bins; ++b)
        for (int iy = 0; iy < P->ny; ++iy)
            for (int ix = 0; ix < P->nx; ++ix) {
                cols[3 * c] = b; cols[3 * c + 1] = iy; cols[3 * c + 2] = ix; ++c;
            }
    int rc = oracle_migrate_columns(P, n_cols, cols, image);
    free(cols);
    return rc;
}

/* Single image points pts[4*k .. 4*k+3] = (b, iy, ix, iz) -> out[k]. */
int oracle_migrate_points(const ko_problem* P, int64_t n_pts, const int32_t* pts, double* out)
{
    if (ko_check(P) || !P->data) return 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n_pts; ++k) {
        const int b = pts[4 * k], iy = pts[4 * k + 1], ix = pts[4 * k + 2], iz = pts[4 * k + 3];
        double acc = 0.0;
        for (int64_t j = 0; j < P->n_traces; ++j) {
            if (P->bin[j] != b) continue;
            double u, w, p = 1.0;
            if (!ko_pair_p(P, j, ix, iy, iz, &u, &w, &p)) continue;
            acc += w * ko_value(P, P->data + j * (int64_t)P->n_t, u, p);
        }
        out[k] = acc;
    }
    return 0;
}

/* Adjoint: data[n_traces][n_t] (overwritten) from image[n_bins][ny][nx][nz]. */
int oracle_demigrate(const ko_problem* P, const double* image, double* data)
{
    if (ko_check(P)) return 1;
    const int32_t nt = P->n_t, nz = P->nz;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < P->n_traces; ++j) {
        double* d = data + j * (int64_t)nt;
        for (int k = 0; k < nt; ++k) d[k] = 0.0;
        const int b = P->bin[j];
        if (b < 0 || b >= P->n_bins) continue;
        for (int iy = 0; iy < P->ny; ++iy)
            for (int ix = 0; ix < P->nx; ++ix) {
                const double* m = image + (((int64_t)b * P->ny + iy) * P->nx + ix) * nz;
                for (int iz = 0; iz < nz; ++iz) {
                    double u, w, p = 1.0;
                    if (!ko_pair_p(P, j, ix, iy, iz, &u, &w, &p)) continue;
                    ko_spread(P, d, u, p, w * m[iz]);
                }
            }
    }
    return 0;
}

/* Adjoint at single samples smp[2*k], smp[2*k+1] = (trace j, sample n) -> out[k]. */
int oracle_demigrate_samples(const ko_problem* P, const double* image, int64_t n_smp, const int64_t* smp,
                             double* out)
{
    if (ko_check(P)) return 1;
    const int32_t nt = P->n_t, nz = P->nz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n_smp; ++k) {
        const int64_t j = smp[2 * k];
        const int64_t n = smp[2 * k + 1];
        const int b = P->bin[j];
        double acc = 0.0;
        if (b >= 0 && b < P->n_bins)
            for (int iy = 0; iy < P->ny; ++iy)
                for (int ix = 0; ix < P->nx; ++ix) {
                    const double* m = image + (((int64_t)b * P->ny + iy) * P->nx + ix) * nz;
                    for (int iz = 0; iz < nz; ++iz) {
                        double u, w, p = 1.0;
                        if (!ko_pair_p(P, j, ix, iy, iz, &u, &w, &p)) continue;
                        if (P->aa_max > 0) {
                            const double fl = floor(u), reach = floor(p) + 2.0;
                            if (!(fl > -reach && fl < (double)nt + reach)) continue;
                            const double f = u - fl;
                            const int64_t i = (int64_t)fl;
                            acc += ((1.0 - f) * ko_tri_weight(p, n - i) + f * ko_tri_weight(p, n - i - 1)) * w * m[iz];
                            continue;
                        }
                        if (!(u > -1.0 && u < (double)nt)) continue;
                        double fl = floor(u);
                        int64_t i = (int64_t)fl;
                        double f = u - fl;
                        if (i == n) acc += (1.0 - f) * w * m[iz];
                        if (i + 1 == n) acc += f * w * m[iz];
                    }
                }
        out[k] = acc;
    }
    return 0;
}

/* Pair counts of Eq. (2): n_aperture = pairs (trace, image point of the
 * trace's bin) passing the aperture test; n_effective = those whose time
 * also falls inside the zero-extended record, -1 < u < n_t. */
int oracle_count(const ko_problem* P, int64_t* n_aperture, int64_t* n_effective)
{
    if (ko_check(P)) return 1;
    int64_t na = 0, ne = 0;
    const int32_t nt = P->n_t;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : na, ne)
    for (int64_t j = 0; j < P->n_traces; ++j) {
        const int b = P->bin[j];
        if (b < 0 || b >= P->n_bins) continue;
        for (int iy = 0; iy < P->ny; ++iy)
            for (int ix = 0; ix < P->nx; ++ix)
                for (int iz = 0; iz < P->nz; ++iz) {
                    double u, w;
                    if (!ko_pair(P, j, ix, iy, iz, &u, &w)) continue;
                    ++na;
                    if (u > -1.0 && u < (double)nt) ++ne;
                }
    }
    *n_aperture = na;
    *n_effective = ne;
    return 0;
}

/* Eq. (2) pair counts restricted to image columns cols[3*c..3*c+2] = (b, iy, ix):
 * out[0] = pairs passing the aperture test, out[1] = of those, -1 < u < n_t. */
int oracle_count_columns(const ko_problem* P, int64_t n_cols, const int32_t* cols, int64_t* out)
{
    if (ko_check(P)) return 1;
    int64_t na = 0, ne = 0;
    const int32_t nt = P->n_t;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : na, ne)
    for (int64_t c = 0; c < n_cols; ++c) {
        const int b = cols[3 * c], iy = cols[3 * c + 1], ix = cols[3 * c + 2];
        for (int64_t j = 0; j < P->n_traces; ++j) {
            if (P->bin[j] != b) continue;
            for (int iz = 0; iz < P->nz; ++iz) {
                double u, w;
                if (!ko_pair(P, j, ix, iy, iz, &u, &w)) continue;
                ++na;
                if (u > -1.0 && u < (double)nt) ++ne;
            }
        }
    }
    out[0] = na;
    out[1] = ne;
    return 0;
}

/* Number of OpenMP threads a parallel region would use. */
int oracle_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}
