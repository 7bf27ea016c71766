// Exact pair counts of Eq. (2) on the host (km_count_contributions_host).
//
// Eq. (2) prices a migration at f_K N_xyz N_tr, N_tr the traces close enough
// to an image point.  The pairs counted here are exactly those the kernels
// evaluate: (trace, image point of the trace's offset bin) pairs that pass
// the float32 aperture decision h^2 <= r2[iz] for both legs, with
// h^2 = fl(fl(dx dx) + fl(dy dy)), dx = fl(x - sx) (n_aperture), and among
// them the pairs whose total time u = (T_s + T_r - t_first) / dt, taken in
// float64 from the float32 tables and coordinates, lies in -1 < u < n_samples,
// where the zero-extended record can give a nonzero value (n_effective).
//
// Work per (image column, trace): the two legs in float32 and the first depth
// inside the aperture.  For a nondecreasing r2 the depths inside are a suffix
// [z_lo, nz), found by a walk from the neighbouring column's z_lo; otherwise
// every depth is tested.  n_effective needs times only on depths whose
// aperture cannot be proven to keep every time inside (-1, n_samples): per
// depth, a bound of u over every leg length the aperture admits (the time
// grows or falls monotonically with h^2 inside the square root) settles the
// others without evaluating a pair.
#include "kirchhoff.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <string>
#include <thread>
#include <vector>

// km_api.cpp: per-thread message of the last failure
km_status km_set_error(km_status st, const char* msg);

namespace {

struct HostProblem {
    int64_t n_traces;
    int32_t nt;
    double t_first, dt;
    const float *src, *rec, *x, *y, *t0sq, *s2, *r2;
    const int32_t* bin;
    int32_t nx, ny, nz, n_bins;
};

// Float32 squared leg length with the kernels' operation order (this file is
// compiled with -ffp-contract=off: nothing is fused).
inline float leg2(float px, float py, float sx, float sy) {
    const float dx = px - sx, dy = py - sy;
    const float a = dx * dx;
    const float b = dy * dy;
    return a + b;
}

// Total time in samples of one pair, float64 (float32 inputs widened exactly).
inline double pair_u(const HostProblem& P, int iz, float px, float py, int64_t j) {
    const double sx = P.src[2 * j], sy = P.src[2 * j + 1], rx = P.rec[2 * j], ry = P.rec[2 * j + 1];
    const double dxs = static_cast<double>(px) - sx, dys = static_cast<double>(py) - sy;
    const double dxr = static_cast<double>(px) - rx, dyr = static_cast<double>(py) - ry;
    const double hs2 = dxs * dxs + dys * dys;
    const double hr2 = dxr * dxr + dyr * dyr;
    const double t0 = P.t0sq[iz], s = P.s2[iz];
    const double a_s = t0 + s * hs2, a_r = t0 + s * hr2;
    return (std::sqrt(a_s) + std::sqrt(a_r) - P.t_first) / P.dt;
}

struct Counts {
    int64_t ap = 0, eff = 0;
};

// Counts of traces [j0, j1).  unsettled: the depths (ascending) whose times
// must be tested pair by pair.
Counts count_range(const HostProblem& P, int64_t j0, int64_t j1, bool monotone, const std::vector<char>& settled,
                   const std::vector<int>& unsettled) {
    Counts c;
    const int nz = P.nz;
    std::vector<float> R(P.r2, P.r2 + nz);
    for (int64_t j = j0; j < j1; ++j) {
        const int b = P.bin[j];
        if (b < 0 || b >= P.n_bins) continue;
        const float sx = P.src[2 * j], sy = P.src[2 * j + 1], rx = P.rec[2 * j], ry = P.rec[2 * j + 1];
        for (int iy = 0; iy < P.ny; ++iy) {
            const float py = P.y[iy];
            int zlo = -1;  // the previous column's first depth inside (-1: none yet in this row)
            for (int ix = 0; ix < P.nx; ++ix) {
                const float px = P.x[ix];
                const float hs = leg2(px, py, sx, sy), hr = leg2(px, py, rx, ry);
                const float hm = std::max(hs, hr);
                if (monotone) {
                    // first iz with hm <= R[iz] (R nondecreasing): a binary search
                    // for the row's first column, then a walk from the neighbour's
                    if (zlo < 0) {
                        zlo = static_cast<int>(std::partition_point(R.begin(), R.end(),
                                                                    [hm](float r) { return !(hm <= r); }) -
                                               R.begin());
                    } else {
                        while (zlo > 0 && hm <= R[zlo - 1]) --zlo;
                        while (zlo < nz && !(hm <= R[zlo])) ++zlo;
                    }
                    c.ap += nz - zlo;
                    int64_t eff = nz - zlo;
                    for (auto it = std::lower_bound(unsettled.begin(), unsettled.end(), zlo); it != unsettled.end();
                         ++it) {
                        const double u = pair_u(P, *it, px, py, j);
                        if (!(u > -1.0 && u < static_cast<double>(P.nt))) --eff;
                    }
                    c.eff += eff;
                } else {
                    for (int iz = 0; iz < nz; ++iz) {
                        if (!(hs <= R[iz] && hr <= R[iz])) continue;
                        ++c.ap;
                        if (settled[iz]) {
                            ++c.eff;
                            continue;
                        }
                        const double u = pair_u(P, iz, px, py, j);
                        if (u > -1.0 && u < static_cast<double>(P.nt)) ++c.eff;
                    }
                }
            }
        }
    }
    return c;
}

}  // namespace

extern "C" km_status km_count_contributions_host(const km_traces* t, const km_grid* g, const km_traveltime* tt,
                                                 int32_t n_threads, int64_t* n_aperture, int64_t* n_effective) {
    if (!t || !g || !tt || !n_aperture || !n_effective)
        return km_set_error(KM_E_INVALID, "km_count_contributions_host: NULL argument");
    if (t->n_traces < 0 || t->n_samples < 0 || g->nx < 0 || g->ny < 0 || g->nz < 0 || g->n_bins < 0)
        return km_set_error(KM_E_INVALID, "km_count_contributions_host: negative size");
    if (!(t->dt > 0.0) || !std::isfinite(t->dt) || !std::isfinite(t->t_first))
        return km_set_error(KM_E_INVALID, "km_count_contributions_host: dt must be finite and > 0, t_first finite");
    const bool empty = g->nx == 0 || g->ny == 0 || g->nz == 0 || g->n_bins == 0 || t->n_traces == 0;
    if (!empty) {
        if (!t->src || !t->rec || !t->bin || !g->x || !g->y || !tt->t0sq || !tt->s2 || !tt->r2)
            return km_set_error(KM_E_INVALID, "km_count_contributions_host: NULL host array");
    }
    *n_aperture = 0;
    *n_effective = 0;
    if (empty) return KM_OK;

    HostProblem P{t->n_traces, t->n_samples, t->t_first, t->dt, t->src, t->rec, g->x, g->y, tt->t0sq, tt->s2,
                  tt->r2, t->bin, g->nx, g->ny, g->nz, g->n_bins};
    const int nz = P.nz;
    bool monotone = true;
    for (int iz = 1; iz < nz; ++iz)
        if (!(P.r2[iz - 1] <= P.r2[iz])) monotone = false;  // also false for NaN entries

    // settled[iz]: every pair the aperture admits at depth iz has -1 < u < nt.
    // The pair's float64 h^2 may exceed r2 by the float32 rounding of h^2 (a
    // relative 2^-23 at most), so the bound takes r2 (1 + 1e-6) and a margin
    // of 1e-6 samples; a depth that cannot be settled is evaluated per pair.
    std::vector<char> settled(nz, 0);
    for (int iz = 0; iz < nz; ++iz) {
        const double t0 = P.t0sq[iz], s = P.s2[iz], r = P.r2[iz];
        if (!(r >= 0.0) || !std::isfinite(r) || !std::isfinite(t0) || !std::isfinite(s)) continue;
        const double a0 = t0, a1 = t0 + s * (r * (1.0 + 1e-6));
        if (!(a0 >= 0.0 && a1 >= 0.0)) continue;
        const double tl = 2.0 * std::sqrt(std::min(a0, a1)), th = 2.0 * std::sqrt(std::max(a0, a1));
        const double ul = (tl - P.t_first) / P.dt, uh = (th - P.t_first) / P.dt;
        settled[iz] = ul > -1.0 + 1e-6 && uh < static_cast<double>(P.nt) - 1e-6;
    }

    std::vector<int> unsettled;
    for (int iz = 0; iz < nz; ++iz)
        if (!settled[iz]) unsettled.push_back(iz);

    int nth = n_threads > 0 ? n_threads : static_cast<int>(std::thread::hardware_concurrency());
    nth = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nth, P.n_traces)));
    std::vector<Counts> part(nth);
    std::atomic<int64_t> next{0};
    const int64_t chunk = 64;
    auto worker = [&](int w) {
        for (;;) {
            const int64_t j0 = next.fetch_add(chunk);
            if (j0 >= P.n_traces) break;
            const Counts c = count_range(P, j0, std::min(P.n_traces, j0 + chunk), monotone, settled, unsettled);
            part[w].ap += c.ap;
            part[w].eff += c.eff;
        }
    };
    std::vector<std::thread> pool;
    try {
        for (int w = 1; w < nth; ++w) pool.emplace_back(worker, w);
    } catch (...) {
        // fewer threads than asked: the running ones (and this one) take the rest
    }
    worker(0);
    for (auto& th : pool) th.join();
    for (const Counts& c : part) {
        *n_aperture += c.ap;
        *n_effective += c.eff;
    }
    return KM_OK;
}
