// Demigration kernel: the transpose of migration as a trace-stationary scatter.
//
// Workgroup = a block of P.tb consecutive traces (of the bin-sorted list).
// The block's output rows live in LDS as float64 accumulators (same
// zero-padded row layout as the migration staging: row[kLead + k] = sample k).
// float64 because gfx950 executes LDS float64 atomic adds at about 8 clocks
// per wavefront instruction and float32 ones at about 190 (measured), and the
// wider sum also keeps the transpose's own rounding negligible.
//
// Wavefronts sweep the image columns that can be inside the aperture of some
// trace of the block (a box computed per depth chunk), one column per
// wavefront at a time; the four 16-lane groups of a wavefront work on four
// different traces of the block (lanes = 16 depths), so the LDS atomics of one
// instruction land in four different rows.  The next column's image values
// are loaded while the current one is evaluated, and the inner loop reads
// nothing from LDS (tables, aperture values and trace geometry are in
// registers), so no wait on a read ever waits behind the queued atomics.
// Each row is written back to HBM exactly once.
#include "km_kernels.h"

namespace km {

// Depth interleave of the adjoint's lanes: neighbouring lanes of a group are two
// depths apart, so their target samples are at least about one sample apart
// within the aperture and the LDS atomics of one instruction seldom share an address.
constexpr int kIL = 2;

// First and last index of v[0..n) with a <= v[i] <= b (compared in float64);
// lo > hi when there is none.  Wavefront-uniform.
__device__ __forceinline__ void index_range(const float* __restrict__ v, int n, double a, double b, int& lo, int& hi) {
    const int lane = threadIdx.x & (kLanes - 1);
    lo = n;
    hi = -1;
    for (int base = 0; base < n; base += kLanes) {
        const int i = base + lane;
        bool in = false;
        if (i < n) {
            const double c = v[i];
            in = c >= a && c <= b;
        }
        const uint64_t m = __builtin_amdgcn_ballot_w64(in);
        if (m) {
            if (lo == n) lo = base + __builtin_ctzll(m);
            hi = base + 63 - __builtin_clzll(m);
        }
    }
}

// Bits of the four 16-lane groups of a ballot, OR-ed / AND-ed into 16 bits.
__device__ __forceinline__ uint32_t fold_or(uint64_t m) {
    return static_cast<uint32_t>((m | (m >> 16) | (m >> 32) | (m >> 48)) & 0xFFFFull);
}
__device__ __forceinline__ uint32_t fold_and(uint64_t m) {
    return static_cast<uint32_t>((m & (m >> 16) & (m >> 32) & (m >> 48)) & 0xFFFFull);
}

// Two slots with a per-lane aperture mask, their taps merged by address.  The
// two slots of a pair are adjacent depths of one lane, so their samples i0 and
// i1 are usually equal or neighbours: the second slot's taps that land on i0
// or i0 + 1 are summed (in float32) into the first slot's, which go out as 2
// float64 atomics; its tap at i1 + 1 needs a third atomic where some lane has
// i1 != i0, its tap at i1 a fourth where some lane has i1 > i0 + 1 (instead
// of 4 atomics for every pair).  A slot outside the aperture contributes
// nothing (its value is zeroed; its clamped sample is still a valid base).  The table,
// extended-precision and anti-alias adjoints keep one pair of atomics per
// slot: with their longer evaluation the merge cost more than it saved.
template <bool TF, int WK>
__device__ __forceinline__ void dem_merged(float A0, float B0, float A1, float B1, float hs2, float hr2, double* row,
                                           float tfo, float wlo, float whi, float x0, float x1, bool act0, bool act1) {
    const Pair p0 = eval_pair<TF, WK, true>(A0, B0, hs2, hr2, tfo, wlo, whi);
    const Pair p1 = eval_pair<TF, WK, true>(A1, B1, hs2, hr2, tfo, wlo, whi);
    float q0 = (WK == W_COSCOS) ? x0 * p0.r : x0;
    float q1 = (WK == W_COSCOS) ? x1 * p1.r : x1;
    q0 = act0 ? q0 : 0.0f;  // a slot outside the aperture: both taps 0
    q1 = act1 ? q1 : 0.0f;
    const float b0 = p0.f * q0, b1 = p1.f * q1;
    const float t0 = q0 - b0, t2 = q1 - b1;
    const bool e0 = p1.i == p0.i, e1 = p1.i == p0.i + 1;
    const float v0 = t0 + (e0 ? t2 : 0.0f);                // at i0
    const float v1 = b0 + (e0 ? b1 : e1 ? t2 : 0.0f);      // at i0 + 1
    if (act0 || act1) {
        atomicAdd(row + p0.i, static_cast<double>(v0));
        atomicAdd(row + p0.i + 1, static_cast<double>(v1));
        if (act1 && !e0) {
            atomicAdd(row + p1.i + 1, static_cast<double>(b1));       // i0 + 2 when i1 = i0 + 1
            if (!e1) atomicAdd(row + p1.i, static_cast<double>(t2));  // i0 + 2 when i1 = i0 + 2
        }
    }
}

// Two slots with the extended-precision time (eval_pair_ext); the two taps
// are formed in float64 from the float64 fraction.
template <bool TF, int WK>
__device__ __forceinline__ void dem_masked_ext(float A0, float B0, float A1, float B1, double Hs, double Hr,
                                               double* row, double inv_dt, double tfo, int ilo, int ihi, double wlo,
                                               double whi, float x0, float x1, bool act0, bool act1) {
    if (act0) {
        const PairX p0 = eval_pair_ext<TF, WK>(A0, B0, Hs, Hr, inv_dt, tfo, ilo, ihi, wlo, whi);
        const double q0 = static_cast<double>((WK == W_COSCOS) ? x0 * p0.r : x0);
        const double b0 = p0.fd * q0;
        atomicAdd(row + p0.i, q0 - b0);
        atomicAdd(row + p0.i + 1, b0);
    }
    if (act1) {
        const PairX p1 = eval_pair_ext<TF, WK>(A1, B1, Hs, Hr, inv_dt, tfo, ilo, ihi, wlo, whi);
        const double q1 = static_cast<double>((WK == W_COSCOS) ? x1 * p1.r : x1);
        const double b1 = p1.fd * q1;
        atomicAdd(row + p1.i, q1 - b1);
        atomicAdd(row + p1.i + 1, b1);
    }
}

// dem_pair_table with extended legs (table_leg_ext).
template <bool TF, bool LAT>
__device__ __forceinline__ void dem_pair_table_ext(const Params& P, TLegX Ls, TLegX Lr, LCol C, int iz0, int iz1,
                                                   double* row, float wlo, float whi, float x0, float x1, bool act0,
                                                   bool act1) {
    if (act0) {
        const PairX p0 = eval_pair_table_ext<TF, LAT>(P, Ls, Lr, iz0, wlo, whi, C);
        const double q0 = static_cast<double>(x0 * p0.r);
        const double b0 = p0.fd * q0;
        atomicAdd(row + p0.i, q0 - b0);
        atomicAdd(row + p0.i + 1, b0);
    }
    if (act1) {
        const PairX p1 = eval_pair_table_ext<TF, LAT>(P, Ls, Lr, iz1, wlo, whi, C);
        const double q1 = static_cast<double>(x1 * p1.r);
        const double b1 = p1.fd * q1;
        atomicAdd(row + p1.i, q1 - b1);
        atomicAdd(row + p1.i + 1, b1);
    }
}

// The two slots of a full depth chunk's slot pair with table times: depths
// iz and iz + 1 of the same legs, read together (table_time_pair); each slot's
// time, weight and taps have the bits of dem_pair_table / dem_pair_table_ext
// (XF: extended legs).
template <bool TF, bool LAT, bool XF, typename Leg>
__device__ __forceinline__ void dem_pair_table2(const Params& P, Leg Ls, Leg Lr, LCol C, int iz, double* row,
                                                float wlo, float whi, float x0, float x1, bool act0, bool act1) {
    double w0, w1;
    if constexpr (XF) {
        const Dbl2 ts = table_time_pair<LAT>(P, Ls.off, Ls.f, C, iz);
        const Dbl2 tr = table_time_pair<LAT>(P, Lr.off, Lr.f, C, iz);
        w0 = (ts.a + tr.a) * P.inv_dt;
        w1 = (ts.b + tr.b) * P.inv_dt;
    } else {
        const TTime2 ts = table_time_pair2<LAT>(P, Ls.off, Ls.f, C, iz);
        const TTime2 tr = table_time_pair2<LAT>(P, Lr.off, Lr.f, C, iz);
        w0 = pair_time(P, ts.a, tr.a);
        w1 = pair_time(P, ts.b, tr.b);
    }
    float r0 = 1.0f, r1 = 1.0f;
    if (P.tamp) {
        const Flt2 as = table_amp_pair<LAT>(P, Ls.off, static_cast<float>(Ls.f), C, iz);
        const Flt2 ar = table_amp_pair<LAT>(P, Lr.off, static_cast<float>(Lr.f), C, iz);
        r0 = as.a * ar.a;
        r1 = as.b * ar.b;
    }
    if (TF) {
        w0 = w0 + P.tf_off_d;
        w1 = w1 + P.tf_off_d;
    }
    w0 = fmin(fmax(w0, static_cast<double>(wlo)), static_cast<double>(whi));
    w1 = fmin(fmax(w1, static_cast<double>(wlo)), static_cast<double>(whi));
    const int i0 = static_cast<int32_t>(w0), i1 = static_cast<int32_t>(w1);
    if (XF) {
        if (act0) {
            const double q = static_cast<double>(x0 * r0), b = (w0 - static_cast<double>(i0)) * q;
            atomicAdd(row + i0, q - b);
            atomicAdd(row + i0 + 1, b);
        }
        if (act1) {
            const double q = static_cast<double>(x1 * r1), b = (w1 - static_cast<double>(i1)) * q;
            atomicAdd(row + i1, q - b);
            atomicAdd(row + i1 + 1, b);
        }
    } else {
        if (act0) {
            const float q = x0 * r0, b = static_cast<float>(w0 - static_cast<double>(i0)) * q;
            atomicAdd(row + i0, static_cast<double>(q - b));
            atomicAdd(row + i0 + 1, static_cast<double>(b));
        }
        if (act1) {
            const float q = x1 * r1, b = static_cast<float>(w1 - static_cast<double>(i1)) * q;
            atomicAdd(row + i1, static_cast<double>(q - b));
            atomicAdd(row + i1 + 1, static_cast<double>(b));
        }
    }
}

// Two slots with table traveltimes (W = A_s A_r with amplitude tables, else
// 1); iz0, iz1 are the lane's depths of the two slots, clamped into the table.  LAT: laterally varying tables, C
// the column on the node grid.
template <bool TF, bool MASKED, bool LAT>
__device__ __forceinline__ void dem_pair_table(const Params& P, TLeg Ls, TLeg Lr, LCol C, int iz0, int iz1,
                                               double* row, float tfo, float wlo, float whi, float x0, float x1,
                                               bool act0, bool act1) {
    if (!MASKED || act0) {
        const Pair p0 = eval_pair_table<TF, true, LAT>(P, Ls, Lr, iz0, tfo, wlo, whi, C);
        const float q0 = x0 * p0.r;  // r = 1 without amplitude tables
        const float b0 = p0.f * q0;
        atomicAdd(row + p0.i, static_cast<double>(q0 - b0));
        atomicAdd(row + p0.i + 1, static_cast<double>(b0));
    }
    if (!MASKED || act1) {
        const Pair p1 = eval_pair_table<TF, true, LAT>(P, Ls, Lr, iz1, tfo, wlo, whi, C);
        const float q1 = x1 * p1.r;
        const float b1 = p1.f * q1;
        atomicAdd(row + p1.i, static_cast<double>(q1 - b1));
        atomicAdd(row + p1.i + 1, static_cast<double>(b1));
    }
}

// One slot with the anti-alias triangle filter: the transpose of the migrate
// value alpha T_L + beta T_{L+1} (second differences of the double running
// sum I2) interpolated between samples i and i + 1.  Each pair adds to the
// dual row G at the eight positions whose I2 it read; the kernel turns G into
// samples at the end (D[k] = sum_{n >= k} (n - k + 1) G[n]).
template <bool TF, int WK>
__device__ __forceinline__ void dem_slot_aa(const PairAA& p, float x, double* row) {
    const float q = (WK == W_COSCOS) ? x * p.r : x;
    const double a = static_cast<double>((1.0f - p.f) * q), b = static_cast<double>(p.f * q);
    const double al = p.alpha, be = p.beta;
    const int i = p.i, L = p.L;
    const double m2 = -2.0 * (al + be);
    atomicAdd(row + i - L - 2, a * be);
    atomicAdd(row + i - L - 1, fma(a, al, b * be));
    atomicAdd(row + i - L, b * al);
    atomicAdd(row + i - 1, a * m2);
    atomicAdd(row + i, b * m2);
    atomicAdd(row + i + L - 1, a * al);
    atomicAdd(row + i + L, fma(a, be, b * al));
    atomicAdd(row + i + L + 1, b * be);
}

// Image values (this lane's depth slots) and coordinates of one swept column.
template <int KS>
struct Column {
    float x[KS];
    float px, py;
};

// Coordinates and image values of column (ix, iy) through buffer loads: the
// resources and offsets are scalar (one resource per column; the lane's depth
// offsets are fixed per chunk), so no VALU instruction computes an address,
// and the loads count on the vector memory counter, so a wait for them never
// waits for the LDS atomics the wavefront has queued (a scalar load's would).
// voff (bytes from the column start): full chunks, voff[m] for the depth pair
// of slots 2m, 2m + 1 (two adjacent depths, one 8-byte load); TAIL (a chunk
// reaching outside [0, nz)), voff[k] per slot, the depth clamped into the
// column (those lanes never pass the aperture test, their value is unused).
template <int KS, bool TAIL>
__device__ __forceinline__ void fetch_column(const Params& P, __amdgpu_buffer_rsrc_t rx, __amdgpu_buffer_rsrc_t ry,
                                             const float* img, int ix, int iy, const int* voff, Column<KS>& c) {
    c.px = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rx, 0, ix * 4, 0));
    c.py = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ry, 0, iy * 4, 0));
    const float* colp = img + (static_cast<int64_t>(iy) * P.nx + ix) * P.nz;
    const __amdgpu_buffer_rsrc_t rc = raw_buffer(colp, static_cast<uint32_t>(P.nz) * 4u);
    if (TAIL) {
#pragma unroll
        for (int k = 0; k < KS; ++k) c.x[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rc, voff[k], 0, 0));
    } else {
#pragma unroll
        for (int m = 0; m < KS / 2; ++m) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(rc, voff[m], 0, 0);
            c.x[2 * m] = __uint_as_float(v[0]);
            c.x[2 * m + 1] = __uint_as_float(v[1]);
        }
    }
}

// Next column of a wavefront's walk: the box columns wave, wave + NW, ... in
// row-major order.  Returns false past the box.
template <int NW>
__device__ __forceinline__ bool next_column(int& ix, int& iy, int ix1, int iy1, int nbx) {
    ix += NW;
    while (ix > ix1) {
        ix -= nbx;
        ++iy;
    }
    return iy <= iy1;
}

// One depth chunk of the segment: wavefront `wave` takes the box columns
// wave, wave + NW, ... in row-major order and scatters every pairing of a
// column with the segment's traces into their rows.  The loop is unrolled by
// two over a pair of column buffers (the next column is loaded while the
// current one is evaluated, with no register copies between them).
template <int NW, int KS, int NQ, bool TF, int WK, bool TAIL, int TT, bool PX>
__device__ __forceinline__ void sweep_columns(const Params& P, const float* img, int z0, int d, int g, int wave, int t0,
                                              int nseg, int nq, int ix0, int ix1, int iy0, int iy1,
                                              const ChunkTables<KS>& T, const float* S, const float4* G, double* sAcc,
                                              const float* sInvSq) {
    static_assert(kIL == 2, "the 8-byte image loads take the two interleaved slots of a depth pair");
    constexpr uint32_t kMask = (KS >= 32) ? ~0u : ((1u << KS) - 1u);
    constexpr bool AA = TT == TT_AA;
    float wlo, whi;
    clamp_bounds<TF>(P.lt, wlo, whi);
    const float tfo = P.tf_off;
    const double tfod = P.tf_off_d;
    const int ilo = static_cast<int>(wlo), ihi = static_cast<int>(whi);
    const double wlod = wlo, whid = whi;
    int rowoff = TF ? 0 : kLead;
    const int lmax = AA ? P.aa_max : 0;
    if (AA) {
        // samples -(lmax + 2) .. nt + lmax + 2 (beyond them every triangle misses
        // the record); row index of sample n is aa_lead + n
        const int koff = TF ? kLead : 0;
        wlo = static_cast<float>(koff - lmax - 2);
        whi = static_cast<float>(koff + P.nt + lmax + 2);
        rowoff = P.aa_lead - koff;
    }
    double* rows[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) rows[q] = sAcc + (t0 + min(kGroupsPerWave * q + g, nseg - 1)) * P.lt + rowoff;
    int voff[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int iz = slot_depth<kIL>(z0, TAIL ? k : 2 * (k % (KS / 2)), d);
        voff[k] = 4 * (TAIL ? min(max(iz, 0), P.nz - 1) : iz);
    }
    const __amdgpu_buffer_rsrc_t rx = raw_buffer(P.x, static_cast<uint32_t>(P.nx) * 4u);
    const __amdgpu_buffer_rsrc_t ry = raw_buffer(P.y, static_cast<uint32_t>(P.ny) * 4u);
    const int nbx = ix1 - ix0 + 1;

    // every pairing of column c with the segment's traces
    constexpr bool LAT = TT == TT_LTABLE;
    auto process = [&](Column<KS>& c) {
        const float px = c.px, py = c.py;
        const LCol lc = LAT ? lateral_col(P, px, py) : LCol{0, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < KS; ++k) c.x[k] *= S[k];
        const float* x = c.x;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            // a segment holds at least one trace, so quad 0 always exists
            if (q > 0 && q >= nq) break;
            const Legs L = legs(px, py, G[q]);
            // lanes d >= KS hold rhi = -inf and rlo = +inf; kMask drops their bits
            const uint32_t any = fold_or(__builtin_amdgcn_ballot_w64(L.hmax <= T.rhi)) & kMask;
            if (!any) continue;
            double* row = rows[q];
            LegsX Lx{0.0, 0.0};
            if (PX) Lx = legs_ext(px, py, G[q]);
            if (AA) {
                // column minus source / receiver of this group's trace
                const float dxs = px - G[q].x, dys = py - G[q].y, dxr = px - G[q].z, dyr = py - G[q].w;
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    if (!((any >> k) & 1u)) continue;
                    if (L.hmax <= T.R[k]) {
                        const PairAA pa = eval_pair_aa<TF, WK>(T.A[k], T.B[k], L.hs2, L.hr2, tfo, wlo, whi, dxs, dys,
                                                               dxr, dyr, P.aa_dx, P.aa_dy, static_cast<float>(lmax),
                                                               sInvSq);
                        dem_slot_aa<TF, WK>(pa, x[k], row);
                    }
                }
                continue;
            }
            if (is_table(TT) && PX) {
                const TLegX Ls = table_leg_ext(P, Lx.hs2), Lr = table_leg_ext(P, Lx.hr2);
#pragma unroll
                for (int k = 0; k < KS; k += 2) {
                    if (!((any >> k) & 3u)) continue;
                    if (!TAIL) {  // every depth of the chunk exists: slot k + 1 is depth + 1
                        dem_pair_table2<TF, LAT, true>(P, Ls, Lr, lc, slot_depth<kIL>(z0, k, d), row, wlo, whi, x[k],
                                                       x[k + 1], L.hmax <= T.R[k], L.hmax <= T.R[k + 1]);
                        continue;
                    }
                    const int iz0 = min(max(slot_depth<kIL>(z0, k, d), 0), P.nz - 1);
                    const int iz1 = min(max(slot_depth<kIL>(z0, k + 1, d), 0), P.nz - 1);
                    dem_pair_table_ext<TF, LAT>(P, Ls, Lr, lc, iz0, iz1, row, wlo, whi, x[k], x[k + 1],
                                                L.hmax <= T.R[k], L.hmax <= T.R[k + 1]);
                }
                continue;
            }
            if (is_table(TT)) {
                const TLeg Ls = table_leg(P, L.hs2), Lr = table_leg(P, L.hr2);
#pragma unroll
                for (int k = 0; k < KS; k += 2) {
                    if (!((any >> k) & 3u)) continue;
                    if (!TAIL) {
                        dem_pair_table2<TF, LAT, false>(P, Ls, Lr, lc, slot_depth<kIL>(z0, k, d), row, wlo, whi,
                                                        x[k], x[k + 1], L.hmax <= T.R[k], L.hmax <= T.R[k + 1]);
                        continue;
                    }
                    const int iz0 = min(max(slot_depth<kIL>(z0, k, d), 0), P.nz - 1);
                    const int iz1 = min(max(slot_depth<kIL>(z0, k + 1, d), 0), P.nz - 1);
                    dem_pair_table<TF, true, LAT>(P, Ls, Lr, lc, iz0, iz1, row, tfo, wlo, whi, x[k], x[k + 1],
                                                  L.hmax <= T.R[k], L.hmax <= T.R[k + 1]);
                }
                continue;
            }
            if (PX) {
#pragma unroll
                for (int k = 0; k < KS; k += 2) {
                    if (!((any >> k) & 3u)) continue;
                    dem_masked_ext<TF, WK>(T.A[k], T.B[k], T.A[k + 1], T.B[k + 1], Lx.hs2, Lx.hr2, row, P.inv_dt,
                                           tfod, ilo, ihi, wlod, whid, x[k], x[k + 1], L.hmax <= T.R[k],
                                           L.hmax <= T.R[k + 1]);
                }
                continue;
            }
            // Every slot pair goes through the masked form: one code path per pair
            // measured faster than a separate unmasked variant for fully-inside pairs.
#pragma unroll
            for (int k = 0; k < KS; k += 2) {
                if (!((any >> k) & 3u)) continue;
                dem_merged<TF, WK>(T.A[k], T.B[k], T.A[k + 1], T.B[k + 1], L.hs2, L.hr2, row, tfo, wlo, whi, x[k],
                                   x[k + 1], L.hmax <= T.R[k], L.hmax <= T.R[k + 1]);
            }
        }
    };

    int ix = ix0 + wave, iy = iy0;
    while (ix > ix1) {
        ix -= nbx;
        ++iy;
    }
    if (iy > iy1) return;
    Column<KS> ca, cb;
    fetch_column<KS, TAIL>(P, rx, ry, img, ix, iy, voff, ca);
    for (;;) {
        const bool more_b = next_column<NW>(ix, iy, ix1, iy1, nbx);
        if (more_b) fetch_column<KS, TAIL>(P, rx, ry, img, ix, iy, voff, cb);
        process(ca);
        if (!more_b) break;
        const bool more_a = next_column<NW>(ix, iy, ix1, iy1, nbx);
        if (more_a) fetch_column<KS, TAIL>(P, rx, ry, img, ix, iy, voff, ca);
        process(cb);
        if (!more_a) break;
    }
}

// Traces t0..t1-1 of the block (one bin b, at most 4 NQ traces).
template <int NW, int KS, int NQ, bool TF, int WK, int TT, bool PX>
__device__ __forceinline__ void demigrate_segment(const Params& P, int b, int t0, int t1, const float4* sGeo,
                                                  double* sAcc, const float* sInvSq) {
    static_assert(KS % 2 == 0, "slots are evaluated in pairs");
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int g = lane / kGroup, d = lane % kGroup;
    const int nseg = t1 - t0;
    const int nq = (nseg + kGroupsPerWave - 1) / kGroupsPerWave;
    const float* img = P.image + static_cast<int64_t>(b) * P.nx * P.ny * P.nz;

    // group g of quad q works on trace 4 q + g of the segment (far away past its end)
    float4 G[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int t = kGroupsPerWave * q + g;
        G[q] = t < nseg ? sGeo[t0 + t] : make_float4(kFar, kFar, kFar, kFar);
    }
    // A column can be inside the aperture of trace j only if both its legs are
    // at most sqrt(r2) long, so in x it lies in [max(sx, rx) - rho, min(sx, rx) + rho]
    // (likewise in y); the union over the segment's traces bounds the columns.
    float ax = __builtin_inff(), bx = -__builtin_inff(), ay = __builtin_inff(), by = -__builtin_inff();
    if (lane < nseg) {
        const float4 s = sGeo[t0 + lane];
        ax = fmaxf(s.x, s.z);
        bx = fminf(s.x, s.z);
        ay = fmaxf(s.y, s.w);
        by = fminf(s.y, s.w);
    }
    ax = wave_min(ax);
    bx = wave_max(bx);
    ay = wave_min(ay);
    by = wave_max(by);

    for (int zc = 0; zc < P.n_zchunks; ++zc) {
        const int z0 = chunk_z0<true>(P.nz, zc, P.n_zchunks, KS * kGroup);
        ChunkTables<KS> T;
        load_chunk_tables<KS, kIL, TT, PX>(P, z0, d, WK == W_COSCOS, T, nullptr);
        if (!(T.rmax >= 0.0f)) continue;
        float S[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int iz = slot_depth<kIL>(z0, k, d);
            S[k] = (iz >= 0 && iz < P.nz) ? depth_factor<PX>(P, iz) : 0.0f;
        }
        // a float32 leg with |dx| > sqrt(r2) (1 + 2^-22) cannot pass the
        // float32 aperture test, so this radius keeps every column that can
        const double rho = sqrt(static_cast<double>(T.rmax)) * (1.0 + 1.0e-6);
        int ix0, ix1, iy0, iy1;
        index_range(P.x, P.nx, static_cast<double>(ax) - rho, static_cast<double>(bx) + rho, ix0, ix1);
        if (ix0 > ix1) continue;
        index_range(P.y, P.ny, static_cast<double>(ay) - rho, static_cast<double>(by) + rho, iy0, iy1);
        if (iy0 > iy1) continue;
        if (z0 < 0)  // the partial (shallowest) chunk
            sweep_columns<NW, KS, NQ, TF, WK, true, TT, PX>(P, img, z0, d, g, wave, t0, nseg, nq, ix0, ix1, iy0, iy1, T,
                                                            S, G, sAcc, sInvSq);
        else
            sweep_columns<NW, KS, NQ, TF, WK, false, TT, PX>(P, img, z0, d, g, wave, t0, nseg, nq, ix0, ix1, iy0, iy1,
                                                             T, S, G, sAcc, sInvSq);
    }
}

// The 4-slot square-root kernels are held to 6 wavefronts per SIMD (80 VGPRs;
// the float32 kernel spills 3 registers in its set-up, outside the column
// loop; the extended-precision one about 20, and ran 2.38 s against 2.56 s at
// its natural 108 on the 3D survey): with 8-wavefront one-quad workgroups that
// is three workgroups per CU, as many as their LDS rows allow.  The other
// kernels need more registers.
template <int NW, int KS, int NQ, bool TF, int WK, int TT = TT_DSR, bool PX = false>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(KS <= 4 && TT == TT_DSR ? 6 : 1)))
void demigrate_kernel(Params P) {
    static_assert(!(PX && TT == TT_AA), "no extended-precision anti-alias kernels");
    extern __shared__ float lds[];
    double* sAcc = reinterpret_cast<double*>(lds);                     // [tb][lt]
    float4* sGeo = reinterpret_cast<float4*>(lds + 2 * P.tb * P.lt);   // [tb]
    float* sInvSq = lds + 2 * P.tb * P.lt + 4 * P.tb;                  // [kAAMaxHalf + 2]: 1 / n^2
    const int64_t j0 = static_cast<int64_t>(blockIdx.x) * P.tb;
    if (TT == TT_AA)
        for (int t = threadIdx.x; t < kAAMaxHalf + 2; t += blockDim.x)
            sInvSq[t] = t > 0 ? 1.0f / static_cast<float>(t * t) : 0.0f;
    const int nb = static_cast<int>(min<int64_t>(P.tb, P.n_traces - j0));

    for (int t = threadIdx.x; t < P.tb; t += blockDim.x) {
        float4 g = make_float4(kFar, kFar, kFar, kFar);
        if (t < nb) {
            const int64_t j = j0 + t;
            g = make_float4(P.src[2 * j], P.src[2 * j + 1], P.rec[2 * j], P.rec[2 * j + 1]);
        }
        sGeo[t] = g;
    }
    for (int e = threadIdx.x; e < P.tb * P.lt; e += blockDim.x) sAcc[e] = 0.0;
    __syncthreads();

    // The block's traces form runs of equal bin (the list is sorted by bin).
    int t0 = 0;
    while (t0 < nb) {
        const int b = P.bin[j0 + t0];
        int t1 = t0 + 1;
        while (t1 < nb && P.bin[j0 + t1] == b) ++t1;
        if (b >= 0 && b < P.n_bins) demigrate_segment<NW, KS, NQ, TF, WK, TT, PX>(P, b, t0, t1, sGeo, sAcc, sInvSq);
        t0 = t1;
    }
    __syncthreads();

    if (TT == TT_AA) {
        // D[k] = sum_{n >= k} (n - k + 1) G[n]: two suffix sums of each row, one
        // wavefront per row, 64 positions at a time from the end.
        const int lane = threadIdx.x & (kLanes - 1);
        for (int t = threadIdx.x / kLanes; t < nb; t += NW) {
            double* row = sAcc + t * P.lt;
            for (int pass = 0; pass < 2; ++pass) {
                double carry = 0.0;
                for (int top = P.lt - 1; top >= 0; top -= kLanes) {
                    const int e = top - lane;
                    double v = e >= 0 ? row[e] : 0.0;
#pragma unroll
                    for (int off = 1; off < kLanes; off <<= 1) {
                        const double u = __shfl_up(v, off, kLanes);
                        if (lane >= off) v += u;
                    }
                    if (e >= 0) row[e] = carry + v;
                    carry += __shfl(v, kLanes - 1, kLanes);
                }
            }
        }
        __syncthreads();
    }

    float* out = static_cast<float*>(P.data);
    for (int t = 0; t < nb; ++t) {
        float* o = out + (j0 + t) * P.stride;
        const double* row = sAcc + t * P.lt + (TT == TT_AA ? P.aa_lead : kLead);
        for (int k = threadIdx.x; k < P.nt; k += blockDim.x) {
            const float v = static_cast<float>(row[k]);
            o[k] = P.accumulate ? o[k] + v : v;
        }
    }
}

// The plain kernels of one time precision (PX) for the weight and t_first cases.
template <int NW, int KS, int NQ, bool PX>
static hipError_t launch_demigrate_dsr(const Params& P, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
    if (P.has_tf) {
        if (P.weight == W_COSCOS)
            return launch_with_lds(demigrate_kernel<NW, KS, NQ, true, W_COSCOS, TT_DSR, PX>, grid, block, lds, s, P);
        return launch_with_lds(demigrate_kernel<NW, KS, NQ, true, W_UNIT, TT_DSR, PX>, grid, block, lds, s, P);
    }
    if (P.weight == W_COSCOS)
        return launch_with_lds(demigrate_kernel<NW, KS, NQ, false, W_COSCOS, TT_DSR, PX>, grid, block, lds, s, P);
    return launch_with_lds(demigrate_kernel<NW, KS, NQ, false, W_UNIT, TT_DSR, PX>, grid, block, lds, s, P);
}

template <int NW, int KS, int NQ>
static hipError_t launch_demigrate_shape(const Params& P, hipStream_t s) {
    if (P.tb < 1 || P.tb > kGroupsPerWave * NQ) return hipErrorInvalidValue;
    const int64_t nblk = (P.n_traces + P.tb - 1) / P.tb;
    dim3 grid(static_cast<unsigned>(nblk)), block(NW * 64);
    const size_t lds = lds_bytes_f64rows(P);
    if (P.ttab && P.n_gx > 0) {  // laterally varying tables: W = 1
        if (P.prec) {
            if (P.has_tf)
                return launch_with_lds(demigrate_kernel<NW, KS, NQ, true, W_UNIT, TT_LTABLE, true>, grid, block, lds, s, P);
            return launch_with_lds(demigrate_kernel<NW, KS, NQ, false, W_UNIT, TT_LTABLE, true>, grid, block, lds, s, P);
        }
        if (P.has_tf) return launch_with_lds(demigrate_kernel<NW, KS, NQ, true, W_UNIT, TT_LTABLE>, grid, block, lds, s, P);
        return launch_with_lds(demigrate_kernel<NW, KS, NQ, false, W_UNIT, TT_LTABLE>, grid, block, lds, s, P);
    }
    if (P.ttab) {  // table traveltimes: W = 1 (the host rejects other weights)
        if (P.prec) {
            if (P.has_tf)
                return launch_with_lds(demigrate_kernel<NW, KS, NQ, true, W_UNIT, TT_TABLE, true>, grid, block, lds, s, P);
            return launch_with_lds(demigrate_kernel<NW, KS, NQ, false, W_UNIT, TT_TABLE, true>, grid, block, lds, s, P);
        }
        if (P.has_tf) return launch_with_lds(demigrate_kernel<NW, KS, NQ, true, W_UNIT, TT_TABLE>, grid, block, lds, s, P);
        return launch_with_lds(demigrate_kernel<NW, KS, NQ, false, W_UNIT, TT_TABLE>, grid, block, lds, s, P);
    }
    if (P.aa_max > 0) {  // anti-alias triangle filter
        if (P.has_tf) {
            if (P.weight == W_COSCOS)
                return launch_with_lds(demigrate_kernel<NW, KS, NQ, true, W_COSCOS, TT_AA>, grid, block, lds, s, P);
            return launch_with_lds(demigrate_kernel<NW, KS, NQ, true, W_UNIT, TT_AA>, grid, block, lds, s, P);
        }
        if (P.weight == W_COSCOS)
            return launch_with_lds(demigrate_kernel<NW, KS, NQ, false, W_COSCOS, TT_AA>, grid, block, lds, s, P);
        return launch_with_lds(demigrate_kernel<NW, KS, NQ, false, W_UNIT, TT_AA>, grid, block, lds, s, P);
    }
    if (P.prec) return launch_demigrate_dsr<NW, KS, NQ, true>(P, grid, block, lds, s);
    return launch_demigrate_dsr<NW, KS, NQ, false>(P, grid, block, lds, s);
}

// (waves, depth slots, trace quads per workgroup, LDS budget for the trace
// accumulators).  The fourth is the default: one quad of traces per
// 8-wavefront workgroup with 4 slots, so that three workgroups share a CU (the
// first, with 8 slots, fits two); one-quad workgroups measured faster than 12
// traces per 16-wavefront workgroup (one per CU), although each workgroup then
// reads its box of image columns for 4 traces instead of 12.
#define KM_DEMIGRATE_SHAPES(X) \
    X(8, 8, 1, 49152)          \
    X(16, 8, 3, 147456)        \
    X(16, 8, 2, 98304)         \
    X(8, 4, 1, 49152)          \
    X(8, 8, 3, 147456)

static const TileShape kDemigrateShapes[] = {
#define X(nw, ks, nq, lb) {nw, 1, ks, lb, nq},
    KM_DEMIGRATE_SHAPES(X)
#undef X
};

int demigrate_shape_count() { return static_cast<int>(sizeof(kDemigrateShapes) / sizeof(kDemigrateShapes[0])); }
const TileShape& demigrate_shape(int i) { return kDemigrateShapes[i]; }

hipError_t launch_demigrate(int shape, const Params& P, hipStream_t s) {
    int i = 0;
#define X(nw, ks, nq, lb) \
    if (shape == i) return launch_demigrate_shape<nw, ks, nq>(P, s); \
    ++i;
    KM_DEMIGRATE_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace km
