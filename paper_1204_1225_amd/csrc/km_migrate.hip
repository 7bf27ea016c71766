// Migration kernel: Eq. (1) as an image-stationary gather.
//
// Workgroup = (offset bin b, column tile, depth chunk).  Each wavefront keeps
// CWQ groups of 4 image columns x (16 * KS) depths of float32 accumulators
// in registers; the traces of bin b stream through LDS in blocks.  A trace
// enters a block only if it can have a pair inside the aperture of the tile
// and chunk, and only the time window its pairs can read is staged (the
// double-square-root time grows with the squared leg lengths, so the window
// follows from the tile's bounding box and the chunk's tables).  For every
// column group the wavefront computes the two squared leg lengths of 16
// traces at once (lane = (column, trace)), hands them to the depth lanes
// through the LDS crossbar, derives from a ballot which 16-depth slots can
// hold a pair inside the aperture, and evaluates those slots two at a time:
// per lane two square roots, the sample index and fraction, one 8-byte LDS
// read of the staged (sample, difference) pair, the interpolation, the weight
// and the lane's aperture mask.  Table times and the anti-alias filter use
// the same blocks with their own staged forms (plain samples; float64 double
// running sums, one slot at a time).  With 16-bit traces the S16 kernels keep
// the samples' 16-bit storage in LDS instead (packed pairs; single samples for
// table times) and widen them on read.
#include "km_kernels.h"

namespace km {

// Sample k of trace j: zero outside [0, nt), times the per-trace scale for
// 16-bit storage.
__device__ __forceinline__ float trace_sample(const Params& P, int64_t j, int k, float sc) {
    if (k < 0 || k >= P.nt) return 0.0f;
    if (P.dtype == F32) return static_cast<const float*>(P.data)[j * P.stride + k];
    return widen16(static_cast<const uint16_t*>(P.data)[j * P.stride + k], P.dtype) * sc;
}

// Stage the window of samples lo .. lo + len - 1 of trace j as len floats
// (the whole-record windows of table traveltimes).  One wavefront.
__device__ __forceinline__ void stage_window_f(const Params& P, int64_t j, int lo, int len, float* dst, int lane) {
    const float sc = (P.dtype != F32 && P.scale) ? P.scale[j] : 1.0f;
    for (int e0 = 0; e0 < len; e0 += 4 * kLanes) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * kLanes + lane;
            v[u] = e < len ? trace_sample(P, j, lo + e, sc) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * kLanes + lane;
            if (e < len) dst[e] = v[u];
        }
    }
}

// 16-bit storage bits of sample k of trace row src (zero bits, +0, outside the record).
__device__ __forceinline__ uint32_t sample_bits16(const Params& P, const uint16_t* src, int k) {
    return (k >= 0 && k < P.nt) ? static_cast<uint32_t>(src[k]) : 0u;
}

// Stage the window of samples lo .. lo + len - 1 of trace j as len - 1 packed
// pairs dst[e] = bits(D[lo + e]) | bits(D[lo + e + 1]) << 16 of the 16-bit
// storage (half the LDS of float (sample, difference) pairs); the reads widen
// them and apply the trace's scale.  One wavefront.
__device__ __forceinline__ void stage_window_16p(const Params& P, int64_t j, int lo, int len, uint32_t* dst, int lane) {
    const uint16_t* src = static_cast<const uint16_t*>(P.data) + j * P.stride;
    for (int e0 = 0; e0 < len - 1; e0 += 2 * kLanes) {
        uint32_t a[2], b[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = e0 + u * kLanes + lane;
            a[u] = 0u;
            b[u] = 0u;
            if (e < len - 1) {
                a[u] = sample_bits16(P, src, lo + e);
                b[u] = sample_bits16(P, src, lo + e + 1);
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = e0 + u * kLanes + lane;
            if (e < len - 1) dst[e] = a[u] | (b[u] << 16);
        }
    }
}

// Stage the window of samples lo .. lo + len - 1 of trace j as len 16-bit
// storage values (half the LDS of float samples: the whole-record windows of
// table traveltimes).  One wavefront.
__device__ __forceinline__ void stage_window_16(const Params& P, int64_t j, int lo, int len, uint16_t* dst, int lane) {
    const uint16_t* src = static_cast<const uint16_t*>(P.data) + j * P.stride;
    for (int e0 = 0; e0 < len; e0 += 4 * kLanes) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * kLanes + lane;
            v[u] = e < len ? sample_bits16(P, src, lo + e) : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * kLanes + lane;
            if (e < len) dst[e] = static_cast<uint16_t>(v[u]);
        }
    }
}

// The two samples of a packed pair (low half: the first), widened.
template <int DT>
__device__ __forceinline__ void widen_pair(uint32_t w, float& a, float& b) {
    if (DT == BF16) {
        a = __uint_as_float(w << 16);
        b = __uint_as_float(w & 0xffff0000u);
    } else {
        a = widen16(w & 0xffffu, DT);
        b = widen16(w >> 16, DT);
    }
}

// Samples k and k + 1 of a window staged by stage_window_16, k counted in
// 16-bit values from s: the two aligned words that hold them, funnel-shifted
// (for even k the second word is not used; it is still inside the
// workgroup's LDS, as the trace block's slot records follow the windows).
__device__ __forceinline__ uint32_t read_pair16(const uint32_t* s, int k) {
    const uint32_t w0 = s[k >> 1], w1 = s[(k >> 1) + 1];
    return __builtin_amdgcn_alignbit(w1, w0, static_cast<uint32_t>(k & 1) << 4);
}

// Stage, for positions lo .. lo + len - 1 of trace j, the double running sum
// I2[n] = sum_{m <= n} sum_{k <= m} D[k] (float64, from position lo; D zero
// outside [0, nt)): the anti-alias triangles are second differences of it.
// One wavefront: running sums over 64 positions at a time.
__device__ __forceinline__ void stage_window_i2(const Params& P, int64_t j, int lo, int len, double* dst, int lane) {
    const float sc = (P.dtype != F32 && P.scale) ? P.scale[j] : 1.0f;
    double c1 = 0.0, c2 = 0.0;  // I1 and I2 at the position before the chunk
    for (int e0 = 0; e0 < len; e0 += kLanes) {
        const int e = e0 + lane;
        double v = e < len ? static_cast<double>(trace_sample(P, j, lo + e, sc)) : 0.0;
#pragma unroll
        for (int off = 1; off < kLanes; off <<= 1) {
            const double t = __shfl_up(v, off, kLanes);
            if (lane >= off) v += t;
        }
        const double i1 = c1 + v;
        double w = i1;
#pragma unroll
        for (int off = 1; off < kLanes; off <<= 1) {
            const double t = __shfl_up(w, off, kLanes);
            if (lane >= off) w += t;
        }
        const double i2 = c2 + w;
        if (e < len) dst[e] = i2;
        c1 = __shfl(i1, kLanes - 1, kLanes);
        c2 = __shfl(i2, kLanes - 1, kLanes);
    }
}

// Stage the window of samples lo .. lo + len - 1 of trace j as len - 1 pairs
// dst[e] = (D[lo + e], D[lo + e + 1] - D[lo + e]): the interpolation then
// reads one pair and needs one FMA.  One wavefront.
__device__ __forceinline__ void stage_window(const Params& P, int64_t j, int lo, int len, float2* dst, int lane) {
    const float sc = (P.dtype != F32 && P.scale) ? P.scale[j] : 1.0f;
    for (int e0 = 0; e0 < len - 1; e0 += 2 * kLanes) {
        float a[2], b[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = e0 + u * kLanes + lane;
            a[u] = 0.0f;
            b[u] = 0.0f;
            if (e < len - 1) {
                a[u] = trace_sample(P, j, lo + e, sc);
                b[u] = trace_sample(P, j, lo + e + 1, sc);
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = e0 + u * kLanes + lane;
            if (e < len - 1) dst[e] = make_float2(a[u], b[u] - a[u]);
        }
    }
}

// Two slots (k, k + 1) of one (column group, trace) pairing.  MASKED: some
// valid lane may be outside the aperture, so each value is kept only where
// hmax <= the lane's aperture value; CLAMP: the time is clamped to the row.
// R0, R1: the lanes' aperture values of the two slots (read only when MASKED).
// row[i] = (D[i], D[i + 1] - D[i]) of the staged window.
template <bool TF, int WK, bool MASKED, bool CLAMP>
__device__ __forceinline__ void mig_pair(float A0, float B0, float A1, float B1, float hs2, float hr2, float hm,
                                         const float2* row, float tfo, float wlo, float whi, float R0, float R1,
                                         float& acc0, float& acc1) {
    const Pair p0 = eval_pair<TF, WK, CLAMP>(A0, B0, hs2, hr2, tfo, wlo, whi);
    const Pair p1 = eval_pair<TF, WK, CLAMP>(A1, B1, hs2, hr2, tfo, wlo, whi);
    const float2 e0 = row[p0.i];
    const float2 e1 = row[p1.i];
    float v0 = fmaf(p0.f, e0.y, e0.x);
    float v1 = fmaf(p1.f, e1.y, e1.x);
    if (MASKED) {
        v0 = (hm <= R0) ? v0 : 0.0f;
        v1 = (hm <= R1) ? v1 : 0.0f;
    }
    acc0 = (WK == W_COSCOS) ? fmaf(v0, p0.r, acc0) : acc0 + v0;
    acc1 = (WK == W_COSCOS) ? fmaf(v1, p1.r, acc1) : acc1 + v1;
}

// mig_pair on a window staged as packed 16-bit pairs (stage_window_16p): the
// pair is widened and interpolated, and the trace's scale joins the weight.
template <bool TF, int WK, int DT>
__device__ __forceinline__ void mig_pair16(float A0, float B0, float A1, float B1, float hs2, float hr2, float hm,
                                           const uint32_t* row, float scl, float tfo, float wlo, float whi,
                                           float R0, float R1, float& acc0, float& acc1) {
    const Pair p0 = eval_pair<TF, WK, true>(A0, B0, hs2, hr2, tfo, wlo, whi);
    const Pair p1 = eval_pair<TF, WK, true>(A1, B1, hs2, hr2, tfo, wlo, whi);
    float a0, b0, a1, b1;
    widen_pair<DT>(row[p0.i], a0, b0);
    widen_pair<DT>(row[p1.i], a1, b1);
    float v0 = fmaf(p0.f, b0 - a0, a0);
    float v1 = fmaf(p1.f, b1 - a1, a1);
    v0 = (hm <= R0) ? v0 : 0.0f;
    v1 = (hm <= R1) ? v1 : 0.0f;
    acc0 = fmaf(v0, (WK == W_COSCOS) ? p0.r * scl : scl, acc0);
    acc1 = fmaf(v1, (WK == W_COSCOS) ? p1.r * scl : scl, acc1);
}

// mig_pair with table traveltimes (W = A_s A_r with amplitude tables, else 1):
// iz0, iz1 are the lane's depths of the two slots, clamped into the table.  LAT: laterally varying tables, C the
// lane's column on the node grid.
template <bool TF, bool MASKED, bool LAT>
__device__ __forceinline__ void mig_pair_table(const Params& P, TLeg Ls, TLeg Lr, LCol C, int iz0, int iz1, float hm,
                                               const float* row, float tfo, float wlo, float whi, float R0, float R1,
                                               float& acc0, float& acc1) {
    const Pair p0 = eval_pair_table<TF, true, LAT>(P, Ls, Lr, iz0, tfo, wlo, whi, C);
    const Pair p1 = eval_pair_table<TF, true, LAT>(P, Ls, Lr, iz1, tfo, wlo, whi, C);
    const float a0 = row[p0.i], b0 = row[p0.i + 1];
    const float a1 = row[p1.i], b1 = row[p1.i + 1];
    float v0 = fmaf(p0.f, b0 - a0, a0);
    float v1 = fmaf(p1.f, b1 - a1, a1);
    if (MASKED) {
        v0 = (hm <= R0) ? v0 : 0.0f;
        v1 = (hm <= R1) ? v1 : 0.0f;
    }
    // r = 1 without amplitude tables: the same bits as acc + v
    acc0 = fmaf(v0, p0.r, acc0);
    acc1 = fmaf(v1, p1.r, acc1);
}

// mig_pair_table on a window staged as 16-bit values (stage_window_16): s is
// the trace block's windows as words, rb the row's offset in 16-bit values.
template <bool TF, bool LAT, int DT>
__device__ __forceinline__ void mig_pair_table16(const Params& P, TLeg Ls, TLeg Lr, LCol C, int iz0, int iz1, float hm,
                                                 const uint32_t* s, int rb, float scl, float tfo, float wlo, float whi,
                                                 float R0, float R1, float& acc0, float& acc1) {
    const Pair p0 = eval_pair_table<TF, true, LAT>(P, Ls, Lr, iz0, tfo, wlo, whi, C);
    const Pair p1 = eval_pair_table<TF, true, LAT>(P, Ls, Lr, iz1, tfo, wlo, whi, C);
    float a0, b0, a1, b1;
    widen_pair<DT>(read_pair16(s, rb + p0.i), a0, b0);
    widen_pair<DT>(read_pair16(s, rb + p1.i), a1, b1);
    float v0 = fmaf(p0.f, b0 - a0, a0);
    float v1 = fmaf(p1.f, b1 - a1, a1);
    v0 = (hm <= R0) ? v0 : 0.0f;
    v1 = (hm <= R1) ? v1 : 0.0f;
    acc0 = fmaf(v0, p0.r * scl, acc0);
    acc1 = fmaf(v1, p1.r * scl, acc1);
}

// One slot with the extended-precision time (eval_pair_ext): leg lengths in
// float64, the clamp as integer bounds [ilo, ihi] (or float64 [wlo, whi] with
// t_first).  One slot at a time: the float64 temporaries of two slots in
// flight would cost more registers than the latency they hide.
template <bool TF, int WK>
__device__ __forceinline__ void mig_slot_ext(float A, float B, double Hs, double Hr, float hm, const float2* row,
                                             double inv_dt, double tfo, int ilo, int ihi, double wlo, double whi,
                                             float R, float& acc) {
    // keep the tables' float64 conversions inside the loop (hoisted, they
    // would hold two more registers per slot)
    asm volatile("" : "+v"(A), "+v"(B));
    const PairX p = eval_pair_ext<TF, WK>(A, B, Hs, Hr, inv_dt, tfo, ilo, ihi, wlo, whi);
    const float2 e = row[p.i];
    float v = fmaf(p.f, e.y, e.x);
    v = (hm <= R) ? v : 0.0f;
    acc = (WK == W_COSCOS) ? fmaf(v, p.r, acc) : acc + v;
}

// mig_pair_table with extended legs (table_leg_ext).
template <bool TF, bool LAT>
__device__ __forceinline__ void mig_pair_table_ext(const Params& P, TLegX Ls, TLegX Lr, LCol C, int iz0, int iz1,
                                                   float hm, const float* row, float wlo, float whi, float R0,
                                                   float R1, float& acc0, float& acc1) {
    const PairX p0 = eval_pair_table_ext<TF, LAT>(P, Ls, Lr, iz0, wlo, whi, C);
    const PairX p1 = eval_pair_table_ext<TF, LAT>(P, Ls, Lr, iz1, wlo, whi, C);
    const float a0 = row[p0.i], b0 = row[p0.i + 1];
    const float a1 = row[p1.i], b1 = row[p1.i + 1];
    float v0 = fmaf(p0.f, b0 - a0, a0);
    float v1 = fmaf(p1.f, b1 - a1, a1);
    v0 = (hm <= R0) ? v0 : 0.0f;
    v1 = (hm <= R1) ? v1 : 0.0f;
    acc0 = fmaf(v0, p0.r, acc0);
    acc1 = fmaf(v1, p1.r, acc1);
}

// Two slots with the anti-alias triangle filter.  row[n] = I2 at window
// position n (staged by stage_window_i2): the smoothed sample at c is
// alpha T_L(c) + beta T_{L+1}(c), T_L(c) = I2[c+L-1] - 2 I2[c-1] + I2[c-L-1],
// read as five (n, n + 1) pairs for c = i and c = i + 1.
template <bool TF, int WK>
__device__ __forceinline__ float aa_value(const PairAA& p, const double* row) {
    const int i = p.i, L = p.L;
    const double a1 = row[i + L - 1], b1 = row[i + L];
    const double a2 = row[i - 1], b2 = row[i];
    const double a3 = row[i - L - 1], b3 = row[i - L];
    const double b4 = row[i + L + 1];
    const double a5 = row[i - L - 2];
    // a4 = b1, b5 = a3
    const double tl0 = fma(-2.0, a2, a1 + a3), tl1 = fma(-2.0, b2, b1 + b3);   // T_L(i), T_L(i + 1)
    const double tm0 = fma(-2.0, a2, b1 + a5), tm1 = fma(-2.0, b2, b4 + a3);   // T_{L+1}(i), T_{L+1}(i + 1)
    const double al = p.alpha, be = p.beta;
    const double v0 = fma(be, tm0, al * tl0), v1 = fma(be, tm1, al * tl1);
    return static_cast<float>(fma(static_cast<double>(p.f), v1 - v0, v0));
}

// One slot at a time (two in flight need more registers than the eight
// float64 reads leave).
template <bool TF, int WK>
__device__ __forceinline__ void mig_slot_aa(float A, float B, float hs2, float hr2, float hm, const double* row,
                                            float tfo, float wlo, float whi, float R, float dxs, float dys, float dxr,
                                            float dyr, float adx, float ady, float lmax, const float* invsq,
                                            float& acc) {
    const PairAA p = eval_pair_aa<TF, WK>(A, B, hs2, hr2, tfo, wlo, whi, dxs, dys, dxr, dyr, adx, ady, lmax, invsq);
    float v = aa_value<TF, WK>(p, row);
    v = (hm <= R) ? v : 0.0f;
    acc = (WK == W_COSCOS) ? fmaf(v, p.r, acc) : acc + v;
}

// RREG: the masked slots take the lanes' aperture values from registers
// (else from the LDS copy, which costs fewer registers).
// TT: traveltime kind (TT_TABLE: one-way time table, W = 1; TT_LTABLE: one
// table per node of a lateral grid, W = 1).
// PX: extended-precision times (eval_pair_ext, table_leg_ext); the squared
// leg lengths then also reach the depth lanes in float64.
//
// LDS (lds_bytes): window storage [P.cap floats; a window of n samples takes
// n - 1 pairs], per block slot the trace geometry (float4) and (float offset,
// first sample, last sample, trace - bin start) (int4) [P.tb each], the aperture values [KS * 16], the tile box
// [4 per wavefront] and the candidates of one pass [NW * 4 x (int2, float4)].
template <int NW, int CWQ, int KS, bool TF, int WK, bool RREG, int TT = TT_DSR, bool PX = false, int S16 = 0>
__device__ __forceinline__ void migrate_tile(const Params& P, int b, int tile, int zc, float* lds) {
    static_assert(!(PX && TT == TT_AA), "no extended-precision anti-alias kernels");
    // S16: the 16-bit storage type (BF16 or F16) staged as it is, 0 for float staging
    static_assert(!(S16 && (PX || TT == TT_AA)), "16-bit staging: float32 time, no anti-alias filter");
    static_assert(KS % 2 == 0, "slots are evaluated in pairs");
    constexpr int NG = NW * kGroupsPerWave;  // candidate traces per pass: one per 16-lane group
    static_assert(NG <= kLanes && NW <= kBoxFloats / 4, "at most 16 wavefronts");
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = threadIdx.x / kLanes;
    const int g = lane / kGroup, d = lane % kGroup;
    const int ncol = P.nx * P.ny;
    const int z0 = chunk_z0<false>(P.nz, zc, P.n_zchunks, KS * kGroup);
    const int nt = P.nt;
    // staged-row index of sample k is k + koff (eval_pair adds kLead with t_first)
    const int koff = TF ? kLead : 0;
    // staged form: (sample, difference) pairs for the square-root times (windows
    // of a few hundred samples), plain samples for the whole-record windows of
    // table times (half the LDS per trace), float64 double running sums with
    // the anti-alias filter
    constexpr bool PAIRS = TT == TT_DSR && !S16;
    constexpr bool AA = TT == TT_AA;
    constexpr bool P16 = TT == TT_DSR && S16;  // packed 16-bit pairs
    constexpr bool T16 = is_table(TT) && S16;  // 16-bit samples
    // anti-aliasing: largest half-width, and the reach of a pair's reads around
    // its sample (L + 2 below, L + 2 above counting the pair's second sample)
    const int lmax = AA ? P.aa_max : 0;

    float* sTr = lds;                                                    // [cap]
    float4* sGeo = reinterpret_cast<float4*>(lds + P.cap);               // [tb]
    int4* sMeta = reinterpret_cast<int4*>(lds + P.cap + 4 * P.tb);       // [tb]
    float* sR = lds + P.cap + 8 * P.tb;                                  // [KS * 16]
    float* sBox = sR + KS * kGroup;                                      // [kBoxFloats]
    int2* sCand = reinterpret_cast<int2*>(sBox + kBoxFloats);            // [kCandMax]
    float4* sCandGeo = reinterpret_cast<float4*>(sBox + kBoxFloats + 2 * kCandMax);  // [kCandMax]
    float* sInvSq = sBox + kBoxFloats + 6 * kCandMax;                    // [kAAMaxHalf + 2]: 1 / n^2
    if (AA)
        for (int t = threadIdx.x; t < kAAMaxHalf + 2; t += blockDim.x)
            sInvSq[t] = t > 0 ? 1.0f / static_cast<float>(t * t) : 0.0f;

    ChunkTables<KS> T;
    load_chunk_tables<KS, 1, TT, PX>(P, z0, d, WK == W_COSCOS, T, sR);

    float px[CWQ], py[CWQ];
    int colv[CWQ];
#pragma unroll
    for (int q = 0; q < CWQ; ++q) {
        const int col = (tile * NW * CWQ + wave * CWQ + q) * kGroupsPerWave + g;
        colv[q] = col;
        px[q] = kFar;
        py[q] = kFar;
        if (col < ncol) {
            px[q] = P.x[col % P.nx];
            py[q] = P.y[col / P.nx];
        }
    }

    // the lane's columns on the node grid of laterally varying tables
    constexpr bool LAT = TT == TT_LTABLE;
    LCol lc[CWQ];
#pragma unroll
    for (int q = 0; q < CWQ; ++q) lc[q] = LAT ? lateral_col(P, px[q], py[q]) : LCol{0, 0.0f, 0.0f};

    float acc[CWQ][KS];
#pragma unroll
    for (int q = 0; q < CWQ; ++q)
#pragma unroll
        for (int k = 0; k < KS; ++k) acc[q][k] = 0.0f;

    const int64_t lo = lower_bound_bin(P.bin, P.n_traces, b);
    const int64_t hi = lower_bound_bin(P.bin, P.n_traces, b + 1);
    const float tfo = P.tf_off;
    const double tfod = P.tf_off_d;

    // Bounding box of the tile's columns.  A leg longer than sqrt(r2)(1 + 2^-22)
    // from every column cannot pass the float32 aperture test, so a trace whose
    // source or receiver lies farther than that from the box (with a 1e-5
    // margin on the squared radius) has no pair in this tile and depth chunk.
    {
        float bx0 = __builtin_inff(), bx1 = -__builtin_inff(), by0 = __builtin_inff(), by1 = -__builtin_inff();
#pragma unroll
        for (int q = 0; q < CWQ; ++q) {
            if (colv[q] < ncol) {
                bx0 = fminf(bx0, px[q]);
                bx1 = fmaxf(bx1, px[q]);
                by0 = fminf(by0, py[q]);
                by1 = fmaxf(by1, py[q]);
            }
        }
        bx0 = wave_min(bx0);
        bx1 = wave_max(bx1);
        by0 = wave_min(by0);
        by1 = wave_max(by1);
        if (lane == 0) {
            sBox[4 * wave] = bx0;
            sBox[4 * wave + 1] = bx1;
            sBox[4 * wave + 2] = by0;
            sBox[4 * wave + 3] = by1;
        }
    }
    __syncthreads();
    float bx0 = sBox[0], bx1 = sBox[1], by0 = sBox[2], by1 = sBox[3];
    for (int w = 1; w < NW; ++w) {
        bx0 = fminf(bx0, sBox[4 * w]);
        bx1 = fmaxf(bx1, sBox[4 * w + 1]);
        by0 = fminf(by0, sBox[4 * w + 2]);
        by1 = fmaxf(by1, sBox[4 * w + 3]);
    }
    // wavefront-uniform: kept in scalar registers
    bx0 = uniform_f(bx0);
    bx1 = uniform_f(bx1);
    by0 = uniform_f(by0);
    by1 = uniform_f(by1);
    const float reach = uniform_f(T.rmax * 1.00001f);

    // Windows need a time that does not decrease with the squared leg length:
    // B >= 0 on every depth that can be inside the aperture (else, and for
    // table times, the whole record is staged).
    bool mono_lane = true;
#pragma unroll
    for (int k = 0; k < KS; ++k) mono_lane = mono_lane && (!(T.R[k] >= 0.0f) || T.B[k] >= 0.0f);
    const bool windows = TT == TT_DSR && __builtin_amdgcn_ballot_w64(!mono_lane) == 0;
    const int first_lo = TF ? -1 : 0;  // lowest staged sample (t_first = 0 gives u >= 0)

    int64_t jn = (T.rmax >= 0.0f) ? lo : hi;
    while (jn < hi) {
        // ---- Build a block: passes of NG candidates; candidate gi is trace jn + gi,
        // evaluated by the 16 lanes of group gi.  Its window [wl, wl + len) of
        // samples covers, with a 2-sample margin, every time of a pair inside the
        // aperture: over the chunk's depths that can hold such a pair, the time at
        // the box's nearest distances bounds it from below, the time at the
        // farthest distances (capped at the depth's aperture) from above.
        int nb = 0, used = 0;
        for (;;) {
            const int gi = wave * kGroupsPerWave + g;
            const int64_t j = jn + gi;
            int wl = 0, len = 0;
            float4 sr = make_float4(kFar, kFar, kFar, kFar);
            if (j < hi) {
                sr = make_float4(P.src[2 * j], P.src[2 * j + 1], P.rec[2 * j], P.rec[2 * j + 1]);
                const float ls = box_dist2(sr.x, sr.y, bx0, bx1, by0, by1);
                const float lr = box_dist2(sr.z, sr.w, bx0, bx1, by0, by1);
                const float m = fmaxf(ls, lr);
                if (m <= reach) {
                    wl = first_lo;
                    len = nt + 2 - first_lo;  // samples first_lo .. nt + 1
                    if (AA) {
                        // positions -(2 lmax + 4) .. nt + 2 lmax + 4: every clamped sample's reads
                        wl = -(2 * lmax + 4);
                        len = nt + 4 * lmax + 9;
                    }
                    if (windows) {
                        const float ms = box_far2(sr.x, sr.y, bx0, bx1, by0, by1);
                        const float mr = box_far2(sr.z, sr.w, bx0, bx1, by0, by1);
                        float umin = __builtin_inff(), umax = -__builtin_inff();
                        bool any = false, bad = false;
#pragma unroll
                        for (int k = 0; k < KS; ++k) {
                            const float R = RREG ? T.R[k] : sR[k * kGroup + d];
                            if (m <= R) {
                                const float a = __builtin_amdgcn_sqrtf(fmaf(T.B[k], ls, T.A[k])) +
                                                __builtin_amdgcn_sqrtf(fmaf(T.B[k], lr, T.A[k]));
                                const float c = __builtin_amdgcn_sqrtf(fmaf(T.B[k], fminf(ms, R), T.A[k])) +
                                                __builtin_amdgcn_sqrtf(fmaf(T.B[k], fminf(mr, R), T.A[k]));
                                any = true;
                                bad = bad || !(a == a && c == c);
                                umin = fminf(umin, a);
                                umax = fmaxf(umax, c);
                            }
                        }
#pragma unroll
                        for (int off = 1; off < kGroup; off <<= 1) {
                            umin = fminf(umin, __shfl_xor(umin, off, kLanes));
                            umax = fmaxf(umax, __shfl_xor(umax, off, kLanes));
                        }
                        if (PX) {  // physical tables: seconds -> samples (a monotone rounding)
                            const float sc = static_cast<float>(P.inv_dt);
                            umin = umin * sc;
                            umax = umax * sc;
                        }
                        const uint32_t gany = static_cast<uint32_t>(__builtin_amdgcn_ballot_w64(any) >> (kGroup * g)) & 0xFFFFu;
                        const uint32_t gbad = static_cast<uint32_t>(__builtin_amdgcn_ballot_w64(bad) >> (kGroup * g)) & 0xFFFFu;
                        if (!gany) {
                            len = 0;  // no depth of the chunk can hold a pair
                        } else if (!gbad) {
                            if (TF) {
                                umin = umin + tfo;
                                umax = umax + tfo;
                            }
                            // sample indices, clamped before conversion
                            const float clo = -static_cast<float>(2 * lmax + 16);
                            const float chi = static_cast<float>(nt + 2 * lmax + 16);
                            const int fmin = static_cast<int>(floorf(fminf(fmaxf(umin, clo), chi))) - koff;
                            const int fmax = static_cast<int>(floorf(fminf(fmaxf(umax, clo), chi))) - koff;
                            if (AA) {
                                // reads reach lmax + 2 around the sample; the clamp range
                                // [wl + lmax + 2, wh - lmax - 2] must hold the pairs' samples
                                const int a0 = max(fmin - lmax - 4, -(2 * lmax + 4));
                                const int a1 = min(fmax + lmax + 4, nt + 2 * lmax + 4);
                                if (a0 + lmax + 2 > a1 - lmax - 2) {
                                    len = 0;  // every triangle lies outside the record
                                } else {
                                    wl = a0;
                                    len = a1 - a0 + 1;
                                }
                            } else if (fmin - 2 > nt - 1 || fmax + 3 < 0) {
                                len = 0;  // every such time reads zeros: nothing to add
                            } else {
                                wl = max(fmin - 2, first_lo);
                                len = max(min(fmax + 3, nt + 1) - wl + 1, 2);
                            }
                        }
                    }
                }
            }
            __syncthreads();  // the previous pass (or block) is done with the candidates and rows
            if (d == 0) {
                sCand[gi] = make_int2(wl, len);
                sCandGeo[gi] = sr;
            }
            __syncthreads();
            // Every wavefront takes the same decision: candidates 0 .. k - 1 join the
            // block (the others do not fit and open the next one).
            int clen = 0, cwl = 0, cn = 0;  // LDS floats of the candidate's window, its first and number of samples
            if (lane < NG) {
                const int2 c = sCand[lane];
                cwl = c.x;
                cn = c.y;
                clen = c.y > 0 ? (AA ? 2 * c.y : T16 ? (c.y + 1) / 2 : P16 ? c.y - 1 : PAIRS ? 2 * (c.y - 1) : c.y)
                               : 0;
            }
            int plen = clen, pcnt = clen > 0 ? 1 : 0;  // inclusive prefix sums
#pragma unroll
            for (int off = 1; off < NG; off <<= 1) {
                const int tl = __shfl_up(plen, off, kLanes), tc = __shfl_up(pcnt, off, kLanes);
                if (lane >= off) {
                    plen += tl;
                    pcnt += tc;
                }
            }
            const bool fits = used + plen <= P.cap && nb + pcnt <= P.tb;
            const uint64_t nofit = __builtin_amdgcn_ballot_w64(lane < NG && !fits);
            const int k = nofit ? static_cast<int>(__builtin_ctzll(nofit)) : NG;
            if (wave == 0 && lane < k && clen > 0) {
                const int slot = nb + pcnt - 1;
                sGeo[slot] = sCandGeo[lane];
                sMeta[slot] = make_int4(used + plen - clen, cwl, cwl + cn - 1, static_cast<int>(jn + lane - lo));
            }
            if (k > 0) {
                nb += __builtin_amdgcn_readlane(pcnt, k - 1);
                used += __builtin_amdgcn_readlane(plen, k - 1);
            }
            jn += k;
            if (k < NG || jn >= hi) break;
        }
        if (nb == 0) continue;  // only when the bin is exhausted
        __syncthreads();        // the block's slots
        for (int t = wave; t < nb; t += NW) {
            const int4 mt = sMeta[t];
            if (AA) stage_window_i2(P, lo + mt.w, mt.y, mt.z - mt.y + 1, reinterpret_cast<double*>(sTr + mt.x), lane);
            else if (T16) stage_window_16(P, lo + mt.w, mt.y, mt.z - mt.y + 1, reinterpret_cast<uint16_t*>(sTr + mt.x), lane);
            else if (P16) stage_window_16p(P, lo + mt.w, mt.y, mt.z - mt.y + 1, reinterpret_cast<uint32_t*>(sTr + mt.x), lane);
            else if (PAIRS) stage_window(P, lo + mt.w, mt.y, mt.z - mt.y + 1, reinterpret_cast<float2*>(sTr + mt.x), lane);
            else stage_window_f(P, lo + mt.w, mt.y, mt.z - mt.y + 1, sTr + mt.x, lane);
        }
        __syncthreads();

        for (int t0 = 0; t0 < nb; t0 += kGroup) {
            const int nbt = min(kGroup, nb - t0);
            // lane (g, d): legs of column group member g and trace t0 + d; the
            // trace's row offset and clamp bounds (window samples wl .. wh)
            const int ts = min(t0 + d, nb - 1);
            const float4 sr = sGeo[ts];
            const int4 mt = sMeta[ts];
            // in pairs / doubles / 16-bit samples / floats or packed 16-bit pairs
            const int lrow = (PAIRS || AA ? mt.x / 2 : T16 ? 2 * mt.x : mt.x) - mt.y - koff;
            // 16-bit staging: the trace's scale, applied per pair with the weight
            const float lscl = (S16 && P.scale) ? P.scale[lo + mt.w] : 1.0f;
            const float lwlo = static_cast<float>(mt.y + koff + (AA ? lmax + 2 : 0));
            const float lwhi = static_cast<float>(mt.z - 1 + koff - (AA ? lmax + 1 : 0));
#pragma unroll
            for (int q = 0; q < CWQ; ++q) {
                const Legs Lp = legs(px[q], py[q], sr);
                LegsX Lx{0.0, 0.0};
                if (PX) Lx = legs_ext(px[q], py[q], sr);
                // extremes of hmax over the four columns, per trace (lanes d, 16 + d, 32 + d, 48 + d)
                float hmin4 = fminf(Lp.hmax, __shfl_xor(Lp.hmax, 16, kLanes));
                hmin4 = fminf(hmin4, __shfl_xor(hmin4, 32, kLanes));
                float hmax4 = fmaxf(Lp.hmax, __shfl_xor(Lp.hmax, 16, kLanes));
                hmax4 = fmaxf(hmax4, __shfl_xor(hmax4, 32, kLanes));
                uint64_t live = __builtin_amdgcn_ballot_w64(hmin4 <= T.rmax) & ((1ull << nbt) - 1ull);
                if (!live) continue;
                // The legs of trace t reach the depth lanes through the LDS crossbar; the
                // next live trace's are requested before trace t is evaluated.
                int t = __builtin_ctzll(live);
                live &= live - 1;
                // (The upper clamp bound also comes through the crossbar, as a vector
                // register: a clamp with two scalar bounds costs a move per pair.)
                float hs2n = lane_read(Lp.hs2, (lane & ~(kGroup - 1)) | t);
                float hr2n = lane_read(Lp.hr2, (lane & ~(kGroup - 1)) | t);
                float whin = lane_read(lwhi, t);
                double Hsn = 0.0, Hrn = 0.0;
                if (PX) {
                    Hsn = lane_read_d(Lx.hs2, (lane & ~(kGroup - 1)) | t);
                    Hrn = lane_read_d(Lx.hr2, (lane & ~(kGroup - 1)) | t);
                }
                for (;;) {
                    const int tc = t;
                    const float hs2 = hs2n, hr2 = hr2n, whi = whin;
                    const double Hs = Hsn, Hr = Hrn;
                    const bool more = live != 0;
                    if (more) {
                        t = __builtin_ctzll(live);
                        live &= live - 1;
                        hs2n = lane_read(Lp.hs2, (lane & ~(kGroup - 1)) | t);
                        hr2n = lane_read(Lp.hr2, (lane & ~(kGroup - 1)) | t);
                        whin = lane_read(lwhi, t);
                        if (PX) {
                            Hsn = lane_read_d(Lx.hs2, (lane & ~(kGroup - 1)) | t);
                            Hrn = lane_read_d(Lx.hr2, (lane & ~(kGroup - 1)) | t);
                        }
                    }
                    const float hmin = uniform_read(hmin4, tc);
                    const float hmaxw = uniform_read(hmax4, tc);
                    uint64_t any, full;
                    slot_masks<KS>(T, hmin, hmaxw, any, full);
                    (void)full;
                    if (!any) {
                        if (!more) break;
                        continue;
                    }
                    const int rb = __builtin_amdgcn_readlane(lrow, tc);
                    const float wlo = uniform_read(lwlo, tc);
                    const float scl = S16 ? uniform_read(lscl, tc) : 1.0f;
                    // max(hs2, hr2): one v_max (fmaxf would first quiet both inputs)
                    float hm;
                    asm("v_max_f32 %0, %1, %2" : "=v"(hm) : "v"(hs2), "v"(hr2));
                    if (is_table(TT) && PX) {
                        const TLegX Ls = table_leg_ext(P, Hs), Lr = table_leg_ext(P, Hr);
#pragma unroll
                        for (int k = 0; k < KS; k += 2) {
                            if ((any >> k) & 3ull) {
                                const int iz0 = min(max(z0 + k * kGroup + d, 0), P.nz - 1);
                                const int iz1 = min(max(z0 + (k + 1) * kGroup + d, 0), P.nz - 1);
                                const float R0 = RREG ? T.R[k] : sR[k * kGroup + d];
                                const float R1 = RREG ? T.R[k + 1] : sR[(k + 1) * kGroup + d];
                                mig_pair_table_ext<TF, LAT>(P, Ls, Lr, lc[q], iz0, iz1, hm, sTr + rb, wlo, whi, R0, R1,
                                                            acc[q][k], acc[q][k + 1]);
                            }
                        }
                    } else if (is_table(TT)) {
                        const TLeg Ls = table_leg(P, hs2), Lr = table_leg(P, hr2);
#pragma unroll
                        for (int k = 0; k < KS; k += 2) {
                            if ((any >> k) & 3ull) {
                                const int iz0 = min(max(z0 + k * kGroup + d, 0), P.nz - 1);
                                const int iz1 = min(max(z0 + (k + 1) * kGroup + d, 0), P.nz - 1);
                                const float R0 = RREG ? T.R[k] : sR[k * kGroup + d];
                                const float R1 = RREG ? T.R[k + 1] : sR[(k + 1) * kGroup + d];
                                if (S16)
                                    mig_pair_table16<TF, LAT, S16>(P, Ls, Lr, lc[q], iz0, iz1, hm,
                                                                   reinterpret_cast<const uint32_t*>(sTr), rb, scl,
                                                                   tfo, wlo, whi, R0, R1, acc[q][k], acc[q][k + 1]);
                                else
                                    mig_pair_table<TF, true, LAT>(P, Ls, Lr, lc[q], iz0, iz1, hm, sTr + rb, tfo, wlo,
                                                                  whi, R0, R1, acc[q][k], acc[q][k + 1]);
                            }
                        }
                    } else if (AA) {
                        // column minus source / receiver of trace tc, for the operator dip
                        const float dxs = px[q] - uniform_read(sr.x, tc), dys = py[q] - uniform_read(sr.y, tc);
                        const float dxr = px[q] - uniform_read(sr.z, tc), dyr = py[q] - uniform_read(sr.w, tc);
                        const double* rowd = reinterpret_cast<const double*>(sTr) + rb;
#pragma unroll
                        for (int k = 0; k < KS; ++k) {
                            if ((any >> k) & 1ull) {
                                const float R = RREG ? T.R[k] : sR[k * kGroup + d];
                                mig_slot_aa<TF, WK>(T.A[k], T.B[k], hs2, hr2, hm, rowd, tfo, wlo, whi, R, dxs, dys, dxr,
                                                    dyr, P.aa_dx, P.aa_dy, static_cast<float>(lmax), sInvSq,
                                                    acc[q][k]);
                            }
                        }
                    } else if (PX) {
                        const int ilo = static_cast<int>(wlo), ihi = static_cast<int>(whi);
                        const double wlod = wlo, whid = whi;
#pragma unroll
                        for (int k = 0; k < KS; ++k) {
                            if ((any >> k) & 1ull) {
                                const float R = RREG ? T.R[k] : sR[k * kGroup + d];
                                mig_slot_ext<TF, WK>(T.A[k], T.B[k], Hs, Hr, hm,
                                                     reinterpret_cast<const float2*>(sTr) + rb, P.inv_dt, tfod, ilo,
                                                     ihi, wlod, whid, R, acc[q][k]);
                            }
                        }
                    } else {
                        // Every slot pair goes through the masked, clamped form: one code path
                        // per pair measured faster than separate unmasked / unclamped variants
                        // (their extra branches and code cost more than the masks they save).
#pragma unroll
                        for (int k = 0; k < KS; k += 2) {
                            if ((any >> k) & 3ull) {
                                const float R0 = RREG ? T.R[k] : sR[k * kGroup + d];
                                const float R1 = RREG ? T.R[k + 1] : sR[(k + 1) * kGroup + d];
                                if (S16)
                                    mig_pair16<TF, WK, S16>(T.A[k], T.B[k], T.A[k + 1], T.B[k + 1], hs2, hr2, hm,
                                                            reinterpret_cast<const uint32_t*>(sTr) + rb, scl, tfo,
                                                       wlo, whi, R0, R1, acc[q][k], acc[q][k + 1]);
                                else
                                    mig_pair<TF, WK, true, true>(T.A[k], T.B[k], T.A[k + 1], T.B[k + 1], hs2, hr2, hm,
                                                                 reinterpret_cast<const float2*>(sTr) + rb,
                                                                 tfo, wlo, whi, R0, R1, acc[q][k], acc[q][k + 1]);
                            }
                        }
                    }
                    if (!more) break;
                }
            }
        }
    }

    float* img = P.image + static_cast<int64_t>(b) * ncol * P.nz;
#pragma unroll
    for (int q = 0; q < CWQ; ++q) {
        if (colv[q] >= ncol) continue;
        float* colp = img + static_cast<int64_t>(colv[q]) * P.nz;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int iz = z0 + k * kGroup + d;
            if (iz >= 0 && iz < P.nz) {
                const float fac = depth_factor<PX>(P, iz);
                const float val = fac != 0.0f ? acc[q][k] * fac : 0.0f;
                colp[iz] = P.accumulate ? colp[iz] + val : val;
            }
        }
    }
}

// Store zeros into a tile whose (column, trace) pairs are all outside the
// aperture (known from the counting kernel): its image values are exactly 0.
template <int NW, int CWQ, int KS>
__device__ __forceinline__ void zero_tile(const Params& P, int b, int tile, int zc) {
    if (P.accumulate) return;
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = threadIdx.x / kLanes;
    const int g = lane / kGroup, d = lane % kGroup;
    const int ncol = P.nx * P.ny;
    const int z0 = chunk_z0<false>(P.nz, zc, P.n_zchunks, KS * kGroup);
    float* img = P.image + static_cast<int64_t>(b) * ncol * P.nz;
#pragma unroll
    for (int q = 0; q < CWQ; ++q) {
        const int col = (tile * NW * CWQ + wave * CWQ + q) * kGroupsPerWave + g;
        if (col >= ncol) continue;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int iz = z0 + k * kGroup + d;
            if (iz >= 0 && iz < P.nz) img[static_cast<int64_t>(col) * P.nz + iz] = 0.0f;
        }
    }
}

// The extended-precision square-root kernels are held to 4 wavefronts per SIMD
// (128 VGPRs, some spilled) so that two 8-wavefront workgroups share a CU:
// 2.28 s against 3.29 s at their natural 165 VGPRs on the 3D survey.
template <int NW, int CWQ, int KS, bool TF, int WK, int TT = TT_DSR, bool PX = false, int S16 = 0>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(PX && TT == TT_DSR && KS <= 8 ? 4 : 1)))
void migrate_kernel(Params P) {
    extern __shared__ float lds[];
    migrate_tile<NW, CWQ, KS, TF, WK, true, TT, PX, S16>(P, blockIdx.z, blockIdx.x, blockIdx.y, lds);
}

// Batched persistent form: work items (problem, bin, column tile, depth
// chunk) are taken from a queue in list order (longest first).  A negative
// tile field -1 - tile marks an item with no pair in aperture: zero store.
// At least 4 wavefronts per SIMD (<= 128 VGPRs) for the 8-slot shapes, so
// that two 8-wavefront workgroups share a CU as they do in single launches.
template <int NW, int CWQ, int KS, bool TF, int WK, bool PX = false>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(KS <= 8 ? 4 : 2)))
void migrate_batch_kernel(const Params* __restrict__ probs,
                                                                const int4* __restrict__ items,
                                                                int64_t n_items, unsigned int* counter) {
    extern __shared__ float lds[];
    __shared__ int64_t s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = static_cast<int64_t>(atomicAdd(counter, 1u));
        __syncthreads();
        const int64_t it = s_item;
        if (it >= n_items) break;
        const int4 w = items[it];  // (problem, bin, tile, zchunk)
        const Params P = probs[w.x];
        if (w.z < 0) zero_tile<NW, CWQ, KS>(P, w.y, -1 - w.z, w.w);
        else migrate_tile<NW, CWQ, KS, TF, WK, false, TT_DSR, PX>(P, w.y, w.z, w.w, lds);
    }
}

// ---------------------------------------------------------------------------
// Launch tables
// ---------------------------------------------------------------------------

// The plain kernels of one time precision (PX) for the weight and t_first cases.
template <int NW, int CWQ, int KS, bool PX>
static hipError_t launch_migrate_dsr(const Params& P, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
    if (P.has_tf) {
        if (P.weight == W_COSCOS)
            return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_COSCOS, TT_DSR, PX>, grid, block, lds, s, P);
        return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_UNIT, TT_DSR, PX>, grid, block, lds, s, P);
    }
    if (P.weight == W_COSCOS)
        return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_COSCOS, TT_DSR, PX>, grid, block, lds, s, P);
    return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_UNIT, TT_DSR, PX>, grid, block, lds, s, P);
}

// The 16-bit staging kernels (float32 time), per storage type: square-root
// times per weight and t_first case, the two table kinds per t_first case.
template <int NW, int CWQ, int KS, int DT>
static hipError_t launch_migrate_s16_dt(const Params& P, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
    if (P.ttab) {
        if (P.n_gx > 0) {
            if (P.has_tf)
                return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_UNIT, TT_LTABLE, false, DT>, grid, block, lds, s, P);
            return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_UNIT, TT_LTABLE, false, DT>, grid, block, lds, s, P);
        }
        if (P.has_tf)
            return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_UNIT, TT_TABLE, false, DT>, grid, block, lds, s, P);
        return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_UNIT, TT_TABLE, false, DT>, grid, block, lds, s, P);
    }
    if (P.has_tf) {
        if (P.weight == W_COSCOS)
            return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_COSCOS, TT_DSR, false, DT>, grid, block, lds, s, P);
        return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_UNIT, TT_DSR, false, DT>, grid, block, lds, s, P);
    }
    if (P.weight == W_COSCOS)
        return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_COSCOS, TT_DSR, false, DT>, grid, block, lds, s, P);
    return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_UNIT, TT_DSR, false, DT>, grid, block, lds, s, P);
}

template <int NW, int CWQ, int KS>
static hipError_t launch_migrate_s16(const Params& P, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
    if (P.dtype == BF16) return launch_migrate_s16_dt<NW, CWQ, KS, BF16>(P, grid, block, lds, s);
    return launch_migrate_s16_dt<NW, CWQ, KS, F16>(P, grid, block, lds, s);
}

template <int NW, int CWQ, int KS>
static hipError_t launch_migrate_shape(const Params& P, hipStream_t s) {
    dim3 grid(P.n_coltiles, P.n_zchunks, P.n_bins), block(NW * 64);
    const size_t lds = lds_bytes(P, KS);
    if (P.s16) return launch_migrate_s16<NW, CWQ, KS>(P, grid, block, lds, s);  // the host checked the kind
    if (P.ttab && P.n_gx > 0) {  // laterally varying tables: W = 1
        if (P.prec) {
            if (P.has_tf)
                return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_UNIT, TT_LTABLE, true>, grid, block, lds, s, P);
            return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_UNIT, TT_LTABLE, true>, grid, block, lds, s, P);
        }
        if (P.has_tf) return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_UNIT, TT_LTABLE>, grid, block, lds, s, P);
        return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_UNIT, TT_LTABLE>, grid, block, lds, s, P);
    }
    if (P.ttab) {  // table traveltimes: W = 1 (the host rejects other weights)
        if (P.prec) {
            if (P.has_tf)
                return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_UNIT, TT_TABLE, true>, grid, block, lds, s, P);
            return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_UNIT, TT_TABLE, true>, grid, block, lds, s, P);
        }
        if (P.has_tf) return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_UNIT, TT_TABLE>, grid, block, lds, s, P);
        return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_UNIT, TT_TABLE>, grid, block, lds, s, P);
    }
    if (P.aa_max > 0) {  // anti-alias triangle filter
        if (P.has_tf) {
            if (P.weight == W_COSCOS)
                return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_COSCOS, TT_AA>, grid, block, lds, s, P);
            return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_UNIT, TT_AA>, grid, block, lds, s, P);
        }
        if (P.weight == W_COSCOS)
            return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_COSCOS, TT_AA>, grid, block, lds, s, P);
        return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_UNIT, TT_AA>, grid, block, lds, s, P);
    }
    if (P.prec) return launch_migrate_dsr<NW, CWQ, KS, true>(P, grid, block, lds, s);
    return launch_migrate_dsr<NW, CWQ, KS, false>(P, grid, block, lds, s);
}

// The batch kernel of (shape, t_first, weight, precision).
template <int NW, int CWQ, int KS>
static const void* batch_kernel_of(int has_tf, int weight, int prec) {
    if (prec) {
        if (has_tf) return weight == W_COSCOS ? (const void*)migrate_batch_kernel<NW, CWQ, KS, true, W_COSCOS, true>
                                              : (const void*)migrate_batch_kernel<NW, CWQ, KS, true, W_UNIT, true>;
        return weight == W_COSCOS ? (const void*)migrate_batch_kernel<NW, CWQ, KS, false, W_COSCOS, true>
                                  : (const void*)migrate_batch_kernel<NW, CWQ, KS, false, W_UNIT, true>;
    }
    if (has_tf) return weight == W_COSCOS ? (const void*)migrate_batch_kernel<NW, CWQ, KS, true, W_COSCOS>
                                          : (const void*)migrate_batch_kernel<NW, CWQ, KS, true, W_UNIT>;
    return weight == W_COSCOS ? (const void*)migrate_batch_kernel<NW, CWQ, KS, false, W_COSCOS>
                              : (const void*)migrate_batch_kernel<NW, CWQ, KS, false, W_UNIT>;
}

template <int NW, int CWQ, int KS>
static hipError_t launch_migrate_batch_shape(const Params* probs, const int4* items, int64_t n_items,
                                             unsigned int* counter, int has_tf, int weight, int prec, int n_wg,
                                             size_t lds, hipStream_t s) {
    dim3 grid(n_wg), block(NW * 64);
    using K = void (*)(const Params*, const int4*, int64_t, unsigned int*);
    const K kern = reinterpret_cast<K>(const_cast<void*>(batch_kernel_of<NW, CWQ, KS>(has_tf, weight, prec)));
    return launch_with_lds(kern, grid, block, lds, s, probs, items, n_items, counter);
}

// (waves, column groups per wave, depth slots, LDS budget for the trace block)
#define KM_MIGRATE_SHAPES(X) \
    X(4, 4, 8, 32768)        \
    X(16, 4, 8, 155648)      \
    X(8, 4, 8, 77824)        \
    X(4, 3, 16, 49152)       \
    X(4, 2, 16, 49152)

static const TileShape kMigrateShapes[] = {
#define X(nw, cwq, ks, lb) {nw, cwq, ks, lb},
    KM_MIGRATE_SHAPES(X)
#undef X
};

int migrate_shape_count() { return static_cast<int>(sizeof(kMigrateShapes) / sizeof(kMigrateShapes[0])); }
const TileShape& migrate_shape(int i) { return kMigrateShapes[i]; }

hipError_t launch_migrate(int shape, const Params& P, hipStream_t s) {
    int i = 0;
#define X(nw, cwq, ks, lb) \
    if (shape == i) return launch_migrate_shape<nw, cwq, ks>(P, s); \
    ++i;
    KM_MIGRATE_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_migrate_batch(int shape, const Params* probs, const int4* items, int64_t n_items,
                                unsigned int* counter, int has_tf, int weight, int prec, int n_wg, size_t lds,
                                hipStream_t s) {
    int i = 0;
#define X(nw, cwq, ks, lb) \
    if (shape == i) return launch_migrate_batch_shape<nw, cwq, ks>(probs, items, n_items, counter, has_tf, weight, prec, n_wg, lds, s); \
    ++i;
    KM_MIGRATE_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

const void* migrate_batch_kernel_ptr(int shape, int has_tf, int weight, int prec) {
    int i = 0;
#define X(nw, cwq, ks, lb) \
    if (shape == i) return batch_kernel_of<nw, cwq, ks>(has_tf, weight, prec); \
    ++i;
    KM_MIGRATE_SHAPES(X)
#undef X
    return nullptr;
}

}  // namespace km
