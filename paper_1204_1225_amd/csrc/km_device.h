// Device-side building blocks shared by the migrate, demigrate, count and
// batched kernels: launch parameters, the per-depth tables of a depth chunk,
// the staged-trace row layout and the per-pair evaluation of Eq. (1)
// (aperture, total time, interpolation index, weight).
//
// Lane layout of the image-domain kernels: a wavefront (64 lanes) is four
// groups of 16 lanes; lane d of a group works on depth z0 + 16 k + d in slot
// k = 0..KS-1 of the depth chunk starting at z0.  A 16-depth slot is the unit
// of work skipping: a slot is evaluated for a (column, trace) pairing only if
// some lane of it can be inside the aperture, and without any per-lane mask
// when every valid lane is inside.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace km {

constexpr int kLanes = 64;
constexpr int kGroup = 16;         // lanes per group (depths per slot)
constexpr int kGroupsPerWave = 4;  // groups per wavefront
constexpr int kLead = 4;           // zero floats before sample 0 in a staged row: row[kLead + k] = D[k]
constexpr float kFar = 3.0e30f;    // coordinate of padding columns / traces: never inside the aperture

enum Dtype : int32_t { F32 = 0, BF16 = 1, F16 = 2 };
enum Weight : int32_t { W_UNIT = 0, W_COSCOS = 1 };

// Everything a kernel needs about one problem.  Plain data, passed by value
// (and, for batches, stored in a device table).
struct Params {
    // traces
    void* data;  // read by migrate, written by demigrate
    const float* scale;
    const float* src;
    const float* rec;
    const int32_t* bin;
    int64_t n_traces;
    int64_t stride;
    int32_t nt;
    int32_t dtype;
    // grid
    const float* x;
    const float* y;
    int32_t nx, ny, nz, n_bins;
    // model (float32 tables in physical units)
    const float* t0sq;
    const float* s2;
    const float* r2;
    double inv_dt2;   // 1 / dt^2: tables -> sample units
    double wscale;    // 1 / dt^4: W = t0sq * wscale / (a_s * a_r) with a in samples^2
    float tf_off;     // kLead - t_first / dt (used when t_first != 0)
    int32_t has_tf;
    int32_t weight;
    // output / input image
    float* image;
    int32_t accumulate;
    // staging geometry
    int32_t lt;       // demigrate: LDS row length (multiple of 4, >= nt + kLead + 2)
    int32_t tb;       // traces per LDS block (migrate: at most)
    int32_t cap;      // migrate: LDS floats for the staged time windows of a block
    int32_t n_zchunks;
    int32_t n_coltiles;
    // table traveltimes (used by the TABLE kernels instead of t0sq / s2)
    const float* ttab;  // [n_h][nz] one-way seconds at h = ih * dh
    int32_t n_h;
    float inv_dh;       // 1 / dh
    double inv_dt;      // 1 / dt
    double tf_off_d;    // kLead - t_first / dt in float64
    // anti-alias triangle filter (the TT_AA kernels)
    float aa_dx, aa_dy;  // image spacings the operator dip is measured over
    int32_t aa_max;      // largest triangle half-width in samples (1 .. kAAMaxHalf)
    int32_t aa_lead;     // demigrate: row index of sample 0 (rows hold samples -aa_lead .. lt - aa_lead - 1)
    // time precision: 0 = float32 evaluation, 1 = extended (the PX kernels)
    int32_t prec;
    double inv_dh_d;     // 1 / dh in float64 (extended table legs)
    // laterally varying tables (the TT_LTABLE kernels): ttab then holds one
    // [n_h][nz] table per node of the grid X_i = gx0 + i gdx, Y_j = gy0 + j gdy,
    // node (i, j) at float offset (j n_gx + i) n_h nz
    int32_t n_gx, n_gy;
    int32_t ldx, ldy;    // floats from a node's table to its +x / +y neighbour's (0 on an axis of one node)
    double gx0, gy0, gdx, gdy;
    uint32_t ttab_bytes; // size of ttab (every node), < 2^31: byte offsets into it fit an int
    // one-way amplitudes of the table kinds (same layout and size as ttab), or
    // NULL: W = A_s A_r instead of 1
    const float* tamp;
    // migrate: 16-bit traces staged in LDS as their 16-bit storage (the S16
    // kernels), widened and scaled per pair
    int32_t s16;
};

// Raw buffer resources (gfx9 family: no format conversion, no swizzle).
// Out-of-range offsets read 0.
constexpr int kRawBufferWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes), kRawBufferWord3);
}

// Traveltime kinds of the kernels: the per-depth double-square-root form
// (t0sq, s2) or a one-way time table T(h, z) interpolated linearly in h.
// TT_AA: the double-square-root form with the anti-alias triangle filter.
// TT_LTABLE: one table per node of a coarse lateral grid, interpolated over
// (image x, image y, h).
enum TravelKind : int32_t { TT_DSR = 0, TT_TABLE = 1, TT_AA = 2, TT_LTABLE = 3 };
constexpr bool is_table(int tt) { return tt == TT_TABLE || tt == TT_LTABLE; }
constexpr int kAAMaxHalf = 32;  // largest anti-alias half-width the kernels accept

// First index in sorted bin[0..n) whose value is >= key.
__device__ __forceinline__ int64_t lower_bound_bin(const int32_t* __restrict__ bin, int64_t n, int32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (bin[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ float widen16(uint32_t bits, int dtype) {
    return dtype == BF16 ? __uint_as_float(bits << 16) : __half2float(__ushort_as_half(static_cast<uint16_t>(bits)));
}

// Horizontal squared leg lengths of a (column, trace) pair, float32 with the
// fixed operation order of the aperture decision (fp-contract is off for all
// device code, so nothing here is fused).
struct Legs {
    float hs2, hr2, hmax;
};

__device__ __forceinline__ Legs legs(float px, float py, float4 sr) {
    const float dxs = px - sr.x, dys = py - sr.y;
    const float dxr = px - sr.z, dyr = py - sr.w;
    Legs L;
    L.hs2 = dxs * dxs + dys * dys;
    L.hr2 = dxr * dxr + dyr * dyr;
    L.hmax = fmaxf(L.hs2, L.hr2);
    return L;
}

// One (trace, image point) pair in sample units:
//   a_s = A + B hs2, a_r = A + B hr2 (A = t0sq / dt^2, B = s2 / dt^2),
//   w   = sqrt(a_s) + sqrt(a_r) [+ tf_off when t_first != 0], clamped to
//         [wlo, whi]; the staged-row index of sample floor(u) is floor(w)
//         (plus kLead through the row pointer when t_first == 0),
//   i   = floor(w), f = w - i, and r = 1 / (a_s a_r) for the weight.
// Migrate and demigrate both call this, so the transpose pair sees
// bit-identical (i, f, r) for every pair.  CLAMP = false skips the clamp (for
// callers that know every w lies in [wlo, whi]; the kernels all clamp).
struct Pair {
    int32_t i;
    float f;
    float r;
};

template <bool TF, int WK, bool CLAMP = true>
__device__ __forceinline__ Pair eval_pair(float A, float B, float hs2, float hr2, float tf_off, float wlo, float whi) {
    const float as = fmaf(B, hs2, A);
    const float ar = fmaf(B, hr2, A);
    float w = __builtin_amdgcn_sqrtf(as) + __builtin_amdgcn_sqrtf(ar);
    if (TF) w = w + tf_off;
    if (CLAMP) w = __builtin_amdgcn_fmed3f(w, wlo, whi);
    Pair p;
    p.i = static_cast<int32_t>(w);
    p.f = __builtin_amdgcn_fractf(w);
    p.r = (WK == W_COSCOS) ? __builtin_amdgcn_rcpf(as * ar) : 1.0f;
    return p;
}

// Extended-precision form of eval_pair (the PX kernels).  A float32 total
// time is rounded to 0.5 ulp of u (6e-5 samples at u = 1000, 1e-3 at 16000)
// after the roundings of A, B, the two products and the two square roots, which
// is a relative image error of about 1e-5 on data that change by O(1) between
// samples.  Here the tables are the physical float32 inputs (A = t0sq in s^2,
// B = s2 in s^2 / m^2, exact in float64), the squared leg lengths Hs, Hr are
// float64 (exact for float32 coordinates), a = A + B H is one float64 FMA, and
// each leg's square root is a float32 reciprocal square root q refined by one
// residual step in float64: y = a q, sqrt(a) = y + (a - y^2) q / 2 to about
// 2^-45 relative (Newton's step from a 2^-23 seed).  Both legs' steps are
// summed in float64 and scaled by 1 / dt, so i = floor(u) and f = u - i come
// from a total time good to about 1e-9 samples.  The weight 1 / (a_s a_r) is
// (q_s q_r)^2 (in s^-4; depth_factor<true> supplies t0sq), from the same seeds,
// with float32 precision.
//   !TF: i = floor(w) clamped to [ilo, ihi] (the two row entries at a clamped
//        index are zeros, or the pair is outside the aperture and masked);
//   TF:  w clamped to [wlo, whi] first (as eval_pair; f = 0 at a bound).
// a = 0 exactly (W = 1 and t0 = 0 at zero offset) would give rsq = inf: the
// tables replace A = 0 by kTinyA (a time of 3e-19 s).
struct PairX {
    int32_t i;
    float f;
    double fd;  // f in float64 (the adjoint's tap weights)
    float r;
};

constexpr float kTinyA = 1.0e-37f;

template <bool TF, int WK>
__device__ __forceinline__ PairX eval_pair_ext(float A, float B, double Hs, double Hr, double inv_dt, double tfo,
                                               int ilo, int ihi, double wlo, double whi) {
    const double Ad = static_cast<double>(A), Bd = static_cast<double>(B);
    const double as = fma(Bd, Hs, Ad);
    const double ar = fma(Bd, Hr, Ad);
    const float qs = __builtin_amdgcn_rsqf(static_cast<float>(as));
    const float qr = __builtin_amdgcn_rsqf(static_cast<float>(ar));
    const double qsd = static_cast<double>(qs), qrd = static_cast<double>(qr);
    const double ys = as * qsd, yr = ar * qrd;
    const double es = fma(-ys, ys, as), er = fma(-yr, yr, ar);
    double w = fma(fma(er, qrd, es * qsd), 0.5, ys + yr) * inv_dt;
    PairX p;
    if (TF) {
        w = fmin(fmax(w + tfo, wlo), whi);
        p.i = static_cast<int32_t>(w);
    } else {
        p.i = min(max(static_cast<int32_t>(w), ilo), ihi);
    }
    p.fd = __builtin_amdgcn_fract(w);
    p.f = static_cast<float>(p.fd);
    const float g = qs * qr;
    p.r = (WK == W_COSCOS) ? g * g : 1.0f;
    return p;
}

// Squared leg lengths in float64 from the float32 coordinates (the
// differences and squares are exact; one rounding in the sum).
struct LegsX {
    double hs2, hr2;
};

__device__ __forceinline__ LegsX legs_ext(float px, float py, float4 sr) {
    const double x = px, y = py;
    const double dxs = x - static_cast<double>(sr.x), dys = y - static_cast<double>(sr.y);
    const double dxr = x - static_cast<double>(sr.z), dyr = y - static_cast<double>(sr.w);
    LegsX L;
    L.hs2 = fma(dxs, dxs, dys * dys);
    L.hr2 = fma(dxr, dxr, dyr * dyr);
    return L;
}

// One pair with the anti-alias triangle filter (Params::aa_*).  As eval_pair
// (clamped), plus the half-width p = |du/dx| dx + |du/dy| dy in samples,
// du/dx = B ((x - x_s) / sqrt(a_s) + (x - x_r) / sqrt(a_r)) (likewise y),
// clamped to [1, aa_max]; L = floor(p) and the blend weights
// alpha = (1 - phi) / L^2, beta = phi / (L + 1)^2 (phi = p - L) of the two
// integer-width unit-area triangles (invsq[n] = 1 / n^2).  (dxs, dys), (dxr,
// dyr): image column minus source / receiver.  Migrate and demigrate call
// this, so both see the same (i, f, r, L, alpha, beta).
struct PairAA {
    int32_t i, L;
    float f, r, alpha, beta;
};

template <bool TF, int WK>
__device__ __forceinline__ PairAA eval_pair_aa(float A, float B, float hs2, float hr2, float tf_off, float wlo,
                                               float whi, float dxs, float dys, float dxr, float dyr, float adx,
                                               float ady, float lmax, const float* invsq) {
    const float as = fmaf(B, hs2, A);
    const float ar = fmaf(B, hr2, A);
    const float ss = __builtin_amdgcn_sqrtf(as), sr = __builtin_amdgcn_sqrtf(ar);
    float w = ss + sr;
    if (TF) w = w + tf_off;
    w = __builtin_amdgcn_fmed3f(w, wlo, whi);
    const float is = __builtin_amdgcn_rcpf(ss), ir = __builtin_amdgcn_rcpf(sr);
    PairAA p;
    p.i = static_cast<int32_t>(w);
    p.f = __builtin_amdgcn_fractf(w);
    // 1 / (a_s a_r) from the legs' reciprocals the dip needs anyway
    const float g = is * ir;
    p.r = (WK == W_COSCOS) ? g * g : 1.0f;
    const float ux = B * fmaf(dxs, is, dxr * ir);
    const float uy = B * fmaf(dys, is, dyr * ir);
    // a NaN (zero leg time) takes the lower bound: no smoothing
    const float q = __builtin_amdgcn_fmed3f(fmaf(fabsf(ux), adx, fabsf(uy) * ady), 1.0f, lmax);
    p.L = static_cast<int32_t>(q);
    const float phi = q - static_cast<float>(p.L);
    p.alpha = (1.0f - phi) * invsq[p.L];
    p.beta = phi * invsq[p.L + 1];
    return p;
}

// Table traveltimes.  A leg's place in the table: the time at horizontal
// distance h = sqrt(h^2) is t[ih][iz] + f (t[ih + 1][iz] - t[ih][iz]) with
// h / dh clamped to [0, n_h - 1] (beyond the table the last row holds); off
// = ih * nz.  Infinite or NaN h^2 (padding) lands on the last row.
struct TLeg {
    int32_t off;
    float f;
};

__device__ __forceinline__ TLeg table_leg(const Params& P, float h2) {
    const float top = static_cast<float>(P.n_h - 1);
    const float hf = fminf(__builtin_amdgcn_sqrtf(h2) * P.inv_dh, top);
    const int ih = min(static_cast<int>(hf), P.n_h - 2);
    TLeg L;
    L.off = ih * P.nz;
    L.f = hf - static_cast<float>(ih);
    return L;
}

// Extended table leg: h = sqrt(H) from the float64 squared length (float32
// reciprocal square root seed and one float64 residual step), h / dh and the
// fraction in float64.  H = 0 (a column above the source) is raised to 1e-30
// so that the seed stays finite (h = 1e-15).
struct TLegX {
    int32_t off;
    double f;
};

__device__ __forceinline__ TLegX table_leg_ext(const Params& P, double H) {
    H = fmax(H, 1.0e-30);
    const double q = static_cast<double>(__builtin_amdgcn_rsqf(static_cast<float>(H)));
    const double y = H * q;
    const double h = fma(fma(-y, y, H), 0.5 * q, y);
    const double hf = fmin(h * P.inv_dh_d, static_cast<double>(P.n_h - 1));
    const int ih = min(static_cast<int>(hf), P.n_h - 2);
    TLegX L;
    L.off = ih * P.nz;
    L.f = hf - static_cast<double>(ih);
    return L;
}

// Table reads go through a raw buffer over the tables: a read's row, node and
// depth displacements are scalar byte offsets, so a leg costs one vector
// address (its row plus the lane's depth) however many values it reads.
// Every read the kernels make lies inside the tables (the buffer's range check
// would return 0 past them).
__device__ __forceinline__ float table_read(const Params& P, int vbyte, int sbyte) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(raw_buffer(P.ttab, P.ttab_bytes), vbyte, sbyte, 0));
}

__device__ __forceinline__ double table_time_ext(const Params& P, TLegX L, int iz) {
    const int vo = (L.off + iz) * 4;
    const double a = table_read(P, vo, 0), b = table_read(P, vo, 4 * P.nz);
    return fma(L.f, b - a, a);
}

// Interpolated one-way time as a float32 table value (exact) plus a small
// float32 increment: b - a of two adjacent table values is exact, and the
// increment f (b - a), at most one row's difference (milliseconds), rounds to
// about 1e-10 s.  The pair's time adds the two bases in float64 (exactly) and
// then the legs' increments (pair_time), so it keeps the table's own precision
// (float32 rounding of the whole time in seconds and again in samples would
// cost about 1e-5 of a band-limited result) for a third of the float64 work
// of a float64 interpolation.
struct TTime {
    float base, inc;
};

__device__ __forceinline__ TTime table_time(const Params& P, TLeg L, int iz) {
    const int vo = (L.off + iz) * 4;
    const float a = table_read(P, vo, 0), b = table_read(P, vo, 4 * P.nz);
    return TTime{a, L.f * (b - a)};
}

// The pair's total time in samples: (T_s + T_r) / dt, the bases summed exactly.
__device__ __forceinline__ double pair_time(const Params& P, TTime s, TTime r) {
    return (static_cast<double>(s.base) + static_cast<double>(r.base) + static_cast<double>(s.inc + r.inc)) *
           P.inv_dt;
}

// Laterally varying tables: the image column's place on the node grid, off
// the float offset of the table of its lower node (i, j), fx and fy the
// fractions towards nodes i + 1 and j + 1 (float32: the time then moves by at
// most 2^-25 of the times' difference between neighbouring nodes).
struct LCol {
    int32_t off;
    float fx, fy;
};

// Lower node and fraction of coordinate c on an axis of n nodes, c clamped
// to the axis (beyond it the edge node holds); one node: no interpolation.
__device__ __forceinline__ void node_axis(double c, double c0, double g, int n, int& i, double& f) {
    if (n <= 1) {
        i = 0;
        f = 0.0;
        return;
    }
    const double a = fmin(fmax((c - c0) / g, 0.0), static_cast<double>(n - 1));
    i = min(static_cast<int>(a), n - 2);
    f = a - static_cast<double>(i);
}

__device__ __forceinline__ LCol lateral_col(const Params& P, float px, float py) {
    int i, j;
    double fx, fy;
    node_axis(px, P.gx0, P.gdx, P.n_gx, i, fx);
    node_axis(py, P.gy0, P.gdy, P.n_gy, j, fy);
    LCol C;
    C.off = (j * P.n_gx + i) * P.n_h * P.nz;
    C.fx = static_cast<float>(fx);
    C.fy = static_cast<float>(fy);
    return C;
}

// One-way time on the laterally varying tables: the interpolation in h on the
// four nodes around the column, then in x, then in y, as a base and an
// increment (as table_time).  The base is node (i, j)'s value a00 at row ih;
// every other term is taken relative to it in float32.  Where neighbouring
// nodes' times at one depth and row lie within a factor of two of each other
// (any smooth medium) their differences from a00 are exact, otherwise such a
// difference rounds once in float32; the interpolated increments are small,
// as in table_time.  Equal nodes give table_time's bits (every difference
// between nodes is 0).
__device__ __forceinline__ TTime ltable_lerp(float fh, LCol C, float a00, float b00, float a10, float b10,
                                             float a01, float b01, float a11, float b11) {
    const float d00 = fh * (b00 - a00);
    const float d10 = fmaf(fh, b10 - a10, a10 - a00);
    const float d01 = fmaf(fh, b01 - a01, a01 - a00);
    const float d11 = fmaf(fh, b11 - a11, a11 - a00);
    const float t0 = fmaf(C.fx, d10 - d00, d00), t1 = fmaf(C.fx, d11 - d01, d01);
    return TTime{a00, fmaf(C.fy, t1 - t0, t0)};
}

__device__ __forceinline__ TTime ltable_time(const Params& P, TLeg L, LCol C, int iz) {
    const int vo = (C.off + L.off + iz) * 4;
    const int nz = 4 * P.nz, dx = 4 * P.ldx, dy = 4 * P.ldy;  // byte offsets (scalar)
    const float a00 = table_read(P, vo, 0), b00 = table_read(P, vo, nz);
    const float a10 = table_read(P, vo, dx), b10 = table_read(P, vo, dx + nz);
    const float a01 = table_read(P, vo, dy), b01 = table_read(P, vo, dy + nz);
    const float a11 = table_read(P, vo, dx + dy), b11 = table_read(P, vo, dx + dy + nz);
    return ltable_lerp(L.f, C, a00, b00, a10, b10, a01, b01, a11, b11);
}

// ltable_time with an extended leg (the h fraction and the differences in float64).
__device__ __forceinline__ double ltable_time_ext(const Params& P, TLegX L, LCol C, int iz) {
    const int vo = (C.off + L.off + iz) * 4;
    const int nz = 4 * P.nz, dx = 4 * P.ldx, dy = 4 * P.ldy;  // byte offsets (scalar)
    const double fh = L.f;
    const double a00 = table_read(P, vo, 0), b00 = table_read(P, vo, nz);
    const double a10 = table_read(P, vo, dx), b10 = table_read(P, vo, dx + nz);
    const double a01 = table_read(P, vo, dy), b01 = table_read(P, vo, dy + nz);
    const double a11 = table_read(P, vo, dx + dy), b11 = table_read(P, vo, dx + dy + nz);
    const double t00 = fma(fh, b00 - a00, a00), t10 = fma(fh, b10 - a10, a10);
    const double t01 = fma(fh, b01 - a01, a01), t11 = fma(fh, b11 - a11, a11);
    const double fx = C.fx, fy = C.fy;
    const double t0 = fma(fx, t10 - t00, t00), t1 = fma(fx, t11 - t01, t01);
    return fma(fy, t1 - t0, t0);
}

// Amplitude of a leg (the table kinds with P.tamp): the amplitude tables
// interpolated as the times are, in float32 (a weight needs no more).
__device__ __forceinline__ float amp_read(const Params& P, int vbyte, int sbyte) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(raw_buffer(P.tamp, P.ttab_bytes), vbyte, sbyte, 0));
}

template <bool LAT>
__device__ __forceinline__ float table_amp(const Params& P, int off, float fh, LCol C, int iz) {
    const int nz = 4 * P.nz;
    if (!LAT) {
        const int vo = (off + iz) * 4;
        const float a = amp_read(P, vo, 0), b = amp_read(P, vo, nz);
        return fmaf(fh, b - a, a);
    }
    const int vo = (C.off + off + iz) * 4;
    const int dx = 4 * P.ldx, dy = 4 * P.ldy;
    const float a00 = amp_read(P, vo, 0), b00 = amp_read(P, vo, nz);
    const float a10 = amp_read(P, vo, dx), b10 = amp_read(P, vo, dx + nz);
    const float a01 = amp_read(P, vo, dy), b01 = amp_read(P, vo, dy + nz);
    const float a11 = amp_read(P, vo, dx + dy), b11 = amp_read(P, vo, dx + dy + nz);
    const float t00 = fmaf(fh, b00 - a00, a00), t10 = fmaf(fh, b10 - a10, a10);
    const float t01 = fmaf(fh, b01 - a01, a01), t11 = fmaf(fh, b11 - a11, a11);
    const float t0 = fmaf(C.fx, t10 - t00, t00), t1 = fmaf(C.fx, t11 - t01, t01);
    return fmaf(C.fy, t1 - t0, t0);
}

// Two adjacent depths iz, iz + 1 of one leg (the adjoint's interleaved slot
// pairs in full depth chunks, iz + 1 < nz): one 8-byte read per row and node
// gives both, where table_time / ltable_time read one value per read.  The
// arithmetic is theirs, so each depth's time has the same bits as the
// single-depth functions give: table_time_pair2 for float32 legs,
// table_time_pair for the extended forms (table_time_ext, ltable_time_ext).
struct Dbl2 {
    double a, b;
};
struct Flt2 {
    float a, b;
};
struct TTime2 {
    TTime a, b;
};

template <bool LAT>
__device__ __forceinline__ TTime2 table_time_pair2(const Params& P, int off, float fh, LCol C, int iz) {
    const __amdgpu_buffer_rsrc_t R = raw_buffer(P.ttab, P.ttab_bytes);
    const int vo = ((LAT ? C.off : 0) + off + iz) * 4;
    const int nz = 4 * P.nz;
    auto rows = [&](int so, float2& a, float2& b) {
        const auto va = __builtin_amdgcn_raw_buffer_load_b64(R, vo, so, 0);       // row ih: iz, iz + 1
        const auto vb = __builtin_amdgcn_raw_buffer_load_b64(R, vo, so + nz, 0);  // row ih + 1
        a = make_float2(__uint_as_float(va[0]), __uint_as_float(va[1]));
        b = make_float2(__uint_as_float(vb[0]), __uint_as_float(vb[1]));
    };
    float2 a00, b00;
    rows(0, a00, b00);
    if (!LAT) return TTime2{TTime{a00.x, fh * (b00.x - a00.x)}, TTime{a00.y, fh * (b00.y - a00.y)}};
    const int dx = 4 * P.ldx, dy = 4 * P.ldy;
    float2 a10, b10, a01, b01, a11, b11;
    rows(dx, a10, b10);
    rows(dy, a01, b01);
    rows(dx + dy, a11, b11);
    return TTime2{ltable_lerp(fh, C, a00.x, b00.x, a10.x, b10.x, a01.x, b01.x, a11.x, b11.x),
                  ltable_lerp(fh, C, a00.y, b00.y, a10.y, b10.y, a01.y, b01.y, a11.y, b11.y)};
}

template <bool LAT>
__device__ __forceinline__ Dbl2 table_time_pair(const Params& P, int off, double fh, LCol C, int iz) {
    const __amdgpu_buffer_rsrc_t R = raw_buffer(P.ttab, P.ttab_bytes);
    const int vo = ((LAT ? C.off : 0) + off + iz) * 4;
    const int nz = 4 * P.nz;
    auto node = [&](int so) {
        const auto a = __builtin_amdgcn_raw_buffer_load_b64(R, vo, so, 0);       // row ih: iz, iz + 1
        const auto b = __builtin_amdgcn_raw_buffer_load_b64(R, vo, so + nz, 0);  // row ih + 1
        const double da0 = __uint_as_float(a[0]), da1 = __uint_as_float(a[1]);
        const double db0 = __uint_as_float(b[0]), db1 = __uint_as_float(b[1]);
        return Dbl2{fma(fh, db0 - da0, da0), fma(fh, db1 - da1, da1)};
    };
    const Dbl2 t00 = node(0);
    if (!LAT) return t00;
    const int dx = 4 * P.ldx, dy = 4 * P.ldy;
    const Dbl2 t10 = node(dx), t01 = node(dy), t11 = node(dx + dy);
    const double fx = C.fx, fy = C.fy;
    Dbl2 t;
    {
        const double t0 = fma(fx, t10.a - t00.a, t00.a), t1 = fma(fx, t11.a - t01.a, t01.a);
        t.a = fma(fy, t1 - t0, t0);
    }
    {
        const double t0 = fma(fx, t10.b - t00.b, t00.b), t1 = fma(fx, t11.b - t01.b, t01.b);
        t.b = fma(fy, t1 - t0, t0);
    }
    return t;
}

// table_amp at two adjacent depths (same bits per depth).
template <bool LAT>
__device__ __forceinline__ Flt2 table_amp_pair(const Params& P, int off, float fh, LCol C, int iz) {
    const __amdgpu_buffer_rsrc_t R = raw_buffer(P.tamp, P.ttab_bytes);
    const int vo = ((LAT ? C.off : 0) + off + iz) * 4;
    const int nz = 4 * P.nz;
    auto node = [&](int so) {
        const auto a = __builtin_amdgcn_raw_buffer_load_b64(R, vo, so, 0);
        const auto b = __builtin_amdgcn_raw_buffer_load_b64(R, vo, so + nz, 0);
        const float a0 = __uint_as_float(a[0]), a1 = __uint_as_float(a[1]);
        const float b0 = __uint_as_float(b[0]), b1 = __uint_as_float(b[1]);
        return Flt2{fmaf(fh, b0 - a0, a0), fmaf(fh, b1 - a1, a1)};
    };
    const Flt2 t00 = node(0);
    if (!LAT) return t00;
    const int dx = 4 * P.ldx, dy = 4 * P.ldy;
    const Flt2 t10 = node(dx), t01 = node(dy), t11 = node(dx + dy);
    Flt2 t;
    {
        const float t0 = fmaf(C.fx, t10.a - t00.a, t00.a), t1 = fmaf(C.fx, t11.a - t01.a, t01.a);
        t.a = fmaf(C.fy, t1 - t0, t0);
    }
    {
        const float t0 = fmaf(C.fx, t10.b - t00.b, t00.b), t1 = fmaf(C.fx, t11.b - t01.b, t01.b);
        t.b = fmaf(C.fy, t1 - t0, t0);
    }
    return t;
}

// eval_pair_table with extended legs (same clamp as eval_pair_table; the
// fraction is returned in float32 and float64).
template <bool TF, bool LAT = false>
__device__ __forceinline__ PairX eval_pair_table_ext(const Params& P, TLegX Ls, TLegX Lr, int iz, float wlo,
                                                     float whi, LCol C = LCol{0, 0.0f, 0.0f}) {
    double w = (LAT ? ltable_time_ext(P, Ls, C, iz) + ltable_time_ext(P, Lr, C, iz)
                    : table_time_ext(P, Ls, iz) + table_time_ext(P, Lr, iz)) * P.inv_dt;
    if (TF) w = w + P.tf_off_d;
    w = fmin(fmax(w, static_cast<double>(wlo)), static_cast<double>(whi));
    PairX p;
    p.i = static_cast<int32_t>(w);
    p.fd = w - static_cast<double>(p.i);
    p.f = static_cast<float>(p.fd);
    p.r = 1.0f;
    if (P.tamp)
        p.r = table_amp<LAT>(P, Ls.off, static_cast<float>(Ls.f), C, iz) *
              table_amp<LAT>(P, Lr.off, static_cast<float>(Lr.f), C, iz);
    return p;
}

// The pair evaluation of eval_pair with table times (iz < nz); the clamp
// bounds are those of clamp_bounds.  LAT: laterally varying tables at column
// C.  r = A_s A_r with amplitude tables, else 1.
template <bool TF, bool CLAMP = true, bool LAT = false>
__device__ __forceinline__ Pair eval_pair_table(const Params& P, TLeg Ls, TLeg Lr, int iz, float tf_off, float wlo,
                                                float whi, LCol C = LCol{0, 0.0f, 0.0f}) {
    (void)tf_off;
    double w = LAT ? pair_time(P, ltable_time(P, Ls, C, iz), ltable_time(P, Lr, C, iz))
                   : pair_time(P, table_time(P, Ls, iz), table_time(P, Lr, iz));
    if (TF) w = w + P.tf_off_d;
    if (CLAMP) w = fmin(fmax(w, static_cast<double>(wlo)), static_cast<double>(whi));
    Pair p;
    p.i = static_cast<int32_t>(w);
    p.f = static_cast<float>(w - static_cast<double>(p.i));
    p.r = 1.0f;
    if (P.tamp) p.r = table_amp<LAT>(P, Ls.off, Ls.f, C, iz) * table_amp<LAT>(P, Lr.off, Lr.f, C, iz);
    return p;
}

// Clamp bounds of eval_pair for a row of lt floats: reads at floor(w) and
// floor(w) + 1 stay in [0, lt).  Without t_first the row pointer is advanced
// by kLead and u >= 0 needs no lower clamp beyond 0.
template <bool TF>
__device__ __forceinline__ void clamp_bounds(int lt, float& wlo, float& whi) {
    wlo = TF ? static_cast<float>(kLead - 1) : 0.0f;
    whi = TF ? static_cast<float>(lt - 2) : static_cast<float>(lt - 2 - kLead);
}

// First depth of depth chunk zc of n_chunks chunks of `span` depths.
// BOTTOM = false: chunks start at depth 0 (a partial chunk holds the deepest
// depths; its lanes past nz are invalid).  BOTTOM = true: chunks end at the
// last depth, so a partial chunk holds the shallowest depths, where the
// aperture is smallest and few pairs fall (its depths below 0 are invalid
// lanes).  The adjoint takes the bottom alignment (5 % faster on the 3D survey:
// its partial chunk no longer wastes half its lanes where the pairs are
// densest); migration and the counting kernel keep the top one (migration ran
// 28 % slower bottom-aligned).
template <bool BOTTOM>
__device__ __forceinline__ int chunk_z0(int nz, int zc, int n_chunks, int span) {
    return BOTTOM ? zc * span - (n_chunks * span - nz) : zc * span;
}

// Depth of lane d in slot k of the chunk starting at z0.  IL = 1: slot k is
// the 16 consecutive depths z0 + 16 k + d.  IL = 2: slots 2m and 2m + 1 share
// the 32 depths z0 + 32 m .. z0 + 32 m + 31, even depths in slot 2m and odd
// ones in 2m + 1, so neighbouring lanes are two depths apart.
template <int IL>
__device__ __forceinline__ int slot_depth(int z0, int k, int d) {
    if (IL == 1) return z0 + k * kGroup + d;
    return z0 + (k >> 1) * (2 * kGroup) + 2 * d + (k & 1);
}

// Per-depth tables of one depth chunk.  Lane d of every group holds depth
// slot_depth(z0, k, d) in slot k.  A lane is valid if its depth exists and (for
// the cos*cos weight) t0sq > 0; elsewhere W = 0 and the image value is 0.
//   A, B     sample-unit traveltime tables per slot
//   R        the aperture table per slot (-1 where the lane is invalid)
//   rlo/rhi  lane d == k < KS of every group holds min / max over the valid
//            lanes of slot k of the aperture table (+inf / -inf when the slot
//            has no valid lane)
//   rmax     max over the chunk (wavefront-uniform)
// PX (extended-precision kernels): A, B are the physical tables t0sq and s2
// (exact float32 inputs; A = kTinyA where t0sq = 0), scaled by 1 / dt after
// the square roots.
// sR[16 k + d] (LDS) holds the aperture value of each lane, -1 where invalid.
template <int KS>
struct ChunkTables {
    float A[KS], B[KS], R[KS];
    float rlo, rhi, rmax;
    uint32_t clean;  // bit k: every lane of slot k is valid (wavefront-uniform)
};

template <int KS, int IL = 1, int TT = TT_DSR, bool PX = false>
__device__ __forceinline__ void load_chunk_tables(const Params& P, int z0, int d, bool zero_weight_guard,
                                                  ChunkTables<KS>& T, float* sR) {
    const int lane = threadIdx.x & (kLanes - 1);
    float rmax = -1.0f;
    float rlo_mine = __builtin_inff(), rhi_mine = -__builtin_inff();
    uint32_t clean = 0;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int iz = slot_depth<IL>(z0, k, d);
        // invalid lanes: a = 1 for every leg (finite time and weight), never inside
        float A = 1.0f, B = 0.0f, R = -1.0f;
        bool valid = false;
        if (iz >= 0 && iz < P.nz) {
            if (is_table(TT)) {
                // table times carry no t0sq / s2; A, B are unused and W = 1
                valid = true;
                A = 0.0f;
                R = P.r2[iz];
            } else {
                const float t0 = P.t0sq[iz];
                valid = !(zero_weight_guard && !(t0 > 0.0f));
                if (valid) {
                    if (PX) {
                        A = t0 == 0.0f ? kTinyA : t0;
                        B = P.s2[iz];
                    } else {
                        A = static_cast<float>(static_cast<double>(t0) * P.inv_dt2);
                        B = static_cast<float>(static_cast<double>(P.s2[iz]) * P.inv_dt2);
                    }
                    R = P.r2[iz];
                }
            }
        }
        T.A[k] = A;
        T.B[k] = B;
        T.R[k] = R;
        if (sR && lane < kGroup) sR[k * kGroup + d] = R;
        if ((__builtin_amdgcn_ballot_w64(valid) & 0xFFFFull) == 0xFFFFull) clean |= 1u << k;
        // min / max over the 16 lanes of the group (all groups hold the same depths)
        float lo = valid ? R : __builtin_inff();
        float hi = valid ? R : -__builtin_inff();
#pragma unroll
        for (int off = 1; off < kGroup; off <<= 1) {
            lo = fminf(lo, __shfl_xor(lo, off, kLanes));
            hi = fmaxf(hi, __shfl_xor(hi, off, kLanes));
        }
        if (d == k) {
            rlo_mine = lo;
            rhi_mine = hi;
        }
        rmax = fmaxf(rmax, hi);
    }
    T.rlo = rlo_mine;
    T.rhi = rhi_mine;
    T.clean = clean;
    // equal in every lane: make them scalar so that branches on them are uniform
    T.rmax = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(rmax)));
}

// Bit k (k < KS) set when slot k may hold a lane inside the aperture
// (hmin <= max R of the slot) / when every valid lane is inside
// (hmax <= min R of the slot).  hmin, hmax: wavefront-uniform.
template <int KS>
__device__ __forceinline__ void slot_masks(const ChunkTables<KS>& T, float hmin, float hmax, uint64_t& any,
                                           uint64_t& full) {
    constexpr uint64_t kMask = (KS >= 64) ? ~0ull : ((1ull << KS) - 1ull);
    any = __builtin_amdgcn_ballot_w64(hmin <= T.rhi) & kMask;
    full = __builtin_amdgcn_ballot_w64(hmax <= T.rlo) & kMask;
}

// Final per-depth factor of the image: t0sq / dt^4 for the cos*cos weight
// (so W = factor * r with r in samples^-4), t0sq for the extended kernels (r in
// s^-4), 1 for the unit weight; 0 where W is defined as 0.
template <bool PX = false>
__device__ __forceinline__ float depth_factor(const Params& P, int iz) {
    if (P.weight != W_COSCOS) return 1.0f;
    const float t0 = P.t0sq[iz];
    if (PX) return t0 > 0.0f ? t0 : 0.0f;
    return t0 > 0.0f ? static_cast<float>(static_cast<double>(t0) * P.wscale) : 0.0f;
}

// A value that is equal in every lane, as a scalar register.
__device__ __forceinline__ float uniform_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Wavefront minimum / maximum (every lane gets it, as a uniform value).
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int off = 1; off < kLanes; off <<= 1) v = fminf(v, __shfl_xor(v, off, kLanes));
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 1; off < kLanes; off <<= 1) v = fmaxf(v, __shfl_xor(v, off, kLanes));
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Squared distance from (x, y) to the box [x0, x1] x [y0, y1] (0 inside), and
// to its farthest point, float32.  Rounding is monotone, so for a column
// (px, py) of the box legs() gives box_dist2 <= h^2 <= box_far2 exactly.
__device__ __forceinline__ float box_dist2(float x, float y, float x0, float x1, float y0, float y1) {
    const float dx = fmaxf(fmaxf(x0 - x, x - x1), 0.0f);
    const float dy = fmaxf(fmaxf(y0 - y, y - y1), 0.0f);
    return dx * dx + dy * dy;
}

__device__ __forceinline__ float box_far2(float x, float y, float x0, float x1, float y0, float y1) {
    const float dx = fmaxf(fabsf(x0 - x), fabsf(x1 - x));
    const float dy = fmaxf(fabsf(y0 - y), fabsf(y1 - y));
    return dx * dx + dy * dy;
}

// v from lane `src` (any lane), through the LDS crossbar.
__device__ __forceinline__ float lane_read(float v, int src) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

// A float64 value from lane `src` (two crossbar reads).
__device__ __forceinline__ double lane_read_d(double v, int src) {
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float uniform_read(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

}  // namespace km
