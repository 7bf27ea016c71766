// Device-side building blocks shared by the migrate, demigrate, count and
// batched kernels: launch parameters, trace staging and the per-pair
// evaluation of Eq. (1) (aperture, total time, interpolation index, weight).
//
// Lane layout used by every image-domain kernel: a wavefront (64 lanes) is
// four groups of 16 lanes; group g works on one image column, lane d of the
// group on depth z0 + 16 k + d for slot k = 0..KS-1.  A 16-depth slot is the
// unit of the aperture mask: a pair (column, trace) enters a slot only if
// some lane of the slot is inside the aperture.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace km {

constexpr int kLanes = 64;
constexpr int kGroup = 16;        // lanes per column group (depths per slot)
constexpr int kGroupsPerWave = 4;  // columns per wavefront slot
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
    float tf_shift;   // 1 - t_first / dt (used when t_first != 0)
    int32_t has_tf;
    int32_t weight;
    // output / input image
    float* image;
    int32_t accumulate;
    // staging geometry
    int32_t lt;       // LDS floats per staged trace (>= nt + 3)
    int32_t tb;       // traces per LDS block
    int32_t n_zchunks;
    int32_t n_coltiles;
};

// First index in sorted bin[0..n) whose value is >= key.
__device__ __forceinline__ int64_t lower_bound_bin(const int32_t* __restrict__ bin, int64_t n, int32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (bin[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ float load_sample(const Params& P, int64_t j, int32_t k) {
    const int64_t off = j * P.stride + k;
    if (P.dtype == F32) return static_cast<const float*>(P.data)[off];
    const uint16_t bits = static_cast<const uint16_t*>(P.data)[off];
    float v;
    if (P.dtype == BF16) {
        v = __uint_as_float(static_cast<uint32_t>(bits) << 16);
    } else {
        v = __half2float(__ushort_as_half(bits));
    }
    return P.scale ? v * P.scale[j] : v;
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
//   u   = sqrt(a_s) + sqrt(a_r) (+ shift when t_first != 0), clamped to
//         [0, umax] so that the staged-trace reads stay inside the row,
//   i   = floor(u), f = u - i, and r = 1 / (a_s a_r) for the weight.
// Migrate and demigrate both call this, so the transpose pair sees
// bit-identical (i, f, r) for every pair.
struct Pair {
    int32_t i;
    float f;
    float r;
};

template <bool TF, int WK>
__device__ __forceinline__ Pair eval_pair(float A, float B, float hs2, float hr2, float tf_shift, float umax) {
    const float as = fmaf(B, hs2, A);
    const float ar = fmaf(B, hr2, A);
    float u = __builtin_amdgcn_sqrtf(as) + __builtin_amdgcn_sqrtf(ar);
    if (TF) u = fmaxf(u + tf_shift, 0.0f);
    u = fminf(u, umax);
    Pair p;
    p.i = static_cast<int32_t>(u);
    p.f = __builtin_amdgcn_fractf(u);
    p.r = (WK == W_COSCOS) ? __builtin_amdgcn_rcpf(as * ar) : 1.0f;
    return p;
}

// Per-depth tables of one depth chunk, in registers: lane d of every group
// holds depth z0 + 16 k + d.  Depths past nz (and, for the cos*cos weight,
// depths with t0sq <= 0 where W = 0) get R = -1 so that no leg is inside.
template <int KS>
struct DepthTables {
    float A[KS], B[KS], R[KS];
    float rmax;  // max over the chunk of R (wavefront-uniform)
};

template <int KS>
__device__ __forceinline__ void load_tables(const Params& P, int z0, int d, bool zero_weight_guard,
                                            DepthTables<KS>& T) {
    float rmax = -1.0f;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int iz = z0 + k * kGroup + d;
        float A = 1.0f, B = 0.0f, R = -1.0f;
        if (iz < P.nz) {
            const float t0 = P.t0sq[iz];
            A = static_cast<float>(static_cast<double>(t0) * P.inv_dt2);
            B = static_cast<float>(static_cast<double>(P.s2[iz]) * P.inv_dt2);
            R = P.r2[iz];
            if (zero_weight_guard && !(t0 > 0.0f)) R = -1.0f;
        }
        T.A[k] = A;
        T.B[k] = B;
        T.R[k] = R;
        rmax = fmaxf(rmax, R);
    }
    // wavefront max (every lane ends with the same value)
#pragma unroll
    for (int off = 1; off < kLanes; off <<= 1) rmax = fmaxf(rmax, __shfl_xor(rmax, off, kLanes));
    T.rmax = rmax;
}

// Final per-depth factor of the image: t0sq / dt^4 for the cos*cos weight
// (so W = factor * r), 1 for the unit weight; 0 where W is defined as 0.
__device__ __forceinline__ float depth_factor(const Params& P, int iz) {
    if (P.weight != W_COSCOS) return 1.0f;
    const float t0 = P.t0sq[iz];
    return t0 > 0.0f ? static_cast<float>(static_cast<double>(t0) * P.wscale) : 0.0f;
}

}  // namespace km
