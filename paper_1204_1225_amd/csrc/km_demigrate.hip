// Demigration kernel: the transpose of migration as a trace-stationary scatter.
//
// Workgroup = a block of P.tb consecutive traces (of the bin-sorted list).
// The block's output rows live in LDS as float32 accumulators (same
// zero-padded row layout as the migration staging: row[1 + k] = sample k).
// Wavefronts sweep the image columns of each bin present in the block (four
// columns per wavefront slot, lanes = depths), load the image value of every
// lane once per column group, and for every trace in aperture scatter
// (1 - f) W I and f W I into the two samples around the total time with LDS
// float atomics.  Each row is written back to HBM exactly once.
#include "km_kernels.h"

namespace km {

template <int NW, int KS, bool TF, int WK>
__device__ __forceinline__ void demigrate_segment(const Params& P, int b, int t0, int t1, const float4* sGeo,
                                                  float* sAcc) {
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = threadIdx.x / kLanes;
    const int g = lane / kGroup, d = lane % kGroup;
    const int ncol = P.nx * P.ny;
    const int nquads = (ncol + kGroupsPerWave - 1) / kGroupsPerWave;
    const float umax = TF ? static_cast<float>(P.lt - 2) : static_cast<float>(P.lt - 3);
    const float tfs = P.tf_shift;
    const float* img = P.image + static_cast<int64_t>(b) * ncol * P.nz;

    for (int zc = 0; zc < P.n_zchunks; ++zc) {
        const int z0 = zc * KS * kGroup;
        DepthTables<KS> T;
        load_tables<KS>(P, z0, d, WK == W_COSCOS, T);
        if (T.rmax < 0.0f) continue;
        for (int qi = wave; qi < nquads; qi += NW) {
            const int col = qi * kGroupsPerWave + g;
            float px = kFar, py = kFar;
            if (col < ncol) {
                px = P.x[col % P.nx];
                py = P.y[col / P.nx];
            }
            // Is any trace of the segment inside the aperture of this column group?
            bool any = false;
            for (int t = t0; t < t1 && !any; ++t) any = legs(px, py, sGeo[t]).hmax <= T.rmax;
            if (!__any(any)) continue;
            float xv[KS];
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                const int iz = z0 + k * kGroup + d;
                xv[k] = (col < ncol && iz < P.nz) ? img[static_cast<int64_t>(col) * P.nz + iz] * depth_factor(P, iz)
                                                  : 0.0f;
            }
            for (int t = t0; t < t1; ++t) {
                const Legs L = legs(px, py, sGeo[t]);
                if (L.hmax <= T.rmax) {
                    float* row = sAcc + t * P.lt + (TF ? 0 : 1);
#pragma unroll
                    for (int k = 0; k < KS; ++k) {
                        if (L.hmax <= T.R[k]) {
                            const Pair pr = eval_pair<TF, WK>(T.A[k], T.B[k], L.hs2, L.hr2, tfs, umax);
                            const float q = (WK == W_COSCOS) ? xv[k] * pr.r : xv[k];
                            const float q1 = pr.f * q;
                            const float q0 = q - q1;
                            atomicAdd(row + pr.i, q0);
                            atomicAdd(row + pr.i + 1, q1);
                        }
                    }
                }
            }
        }
    }
}

template <int NW, int KS, bool TF, int WK>
__global__ __launch_bounds__(NW * 64) void demigrate_kernel(Params P) {
    extern __shared__ float lds[];
    float4* sGeo = reinterpret_cast<float4*>(lds);
    float* sAcc = lds + 4 * P.tb;
    const int64_t j0 = static_cast<int64_t>(blockIdx.x) * P.tb;
    const int nb = static_cast<int>(min<int64_t>(P.tb, P.n_traces - j0));

    for (int t = threadIdx.x; t < P.tb; t += blockDim.x) {
        float4 g = make_float4(kFar, kFar, kFar, kFar);
        if (t < nb) {
            const int64_t j = j0 + t;
            g = make_float4(P.src[2 * j], P.src[2 * j + 1], P.rec[2 * j], P.rec[2 * j + 1]);
        }
        sGeo[t] = g;
    }
    for (int e = threadIdx.x; e < P.tb * P.lt; e += blockDim.x) sAcc[e] = 0.0f;
    __syncthreads();

    // The block's traces form runs of equal bin (the list is sorted by bin).
    int t0 = 0;
    while (t0 < nb) {
        const int b = P.bin[j0 + t0];
        int t1 = t0 + 1;
        while (t1 < nb && P.bin[j0 + t1] == b) ++t1;
        if (b >= 0 && b < P.n_bins) demigrate_segment<NW, KS, TF, WK>(P, b, t0, t1, sGeo, sAcc);
        t0 = t1;
    }
    __syncthreads();

    float* out = static_cast<float*>(P.data);
    for (int t = 0; t < nb; ++t) {
        float* o = out + (j0 + t) * P.stride;
        const float* row = sAcc + t * P.lt + 1;
        for (int k = threadIdx.x; k < P.nt; k += blockDim.x) o[k] = P.accumulate ? o[k] + row[k] : row[k];
    }
}

template <int NW, int KS>
static hipError_t launch_demigrate_shape(const Params& P, hipStream_t s) {
    const int64_t nblk = (P.n_traces + P.tb - 1) / P.tb;
    dim3 grid(static_cast<unsigned>(nblk)), block(NW * 64);
    const size_t lds = lds_bytes(P);
    if (P.has_tf) {
        if (P.weight == W_COSCOS) return launch_with_lds(demigrate_kernel<NW, KS, true, W_COSCOS>, grid, block, lds, s, P);
        return launch_with_lds(demigrate_kernel<NW, KS, true, W_UNIT>, grid, block, lds, s, P);
    }
    if (P.weight == W_COSCOS) return launch_with_lds(demigrate_kernel<NW, KS, false, W_COSCOS>, grid, block, lds, s, P);
    return launch_with_lds(demigrate_kernel<NW, KS, false, W_UNIT>, grid, block, lds, s, P);
}

#define KM_DEMIGRATE_SHAPES(X) \
    X(8, 16, 98304)            \
    X(4, 16, 65536)            \
    X(8, 8, 98304)

static const TileShape kDemigrateShapes[] = {
#define X(nw, ks, lb) {nw, 1, ks, lb},
    KM_DEMIGRATE_SHAPES(X)
#undef X
};

int demigrate_shape_count() { return static_cast<int>(sizeof(kDemigrateShapes) / sizeof(kDemigrateShapes[0])); }
const TileShape& demigrate_shape(int i) { return kDemigrateShapes[i]; }

hipError_t launch_demigrate(int shape, const Params& P, hipStream_t s) {
    int i = 0;
#define X(nw, ks, lb) \
    if (shape == i) return launch_demigrate_shape<nw, ks>(P, s); \
    ++i;
    KM_DEMIGRATE_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace km
