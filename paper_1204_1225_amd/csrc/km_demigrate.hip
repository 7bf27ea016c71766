// Demigration kernel: the transpose of migration as a trace-stationary scatter.
//
// Workgroup = a block of P.tb consecutive traces (of the bin-sorted list).
// The block's output rows live in LDS as float64 accumulators (same
// zero-padded row layout as the migration staging: row[kLead + k] = sample k).
// float64 because gfx950 executes LDS float64 atomic adds at about 8 clocks
// per wavefront instruction and float32 ones at about 190 (measured), and the
// wider sum also keeps the transpose's own rounding negligible.
// Wavefronts sweep the image columns of each bin present in the block, one
// column per wavefront at a time; the four 16-lane groups of a wavefront work
// on four different traces of the block (lanes = 16 consecutive depths), so
// that the LDS float atomics of one instruction land in four different rows
// and seldom on the same address.  The image values of the column are loaded
// once and serve every trace of the block.  Each row is written back to HBM
// exactly once.
#include "km_kernels.h"

namespace km {

// Depth interleave of the adjoint's lanes: neighbouring lanes of a group are two
// depths apart, so their target samples are at least about one sample apart
// within the aperture and the LDS atomics of one instruction seldom share an address.
constexpr int kIL = 2;

// Two slots of one lane: with the depth interleave they are neighbouring
// depths z, z + 1 of the same (column, trace) pairing, whose first samples i0,
// i1 usually differ by 0 or 1.  Contributions landing on the same sample are
// summed (in float32) before the LDS atomic, so a lane issues 2 to 4 atomics
// for its 4 (sample, value) contributions instead of always 4.  Lanes with
// nothing to add (image value 0, padding lanes, outside the aperture) issue
// none.  MASKED: keep only lanes with hmax <= their aperture value.
template <bool TF, int WK, bool MASKED, bool CLAMP>
__device__ __forceinline__ void dem_pair(float A0, float B0, float A1, float B1, float hs2, float hr2, float hm,
                                         double* row, float tfo, float wlo, float whi, const float* sRk, float x0,
                                         float x1) {
    bool act0 = x0 != 0.0f, act1 = x1 != 0.0f;
    if (MASKED) {
        act0 = act0 && hm <= sRk[0];
        act1 = act1 && hm <= sRk[kGroup];
    }
    if (!(act0 || act1)) return;
    const Pair p0 = eval_pair<TF, WK, CLAMP>(A0, B0, hs2, hr2, tfo, wlo, whi);
    const Pair p1 = eval_pair<TF, WK, CLAMP>(A1, B1, hs2, hr2, tfo, wlo, whi);
    float q0 = (WK == W_COSCOS) ? x0 * p0.r : x0;
    float q1 = (WK == W_COSCOS) ? x1 * p1.r : x1;
    q0 = act0 ? q0 : 0.0f;
    q1 = act1 ? q1 : 0.0f;
    const float b0 = p0.f * q0, a0 = q0 - b0;  // to samples i0, i0 + 1
    const float b1 = p1.f * q1, a1 = q1 - b1;  // to samples i1, i1 + 1
    const int delta = p1.i - p0.i;
    const bool same = delta == 0, next = delta == 1;
    // float32 pre-sums (each term is a float32 product already); the row is float64
    const float c0 = a0 + (same ? a1 : 0.0f);
    const float c1 = b0 + (same ? b1 : (next ? a1 : 0.0f));
    if (act0 || (act1 && (same || next))) {
        atomicAdd(row + p0.i, static_cast<double>(c0));
        atomicAdd(row + p0.i + 1, static_cast<double>(c1));
    }
    if (act1 && !same) {
        atomicAdd(row + p1.i + 1, static_cast<double>(b1));
        if (!next) atomicAdd(row + p1.i, static_cast<double>(a1));
    }
}

// The same two slots without merging: 4 atomics per lane with something to add.
template <bool TF, int WK, bool MASKED, bool CLAMP>
__device__ __forceinline__ void dem_pair_plain(float A0, float B0, float A1, float B1, float hs2, float hr2, float hm,
                                               double* row, float tfo, float wlo, float whi, const float* sRk,
                                               float x0, float x1) {
    bool act0 = x0 != 0.0f, act1 = x1 != 0.0f;
    if (MASKED) {
        act0 = act0 && hm <= sRk[0];
        act1 = act1 && hm <= sRk[kGroup];
    }
    if (act0) {
        const Pair p0 = eval_pair<TF, WK, CLAMP>(A0, B0, hs2, hr2, tfo, wlo, whi);
        const float q0 = (WK == W_COSCOS) ? x0 * p0.r : x0;
        const float b0 = p0.f * q0;
        atomicAdd(row + p0.i, static_cast<double>(q0 - b0));
        atomicAdd(row + p0.i + 1, static_cast<double>(b0));
    }
    if (act1) {
        const Pair p1 = eval_pair<TF, WK, CLAMP>(A1, B1, hs2, hr2, tfo, wlo, whi);
        const float q1 = (WK == W_COSCOS) ? x1 * p1.r : x1;
        const float b1 = p1.f * q1;
        atomicAdd(row + p1.i, static_cast<double>(q1 - b1));
        atomicAdd(row + p1.i + 1, static_cast<double>(b1));
    }
}

template <bool MERGE, bool TF, int WK, bool MASKED, bool CLAMP>
__device__ __forceinline__ void dem_two(float A0, float B0, float A1, float B1, float hs2, float hr2, float hm,
                                        double* row, float tfo, float wlo, float whi, const float* sRk, float x0,
                                        float x1) {
    if (MERGE) dem_pair<TF, WK, MASKED, CLAMP>(A0, B0, A1, B1, hs2, hr2, hm, row, tfo, wlo, whi, sRk, x0, x1);
    else dem_pair_plain<TF, WK, MASKED, CLAMP>(A0, B0, A1, B1, hs2, hr2, hm, row, tfo, wlo, whi, sRk, x0, x1);
}

template <int NW, int KS, bool MERGE, bool TF, int WK>
__device__ __forceinline__ void demigrate_segment(const Params& P, int b, int t0, int t1, const float4* sGeo,
                                                  double* sAcc, float* sR) {
    static_assert(KS % 2 == 0, "slots are evaluated in pairs");
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = threadIdx.x / kLanes;
    const int g = lane / kGroup, d = lane % kGroup;
    const int ncol = P.nx * P.ny;
    const int nseg = t1 - t0;  // <= tb <= 64
    const int nquads = (nseg + kGroupsPerWave - 1) / kGroupsPerWave;
    float wlo, whi;
    clamp_bounds<TF>(P.lt, wlo, whi);
    const float tfo = P.tf_off;
    const int rowoff = TF ? 0 : kLead;
    const float* img = P.image + static_cast<int64_t>(b) * ncol * P.nz;
    const uint64_t segmask = nseg >= 64 ? ~0ull : ((1ull << nseg) - 1ull);
    // lane-parallel geometry: lane l <-> trace t0 + l (far away past the segment)
    const float4 srl = lane < nseg ? sGeo[t0 + lane] : make_float4(kFar, kFar, kFar, kFar);

    for (int zc = 0; zc < P.n_zchunks; ++zc) {
        const int z0 = zc * KS * kGroup;
        ChunkTables<KS> T;
        __syncthreads();  // previous chunk's readers of sR are done
        load_chunk_tables<KS, kIL>(P, z0, d, WK == W_COSCOS, T, sR);
        const bool noclamp = !TF && T.wmax <= whi;
        float S[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int iz = slot_depth<kIL>(z0, k, d);
            S[k] = (iz < P.nz) ? depth_factor(P, iz) : 0.0f;
        }
        __syncthreads();
        if (T.rmax < 0.0f) continue;
        for (int col = wave; col < ncol; col += NW) {
            const float px = P.x[col % P.nx], py = P.y[col / P.nx];
            const Legs Lp = legs(px, py, srl);
            const uint64_t live = __builtin_amdgcn_ballot_w64(Lp.hmax <= T.rmax) & segmask;
            if (!live) continue;
            // extremes of hmax over each aligned quad of traces (the four groups of a slot)
            float qmin = fminf(Lp.hmax, __shfl_xor(Lp.hmax, 1, kLanes));
            qmin = fminf(qmin, __shfl_xor(qmin, 2, kLanes));
            float qmax = fmaxf(Lp.hmax, __shfl_xor(Lp.hmax, 1, kLanes));
            qmax = fmaxf(qmax, __shfl_xor(qmax, 2, kLanes));
            float x[KS];
            const float* colp = img + static_cast<int64_t>(col) * P.nz;
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                const int iz = slot_depth<kIL>(z0, k, d);
                x[k] = (iz < P.nz) ? colp[iz] * S[k] : 0.0f;
            }
            for (int qt = 0; qt < nquads; ++qt) {
                if (!((live >> (kGroupsPerWave * qt)) & 0xFull)) continue;
                const float hmin = uniform_read(qmin, kGroupsPerWave * qt);
                const float hmaxw = uniform_read(qmax, kGroupsPerWave * qt);
                uint64_t any, full;
                slot_masks<KS>(T, hmin, hmaxw, any, full);
                if (!any) continue;
                const int src = kGroupsPerWave * qt + g;  // this group's trace (segment-relative)
                const float hs2 = lane_read(Lp.hs2, src);
                const float hr2 = lane_read(Lp.hr2, src);
                const float hm = fmaxf(hs2, hr2);
                double* row = sAcc + (t0 + min(src, nseg - 1)) * P.lt + rowoff;
#pragma unroll
                for (int k = 0; k < KS; k += 2) {
                    if ((any >> k) & 3ull) {
                        if (((full >> k) & 3ull) == 3ull) {
                            if (noclamp)
                                dem_two<MERGE, TF, WK, false, false>(T.A[k], T.B[k], T.A[k + 1], T.B[k + 1], hs2, hr2, hm, row,
                                                               tfo, wlo, whi, nullptr, x[k], x[k + 1]);
                            else
                                dem_two<MERGE, TF, WK, false, true>(T.A[k], T.B[k], T.A[k + 1], T.B[k + 1], hs2, hr2, hm, row,
                                                              tfo, wlo, whi, nullptr, x[k], x[k + 1]);
                        } else {
                            dem_two<MERGE, TF, WK, true, true>(T.A[k], T.B[k], T.A[k + 1], T.B[k + 1], hs2, hr2, hm, row, tfo,
                                                         wlo, whi, sR + k * kGroup + d, x[k], x[k + 1]);
                        }
                    }
                }
            }
        }
    }
}

template <int NW, int KS, bool MERGE, bool TF, int WK>
__global__ __launch_bounds__(NW * 64) void demigrate_kernel(Params P) {
    extern __shared__ float lds[];
    double* sAcc = reinterpret_cast<double*>(lds);                     // [tb][lt]
    float4* sGeo = reinterpret_cast<float4*>(lds + 2 * P.tb * P.lt);   // [tb]
    float* sR = lds + 2 * P.tb * P.lt + 4 * P.tb;                      // [KS * 16]
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
    for (int e = threadIdx.x; e < P.tb * P.lt; e += blockDim.x) sAcc[e] = 0.0;
    __syncthreads();

    // The block's traces form runs of equal bin (the list is sorted by bin).
    int t0 = 0;
    while (t0 < nb) {
        const int b = P.bin[j0 + t0];
        int t1 = t0 + 1;
        while (t1 < nb && P.bin[j0 + t1] == b) ++t1;
        if (b >= 0 && b < P.n_bins) demigrate_segment<NW, KS, MERGE, TF, WK>(P, b, t0, t1, sGeo, sAcc, sR);
        t0 = t1;
    }
    __syncthreads();

    float* out = static_cast<float*>(P.data);
    for (int t = 0; t < nb; ++t) {
        float* o = out + (j0 + t) * P.stride;
        const double* row = sAcc + t * P.lt + kLead;
        for (int k = threadIdx.x; k < P.nt; k += blockDim.x) {
            const float v = static_cast<float>(row[k]);
            o[k] = P.accumulate ? o[k] + v : v;
        }
    }
}

template <int NW, int KS, bool MERGE>
static hipError_t launch_demigrate_shape(const Params& P, hipStream_t s) {
    const int64_t nblk = (P.n_traces + P.tb - 1) / P.tb;
    dim3 grid(static_cast<unsigned>(nblk)), block(NW * 64);
    const size_t lds = lds_bytes_f64rows(P, KS);
    if (P.has_tf) {
        if (P.weight == W_COSCOS) return launch_with_lds(demigrate_kernel<NW, KS, MERGE, true, W_COSCOS>, grid, block, lds, s, P);
        return launch_with_lds(demigrate_kernel<NW, KS, MERGE, true, W_UNIT>, grid, block, lds, s, P);
    }
    if (P.weight == W_COSCOS) return launch_with_lds(demigrate_kernel<NW, KS, MERGE, false, W_COSCOS>, grid, block, lds, s, P);
    return launch_with_lds(demigrate_kernel<NW, KS, MERGE, false, W_UNIT>, grid, block, lds, s, P);
}

// (waves, depth slots, LDS budget for the trace accumulators, merge same-sample atomics)
#define KM_DEMIGRATE_SHAPES(X) \
    X(16, 8, 131072, true)     \
    X(16, 8, 131072, false)    \
    X(8, 8, 98304, false)      \
    X(12, 16, 131072, false)

static const TileShape kDemigrateShapes[] = {
#define X(nw, ks, lb, mg) {nw, 1, ks, lb},
    KM_DEMIGRATE_SHAPES(X)
#undef X
};

int demigrate_shape_count() { return static_cast<int>(sizeof(kDemigrateShapes) / sizeof(kDemigrateShapes[0])); }
const TileShape& demigrate_shape(int i) { return kDemigrateShapes[i]; }

hipError_t launch_demigrate(int shape, const Params& P, hipStream_t s) {
    int i = 0;
#define X(nw, ks, lb, mg) \
    if (shape == i) return launch_demigrate_shape<nw, ks, mg>(P, s); \
    ++i;
    KM_DEMIGRATE_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace km
