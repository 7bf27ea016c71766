// Migration kernel: Eq. (1) as an image-stationary gather.
//
// Workgroup = (offset bin b, column tile, depth chunk).  Each wavefront keeps
// CWQ x 4 image columns x (16 * KS) depths of float32 accumulators in
// registers; the traces of bin b stream through LDS in blocks of P.tb rows
// (zero-padded so that every interpolation read stays in its row).  For each
// (column group, trace) the wavefront computes both squared leg lengths once
// and then, slot by slot, every lane evaluates its depth: two square roots,
// the sample index and fraction, a two-sample LDS gather and the weight.
#include "km_kernels.h"

namespace km {

// Stage traces [j0, j0 + nb) of the sorted trace list into LDS rows of
// P.lt floats: row[0] = 0 (lead pad), row[1 + k] = D_j[k], zeros after.
// Rows nb..tb-1 are zero and their geometry is far away.
__device__ __forceinline__ void stage_block(const Params& P, int64_t j0, int nb, float4* sGeo, float* sTr) {
    const int nthr = blockDim.x;
    for (int t = threadIdx.x; t < P.tb; t += nthr) {
        float4 g = make_float4(kFar, kFar, kFar, kFar);
        if (t < nb) {
            const int64_t j = j0 + t;
            g = make_float4(P.src[2 * j], P.src[2 * j + 1], P.rec[2 * j], P.rec[2 * j + 1]);
        }
        sGeo[t] = g;
    }
    for (int t = 0; t < P.tb; ++t) {
        float* row = sTr + static_cast<int64_t>(t) * P.lt;
        if (t < nb) {
            const int64_t j = j0 + t;
            for (int k = threadIdx.x; k < P.lt; k += nthr) {
                const int ks = k - 1;
                row[k] = (ks >= 0 && ks < P.nt) ? load_sample(P, j, ks) : 0.0f;
            }
        } else {
            for (int k = threadIdx.x; k < P.lt; k += nthr) row[k] = 0.0f;
        }
    }
}

template <int NW, int CWQ, int KS, bool TF, int WK>
__device__ __forceinline__ void migrate_tile(const Params& P, int b, int tile, int zc, float* lds) {
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = threadIdx.x / kLanes;
    const int g = lane / kGroup, d = lane % kGroup;
    const int ncol = P.nx * P.ny;
    const int z0 = zc * KS * kGroup;

    DepthTables<KS> T;
    load_tables<KS>(P, z0, d, WK == W_COSCOS, T);

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

    float acc[CWQ][KS];
#pragma unroll
    for (int q = 0; q < CWQ; ++q)
#pragma unroll
        for (int k = 0; k < KS; ++k) acc[q][k] = 0.0f;

    const int64_t lo = lower_bound_bin(P.bin, P.n_traces, b);
    const int64_t hi = lower_bound_bin(P.bin, P.n_traces, b + 1);

    float4* sGeo = reinterpret_cast<float4*>(lds);
    float* sTr = lds + 4 * P.tb;
    const float umax = TF ? static_cast<float>(P.lt - 2) : static_cast<float>(P.lt - 3);
    const float tfs = P.tf_shift;

    // A wavefront whose depth chunk has no valid depth (rmax < 0) still takes
    // part in staging and barriers but skips all evaluation.
    for (int64_t j0 = lo; j0 < hi; j0 += P.tb) {
        const int nb = static_cast<int>(min<int64_t>(P.tb, hi - j0));
        __syncthreads();
        stage_block(P, j0, nb, sGeo, sTr);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < CWQ; ++q) {
            for (int t = 0; t < nb; ++t) {
                const Legs L = legs(px[q], py[q], sGeo[t]);
                if (L.hmax <= T.rmax) {
                    const float* row = sTr + t * P.lt + (TF ? 0 : 1);
#pragma unroll
                    for (int k = 0; k < KS; ++k) {
                        if (L.hmax <= T.R[k]) {
                            const Pair pr = eval_pair<TF, WK>(T.A[k], T.B[k], L.hs2, L.hr2, tfs, umax);
                            const float d0 = row[pr.i];
                            const float d1 = row[pr.i + 1];
                            const float v = fmaf(pr.f, d1 - d0, d0);
                            acc[q][k] = (WK == W_COSCOS) ? fmaf(v, pr.r, acc[q][k]) : acc[q][k] + v;
                        }
                    }
                }
            }
        }
    }

    const int64_t plane = static_cast<int64_t>(ncol) * P.nz;
    float* img = P.image + static_cast<int64_t>(b) * plane;
#pragma unroll
    for (int q = 0; q < CWQ; ++q) {
        if (colv[q] >= ncol) continue;
        float* colp = img + static_cast<int64_t>(colv[q]) * P.nz;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int iz = z0 + k * kGroup + d;
            if (iz < P.nz) {
                const float val = acc[q][k] * depth_factor(P, iz);
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
    const int z0 = zc * KS * kGroup;
    float* img = P.image + static_cast<int64_t>(b) * ncol * P.nz;
#pragma unroll
    for (int q = 0; q < CWQ; ++q) {
        const int col = (tile * NW * CWQ + wave * CWQ + q) * kGroupsPerWave + g;
        if (col >= ncol) continue;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int iz = z0 + k * kGroup + d;
            if (iz < P.nz) img[static_cast<int64_t>(col) * P.nz + iz] = 0.0f;
        }
    }
}

template <int NW, int CWQ, int KS, bool TF, int WK>
__global__ __launch_bounds__(NW * 64) void migrate_kernel(Params P) {
    extern __shared__ float lds[];
    migrate_tile<NW, CWQ, KS, TF, WK>(P, blockIdx.z, blockIdx.x, blockIdx.y, lds);
}

// Batched persistent form: work items (problem, bin, column tile, depth
// chunk) are taken from a queue in list order (longest first).  A negative
// tile field -1 - tile marks an item with no pair in aperture: zero store.
template <int NW, int CWQ, int KS, bool TF, int WK>
__global__ __launch_bounds__(NW * 64) void migrate_batch_kernel(const Params* __restrict__ probs,
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
        else migrate_tile<NW, CWQ, KS, TF, WK>(P, w.y, w.z, w.w, lds);
    }
}

// ---------------------------------------------------------------------------
// Launch tables
// ---------------------------------------------------------------------------

template <int NW, int CWQ, int KS>
static hipError_t launch_migrate_shape(const Params& P, hipStream_t s) {
    dim3 grid(P.n_coltiles, P.n_zchunks, P.n_bins), block(NW * 64);
    const size_t lds = lds_bytes(P);
    if (P.has_tf) {
        if (P.weight == W_COSCOS) return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_COSCOS>, grid, block, lds, s, P);
        return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_UNIT>, grid, block, lds, s, P);
    }
    if (P.weight == W_COSCOS) return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_COSCOS>, grid, block, lds, s, P);
    return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_UNIT>, grid, block, lds, s, P);
}

template <int NW, int CWQ, int KS>
static hipError_t launch_migrate_batch_shape(const Params* probs, const int4* items, int64_t n_items,
                                             unsigned int* counter, int has_tf, int weight, int n_wg, size_t lds,
                                             hipStream_t s) {
    dim3 grid(n_wg), block(NW * 64);
    if (has_tf) {
        if (weight == W_COSCOS)
            return launch_with_lds(migrate_batch_kernel<NW, CWQ, KS, true, W_COSCOS>, grid, block, lds, s, probs, items, n_items, counter);
        return launch_with_lds(migrate_batch_kernel<NW, CWQ, KS, true, W_UNIT>, grid, block, lds, s, probs, items, n_items, counter);
    }
    if (weight == W_COSCOS)
        return launch_with_lds(migrate_batch_kernel<NW, CWQ, KS, false, W_COSCOS>, grid, block, lds, s, probs, items, n_items, counter);
    return launch_with_lds(migrate_batch_kernel<NW, CWQ, KS, false, W_UNIT>, grid, block, lds, s, probs, items, n_items, counter);
}

#define KM_MIGRATE_SHAPES(X) \
    X(4, 4, 16, 65536)       \
    X(4, 2, 16, 65536)       \
    X(8, 2, 16, 98304)       \
    X(4, 4, 8, 49152)

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
                                unsigned int* counter, int has_tf, int weight, int n_wg, size_t lds,
                                hipStream_t s) {
    int i = 0;
#define X(nw, cwq, ks, lb) \
    if (shape == i) return launch_migrate_batch_shape<nw, cwq, ks>(probs, items, n_items, counter, has_tf, weight, n_wg, lds, s); \
    ++i;
    KM_MIGRATE_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

const void* migrate_batch_kernel_ptr(int shape, int has_tf, int weight) {
    int i = 0;
#define X(nw, cwq, ks, lb)                                                                                   \
    if (shape == i) {                                                                                      \
        if (has_tf) return weight == W_COSCOS ? (const void*)migrate_batch_kernel<nw, cwq, ks, true, W_COSCOS> \
                                              : (const void*)migrate_batch_kernel<nw, cwq, ks, true, W_UNIT>;  \
        return weight == W_COSCOS ? (const void*)migrate_batch_kernel<nw, cwq, ks, false, W_COSCOS>          \
                                  : (const void*)migrate_batch_kernel<nw, cwq, ks, false, W_UNIT>;           \
    }                                                                                                      \
    ++i;
    KM_MIGRATE_SHAPES(X)
#undef X
    return nullptr;
}

}  // namespace km
