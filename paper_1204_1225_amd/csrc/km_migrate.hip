// Migration kernel: Eq. (1) as an image-stationary gather.
//
// Workgroup = (offset bin b, column tile, depth chunk).  Each wavefront keeps
// CWQ groups of 4 image columns x (16 * KS) depths of float32 accumulators
// in registers; the traces of bin b stream through LDS in blocks of P.tb
// zero-padded rows.  For every column group the wavefront computes the two
// squared leg lengths of 16 traces at once (lane = (column, trace)), hands
// them to the depth lanes through the LDS crossbar, derives from a ballot
// which 16-depth slots can hold a pair inside the aperture, and evaluates
// those slots two at a time: per lane two square roots, the sample index and
// fraction, a two-sample LDS gather, the interpolation, the weight and the
// lane's aperture mask.
#include "km_kernels.h"

namespace km {

// Stage traces [j0, j0 + nb) of the sorted list into rows 0..tb-1 (rows past
// nb are zero with far-away geometry).
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
            stage_row(P, j0 + t, row, threadIdx.x, nthr);
        } else {
            float4* row4 = reinterpret_cast<float4*>(row);
            for (int m = threadIdx.x; m < (P.lt >> 2); m += nthr) row4[m] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

// Two slots (k, k + 1) of one (column group, trace) pairing.  MASKED: some
// valid lane may be outside the aperture, so each value is kept only where
// hmax <= the lane's aperture value; CLAMP: the time is clamped to the row.
// R0, R1: the lanes' aperture values of the two slots (read only when MASKED).
template <bool TF, int WK, bool MASKED, bool CLAMP>
__device__ __forceinline__ void mig_pair(float A0, float B0, float A1, float B1, float hs2, float hr2, float hm,
                                         const float* row, float tfo, float wlo, float whi, float R0, float R1,
                                         float& acc0, float& acc1) {
    const Pair p0 = eval_pair<TF, WK, CLAMP>(A0, B0, hs2, hr2, tfo, wlo, whi);
    const Pair p1 = eval_pair<TF, WK, CLAMP>(A1, B1, hs2, hr2, tfo, wlo, whi);
    const float a0 = row[p0.i], b0 = row[p0.i + 1];
    const float a1 = row[p1.i], b1 = row[p1.i + 1];
    float v0 = fmaf(p0.f, b0 - a0, a0);
    float v1 = fmaf(p1.f, b1 - a1, a1);
    if (MASKED) {
        v0 = (hm <= R0) ? v0 : 0.0f;
        v1 = (hm <= R1) ? v1 : 0.0f;
    }
    acc0 = (WK == W_COSCOS) ? fmaf(v0, p0.r, acc0) : acc0 + v0;
    acc1 = (WK == W_COSCOS) ? fmaf(v1, p1.r, acc1) : acc1 + v1;
}

// mig_pair with table traveltimes (W = 1): iz0, iz1 are the lane's depths of
// the two slots, clamped into the table.
template <bool TF, bool MASKED>
__device__ __forceinline__ void mig_pair_table(const Params& P, TLeg Ls, TLeg Lr, int iz0, int iz1, float hm,
                                               const float* row, float tfo, float wlo, float whi, float R0, float R1,
                                               float& acc0, float& acc1) {
    const Pair p0 = eval_pair_table<TF>(P, Ls, Lr, iz0, tfo, wlo, whi);
    const Pair p1 = eval_pair_table<TF>(P, Ls, Lr, iz1, tfo, wlo, whi);
    const float a0 = row[p0.i], b0 = row[p0.i + 1];
    const float a1 = row[p1.i], b1 = row[p1.i + 1];
    float v0 = fmaf(p0.f, b0 - a0, a0);
    float v1 = fmaf(p1.f, b1 - a1, a1);
    if (MASKED) {
        v0 = (hm <= R0) ? v0 : 0.0f;
        v1 = (hm <= R1) ? v1 : 0.0f;
    }
    acc0 += v0;
    acc1 += v1;
}

// RREG: the masked slots take the lanes' aperture values from registers
// (else from the LDS copy, which costs fewer registers).
// TT: traveltime kind (TT_TABLE: one-way time table, W = 1).
template <int NW, int CWQ, int KS, bool TF, int WK, bool RREG, int TT = TT_DSR>
__device__ __forceinline__ void migrate_tile(const Params& P, int b, int tile, int zc, float* lds) {
    static_assert(KS % 2 == 0, "slots are evaluated in pairs");
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = threadIdx.x / kLanes;
    const int g = lane / kGroup, d = lane % kGroup;
    const int ncol = P.nx * P.ny;
    const int z0 = zc * KS * kGroup;

    // LDS: rows first, so that a row's lead pad folds into the gather's offset field
    float* sTr = lds;                                                      // [tb][lt]
    float4* sGeo = reinterpret_cast<float4*>(lds + P.tb * P.lt);           // [tb]
    float* sR = lds + P.tb * P.lt + 4 * P.tb;                              // [KS * 16]
    float* sBox = sR + KS * kGroup;                                        // [NW][4]

    ChunkTables<KS> T;
    load_chunk_tables<KS, 1, TT>(P, z0, d, WK == W_COSCOS, T, sR);

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
    float wlo, whi;
    clamp_bounds<TF>(P.lt, wlo, whi);
    const float tfo = P.tf_off;
    const int rowoff = TF ? 0 : kLead;

    // Bounding box of the tile's columns.  A leg longer than sqrt(r2)(1 + 2^-22)
    // from every column cannot pass the float32 aperture test, so a trace whose
    // source or receiver lies farther than that from the box (with a 1e-5
    // margin on the squared radius) has no pair in this tile and depth chunk,
    // and a block of such traces is neither staged nor evaluated.
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
    const float reach = T.rmax * 1.00001f;

    for (int64_t j0 = lo; j0 < hi; j0 += P.tb) {
        const int nb = static_cast<int>(min<int64_t>(P.tb, hi - j0));
        bool live = false;
        if (T.rmax >= 0.0f) {
            for (int t = threadIdx.x; t < nb; t += blockDim.x) {
                const int64_t j = j0 + t;
                live |= !(box_dist2(P.src[2 * j], P.src[2 * j + 1], bx0, bx1, by0, by1) > reach) &&
                        !(box_dist2(P.rec[2 * j], P.rec[2 * j + 1], bx0, bx1, by0, by1) > reach);
            }
        }
        // (also the barrier before the rows of the previous block are overwritten)
        if (!__syncthreads_or(live)) continue;
        stage_block(P, j0, nb, sGeo, sTr);
        __syncthreads();
        for (int t0 = 0; t0 < nb; t0 += kGroup) {
            const int nbt = min(kGroup, nb - t0);
            // lane (g, d): legs of column group member g and trace t0 + d
            const float4 sr = sGeo[min(t0 + d, P.tb - 1)];
#pragma unroll
            for (int q = 0; q < CWQ; ++q) {
                const Legs Lp = legs(px[q], py[q], sr);
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
                float hs2n = lane_read(Lp.hs2, (lane & ~(kGroup - 1)) | t);
                float hr2n = lane_read(Lp.hr2, (lane & ~(kGroup - 1)) | t);
                for (;;) {
                    const int tc = t;
                    const float hs2 = hs2n, hr2 = hr2n;
                    const bool more = live != 0;
                    if (more) {
                        t = __builtin_ctzll(live);
                        live &= live - 1;
                        hs2n = lane_read(Lp.hs2, (lane & ~(kGroup - 1)) | t);
                        hr2n = lane_read(Lp.hr2, (lane & ~(kGroup - 1)) | t);
                    }
                    const float hmin = uniform_read(hmin4, tc);
                    const float hmaxw = uniform_read(hmax4, tc);
                    uint64_t any, full;
                    slot_masks<KS>(T, hmin, hmaxw, any, full);
                    (void)full;
                    if (any && TT == TT_TABLE) {
                        const float hm = fmaxf(hs2, hr2);
                        const float* row = sTr + (t0 + tc) * P.lt + rowoff;
                        const TLeg Ls = table_leg(P, hs2), Lr = table_leg(P, hr2);
#pragma unroll
                        for (int k = 0; k < KS; k += 2) {
                            if ((any >> k) & 3ull) {
                                const int iz0 = min(z0 + k * kGroup + d, P.nz - 1);
                                const int iz1 = min(z0 + (k + 1) * kGroup + d, P.nz - 1);
                                const float R0 = RREG ? T.R[k] : sR[k * kGroup + d];
                                const float R1 = RREG ? T.R[k + 1] : sR[(k + 1) * kGroup + d];
                                mig_pair_table<TF, true>(P, Ls, Lr, iz0, iz1, hm, row, tfo, wlo, whi, R0, R1, acc[q][k],
                                                         acc[q][k + 1]);
                            }
                        }
                    } else if (any) {
                        // Every slot pair goes through the masked, clamped form: one code path
                        // per pair measured faster than separate unmasked / unclamped variants
                        // (their extra branches and code cost more than the masks they save).
                        const float hm = fmaxf(hs2, hr2);
                        const float* row = sTr + (t0 + tc) * P.lt + rowoff;
#pragma unroll
                        for (int k = 0; k < KS; k += 2) {
                            if ((any >> k) & 3ull) {
                                const float R0 = RREG ? T.R[k] : sR[k * kGroup + d];
                                const float R1 = RREG ? T.R[k + 1] : sR[(k + 1) * kGroup + d];
                                mig_pair<TF, WK, true, true>(T.A[k], T.B[k], T.A[k + 1], T.B[k + 1], hs2, hr2, hm, row,
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
            if (iz < P.nz) {
                const float fac = depth_factor(P, iz);
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

template <int NW, int CWQ, int KS, bool TF, int WK, int TT = TT_DSR>
__global__ __launch_bounds__(NW * 64) void migrate_kernel(Params P) {
    extern __shared__ float lds[];
    migrate_tile<NW, CWQ, KS, TF, WK, true, TT>(P, blockIdx.z, blockIdx.x, blockIdx.y, lds);
}

// Batched persistent form: work items (problem, bin, column tile, depth
// chunk) are taken from a queue in list order (longest first).  A negative
// tile field -1 - tile marks an item with no pair in aperture: zero store.
// At least 4 wavefronts per SIMD (<= 128 VGPRs) for the 8-slot shapes, so
// that two 8-wavefront workgroups share a CU as they do in single launches.
template <int NW, int CWQ, int KS, bool TF, int WK>
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
        else migrate_tile<NW, CWQ, KS, TF, WK, false>(P, w.y, w.z, w.w, lds);
    }
}

// ---------------------------------------------------------------------------
// Launch tables
// ---------------------------------------------------------------------------

template <int NW, int CWQ, int KS>
static hipError_t launch_migrate_shape(const Params& P, hipStream_t s) {
    dim3 grid(P.n_coltiles, P.n_zchunks, P.n_bins), block(NW * 64);
    const size_t lds = lds_bytes(P, KS);
    if (P.ttab) {  // table traveltimes: W = 1 (the host rejects other weights)
        if (P.has_tf) return launch_with_lds(migrate_kernel<NW, CWQ, KS, true, W_UNIT, TT_TABLE>, grid, block, lds, s, P);
        return launch_with_lds(migrate_kernel<NW, CWQ, KS, false, W_UNIT, TT_TABLE>, grid, block, lds, s, P);
    }
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
