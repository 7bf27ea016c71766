// Internal interface between the C ABI (km_api.cpp) and the kernel files.
#pragma once

#include "km_device.h"

namespace km {

// One compiled tile shape.  lds_budget bounds the bytes of LDS a workgroup
// spends on its trace block (migrate) or trace accumulators (demigrate).
struct TileShape {
    int waves;          // wavefronts per workgroup
    int column_groups;  // groups of 4 columns per wavefront (migrate); unused by demigrate
    int depth_slots;    // KS: 16-depth slots per lane
    int lds_budget;
    int max_quads;      // demigrate: at most 4 * max_quads traces per workgroup (0: no cap)
};

// Launch with `lds` bytes of dynamic LDS (raising the kernel's limit first
// when more than the default 64 KiB is requested).
template <typename Kernel, typename... Args>
inline hipError_t launch_with_lds(Kernel kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, Args... args) {
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    return hipGetLastError();
}

// LDS of a migrate workgroup: the staged time windows (cap floats), per
// block slot the trace geometry and window record (8 words), the chunk's
// aperture table (16 * ks floats), the column tile's bounding box (4 floats
// per wavefront, at most 16 wavefronts), one pass's candidates (6 words
// each, at most 64) and the anti-alias table 1 / n^2.
constexpr int kBoxFloats = 64;
constexpr int kCandMax = 64;
inline size_t migrate_lds_words(int cap, int tb, int ks) {
    return static_cast<size_t>(cap) + static_cast<size_t>(8) * tb + static_cast<size_t>(16) * ks + kBoxFloats +
           static_cast<size_t>(6) * kCandMax + ((kAAMaxHalf + 2 + 3) & ~3);
}
inline size_t lds_bytes(const Params& P, int ks) { return migrate_lds_words(P.cap, P.tb, ks) * sizeof(float); }

// Demigrate workgroups keep their rows as float64 next to the staged geometry
// (and the anti-alias table 1 / n^2).
inline size_t lds_bytes_f64rows(const Params& P) {
    return (static_cast<size_t>(4) * P.tb + static_cast<size_t>(2) * P.tb * P.lt + ((kAAMaxHalf + 2 + 3) & ~3)) *
           sizeof(float);
}

// migrate (km_migrate.hip)
int migrate_shape_count();
const TileShape& migrate_shape(int i);
hipError_t launch_migrate(int shape, const Params& P, hipStream_t s);
hipError_t launch_migrate_batch(int shape, const Params* probs, const int4* items, int64_t n_items,
                                unsigned int* counter, int has_tf, int weight, int prec, int n_wg, size_t lds,
                                hipStream_t s);
const void* migrate_batch_kernel_ptr(int shape, int has_tf, int weight, int prec);

// demigrate (km_demigrate.hip)
int demigrate_shape_count();
const TileShape& demigrate_shape(int i);
hipError_t launch_demigrate(int shape, const Params& P, hipStream_t s);

// offset stack and moveout (km_cig.hip)
size_t cig_lds_bytes(int n_bins, int nz, int max_lag);
hipError_t launch_stack(const float* img, int n_bins, int64_t n_points, float* out, hipStream_t s);
hipError_t launch_cig(const float* img, int n_bins, int ny, int nx, int nz, int max_lag, int z_lo, int z_hi,
                      const float* offsets, float* stack, float* shift, float* peak, float* curvature,
                      hipStream_t s);

// trace pre-filter (km_filter.hip)
size_t fir_lds_bytes(int n, int K);
hipError_t launch_fir(const float* in, int64_t in_stride, float* out, int64_t out_stride, int64_t n_traces, int n,
                      const float* taps, int K, int c, int adjoint, hipStream_t s);

// counting, reductions, probes (km_misc.hip)
hipError_t launch_count(const Params& P, unsigned long long* counts, hipStream_t s);
hipError_t launch_dot_f64(const float* a, const float* b, int64_t n, double* out, hipStream_t s);
hipError_t launch_axpby(float alpha, const float* x, float beta, float* y, int64_t n, hipStream_t s);
hipError_t launch_item_costs(const Params& P, int shape_ks, int cols_per_tile, unsigned long long* costs,
                             hipStream_t s);
hipError_t launch_reset_counter(unsigned int* counter, hipStream_t s);
hipError_t launch_probe(int kind, int n_waves, int iters, float* sink, hipStream_t s);

}  // namespace km
