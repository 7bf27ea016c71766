// Counting (Eq. (2) pair counts and per-work-item costs), float64 reductions,
// the axpby update used by least-squares migration, the queue reset of the
// batched launch and the issue-rate probe.
#include "km_kernels.h"

namespace km {

// ---------------------------------------------------------------------------
// Pair counts.  Same lane layout as migration (4 column groups x 16 depths per
// wavefront slot); the aperture decision is the kernels' float32 one.
// Grid (column tiles, depth chunks, bins); tile = cpt columns, chunk = 16 ks
// depths.  counts (optional) gets the totals, costs (optional) one in-aperture
// count per workgroup at ((bin * n_zchunks + zchunk) * n_coltiles + tile).
// ---------------------------------------------------------------------------
constexpr int kCountWaves = 4;

__global__ __launch_bounds__(kCountWaves * 64) void count_kernel(Params P, int cpt, int ks,
                                                                 unsigned long long* counts,
                                                                 unsigned long long* costs) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x / 64;
    const int g = lane / kGroup, d = lane % kGroup;
    const int b = blockIdx.z, zc = blockIdx.y, tile = blockIdx.x;
    const int ncol = P.nx * P.ny;
    const int z0 = chunk_z0<false>(P.nz, zc, gridDim.y, ks * kGroup);
    const int64_t lo = lower_bound_bin(P.bin, P.n_traces, b);
    const int64_t hi = lower_bound_bin(P.bin, P.n_traces, b + 1);
    const float tfu = P.has_tf ? static_cast<float>(kLead) - P.tf_off : 0.0f;  // t_first / dt
    constexpr int kMaxSlots = 16;  // host guarantees ks <= kMaxSlots
    float Rk[kMaxSlots], Ak[kMaxSlots], Bk[kMaxSlots];
    float rmax = -1.0f;
#pragma unroll
    for (int k = 0; k < kMaxSlots; ++k) {
        const int iz = z0 + k * kGroup + d;
        Rk[k] = -1.0f;
        Ak[k] = 1.0f;
        Bk[k] = 0.0f;
        if (k < ks && iz >= 0 && iz < P.nz) {
            Rk[k] = P.r2[iz];
            Ak[k] = static_cast<float>(static_cast<double>(P.t0sq[iz]) * P.inv_dt2);
            Bk[k] = static_cast<float>(static_cast<double>(P.s2[iz]) * P.inv_dt2);
        }
        rmax = fmaxf(rmax, Rk[k]);
    }
    unsigned long long na = 0, ne = 0;
    for (int cg = wave; cg * kGroupsPerWave < cpt; cg += kCountWaves) {
        const int col = tile * cpt + cg * kGroupsPerWave + g;
        const bool valid = cg * kGroupsPerWave + g < cpt && col < ncol;
        const float px = valid ? P.x[col % P.nx] : kFar;
        const float py = valid ? P.y[col / P.nx] : kFar;
        for (int64_t j = lo; j < hi; ++j) {
            const float4 sr = make_float4(P.src[2 * j], P.src[2 * j + 1], P.rec[2 * j], P.rec[2 * j + 1]);
            const Legs L = legs(px, py, sr);
            if (!(L.hmax <= rmax)) continue;
#pragma unroll
            for (int k = 0; k < kMaxSlots; ++k) {
                if (L.hmax <= Rk[k]) {
                    ++na;
                    if (counts) {
                        const float u = __builtin_amdgcn_sqrtf(fmaf(Bk[k], L.hs2, Ak[k])) +
                                        __builtin_amdgcn_sqrtf(fmaf(Bk[k], L.hr2, Ak[k])) - tfu;
                        if (u > -1.0f && u < static_cast<float>(P.nt)) ++ne;
                    }
                }
            }
        }
    }
    // workgroup reduction through LDS
    __shared__ unsigned long long s_na[kCountWaves * 64], s_ne[kCountWaves * 64];
    s_na[threadIdx.x] = na;
    s_ne[threadIdx.x] = ne;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s_na[threadIdx.x] += s_na[threadIdx.x + off];
            s_ne[threadIdx.x] += s_ne[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (counts) {
            atomicAdd(&counts[0], s_na[0]);
            atomicAdd(&counts[1], s_ne[0]);
        }
        if (costs) {
            const int64_t slot = (static_cast<int64_t>(b) * gridDim.y + zc) * gridDim.x + tile;
            costs[slot] = s_na[0];
        }
    }
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_count(const Params& P, unsigned long long* counts, hipStream_t s) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, counts, 2);
    const int cpt = 64, ks = 16;
    const int ncol = P.nx * P.ny;
    dim3 grid((ncol + cpt - 1) / cpt, (P.nz + ks * kGroup - 1) / (ks * kGroup), P.n_bins);
    if (grid.x && grid.y && grid.z)
        hipLaunchKernelGGL(count_kernel, grid, dim3(kCountWaves * 64), 0, s, P, cpt, ks, counts, nullptr);
    return hipGetLastError();
}

hipError_t launch_item_costs(const Params& P, int shape_ks, int cols_per_tile, unsigned long long* costs,
                             hipStream_t s) {
    dim3 grid(P.n_coltiles, P.n_zchunks, P.n_bins);
    if (grid.x && grid.y && grid.z)
        hipLaunchKernelGGL(count_kernel, grid, dim3(kCountWaves * 64), 0, s, P, cols_per_tile, shape_ks, nullptr,
                           costs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// float64 dot product of float32 vectors
// ---------------------------------------------------------------------------
__global__ void zero_f64_kernel(double* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0.0;
}

__global__ __launch_bounds__(256) void dot_f64_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                      int64_t n, double* out) {
    double acc = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        acc += static_cast<double>(a[i]) * static_cast<double>(b[i]);
    __shared__ double s[256];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, s[0]);
}

hipError_t launch_dot_f64(const float* a, const float* b, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(zero_f64_kernel, dim3(1), dim3(64), 0, s, out);
    if (n > 0) {
        const int64_t want = (n + 255) / 256;
        const int blocks = static_cast<int>(want < 4096 ? want : 4096);
        hipLaunchKernelGGL(dot_f64_kernel, dim3(blocks), dim3(256), 0, s, a, b, n, out);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// y = alpha x + beta y
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void axpby_kernel(float alpha, const float* x, float beta, float* y, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        y[i] = beta == 0.0f ? alpha * x[i] : fmaf(alpha, x[i], beta * y[i]);
}

hipError_t launch_axpby(float alpha, const float* x, float beta, float* y, int64_t n, hipStream_t s) {
    if (n > 0) {
        const int64_t want = (n + 255) / 256;
        const int blocks = static_cast<int>(want < 8192 ? want : 8192);
        hipLaunchKernelGGL(axpby_kernel, dim3(blocks), dim3(256), 0, s, alpha, x, beta, y, n);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Queue reset for the batched launch (a kernel, so that it can sit in a graph).
// ---------------------------------------------------------------------------
__global__ void reset_counter_kernel(unsigned int* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0u;
}

hipError_t launch_reset_counter(unsigned int* counter, hipStream_t s) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Issue-rate probe: 8 independent chains per lane of one instruction kind.
// ---------------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(256) void probe_kernel(int iters, float* sink) {
    float v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = 1.0f + 1e-3f * (threadIdx.x + c);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (KIND == 0) v[c] = fmaf(v[c], 0.999999f, 1e-7f);
            else if (KIND == 1) v[c] = __builtin_amdgcn_sqrtf(v[c]);
            else v[c] = __builtin_amdgcn_rcpf(v[c]);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += v[c];
    if (s == 12345.678f) sink[threadIdx.x] = s;
}

hipError_t launch_probe(int kind, int n_waves, int iters, float* sink, hipStream_t s) {
    const int blocks = (n_waves + 3) / 4;
    if (kind == 0) hipLaunchKernelGGL(probe_kernel<0>, dim3(blocks), dim3(256), 0, s, iters, sink);
    else if (kind == 1) hipLaunchKernelGGL(probe_kernel<1>, dim3(blocks), dim3(256), 0, s, iters, sink);
    else hipLaunchKernelGGL(probe_kernel<2>, dim3(blocks), dim3(256), 0, s, iters, sink);
    return hipGetLastError();
}

}  // namespace km
