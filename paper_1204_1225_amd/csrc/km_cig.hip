// Offset stack and the moveout measure of the offset images (the redundant
// images of the Introduction: their disagreement in reflector depth measures
// the velocity error; once they agree they are summed).
//
// stack_kernel   stack[p] = sum_b image[b][p]: one pass over the image, float4
//                when aligned; HBM-bound.
// cig_kernel     one workgroup per image column: the column's n_bins depth
//                vectors are staged in LDS (zero-padded by max_lag on both
//                sides), the stack is formed in float64, every (bin, lag)
//                correlation over the depth window is a float64 dot product
//                of LDS rows, then one thread per bin picks the best lag (ties
//                to the smaller |lag|, then the negative one) and refines it
//                by the parabola through its neighbours; thread 0 fits the
//                shift against offset^2.
#include <algorithm>

#include "km_kernels.h"

namespace km {

constexpr int kCigThreads = 256;

__global__ __launch_bounds__(256) void stack_kernel(const float* __restrict__ img, int n_bins, int64_t n_points,
                                                    int vec, float* __restrict__ out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (vec) {
        const int64_t n4 = n_points >> 2;
        const float4* in4 = reinterpret_cast<const float4*>(img);
        float4* out4 = reinterpret_cast<float4*>(out);
        for (int64_t i = t0; i < n4; i += stride) {
            float4 s = in4[i];
            for (int b = 1; b < n_bins; ++b) {
                const float4 v = in4[static_cast<int64_t>(b) * n4 + i];
                s.x += v.x;
                s.y += v.y;
                s.z += v.z;
                s.w += v.w;
            }
            out4[i] = s;
        }
    } else {
        for (int64_t i = t0; i < n_points; i += stride) {
            float s = img[i];
            for (int b = 1; b < n_bins; ++b) s += img[static_cast<int64_t>(b) * n_points + i];
            out[i] = s;
        }
    }
}

// LDS of one workgroup (one column): stack [nz] double, correlations
// [n_bins][2 L + 1] double, depth-part partial sums [zs][n_bins][2 L + 1]
// double, shifts and peaks [n_bins] double each, rows [n_bins][rl] float
// with rl = nz + 2 L + 2 kLagBlock (even), zero outside the column.
constexpr int kLagBlock = 5;  // lags per thread in the correlation phase

__host__ __device__ inline int cig_row_len(int nz, int L) { return (nz + 2 * L + 2 * kLagBlock + 1) & ~1; }

__host__ __device__ inline int cig_lag_blocks(int L) { return (2 * L + 1 + kLagBlock - 1) / kLagBlock; }

// depth parts per (bin, lag block) so that the items fill the workgroup
__host__ __device__ inline int cig_depth_parts(int n_bins, int L) {
    const int items = n_bins * cig_lag_blocks(L);
    return items >= kCigThreads ? 1 : kCigThreads / items;
}

__host__ __device__ inline size_t cig_doubles(int n_bins, int nz, int L) {
    const size_t nl = 2 * static_cast<size_t>(L) + 1;
    return static_cast<size_t>(nz) + static_cast<size_t>(n_bins) * nl * (1 + cig_depth_parts(n_bins, L)) +
           2 * static_cast<size_t>(n_bins) + static_cast<size_t>(n_bins) * cig_row_len(nz, L) / 2;
}

// Partial C_b(l) over depths [za, zb) for l = lag0 .. lag0 + kLagBlock - 1:
// a rotating window of the row in registers (slot (u + j) % kLagBlock holds
// row[z + u + lag0 + j]), so each depth step costs one row read, one stack
// read and kLagBlock FMAs.  Steps past zb use a zero stack value.
__device__ __forceinline__ void lag_block(const double* sS, const float* row, int lag0, int za, int zb, double* c) {
    constexpr int LB = kLagBlock;
    double w[LB];
#pragma unroll
    for (int j = 0; j < LB; ++j) c[j] = 0.0;
    if (za >= zb) return;
#pragma unroll
    for (int m = 0; m < LB - 1; ++m) w[m] = static_cast<double>(row[za + lag0 + m]);
    for (int z = za; z < zb; z += LB) {
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            w[(u + LB - 1) % LB] = static_cast<double>(row[z + u + lag0 + LB - 1]);
            const double sv = (z + u < zb) ? sS[z + u] : 0.0;
#pragma unroll
            for (int j = 0; j < LB; ++j) c[j] = fma(sv, w[(u + j) % LB], c[j]);
        }
    }
}

__global__ __launch_bounds__(kCigThreads) void cig_kernel(const float* __restrict__ img, int n_bins, int ny, int nx,
                                                         int nz, int L, int z_lo, int z_hi,
                                                         const float* __restrict__ offsets, float* stack,
                                                         float* shift, float* peak, float* curvature) {
    extern __shared__ double cig_lds[];
    const int nl = 2 * L + 1;
    const int rl = cig_row_len(nz, L);
    const int nblk = cig_lag_blocks(L);
    const int zs = cig_depth_parts(n_bins, L);
    const int items = n_bins * nblk * zs;
    const int zlen = (z_hi - z_lo + zs - 1) / zs;
    double* sS = cig_lds;                                           // [nz]
    double* sC = sS + nz;                                           // [n_bins][nl]
    double* sP = sC + n_bins * nl;                                  // [zs][n_bins][nl]
    double* sShift = sP + static_cast<int64_t>(zs) * n_bins * nl;   // [n_bins]
    double* sPeak = sShift + n_bins;                                // [n_bins]
    float* sRow = reinterpret_cast<float*>(sPeak + n_bins);         // [n_bins][rl]
    const int64_t ncol = static_cast<int64_t>(ny) * nx;
    const int64_t bin_stride = ncol * nz;
    const int tid = threadIdx.x;

    for (int64_t col = blockIdx.x; col < ncol; col += gridDim.x) {
        __syncthreads();  // the previous column's readers are done
        const float* src = img + col * nz;
        for (int b = 0; b < n_bins; ++b) {
            float* dst = sRow + b * rl;
            for (int r = tid; r < rl; r += kCigThreads) {
                const int k = r - L;
                dst[r] = (k >= 0 && k < nz) ? src[b * bin_stride + k] : 0.0f;
            }
        }
        __syncthreads();
        for (int z = tid; z < nz; z += kCigThreads) {
            double s = 0.0;
            for (int b = 0; b < n_bins; ++b) s += static_cast<double>(sRow[b * rl + L + z]);
            sS[z] = s;
            if (stack) stack[col * nz + z] = static_cast<float>(s);
        }
        __syncthreads();
        for (int it = tid; it < items; it += kCigThreads) {
            const int part = it % zs, rest = it / zs;
            const int b = rest / nblk, blk = rest % nblk;
            const int lag0 = -L + blk * kLagBlock;
            const int za = z_lo + part * zlen, zb = min(z_hi, za + zlen);
            double cc[kLagBlock];
            lag_block(sS, sRow + b * rl + L, lag0, za, zb, cc);
            double* out = sP + (static_cast<int64_t>(part) * n_bins + b) * nl + lag0 + L;
#pragma unroll
            for (int j = 0; j < kLagBlock; ++j)
                if (lag0 + j <= L) out[j] = cc[j];
        }
        __syncthreads();
        for (int w = tid; w < n_bins * nl; w += kCigThreads) {
            double c = 0.0;
            for (int part = 0; part < zs; ++part) c += sP[static_cast<int64_t>(part) * n_bins * nl + w];
            sC[w] = c;
        }
        __syncthreads();
        for (int b = tid; b < n_bins; b += kCigThreads) {
            const double* c = sC + b * nl + L;  // c[lag]
            int best = 0;
            for (int m = 1; m <= L; ++m) {
                if (c[-m] > c[best]) best = -m;
                if (c[m] > c[best]) best = m;
            }
            double sh = best;
            if (best > -L && best < L) {
                const double cm = c[best - 1], c0 = c[best], cp = c[best + 1];
                const double den = cm - 2.0 * c0 + cp;
                if (den < 0.0) sh = best + 0.5 * (cm - cp) / den;
            }
            sShift[b] = sh;
            sPeak[b] = c[best];
            shift[b * ncol + col] = static_cast<float>(sh);
            if (peak) peak[b * ncol + col] = static_cast<float>(c[best]);
        }
        __syncthreads();
        if (curvature && tid == 0) {
            int n = 0;
            double mq = 0.0, ms = 0.0;
            for (int b = 0; b < n_bins; ++b) {
                if (sPeak[b] > 0.0) {
                    const double h = offsets[b];
                    mq += h * h;
                    ms += sShift[b];
                    ++n;
                }
            }
            double g = 0.0;
            if (n >= 2) {
                mq /= n;
                ms /= n;
                double num = 0.0, den = 0.0;
                for (int b = 0; b < n_bins; ++b) {
                    if (sPeak[b] > 0.0) {
                        const double h = offsets[b];
                        const double dq = h * h - mq;
                        num += dq * (sShift[b] - ms);
                        den += dq * dq;
                    }
                }
                if (den > 0.0) g = num / den;
            }
            curvature[col] = static_cast<float>(g);
        }
    }
}

size_t cig_lds_bytes(int n_bins, int nz, int max_lag) { return sizeof(double) * cig_doubles(n_bins, nz, max_lag); }

hipError_t launch_stack(const float* img, int n_bins, int64_t n_points, float* out, hipStream_t s) {
    const int vec = (n_points % 4 == 0) && (reinterpret_cast<uintptr_t>(img) % 16 == 0) &&
                    (reinterpret_cast<uintptr_t>(out) % 16 == 0);
    const int64_t work = vec ? n_points / 4 : n_points;
    const int64_t blocks = std::min<int64_t>((work + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(stack_kernel, dim3(static_cast<unsigned>(std::max<int64_t>(blocks, 1))), dim3(256), 0, s,
                       img, n_bins, n_points, vec, out);
    return hipGetLastError();
}

hipError_t launch_cig(const float* img, int n_bins, int ny, int nx, int nz, int max_lag, int z_lo, int z_hi,
                      const float* offsets, float* stack, float* shift, float* peak, float* curvature,
                      hipStream_t s) {
    const int64_t ncol = static_cast<int64_t>(ny) * nx;
    const int64_t blocks = std::min<int64_t>(ncol, 1 << 20);
    return launch_with_lds(cig_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kCigThreads),
                           cig_lds_bytes(n_bins, nz, max_lag), s, img, n_bins, ny, nx, nz, max_lag, z_lo, z_hi,
                           offsets, stack, shift, peak, curvature);
}

}  // namespace km
