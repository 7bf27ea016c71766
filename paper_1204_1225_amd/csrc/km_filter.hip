// Trace pre-filter: a finite impulse response applied to every trace before
// migration (the rho filter that makes the summation of Eq. (1) return a
// zero-phase wavelet), and its transpose after demigration.
//
//   forward  y[n] = sum_k h[k] x[n + c - k]
//   adjoint  x[m] = sum_k h[k] y[m - c + k]
// (zero outside [0, N)).  Both are correlations out[n] = sum_k w[k] in[n + off + k]:
// forward with the reversed taps and off = c - (K - 1), adjoint with the taps
// and off = -c.
//
// One workgroup per trace at a time: the trace is staged in LDS between K
// zeros on each side, the (possibly reversed) taps next to it; each thread
// produces kOut consecutive outputs from a rotating window of kOut input
// values in registers (slot (k + r) % kOut holds in[n0 + off + k + r]), so a
// tap costs one LDS read of the input and one broadcast read of the tap for
// kOut FMAs.  The trace is fully staged before any output is written, so the
// output may be the input.
#include <algorithm>

#include "km_kernels.h"

namespace km {

constexpr int kFirThreads = 256;
constexpr int kOut = 4;

__global__ __launch_bounds__(kFirThreads) void fir_kernel(const float* in, int64_t in_stride, float* out,
                                                         int64_t out_stride, int64_t n_traces, int n, int K,
                                                         const float* __restrict__ taps, int c, int adjoint) {
    extern __shared__ float fir_lds[];
    float* sW = fir_lds;                 // [K] correlation weights
    float* sIn = fir_lds + ((K + 3) & ~3);  // [n + 2 K]: sIn[K + p] = in[p]
    const int off = adjoint ? -c : c - (K - 1);
    const int tid = threadIdx.x;
    for (int k = tid; k < K; k += kFirThreads) sW[k] = adjoint ? taps[k] : taps[K - 1 - k];
    for (int64_t j = blockIdx.x; j < n_traces; j += gridDim.x) {
        __syncthreads();  // the previous trace's readers are done (and sW is written)
        const float* src = in + j * in_stride;
        for (int p = tid; p < n + 2 * K; p += kFirThreads) {
            const int q = p - K;
            sIn[p] = (q >= 0 && q < n) ? src[q] : 0.0f;
        }
        __syncthreads();
        float* dst = out + j * out_stride;
        for (int n0 = tid * kOut; n0 < n; n0 += kFirThreads * kOut) {
            // sIn[base + k + r] = in[n0 + r + off + k].  An index past the staged row only
            // arises for an output past n or a tap past K (both discarded); it is clamped
            // so that the read stays inside the row.
            const int base = n0 + off + K;
            float acc[kOut], w[kOut];
#pragma unroll
            for (int r = 0; r < kOut; ++r) acc[r] = 0.0f;
#pragma unroll
            for (int m = 0; m < kOut - 1; ++m) w[m] = sIn[min(base + m, n + 2 * K - 1)];
            for (int k0 = 0; k0 < K; k0 += kOut) {
#pragma unroll
                for (int u = 0; u < kOut; ++u) {
                    const int k = k0 + u;
                    w[(u + kOut - 1) % kOut] = sIn[min(base + k + kOut - 1, n + 2 * K - 1)];
                    const float hk = k < K ? sW[min(k, K - 1)] : 0.0f;
#pragma unroll
                    for (int r = 0; r < kOut; ++r) acc[r] = fmaf(hk, w[(u + r) % kOut], acc[r]);
                }
            }
#pragma unroll
            for (int r = 0; r < kOut; ++r)
                if (n0 + r < n) dst[n0 + r] = acc[r];
        }
    }
}

size_t fir_lds_bytes(int n, int K) { return sizeof(float) * (static_cast<size_t>((K + 3) & ~3) + n + 2 * static_cast<size_t>(K)); }

hipError_t launch_fir(const float* in, int64_t in_stride, float* out, int64_t out_stride, int64_t n_traces, int n,
                      const float* taps, int K, int c, int adjoint, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>(n_traces, 256 * 16);
    return launch_with_lds(fir_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kFirThreads), fir_lds_bytes(n, K), s,
                           in, in_stride, out, out_stride, n_traces, n, K, taps, c, adjoint);
}

}  // namespace km
