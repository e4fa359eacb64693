// Vector kernels of the adjoint step through Euler-Maruyama steps: bead
// means, the centre-of-mass projection, dot products and updates of [n][3]
// arrays in ABI order.  Sums run over fixed blocks of 256 beads and are
// combined in a fixed order, so every result is the same bits run to run.
#include "tild_device.h"

namespace tild {

// part[blk][a] = sum over the block's beads of v[3 j + a] (float64).
template <typename TV>
__global__ void __launch_bounds__(256) k_sum3(const TV* __restrict__ v, long long n, double* __restrict__ part) {
    __shared__ double red[3 * 4];
    const long long j = blockIdx.x * 256LL + threadIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    if (j < n)
        for (int a = 0; a < 3; ++a) s[a] = (double)v[3 * j + a];
    block_sum<double, 3>(s, red, threadIdx.x, 256);
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) part[3 * blockIdx.x + a] = s[a];
}

// The partial sums of one reduction, combined in a fixed order by one block of
// kSumBlock threads: thread t adds blocks t, t + kSumBlock, ... in turn, then
// the threads' sums are added by a fixed tree (block_sum).
constexpr int kSumBlock = 256;

// mean[a] = (sum of part[blk][a] over the blocks) / n.
__global__ void __launch_bounds__(kSumBlock) k_mean3(const double* __restrict__ part, int nblk, long long n,
                                                     double* __restrict__ mean) {
    __shared__ double red[3 * (kSumBlock / 64)];
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += kSumBlock)
        for (int a = 0; a < 3; ++a) s[a] += part[3 * b + a];
    block_sum<double, 3>(s, red, threadIdx.x, kSumBlock);
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) mean[a] = n > 0 ? s[a] / (double)n : 0.0;
}

// pl = v - mean (mean may be NULL: pl = v).
template <typename TV>
__global__ void __launch_bounds__(256) k_project3(const TV* __restrict__ v, const double* __restrict__ mean, long long n,
                                                  TV* __restrict__ pl) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= 3 * n) return;
    pl[i] = mean ? (TV)((double)v[i] - mean[i % 3]) : v[i];
}

// part[blk] = sum over the block's beads of a[3 j + k] b[3 j + k] (float64).
template <typename TV>
__global__ void __launch_bounds__(256) k_dot3(const TV* __restrict__ a, const double* __restrict__ b, long long n,
                                              double* __restrict__ part) {
    __shared__ double red[4];
    const long long j = blockIdx.x * 256LL + threadIdx.x;
    double s[1] = {0.0};
    if (j < n)
        for (int k = 0; k < 3; ++k) s[0] += (double)a[3 * j + k] * b[3 * j + k];
    block_sum<double, 1>(s, red, threadIdx.x, 256);
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// acc[0] += scale * (sum of part[blk] over the blocks).
__global__ void __launch_bounds__(kSumBlock) k_add_sum(const double* __restrict__ part, int nblk, double scale,
                                                       double* __restrict__ acc) {
    __shared__ double red[kSumBlock / 64];
    double s[1] = {0.0};
    for (int b = threadIdx.x; b < nblk; b += kSumBlock) s[0] += part[b];
    block_sum<double, 1>(s, red, threadIdx.x, kSumBlock);
    if (threadIdx.x == 0) acc[0] += scale * s[0];
}

// y += alpha x over 3 n values.
template <typename TV>
__global__ void __launch_bounds__(256) k_axpy3(TV* __restrict__ y, const double* __restrict__ x, double alpha,
                                               long long n) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= 3 * n) return;
    y[i] = (TV)((double)y[i] + alpha * x[i]);
}

// v *= alpha over 3 n values.
template <typename TV>
__global__ void __launch_bounds__(256) k_scale3(TV* __restrict__ v, double alpha, long long n) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= 3 * n) return;
    v[i] = (TV)(alpha * (double)v[i]);
}

template <typename TV>
static hipError_t adjoint_vectors(const Launch& L, DeviceState& S, AdjointOp op, void* v, void* w, double alpha,
                                  double* out) {
    const long long n = S.n;
    const unsigned gb = blocks_for(n > 0 ? n : 1, 256), g3 = blocks_for(3 * (n > 0 ? n : 1), 256);
    double* part = S.apart;
    switch (op) {
        case AdjointOp::kMean:  // out[0..2] = mean of v
            hipLaunchKernelGGL(k_sum3<TV>, dim3(gb), dim3(256), 0, L.stream, (const TV*)v, n, part);
            hipLaunchKernelGGL(k_mean3, dim3(1), dim3(kSumBlock), 0, L.stream, (const double*)part, (int)gb, n, out);
            break;
        case AdjointOp::kProject:  // w (TV) = v - out[0..2] (out may be NULL)
            hipLaunchKernelGGL(k_project3<TV>, dim3(g3), dim3(256), 0, L.stream, (const TV*)v, (const double*)out, n,
                               (TV*)w);
            break;
        case AdjointOp::kDotAdd:  // out[0] += alpha v . w (w float64)
            hipLaunchKernelGGL(k_dot3<TV>, dim3(gb), dim3(256), 0, L.stream, (const TV*)v, (const double*)w, n, part);
            hipLaunchKernelGGL(k_add_sum, dim3(1), dim3(kSumBlock), 0, L.stream, (const double*)part, (int)gb, alpha,
                               out);
            break;
        case AdjointOp::kAxpy:  // v += alpha w (w float64)
            hipLaunchKernelGGL(k_axpy3<TV>, dim3(g3), dim3(256), 0, L.stream, (TV*)v, (const double*)w, alpha, n);
            break;
        case AdjointOp::kScale:  // v *= alpha
            hipLaunchKernelGGL(k_scale3<TV>, dim3(g3), dim3(256), 0, L.stream, (TV*)v, alpha, n);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_vectors(const Launch& L, DeviceState& S, AdjointOp op, void* v, void* w, int dtype,
                                  double alpha, double* out) {
    return dtype == 0 ? adjoint_vectors<float>(L, S, op, v, w, alpha, out)
                      : adjoint_vectors<double>(L, S, op, v, w, alpha, out);
}

}  // namespace tild
