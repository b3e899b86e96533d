// Small vector kernels of the learned warm start: statistics of a vector
// pair in FP64, the label weights of the l1 residual, and scaling.
//
// ashrt_vec_stats sums in one 1024-thread workgroup: each thread takes a
// fixed stride of elements, the partial sums combine in a fixed tree, so the
// result does not depend on timing.  Most calls are on one gather's data (a
// few hundred thousand samples); the one call per training run on the
// model-label buffer (~10^9 elements) is slow at one workgroup but rare.
#include "block_reduce.h"
#include "kernels.h"

namespace ashrt {

constexpr int kStatThreads = 1024;

// out[0] = sum |a - alpha b|^p (p = 1 or 2), out[1] = sum a b, out[2] = sum b b;
// b == nullptr is a zero vector.
__global__ __launch_bounds__(kStatThreads) void k_vec_stats(const float* __restrict__ a, const float* __restrict__ b,
                                                            long long n, double alpha, int p, double* out) {
  __shared__ double sh[kStatThreads / 64];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (long long i = threadIdx.x; i < n; i += kStatThreads) {
    const double x = a[i];
    const double y = b ? (double)b[i] : 0.0;
    const double r = x - alpha * y;
    s0 += p == 1 ? fabs(r) : r * r;
    s1 += x * y;
    s2 += y * y;
  }
  const double t0 = block_sum(s0, sh);
  const double t1 = block_sum(s1, sh);
  const double t2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    out[0] = t0;
    out[1] = t1;
    out[2] = t2;
  }
}

// w = sqrt(eps / max(|d - drec|, eps))
__global__ void k_weight_target(const float* __restrict__ d, const float* __restrict__ drec, long long n, float eps,
                                float* __restrict__ w) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float r = fabsf(d[i] - drec[i]);
    w[i] = sqrtf(eps / fmaxf(r, eps));
  }
}

__global__ void k_vec_scale(const float* __restrict__ x, long long n, float s, float* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = s * x[i];
}

static int grid_for(long long n) {
  const long long g = (n + kThreads - 1) / kThreads;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

hipError_t launch_vec_stats(const float* a, const float* b, long long n, double alpha, int p, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_vec_stats, dim3(1), dim3(kStatThreads), 0, s, a, b, n, alpha, p, out);
  return hipGetLastError();
}

hipError_t launch_weight_target(const float* d, const float* drec, long long n, float eps, float* w, hipStream_t s) {
  hipLaunchKernelGGL(k_weight_target, dim3(grid_for(n)), dim3(kThreads), 0, s, d, drec, n, eps, w);
  return hipGetLastError();
}

hipError_t launch_vec_scale(const float* x, long long n, float sc, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_vec_scale, dim3(grid_for(n)), dim3(kThreads), 0, s, x, n, sc, y);
  return hipGetLastError();
}

}  // namespace ashrt
