// Numerical blending and pseudo-deblending of a multi-source survey (thesis
// Chapter 2, equations ch2_blending and pseudodeblending_equ), and the
// source <-> receiver re-sort of a cube.
//
// Blending:  b[r][tau] = sum_s D[s][r][tau - T_s]  (0 <= tau - T_s < nt),
// written as a gather (one thread per record sample, no atomics);
// pseudo-deblending (its adjoint): D~[s][r][t] = b[r][T_s + t], written in
// either the source-major [s][r][t] or the receiver-major [r][s][t] order
// (the latter is the batch of common receiver gathers the separation
// consumes, so no separate sort is needed).
#include "kernels.h"

namespace ashrt {

__global__ __launch_bounds__(256) void k_blend(const float* __restrict__ D, int ns, int nr, int nt,
                                              const int* __restrict__ fire, float* __restrict__ b, int nrec) {
  const long long n = (long long)nr * nrec;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int tau = (int)(i % nrec), r = (int)(i / nrec);
    float acc = 0.f;
    for (int s = 0; s < ns; ++s) {
      const int t = tau - fire[s];
      if (t >= 0 && t < nt) acc += D[((long long)s * nr + r) * nt + t];
    }
    b[i] = acc;
  }
}

__global__ __launch_bounds__(256) void k_deblend(const float* __restrict__ b, int ns, int nr, int nt,
                                                const int* __restrict__ fire, int nrec, float* __restrict__ out,
                                                int receiver_major) {
  const long long n = (long long)ns * nr * nt;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(i % nt);
    const long long q = i / nt;
    int s, r;
    if (receiver_major) {
      s = (int)(q % ns);
      r = (int)(q / ns);
    } else {
      r = (int)(q % nr);
      s = (int)(q / nr);
    }
    const int tau = fire[s] + t;
    out[i] = (tau >= 0 && tau < nrec) ? b[(long long)r * nrec + tau] : 0.f;
  }
}

__global__ __launch_bounds__(256) void k_resort(const float* __restrict__ in, int na, int nb, int nt,
                                               float* __restrict__ out) {
  const long long n = (long long)na * nb * nt;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(i % nt);
    const long long q = i / nt;
    const int a = (int)(q % na), bb = (int)(q / na);  // out[bb][a][t] = in[a][bb][t]
    out[i] = in[((long long)a * nb + bb) * nt + t];
  }
}

static unsigned grid_of(long long n) {
  long long g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

hipError_t launch_blend(const float* D, int ns, int nr, int nt, const int* fire, float* b, int nrec, hipStream_t s) {
  hipLaunchKernelGGL(k_blend, dim3(grid_of((long long)nr * nrec)), dim3(256), 0, s, D, ns, nr, nt, fire, b, nrec);
  return hipGetLastError();
}

hipError_t launch_deblend(const float* b, int ns, int nr, int nt, const int* fire, int nrec, float* out, int rmaj,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_deblend, dim3(grid_of((long long)ns * nr * nt)), dim3(256), 0, s, b, ns, nr, nt, fire, nrec,
                     out, rmaj);
  return hipGetLastError();
}

hipError_t launch_resort(const float* in, int na, int nb, int nt, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_resort, dim3(grid_of((long long)na * nb * nt)), dim3(256), 0, s, in, na, nb, nt, out);
  return hipGetLastError();
}

}  // namespace ashrt
