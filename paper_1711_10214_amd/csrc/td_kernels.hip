// Time-domain (classical) ASHRT / AASHRT operator pair, the O(P nx^2 nt)
// reference the Stolt operator is compared against (thesis Chapter 3, the
// ASHRT and AASHRT rows of the Radon-operator table; Chapter 6, equations
// ch6_AASHRT_forward and ch6_AASHRT_adjoint; Chapter 5's speed comparison).
//
// A model sample at apex time tau (samples), apex trace xa and panel p lies
// on the data curve T = n0_p + sqrt(tau^2 + (x - xa)^2 q_p), q_p =
// (dx / (v_p dt))^2, read with linear interpolation: the adjoint gathers
// m[p][xa][tau] = sum_x (1 - f) d[x][i0] + f d[x][i0 + 1] (i0 = floor T,
// f = T - i0, samples outside [0, nt) dropped); the forward is its exact
// transpose written as a gather: d[x][t] = sum_{p, xa, tau} hat(T - t)
// m[p][xa][tau] with hat(s) = max(0, 1 - |s|), over the tau whose curve
// passes within one sample of t (found from the inverse of T).  T is FP64
// (its fractional part is the interpolation weight); sums are FP32.  No
// atomics: every output is owned by one thread.
#include "kernels.h"

namespace ashrt {

// (dx / (v dt))^2 from the panel's Stolt bin scale c2 = (v ntp dt / (nxp dx))^2
// (0 for v = 0, which restricts the curve to its apex trace).
__device__ __forceinline__ double td_q(const PanelDev& P, const GatherDev& G) {
  if (P.c2 <= 0.0) return -1.0;
  const double r = (double)G.ntp / (double)G.nxp;
  return r * r / P.c2;
}

__device__ __forceinline__ bool td_h2(double q, int dxa, double* h2) {
  if (q < 0.0) {  // v = 0: only the apex trace
    *h2 = 0.0;
    return dxa == 0;
  }
  *h2 = (double)dxa * (double)dxa * q;
  return true;
}

// Adjoint: one thread per model sample (p, xa, tau); loops over the traces.
__global__ __launch_bounds__(256) void k_td_adjoint(TdArgs A) {
  const GatherDev G = A.gd[0];
  const int nt = G.nt, nx = G.nx;
  const long long n = (long long)G.npanel * nx * nt;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int tau = (int)(i % nt);
    const long long r = i / nt;
    const int xa = (int)(r % nx), p = (int)(r / nx);
    const PanelDev P = A.panels[G.panel_off + p];
    const double q = td_q(P, G);
    const double t2 = (double)tau * (double)tau;
    float acc = 0.f;
    for (int x = 0; x < nx; ++x) {
      if (A.tmask && A.tmask[x] == 0) continue;
      double h2;
      if (!td_h2(q, x - xa, &h2)) continue;
      const double T = (double)P.n0 + sqrt(t2 + h2);
      const double fl = floor(T);
      if (fl >= (double)nt) continue;
      const int i0 = (int)fl;
      const float f = (float)(T - fl);
      const float* dr = A.d + (long long)x * nt;
      if (i0 >= 0) acc = fmaf(1.f - f, dr[i0], acc);
      if (i0 + 1 >= 0 && i0 + 1 < nt) acc = fmaf(f, dr[i0 + 1], acc);
    }
    A.m[i] = acc;
  }
}

// Forward: one thread per data sample (x, t); loops over panels, apexes and
// the apex times whose curve passes within one sample of t.
__global__ __launch_bounds__(256) void k_td_forward(TdArgs A) {
  const GatherDev G = A.gd[0];
  const int nt = G.nt, nx = G.nx;
  const long long n = (long long)nx * nt;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(i % nt), x = (int)(i / nt);
    float acc = 0.f;
    if (!(A.tmask && A.tmask[x] == 0)) {
      for (int p = 0; p < G.npanel; ++p) {
        const PanelDev P = A.panels[G.panel_off + p];
        const double q = td_q(P, G);
        const double s1 = (double)(t - 1 - P.n0), s2 = (double)(t + 1 - P.n0);
        if (s2 <= 0.0) continue;
        const float* mp = A.m + (long long)p * nx * nt;
        for (int xa = 0; xa < nx; ++xa) {
          double h2;
          if (!td_h2(q, x - xa, &h2)) continue;
          if (s2 * s2 <= h2) continue;  // the curve starts after t + 1
          // tau range whose T lies in (t - 1, t + 1), widened by one sample
          const int lo = (s1 > 0.0 && s1 * s1 > h2) ? max(0, (int)floor(sqrt(s1 * s1 - h2)) - 1) : 0;
          const int hi = min(nt - 1, (int)ceil(sqrt(s2 * s2 - h2)) + 1);
          const float* mr = mp + (long long)xa * nt;
          for (int tau = lo; tau <= hi; ++tau) {
            const double T = (double)P.n0 + sqrt((double)tau * (double)tau + h2);
            const double w = 1.0 - fabs(T - (double)t);
            if (w > 0.0) acc = fmaf((float)w, mr[tau], acc);
          }
        }
      }
    }
    A.d[i] = acc;
  }
}

hipError_t launch_td(const TdArgs& a, bool forward, hipStream_t s) {
  const long long n = a.n_out;
  long long g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  if (forward) hipLaunchKernelGGL(k_td_forward, dim3((unsigned)g), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_td_adjoint, dim3((unsigned)g), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace ashrt
