// In-LDS mixed-radix (2, 3, 4) Stockham FFT for a 256-thread workgroup.
//
// A batch of `nb` transforms of length N (2^a or 3*2^a) sits in LDS at
// buf + b*bstride.  Each stage reads its radix-R butterflies into registers,
// waits at a barrier, then writes the autosorted outputs in place, so one
// buffer suffices.  Twiddles come from a table tw[m] = exp(-2 pi i m / N)
// built in FP64 on the host; the inverse uses their conjugates and is
// unnormalised.  Stage recursion (Ns = product of the radices done so far):
//   in : v_r = x[j + r N/R] * w^(r (j mod Ns))   with w = exp(-2 pi i / (Ns R))
//   out: y[(j div Ns) Ns R + (j mod Ns) + r Ns] = DFT_R(v)_r
// The caller must place a barrier between writing `buf` and calling fft_lds;
// fft_lds ends with a barrier.
#pragma once

#include <hip/hip_runtime.h>

namespace ashrt {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulconj(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cfma(float s, float2 a, float2 acc) {  // acc + s a
  return make_float2(fmaf(s, a.x, acc.x), fmaf(s, a.y, acc.y));
}

// Division by a runtime n of the form 2^s or 3*2^s.
struct Div23 {
  int s;
  int three;
};
__device__ __forceinline__ Div23 make_div23(int n) {
  const int s = __ffs(n) - 1;
  return Div23{s, (n >> s) == 3};
}
__device__ __forceinline__ int div23(int a, Div23 d) {
  const unsigned q = (unsigned)a >> d.s;
  return d.three ? (int)(q / 3u) : (int)q;
}

template <int R, bool INV>
__device__ __forceinline__ void butterfly(float2 (&v)[R]) {
  if constexpr (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const float2 a0 = cadd(v[0], v[2]);
    const float2 a1 = csub(v[0], v[2]);
    const float2 a2 = cadd(v[1], v[3]);
    const float2 d = csub(v[1], v[3]);
    // forward: -i d ; inverse: +i d
    const float2 a3 = INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = cadd(a1, a3);
    v[3] = csub(a1, a3);
  } else if constexpr (R == 3) {
    constexpr float kS = 0.86602540378443864676f;  // sqrt(3)/2
    const float2 t1 = cadd(v[1], v[2]);
    const float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    const float2 d = csub(v[1], v[2]);
    // forward: s = -i (sqrt3/2) d ; inverse: +i (sqrt3/2) d
    const float2 s = INV ? make_float2(-kS * d.y, kS * d.x) : make_float2(kS * d.y, -kS * d.x);
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, s);
    v[2] = csub(t2, s);
  }
}

template <int R, int NT, int MAXB, bool INV>
__device__ __forceinline__ void fft_stage(float2* buf, int N, int nb, int bstride, int Ns,
                                          const float2* __restrict__ tw) {
  const int nbf = N / R;
  const int total = nbf * nb;
  const Div23 dnbf = make_div23(nbf);
  const Div23 dns = make_div23(Ns);
  const int twstep = N / (Ns * R);
  float2 v[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int id = (int)threadIdx.x + i * NT;
    dst[i] = -1;
    if (id < total) {
      const int b = div23(id, dnbf);
      const int j = id - b * nbf;
      const int jq = div23(j, dns);
      const int jm = j - jq * Ns;
      const float2* src = buf + b * bstride + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src[r * nbf];
      if (jm != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[jm * r * twstep];
          if (INV) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      butterfly<R, INV>(v[i]);
      dst[i] = b * bstride + jq * Ns * R + jm;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    if (dst[i] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[i] + r * Ns] = v[i][r];
    }
  }
  __syncthreads();
}

// Batched FFT of nb transforms of length N in LDS; N * nb <= MAXTOT.
template <int NT, int MAXTOT, bool INV>
__device__ void fft_lds(float2* buf, int N, int nb, int bstride, const float2* __restrict__ tw) {
  constexpr int MB4 = (MAXTOT / 4 + NT - 1) / NT;
  constexpr int MB2 = (MAXTOT / 2 + NT - 1) / NT;
  constexpr int MB3 = (MAXTOT / 3 + NT - 1) / NT;
  int Ns = 1;
  const int s2 = __ffs(N) - 1;
  if ((N >> s2) == 3) {
    fft_stage<3, NT, MB3, INV>(buf, N, nb, bstride, Ns, tw);
    Ns = 3;
  }
  int rem = s2;
  while (rem >= 2) {
    fft_stage<4, NT, MB4, INV>(buf, N, nb, bstride, Ns, tw);
    Ns *= 4;
    rem -= 2;
  }
  if (rem == 1) {
    fft_stage<2, NT, MB2, INV>(buf, N, nb, bstride, Ns, tw);
  }
}

}  // namespace ashrt
