// HIP kernels of the Stolt (A)ASHRT operator pair for gfx950.
//
// Data flow (the same linear operator as F^-1 M F of the thesis' Chapter 5
// operator factorisation, with the two FFT axes taken in the order that lets
// the Stolt map run in LDS):
//
//   forward  m_p[x][t] --(x-RFFT, per time column)--> X_p[l][t]     (HBM)
//            per wavenumber row l (+ its mirror -l): time FFT of X_p[l][:]
//            in LDS, Stolt map (gather over 2R taps) + phase ramp + scale,
//            accumulated over the panels in LDS --> partial D (HBM)
//            sum of partials, Hermitian completion, inverse time FFT --> H[l][t]
//            x-C2R per time column --> d[x][t] (+ mask, residual, weights)
//   adjoint  the transposes in reverse: x-RFFT of the data, per row a time
//            FFT, the Stolt map's transpose as a gather over the data bins
//            that tap each model bin, inverse time FFT per panel --> G_p[l][t],
//            x-C2R per panel --> m_p[x][t].
//
// Real-signal packing: the x-RFFT transforms two time columns as one complex
// sequence; row l = 0 carries the kx = 0 and kx = Nyquist spectra as the real
// and imaginary parts of one complex time signal; rows l >= 1 produce the
// spectra of +l (bins j) and -l (conjugated bins ntp - j) from one complex
// time FFT.  Only interior bins 1..ntp/2-1 are mapped (Chapter 5: positive
// frequencies, the negative ones by symmetry).
//
// FFT lengths in ASHRT_TPL_SIZES use the compile-time radix-8 Stockham FFT
// with its pass twiddle table staged in LDS; other lengths use the generic
// runtime FFT with the plain table exp(-2 pi i m / N).
#include "block_reduce.h"
#include "fft_tpl.h"
#include "kernels.h"

#include <type_traits>
#include "tap_poly.h"

namespace ashrt {

// ------------------------------------------------------------ interpolation taps
//
// Hann-windowed sinc h(x) = sinc(x) (1/2 + 1/2 cos(pi x / R)), |x| < R, at
// x = delta - t for the 2R taps t = -R+1..R around floor(u).  With
// theta = pi delta / R, sin(pi (delta - t)) = (-1)^t sin(R theta) and
// cos(pi (delta - t) / R) = cos(theta) cos(pi t/R) + sin(theta) sin(pi t/R),
// so one sine/cosine pair of theta per output bin gives all 2R weights.
struct Taps {
  int k0;       // floor(u), or a large negative sentinel outside the cone
  float4 trig;  // (delta, sin(pi delta)/pi, cos(theta), sin(theta))
};

constexpr int kNoTap = -(1 << 28);

// sin and cos on [0, pi/2] by their Taylor series to the x^13 / x^12 terms
// (truncation below 1e-8 there).
__device__ __forceinline__ void sincos_quadrant(float x, float* s, float* c) {
  const float z = x * x;
  float ps = 1.0f / 6227020800.0f;
  ps = fmaf(ps, -z, 1.0f / 39916800.0f);
  ps = fmaf(ps, -z, 1.0f / 362880.0f);
  ps = fmaf(ps, -z, 1.0f / 5040.0f);
  ps = fmaf(ps, -z, 1.0f / 120.0f);
  ps = fmaf(ps, -z, 1.0f / 6.0f);
  ps = fmaf(ps, -z, 1.0f);       // sin x / x
  *s = x * ps;
  float pc = 1.0f / 479001600.0f;
  pc = fmaf(pc, -z, 1.0f / 3628800.0f);
  pc = fmaf(pc, -z, 1.0f / 40320.0f);
  pc = fmaf(pc, -z, 1.0f / 720.0f);
  pc = fmaf(pc, -z, 1.0f / 24.0f);
  pc = fmaf(pc, -z, 0.5f);
  *c = fmaf(pc, -z, 1.0f);
}

// u = sqrt(j^2 - a^2) in FP64 (the coordinate sets the phase of the
// interpolated spectrum, so it must be exact to ~1e-7 bins).
template <int R>
__device__ __forceinline__ Taps make_taps(int j, double a2) {
  Taps T;
  const double jj = (double)j * (double)j;
  if (jj < a2) {
    T.k0 = kNoTap;
    T.trig = make_float4(0.f, 0.f, 1.f, 0.f);
    return T;
  }
  const double u = sqrt(jj - a2);
  const double f = floor(u);
  T.k0 = (int)f;
  const float dl = (float)(u - f);
  constexpr float kPi = 3.14159265358979323846f;
  float st, ct, sR;
  if constexpr (R == 1) {
    sincospif(dl, &st, &ct);
    sR = st;
  } else {
    // window angle theta = pi delta / R <= pi / 2
    sincos_quadrant(dl * (kPi / (float)R), &st, &ct);
    // sin(pi delta) = sin(pi min(delta, 1 - delta)): the reflection is exact
    // in FP32 and keeps the relative accuracy where the sine is small (the
    // sinc divides it by delta - t, which is small there too)
    float s2, c2;
    sincos_quadrant(kPi * fminf(dl, 1.0f - dl), &s2, &c2);
    sR = s2;
  }
  T.trig = make_float4(dl, sR * 0.31830988618379067154f, ct, st);
  return T;
}

// Runtime half-width (generic kernels): same quantities, R not known at
// compile time.
__device__ __forceinline__ Taps make_taps_rt(int j, double a2, int R) {
  Taps T;
  const double jj = (double)j * (double)j;
  if (jj < a2) {
    T.k0 = kNoTap;
    T.trig = make_float4(0.f, 0.f, 1.f, 0.f);
    return T;
  }
  const double u = sqrt(jj - a2);
  const double f = floor(u);
  T.k0 = (int)f;
  const float dl = (float)(u - f);
  float s1, c1, st, ct;
  sincospif(dl, &s1, &c1);
  sincospif(dl / (float)R, &st, &ct);
  T.trig = make_float4(dl, s1 * 0.31830988618379067154f, ct, st);
  return T;
}

// Weight of tap t (k = k0 + t); ct/st = cos/sin(pi t / R).
__device__ __forceinline__ float tap_weight(float4 tr, int t, float ct, float st) {
  const float x = tr.x - (float)t;
  if (x == 0.0f) return 1.0f;
  const float sg = (t & 1) ? -tr.y : tr.y;
  const float win = fmaf(0.5f, fmaf(tr.z, ct, tr.w * st), 0.5f);
  return sg * __builtin_amdgcn_rcpf(x) * win;
}

__device__ __forceinline__ void init_tap_trig(float* ct, float* st, int R) {
  if ((int)threadIdx.x < 2 * R) {
    const int t = (int)threadIdx.x - R + 1;
    ct[threadIdx.x] = (float)cospi((double)t / (double)R);
    st[threadIdx.x] = (float)sinpi((double)t / (double)R);
  }
}

// Smallest j >= 0 with j^2 >= a2 (in FP64, as make_taps tests it): bins
// below it have no taps.
__device__ __forceinline__ int cone_first_bin(double a2) {
  if (!(a2 > 0.0)) return 0;
  int j = (int)ceil(sqrt(a2));
  if (j > 0 && (double)(j - 1) * (double)(j - 1) >= a2) --j;
  if ((double)j * (double)j < a2) ++j;
  return j;
}

// Half-width 4 (the compile-time row kernels): coordinates in FP32 and the
// eight weights from polynomials.
//
// a^2 of a (panel, wavenumber) row as an exact integer part and an FP32
// fraction f, so a row's a^2 is taken as a2i + f (within 3e-8 of the FP64
// value).  For a data bin j in the cone, u^2 = K - f with K = j^2 - a2i an
// exact integer.  k0 = floor(u) is the FP32 root's integer part corrected
// by one where needed, with integer tests (k0^2 <= K - [f > 0] <
// (k0 + 1)^2), so it is exact for this u^2: it rises by at least 1 from one
// bin to the next (u_{j+1} - u_j = (2j+1) / (u_{j+1} + u_j) >= 1), which the
// adjoint's ordered scatter relies on.  delta = (K - k0^2 - f) / (u + k0)
// takes the integer part exactly and the root only in the denominator, so
// it is good to ~1e-7.  Where u^2 lies within the 3e-8 change of a^2 of a
// perfect square, k0 may differ by one from the FP64 floor: the taps then
// shift by one place, and the tap that leaves or enters sits at
// |u - k| = R, where the weight is ~1e-14.
struct RowA2 {
  int i;
  float f;
};

__device__ __forceinline__ RowA2 split_a2(double a2) {
  RowA2 r;
  if (!(a2 < 1073741824.0)) {  // no bin of such a row is in the cone (j < 2^12)
    r.i = 1 << 30;
    r.f = 0.f;
    return r;
  }
  const double f = floor(a2);
  r.i = (int)f;
  r.f = (float)(a2 - f);
  return r;
}

struct Taps4 {
  int k0;       // floor(u): the taps are k0 - 3 .. k0 + 4
  float w[8];   // h(delta - t), t = -3 .. 4
};

// Data bin j (j^2 >= a^2, j < 2^12) of a row: tap base and weights.  The
// weight of tap t is a degree-9 polynomial in z = (2 delta - 1) * scale
// (tap_poly.h); taps t and 1 - t share the even and odd parts.
__device__ __forceinline__ Taps4 taps4(int j, RowA2 a) {
  Taps4 T;
  const int jj = (int)__umul24((unsigned)j, (unsigned)j) - a.i;
  const float u2 = (float)jj - a.f;
  const float u = __builtin_amdgcn_sqrtf(fmaxf(u2, 0.f));
  // exact floor of sqrt(jj - f): k0^2 <= kf < (k0 + 1)^2 with kf = jj - [f > 0]
  const int kf = jj - (a.f > 0.f ? 1 : 0);
  // (no branch: at most one of the two corrections applies)
  int k0 = (int)u;
  const int m0 = (int)__umul24((unsigned)k0, (unsigned)k0);
  k0 += (m0 + 2 * k0 + 1 <= kf ? 1 : 0) - (m0 > kf ? 1 : 0);
  const float rem = (float)(jj - (int)__umul24((unsigned)k0, (unsigned)k0)) - a.f;
  const float dl = rem * __builtin_amdgcn_rcpf(fmaxf(u + (float)k0, 1e-30f));
  const float z = fmaf(2.0f * kTapZScale, dl, -kTapZScale);
  const float z2 = z * z;
  T.k0 = k0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float e = fmaf(kTapEven[q][4], z2, kTapEven[q][3]);
    e = fmaf(e, z2, kTapEven[q][2]);
    e = fmaf(e, z2, kTapEven[q][1]);
    e = fmaf(e, z2, kTapEven[q][0]);
    float o = fmaf(kTapOdd[q][4], z2, kTapOdd[q][3]);
    o = fmaf(o, z2, kTapOdd[q][2]);
    o = fmaf(o, z2, kTapOdd[q][1]);
    o = fmaf(o, z2, kTapOdd[q][0]);
    T.w[4 + q] = fmaf(z, o, e);    // tap t = q + 1
    T.w[3 - q] = fmaf(-z, o, e);   // tap t = -q
  }
  return T;
}

template <int R>
__device__ __forceinline__ Taps taps_of(int j, double a2, int Rrt) {
  if constexpr (R > 0) return make_taps<R>(j, a2);
  else return make_taps_rt(j, a2, Rrt);
}

// Per data bin j of panel p: W_j s_p exp(-2 pi i j n0 / ntp), from the exact
// FFT twiddle table in global memory (the ramp index is reduced with integer
// arithmetic).
__device__ __forceinline__ float2 bin_factor(const GatherDev& G, const PanelDev& P,
                                             const float2* __restrict__ tw,
                                             const float* __restrict__ wav, int j) {
  float2 e = make_float2(1.0f, 0.0f);
  if (P.n0 != 0) e = tw[G.tw_t_off + (int)(((long long)j * P.n0) % G.ntp)];
  float s = P.scale;
  if (G.wav_off >= 0) s *= wav[G.wav_off + j];
  return cscale(e, s);
}

// ------------------------------------------------------------ FFT dispatch
// Copy the twiddles an FFT of length n needs into LDS (pass table for the
// compile-time lengths, plain table otherwise).  No barrier.
template <int N, int NT = kThreads>
__device__ __forceinline__ void stage_twiddles(float2* dst, const float2* __restrict__ tw, int plain_off,
                                               int pass_off, int n) {
  if constexpr (N > 0) {
    constexpr int ntw = FftPlan<N>::twsize();
    for (int i = threadIdx.x; i < ntw; i += NT) dst[i] = tw[pass_off + i];
  } else {
    for (int i = threadIdx.x; i < n; i += NT) dst[i] = tw[plain_off + i];
  }
}

// Batched x-axis FFTs of a tile: nb transforms of length n at stride
// bstride, run in groups of at most kXfftBatch points per call (bounded
// registers).  N > 0: compile-time length; N == 0: generic runtime FFT.
// Compile-time lengths: the forward reads only the nx trace slots (the pad
// to nxp is zero and never filled), the inverse writes only the nx traces.
template <int N, bool INV>
__device__ __forceinline__ void xfft_tile(float2* buf, int n, int nb, int bstride, const float2* twl, int nx) {
  if constexpr (N > 0) {
    static_assert(N <= kXfftBatch, "compile-time x-FFT longer than one batch");
    constexpr int per = kXfftBatch / N;
    for (int b0 = 0; b0 < nb; b0 += per)
      fft_tpl_masked<N, kXfftBatch, INV, !INV, INV>(buf + b0 * bstride, min(per, nb - b0), bstride, twl, nx);
  } else {
    // generic: n <= 4096 = kXfftGenericBatch, so per >= 1
    const int per = max(1, kXfftGenericBatch / n);
    for (int b0 = 0; b0 < nb; b0 += per)
      fft_lds<kThreads, kXfftGenericBatch, INV>(buf + b0 * bstride, n, min(per, nb - b0), bstride, twl);
  }
}

// Division by a workgroup-uniform d >= 1 through a precomputed reciprocal:
// m = floor((2^32 - 1) / d) + 1 gives floor(n / d) = mulhi(n, m) whenever
// n d < 2^32 (the tile loops below stay far inside that: the LDS limit keeps
// tile width times nxp under 2^16).
struct UDiv {
  unsigned m;
  int d;
  __device__ __forceinline__ explicit UDiv(int dd) : m(dd > 1 ? 0xffffffffu / (unsigned)dd + 1u : 0u), d(dd) {}
  __device__ __forceinline__ int div(int n) const { return d == 1 ? n : (int)__umulhi((unsigned)n, m); }
};

// A workgroup-uniform 64-bit value moved to scalar registers (values read
// through vector loads are not known to be uniform), so that addresses built
// from it take a scalar base plus one 32-bit VGPR offset.
__device__ __forceinline__ long long uniform64(long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long long)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
template <class V, class T>
__device__ __forceinline__ V& at_byte(T* base, unsigned off) {
  return *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + off);
}
template <class V, class T>
__device__ __forceinline__ const V& at_byte(const T* base, unsigned off) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + off);
}

// Input of a full model tile (nt even, t0 + T <= nt): the element pairs
// (t, t+1) of the nx columns go to the LDS column pairs.  CG: the previous
// CG iteration's update of the pair (u += ca p, p = g + cb p) comes first
// and the new p is the input; MUL: the input is scaled by mul.  The loads
// of kXLoadBatch loop iterations are issued before any of them is used (one
// iteration at a time leaves a wave with a single load in flight); indices
// past the tile are clamped for the loads and skipped for the stores.
template <int NX, bool CG, bool MUL>
__device__ __forceinline__ void xfwd_model_full_tile(float2* buf, int bs, const UDiv& dh, int half, int nx,
                                                     int nt, int t0, const float* __restrict__ src,
                                                     const float* __restrict__ mul, float* pp, float* uu,
                                                     const float* gg, float ca, float cb) {
  const int nin = nx * half;
  for (int base = threadIdx.x; base < nin; base += kXLoadBatch * kThreads) {
    float2 va[kXLoadBatch], vg[kXLoadBatch], vu[kXLoadBatch], vm[kXLoadBatch];
    unsigned off[kXLoadBatch];  // byte offsets in the panel (4 nx nt < 2^32)
#pragma unroll
    for (int u = 0; u < kXLoadBatch; ++u) {
      const int idx = min(base + u * kThreads, nin - 1);
      const int x = dh.div(idx);
      off[u] = 4u * (unsigned)(x * nt + t0 + 2 * (idx - x * half));
      if constexpr (CG) {
        va[u] = at_byte<float2>(pp, off[u]);
        vg[u] = at_byte<float2>(gg, off[u]);
        vu[u] = at_byte<float2>(uu, off[u]);
      } else {
        va[u] = at_byte<float2>(src, off[u]);
      }
      if constexpr (MUL) vm[u] = at_byte<float2>(mul, off[u]);
    }
#pragma unroll
    for (int u = 0; u < kXLoadBatch; ++u) {
      const int idx = base + u * kThreads;
      if (idx < nin) {
        const int x = dh.div(idx);
        const int i = idx - x * half;
        float2 v = va[u];
        if constexpr (CG) {
          at_byte<float2>(uu, off[u]) = make_float2(fmaf(ca, v.x, vu[u].x), fmaf(ca, v.y, vu[u].y));
          v = make_float2(fmaf(cb, v.x, vg[u].x), fmaf(cb, v.y, vg[u].y));
          at_byte<float2>(pp, off[u]) = v;
        }
        if constexpr (MUL) v = make_float2(v.x * vm[u].x, v.y * vm[u].y);
        buf[i * bs + px<NX>(x)] = v;
      }
    }
  }
}

// Input of a full data tile (nt even, t0 + T <= nt), loads batched as in
// xfwd_model_full_tile.  SCG: the CG step s -= alpha q first (s is written
// back) and the new s is the input; MUL: times mul; traces with tm[x] == 0
// (tm non-null) give zero.
template <int NX, bool SCG, bool MUL>
__device__ __forceinline__ void xfwd_data_full_tile(float2* buf, int bs, const UDiv& dh, int half, int nx,
                                                    int nt, int t0, const float* __restrict__ src,
                                                    const float* __restrict__ mul,
                                                    const uint8_t* __restrict__ tm, float* sv,
                                                    const float* qv, float alpha) {
  const int nin = nx * half;
  for (int base = threadIdx.x; base < nin; base += kXLoadBatch * kThreads) {
    float2 va[kXLoadBatch], vq[kXLoadBatch], vm[kXLoadBatch];
    int live[kXLoadBatch];  // trace index, then its mask byte
    unsigned off[kXLoadBatch];  // byte offsets in the gather (4 nx nt < 2^32)
#pragma unroll
    for (int u = 0; u < kXLoadBatch; ++u) {
      const int idx = min(base + u * kThreads, nin - 1);
      const int x = dh.div(idx);
      off[u] = 4u * (unsigned)(x * nt + t0 + 2 * (idx - x * half));
      if constexpr (SCG) {
        va[u] = at_byte<float2>(sv, off[u]);
        vq[u] = at_byte<float2>(qv, off[u]);
      } else {
        va[u] = at_byte<float2>(src, off[u]);
      }
      if constexpr (MUL) vm[u] = at_byte<float2>(mul, off[u]);
      live[u] = x;
    }
    // mask bytes after every other load of the batch is issued
    if (tm) {
#pragma unroll
      for (int u = 0; u < kXLoadBatch; ++u) live[u] = tm[live[u]];
    } else {
#pragma unroll
      for (int u = 0; u < kXLoadBatch; ++u) live[u] = 1;
    }
#pragma unroll
    for (int u = 0; u < kXLoadBatch; ++u) {
      const int idx = base + u * kThreads;
      if (idx < nin) {
        const int x = dh.div(idx);
        const int i = idx - x * half;
        float2 v = va[u];
        if constexpr (SCG) {
          v = make_float2(fmaf(-alpha, vq[u].x, v.x), fmaf(-alpha, vq[u].y, v.y));
          at_byte<float2>(sv, off[u]) = v;
        }
        if constexpr (MUL) v = make_float2(v.x * vm[u].x, v.y * vm[u].y);
        if (live[u] == 0) v = make_float2(0.f, 0.f);
        buf[i * bs + px<NX>(x)] = v;
      }
    }
  }
}

// Input of a full tile of the x-spectrum rows (nt even, t0 + T <= nt) into
// the LDS column pairs, Hermitian-completed: rows l >= 1 fill slots l and
// nxp - l, row 0 packs (DC, Nyquist).  Rows nrw .. nrows-1 are zero and not
// read.  Loads batched as in xfwd_model_full_tile.
template <int NX>
__device__ __forceinline__ void xinv_rows_full_tile(float2* buf, int bs, const UDiv& dh, int half, int nrows,
                                                    int nrw, int nxp, int nt, int t0,
                                                    const float2* __restrict__ src) {
  const int nin = nrw * half;
  for (int base = threadIdx.x; base < nin; base += kXLoadBatch * kThreads) {
    float4 hv[kXLoadBatch];
#pragma unroll
    for (int u = 0; u < kXLoadBatch; ++u) {
      const int idx = min(base + u * kThreads, nin - 1);
      const int l = dh.div(idx);
      // byte offset in the panel's rows (8 nrows nt < 2^32)
      hv[u] = at_byte<float4>(src, 8u * (unsigned)(l * nt + t0 + 2 * (idx - l * half)));
    }
#pragma unroll
    for (int u = 0; u < kXLoadBatch; ++u) {
      const int idx = base + u * kThreads;
      if (idx < nin) {
        const int l = dh.div(idx);
        const int i = idx - l * half;
        const float2 h1 = make_float2(hv[u].x, hv[u].y), h2 = make_float2(hv[u].z, hv[u].w);
        float2* Z = buf + i * bs;
        if (l == 0) {
          Z[0] = make_float2(h1.x, h2.x);
          Z[px<NX>(nrows)] = make_float2(h1.y, h2.y);
        } else {
          Z[px<NX>(l)] = make_float2(h1.x - h2.y, h1.y + h2.x);
          Z[px<NX>(nxp - l)] = make_float2(h1.x + h2.y, -h1.y + h2.x);
        }
      }
    }
  }
  for (int idx = nin + (int)threadIdx.x; idx < nrows * half; idx += kThreads) {
    const int l = dh.div(idx);  // >= nrw >= 1
    const int i = idx - l * half;
    float2* Z = buf + i * bs;
    Z[px<NX>(l)] = make_float2(0.f, 0.f);
    Z[px<NX>(nxp - l)] = make_float2(0.f, 0.f);
  }
}

// Work-item order for a one-item-per-workgroup launch of n items on the 8
// XCDs.  Workgroup b runs on XCD b mod 8; this gives XCD x the consecutive
// items [x q + min(x, r), ...) (q = n div 8, r = n mod 8), so neighbouring
// time tiles, which share 128-byte lines of the trace-major arrays, are read
// through one L2.
__device__ __forceinline__ int xcd_item(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
  return x * q + min(x, r) + k;
}

// ------------------------------------------------------------ x-direction RFFT
template <int NX>
__global__ __launch_bounds__(kThreads) void k_xfft_fwd(XfwdArgs A) {
  extern __shared__ float2 lds[];
  __shared__ float s_alpha;
  __shared__ float s_ab[2];
  __shared__ double s_red[kThreads / 64];
  for (int it0 = blockIdx.x; it0 < A.nitems; it0 += gridDim.x) {
    const int it = (int)gridDim.x == A.nitems ? xcd_item(it0, A.nitems) : it0;
    const WorkItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    float alpha = 0.f;
    if (A.s_inout) {
      double dsum = 0.0;
      if (A.part_red) {
        double part = 0.0;
        for (int i = G.xd_lo + (int)threadIdx.x; i < G.xd_hi; i += kThreads) part += A.part_red[i];
        dsum = block_sum(part, s_red);
      }
      if (threadIdx.x == 0) {
        double* sc = A.sc + (long long)w.g * kNScal;
        const double delta = A.part_red ? dsum : sc[SC_DELTA];
        const double gm = sc[SC_GAMMA0 + A.par];
        const bool stop = sc[SC_DONE] != 0.0 || gm == 0.0 || delta == 0.0 || !isfinite(gm) || !isfinite(delta);
        const double al = stop ? 0.0 : gm / delta;
        s_alpha = (float)al;
        if (A.item_base + it == G.xd_lo) {
          sc[SC_ALPHA] = al;
          if (stop) sc[SC_DONE] = 1.0;
          else sc[SC_NINNER] += 1.0;
        }
      }
      __syncthreads();
      alpha = s_alpha;
    }
    float cg_a = 0.f, cg_b = 0.f;
    if (A.cg_upd) {
      double gsum = 0.0;
      if (A.part_red) {
        double part = 0.0;
        for (int i = G.xm_lo + (int)threadIdx.x; i < G.xm_hi; i += kThreads) part += A.part_red[i];
        gsum = block_sum(part, s_red);
      }
      if (threadIdx.x == 0) {
        double* sc = A.sc + (long long)w.g * kNScal;
        const double gnew = A.part_red ? gsum : sc[SC_GNEW];
        const bool done = sc[SC_DONE] != 0.0;
        const double gold = sc[SC_GAMMA0 + A.cg_par];
        const double beta = (done || gold == 0.0) ? 0.0 : gnew / gold;
        s_ab[0] = done ? 0.f : (float)sc[SC_ALPHA];
        s_ab[1] = (float)beta;
        if (A.item_base + it == G.xm_lo) {
          sc[SC_GAMMA0 + (A.cg_par ^ 1)] = gnew;
          sc[SC_BETA] = beta;
        }
      }
      __syncthreads();
      cg_a = s_ab[0];
      cg_b = s_ab[1];
    }
    const int p = w.a;
    const int nx = G.nx, nt = G.nt, nxp = G.nxp, nrows = G.nrows;
    const int T = A.is_model ? G.tileT : G.tileTd, half = T >> 1;
    const int bs = ((NX > 0 ? fft_padlen(nxp) : nxp) | 1);  // odd slot stride between columns
    const int t0 = w.b * T;
    float2* twl = lds;                          // x twiddles
    float2* buf = lds + fft_tw_slots(NX, nxp);  // T/2 packed column pairs, odd slot stride bs
    stage_twiddles<NX>(twl, A.tw, G.tw_x_off, G.twp_x_off, nxp);
    const long long fbase = uniform64(A.is_model ? (G.m_off + (long long)p * nx * nt) : G.d_off);
    const float* __restrict__ src = A.src + fbase;
    const float* __restrict__ mul = A.mul ? A.mul + fbase : nullptr;
    const uint8_t* __restrict__ tm = A.tmask ? A.tmask + G.mask_off : nullptr;
    const bool even = (nt & 1) == 0;

    const UDiv dh(half);
    if (!A.is_model && even && t0 + T <= nt && G.nudft_off < 0) {
      // a full data tile (all but a ragged last one)
      float* sv = A.s_inout ? A.s_inout + fbase : nullptr;
      const float* qv = A.s_inout ? A.qv + fbase : nullptr;
      if (A.s_inout) {
        if (mul) xfwd_data_full_tile<NX, true, true>(buf, bs, dh, half, nx, nt, t0, src, mul, tm, sv, qv, alpha);
        else xfwd_data_full_tile<NX, true, false>(buf, bs, dh, half, nx, nt, t0, src, mul, tm, sv, qv, alpha);
      } else {
        if (mul) xfwd_data_full_tile<NX, false, true>(buf, bs, dh, half, nx, nt, t0, src, mul, tm, sv, qv, alpha);
        else xfwd_data_full_tile<NX, false, false>(buf, bs, dh, half, nx, nt, t0, src, mul, tm, sv, qv, alpha);
      }
    } else if (A.is_model && even && t0 + T <= nt) {
      // a full model tile (all but a ragged last one)
      float* pp = A.cg_upd ? A.cg_p + fbase : nullptr;
      float* uu = A.cg_upd ? A.cg_u + fbase : nullptr;
      const float* gg = A.cg_upd ? A.cg_g + fbase : nullptr;
      if (A.cg_upd) {
        if (mul) xfwd_model_full_tile<NX, true, true>(buf, bs, dh, half, nx, nt, t0, src, mul, pp, uu, gg, cg_a, cg_b);
        else xfwd_model_full_tile<NX, true, false>(buf, bs, dh, half, nx, nt, t0, src, mul, pp, uu, gg, cg_a, cg_b);
      } else {
        if (mul) xfwd_model_full_tile<NX, false, true>(buf, bs, dh, half, nx, nt, t0, src, mul, pp, uu, gg, 0.f, 0.f);
        else xfwd_model_full_tile<NX, false, false>(buf, bs, dh, half, nx, nt, t0, src, mul, pp, uu, gg, 0.f, 0.f);
      }
    } else
    for (int idx = threadIdx.x; idx < nx * half; idx += kThreads) {
      const int x = dh.div(idx);
      const int i = idx - x * half;
      const int t = t0 + 2 * i;
      const long long o = (long long)x * nt + t;
      float a = 0.f, b = 0.f;
      if (A.cg_upd) {
        // the previous iteration's CG update of this element pair; the new
        // search direction is the input
        float* pp = A.cg_p + fbase;
        float* uu = A.cg_u + fbase;
        const float* gg = A.cg_g + fbase;
        if (even && t < nt) {
          const float2 pv = *reinterpret_cast<const float2*>(pp + o);
          const float2 gv = *reinterpret_cast<const float2*>(gg + o);
          const float2 uv = *reinterpret_cast<const float2*>(uu + o);
          *reinterpret_cast<float2*>(uu + o) = make_float2(fmaf(cg_a, pv.x, uv.x), fmaf(cg_a, pv.y, uv.y));
          a = fmaf(cg_b, pv.x, gv.x);
          b = fmaf(cg_b, pv.y, gv.y);
          *reinterpret_cast<float2*>(pp + o) = make_float2(a, b);
        } else {
          if (t < nt) {
            const float pv = pp[o];
            uu[o] = fmaf(cg_a, pv, uu[o]);
            a = fmaf(cg_b, pv, gg[o]);
            pp[o] = a;
          }
          if (t + 1 < nt) {
            const float pv = pp[o + 1];
            uu[o + 1] = fmaf(cg_a, pv, uu[o + 1]);
            b = fmaf(cg_b, pv, gg[o + 1]);
            pp[o + 1] = b;
          }
        }
        if (mul) {
          a *= (t < nt) ? mul[o] : 0.f;
          b *= (t + 1 < nt) ? mul[o + 1] : 0.f;
        }
      } else if (A.s_inout) {
        float* sv = A.s_inout + fbase;
        const float* qv = A.qv + fbase;
        if (t < nt) {
          a = fmaf(-alpha, qv[o], sv[o]);
          sv[o] = a;
        }
        if (t + 1 < nt) {
          b = fmaf(-alpha, qv[o + 1], sv[o + 1]);
          sv[o + 1] = b;
        }
        if (mul) {
          a *= (t < nt) ? mul[o] : 0.f;
          b *= (t + 1 < nt) ? mul[o + 1] : 0.f;
        }
      } else if (even && t < nt) {
        // nt even: (t, t+1) is an aligned pair inside the trace
        const float2 v = *reinterpret_cast<const float2*>(src + o);
        a = v.x;
        b = v.y;
        if (mul) {
          const float2 wv = *reinterpret_cast<const float2*>(mul + o);
          a *= wv.x;
          b *= wv.y;
        }
      } else {
        if (t < nt) {
          a = src[o];
          if (mul) a *= mul[o];
        }
        if (t + 1 < nt) {
          b = src[o + 1];
          if (mul) b *= mul[o + 1];
        }
      }
      if (tm && tm[x] == 0) {
        a = 0.f;
        b = 0.f;
      }
      buf[i * bs + px<NX>(x)] = make_float2(a, b);
    }
    if constexpr (NX == 0) {  // the generic FFT reads the pad
      for (int idx = threadIdx.x; idx < (nxp - nx) * half; idx += kThreads) {
        const int xx = dh.div(idx);
        const int i = idx - xx * half;
        buf[i * bs + px<NX>(nx + xx)] = make_float2(0.f, 0.f);
      }
    }
    __syncthreads();
    if (!A.is_model && G.nudft_off >= 0) {
      // irregular traces: non-uniform DFT over the trace positions,
      // H_t[r] = sum_x d_t[x] exp(-2 pi i r x_pos / (nxp dx)); row 0 packs
      // (H_t[0], 0) (no Nyquist wavenumber off the grid)
      const float2* __restrict__ E = A.tw + G.nudft_off;
      float2* __restrict__ dst = A.dst + G.H_off;
      for (int idx = threadIdx.x; idx < nrows * T; idx += kThreads) {
        const int r = idx / T, c = idx - r * T, t = t0 + c;
        if (t >= nt) continue;
        const float2* Z = buf + (c >> 1) * bs;
        float2 acc = make_float2(0.f, 0.f);
        if (r == 0) {
          for (int x = 0; x < nx; ++x) acc.x += (c & 1) ? Z[px<NX>(x)].y : Z[px<NX>(x)].x;
        } else {
          const float2* Er = E + (long long)r * nx;
          for (int x = 0; x < nx; ++x) {
            const float v = (c & 1) ? Z[px<NX>(x)].y : Z[px<NX>(x)].x;
            acc = cfma(v, Er[x], acc);
          }
        }
        dst[(long long)r * nt + t] = acc;
      }
      __syncthreads();
      continue;
    }
    xfft_tile<NX, false>(buf, nxp, half, bs, twl, nx);

    // column pair i holds the packed spectra of columns t0 + 2i (real part)
    // and t0 + 2i + 1 (imaginary part); both outputs of a row are written
    // together (one 16-byte store when nt is even)
    float2* __restrict__ dst = A.dst + (A.is_model ? G.X_off + (long long)p * nrows * nt : G.H_off);
    // model panels: rows at or above the panel's live-row count are never read
    const int nrw = A.is_model ? min(nrows, A.panels[G.panel_off + p].rlive) : nrows;
    for (int idx = threadIdx.x; idx < nrw * half; idx += kThreads) {
      const int r = dh.div(idx);
      const int i = idx - r * half;
      const int t = t0 + 2 * i;
      if (t >= nt) continue;
      const float2* Z = buf + i * bs;
      float2 o0, o1;
      if (r == 0) {
        const float2 z0 = Z[0], zn = Z[px<NX>(nrows)];
        o0 = make_float2(z0.x, zn.x);
        o1 = make_float2(z0.y, zn.y);
      } else {
        const float2 a = Z[px<NX>(r)];
        const float2 b = cconj(Z[px<NX>(nxp - r)]);
        o0 = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y + b.y));
        o1 = make_float2(0.5f * (a.y - b.y), -0.5f * (a.x - b.x));
      }
      float2* d = dst + (long long)r * nt + t;
      if (even) {
        *reinterpret_cast<float4*>(d) = make_float4(o0.x, o0.y, o1.x, o1.y);
      } else {
        d[0] = o0;
        if (t + 1 < nt) d[1] = o1;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ x-direction C2R
template <int NX>
__global__ __launch_bounds__(kThreads) void k_xfft_inv(XinvArgs A) {
  extern __shared__ float2 lds[];
  __shared__ double sh[kThreads / 64];
  for (int it0 = blockIdx.x; it0 < A.nitems; it0 += gridDim.x) {
    const int it = (int)gridDim.x == A.nitems ? xcd_item(it0, A.nitems) : it0;
    const WorkItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    const int p = w.a;
    const int nx = G.nx, nt = G.nt, nxp = G.nxp, nrows = G.nrows;
    const int T = A.is_model ? G.tileT : G.tileTd, half = T >> 1;
    const int bs = ((NX > 0 ? fft_padlen(nxp) : nxp) | 1);  // odd slot stride between columns
    const int t0 = w.b * T;
    const float2* __restrict__ src = A.src + uniform64(A.is_model ? G.X_off + (long long)p * nrows * nt : G.H_off);
    float2* twl = lds;
    float2* buf = lds + fft_tw_slots(NX, nxp);
    if (!A.is_model && G.nudft_off >= 0) {
      // irregular traces: d_t[x] = (1/nxp) (Re H_t[0] + 2 Re sum_{r>=1} H_t[r]
      // exp(+2 pi i r x_pos / (nxp dx))), the rows staged column by column
      for (int idx = threadIdx.x; idx < nrows * T; idx += kThreads) {
        const int l = idx / T, c = idx - l * T, t = t0 + c;
        buf[c * nrows + l] = (t < nt) ? src[(long long)l * nt + t] : make_float2(0.f, 0.f);
      }
      __syncthreads();
      const float2* __restrict__ E = A.tw + G.nudft_off;
      const float inv = 1.0f / (float)nxp;
      const long long fbase = G.d_off;
      const uint8_t* __restrict__ tm = A.tmask ? A.tmask + G.mask_off : nullptr;
      double ss = 0.0;
      for (int idx = threadIdx.x; idx < nx * T; idx += kThreads) {
        const int x = idx / T, c = idx - x * T, t = t0 + c;
        if (t >= nt) continue;
        const float2* hc = buf + c * nrows;
        float acc = 0.f;
        for (int r = 1; r < nrows; ++r) {
          const float2 e = E[(long long)r * nx + x];
          acc = fmaf(hc[r].x, e.x, fmaf(hc[r].y, e.y, acc));
        }
        float v = (hc[0].x + 2.0f * acc) * inv;
        const long long o = fbase + (long long)x * nt + t;
        if (A.raw_out) A.raw_out[o] = v;
        if (A.sub) v = A.sub[o] - v;
        if (tm && tm[x] == 0) v = 0.f;
        if (A.wmul) v *= A.wmul[o];
        A.out[o] = v;
        ss += (double)v * (double)v;
      }
      if (A.part) {
        const double tot = block_sum(ss, sh);
        if (threadIdx.x == 0) A.part[A.item_base + it] = tot;
      }
      __syncthreads();
      continue;
    }
    stage_twiddles<NX>(twl, A.tw, G.tw_x_off, G.twp_x_off, nxp);

    const UDiv dh(half);
    const bool even = (nt & 1) == 0;
    // model panels: rows at or above the panel's live-row count are zero (not stored)
    const int nrw = A.is_model ? min(nrows, A.panels[G.panel_off + p].rlive) : nrows;
    if (even && t0 + T <= nt) {
      // a full tile (all but a ragged last one)
      xinv_rows_full_tile<NX>(buf, bs, dh, half, nrows, nrw, nxp, nt, t0, src);
    } else
    for (int idx = threadIdx.x; idx < nrows * half; idx += kThreads) {
      const int l = dh.div(idx);
      const int i = idx - l * half;
      const int t = t0 + 2 * i;
      float2 h1 = make_float2(0.f, 0.f), h2 = make_float2(0.f, 0.f);
      if (l >= nrw) {
        // zero row
      } else if (even && t < nt) {
        // nt even: (t, t+1) is an aligned pair inside the row
        const float4 h = *reinterpret_cast<const float4*>(src + (long long)l * nt + t);
        h1 = make_float2(h.x, h.y);
        h2 = make_float2(h.z, h.w);
      } else {
        if (t < nt) h1 = src[(long long)l * nt + t];
        if (t + 1 < nt) h2 = src[(long long)l * nt + t + 1];
      }
      float2* Z = buf + i * bs;
      if (l == 0) {
        Z[0] = make_float2(h1.x, h2.x);
        Z[px<NX>(nrows)] = make_float2(h1.y, h2.y);
      } else {
        Z[px<NX>(l)] = make_float2(h1.x - h2.y, h1.y + h2.x);
        Z[px<NX>(nxp - l)] = make_float2(h1.x + h2.y, -h1.y + h2.x);
      }
    }
    __syncthreads();
    xfft_tile<NX, true>(buf, nxp, half, bs, twl, nx);

    const float inv = 1.0f / (float)nxp;
    const long long fbase = uniform64(A.is_model ? (G.m_off + (long long)p * nx * nt) : G.d_off);
    const uint8_t* __restrict__ tm = A.tmask ? A.tmask + G.mask_off : nullptr;
    double ss = 0.0;
    if (even && t0 + T <= nt && (A.wmul || A.sub)) {
      // a full tile whose epilogue reads memory (wmul, sub): the loads of
      // kXLoadBatch loop iterations are issued together (indices past the
      // tile clamped)
      const float* __restrict__ wm = A.wmul ? A.wmul + fbase : nullptr;
      const bool wsq = A.wmul && A.wmul_sq;
      const float* __restrict__ sb = A.sub ? A.sub + fbase : nullptr;
      float* __restrict__ raw = A.raw_out ? A.raw_out + fbase : nullptr;
      float* __restrict__ out = A.out + fbase;
      const int nin = nx * half;
      for (int base = threadIdx.x; base < nin; base += kXLoadBatch * kThreads) {
        float2 wv[kXLoadBatch], sv[kXLoadBatch];
        int live[kXLoadBatch];  // trace index, then its mask byte
        unsigned off[kXLoadBatch];  // byte offsets (4 nx nt < 2^32)
#pragma unroll
        for (int u = 0; u < kXLoadBatch; ++u) {
          const int idx = min(base + u * kThreads, nin - 1);
          const int x = dh.div(idx);
          off[u] = 4u * (unsigned)(x * nt + t0 + 2 * (idx - x * half));
          if (wm) wv[u] = at_byte<float2>(wm, off[u]);
          if (sb) sv[u] = at_byte<float2>(sb, off[u]);
          live[u] = x;
        }
        // mask bytes after every other load of the batch is issued
        if (tm) {
#pragma unroll
          for (int u = 0; u < kXLoadBatch; ++u) live[u] = tm[live[u]];
        } else {
#pragma unroll
          for (int u = 0; u < kXLoadBatch; ++u) live[u] = 1;
        }
#pragma unroll
        for (int u = 0; u < kXLoadBatch; ++u) {
          const int idx = base + u * kThreads;
          if (idx < nin) {
            const int x = dh.div(idx);
            const int i = idx - x * half;
            const float2 z = buf[i * bs + px<NX>(x)];
            float2 v = make_float2(z.x * inv, z.y * inv);
            if (raw) at_byte<float2>(raw, off[u]) = v;
            if (sb) v = make_float2(sv[u].x - v.x, sv[u].y - v.y);
            if (live[u] == 0) v = make_float2(0.f, 0.f);
            if (wm) v = make_float2(v.x * wv[u].x, v.y * wv[u].y);
            ss += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            if (wsq) v = make_float2(v.x * wv[u].x, v.y * wv[u].y);
            at_byte<float2>(out, off[u]) = v;
          }
        }
      }
    } else
    for (int idx = threadIdx.x; idx < nx * half; idx += kThreads) {
      const int x = dh.div(idx);
      const int i = idx - x * half;
      const int t = t0 + 2 * i;
      if (t >= nt) continue;
      const float2 z = buf[i * bs + px<NX>(x)];
      const bool live = !(tm && tm[x] == 0);
      const long long o = fbase + (long long)x * nt + t;
      if (even) {
        // nt even: columns t, t+1 form an aligned pair inside the trace
        float2 v = make_float2(z.x * inv, z.y * inv);
        if (A.raw_out) *reinterpret_cast<float2*>(A.raw_out + o) = v;
        if (A.sub) {
          const float2 sv = *reinterpret_cast<const float2*>(A.sub + o);
          v = make_float2(sv.x - v.x, sv.y - v.y);
        }
        if (!live) v = make_float2(0.f, 0.f);
        if (A.wmul) {
          const float2 wv = *reinterpret_cast<const float2*>(A.wmul + o);
          v = make_float2(v.x * wv.x, v.y * wv.y);
          ss += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
          if (A.wmul_sq) v = make_float2(v.x * wv.x, v.y * wv.y);
        } else {
          ss += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
        *reinterpret_cast<float2*>(A.out + o) = v;
      } else {
        for (int c = 0; c < 2 && t + c < nt; ++c) {
          float v = (c ? z.y : z.x) * inv;
          if (A.raw_out) A.raw_out[o + c] = v;
          if (A.sub) v = A.sub[o + c] - v;
          if (!live) v = 0.f;
          if (A.wmul) v *= A.wmul[o + c];
          ss += (double)v * (double)v;
          if (A.wmul && A.wmul_sq) v *= A.wmul[o + c];
          A.out[o + c] = v;
        }
      }
    }
    if (A.part) {
      const double tot = block_sum(ss, sh);
      if (threadIdx.x == 0) A.part[A.item_base + it] = tot;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ rows: shared steps
// Natural (unpadded, generic-length) layout <-> pair layout (fft_tpl.h),
// in place: every thread first reads its bins, then all write.
template <int NT>
__device__ __forceinline__ void natural_to_pairs(float2* buf, int n) {
  constexpr int MAXK = (kRowMaxN / 2 + NT - 1) / NT;
  float2 a[MAXK], b[MAXK];
#pragma unroll
  for (int i = 0; i < MAXK; ++i) {
    const int k = 1 + (int)threadIdx.x + i * NT;
    if (k < n / 2) {
      a[i] = buf[k];
      b[i] = buf[n - k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXK; ++i) {
    const int k = 1 + (int)threadIdx.x + i * NT;
    if (k < n / 2) {
      buf[2 * k] = a[i];
      buf[2 * k + 1] = b[i];
    }
  }
  __syncthreads();
}

template <int NT>
__device__ __forceinline__ void pairs_to_natural(float2* buf, int n) {
  constexpr int MAXK = (kRowMaxN / 2 + NT - 1) / NT;
  float2 a[MAXK], b[MAXK];
#pragma unroll
  for (int i = 0; i < MAXK; ++i) {
    const int k = 1 + (int)threadIdx.x + i * NT;
    if (k < n / 2) {
      a[i] = buf[2 * k];
      b[i] = buf[2 * k + 1];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXK; ++i) {
    const int k = 1 + (int)threadIdx.x + i * NT;
    if (k < n / 2) {
      buf[k] = a[i];
      buf[n - k] = b[i];
    }
  }
  if (threadIdx.x == 0) {
    buf[0] = make_float2(0.f, 0.f);
    buf[n / 2] = make_float2(0.f, 0.f);
  }
  __syncthreads();
}

// Load row r of a [nrows][nt] complex field into buf[0..nt), zero to ntp,
// forward time FFT, leaving the spectrum in the pair layout: pair k holds
// (Q[k], Q[ntp-k]).  Rows >= 1 then read "up = Q[k], lo = conj Q[ntp-k]"
// (the +l and -l spectra); row 0 separates the packed kx = 0 / Nyquist
// spectra so that the same reading gives them.
template <int N, int NT>
__device__ __forceinline__ void row_spectrum_lds(float2* buf, int r, int ntp, const float2* twl);

template <int N, int NT>
__device__ __forceinline__ void row_spectrum(float2* buf, const float2* __restrict__ src, int r, int nt,
                                             int ntp, const float2* twl) {
  for (int t = threadIdx.x; t < ntp; t += NT) buf[px<N>(t)] = (t < nt) ? src[t] : make_float2(0.f, 0.f);
  row_spectrum_lds<N, NT>(buf, r, ntp, twl);
}

// Forward time FFT of the row held in buf (natural order, zero-padded to
// ntp), leaving the pair layout described above.
template <int N, int NT>
__device__ __forceinline__ void row0_separate(float2* buf, int ntp);

template <int N, int NT>
__device__ __forceinline__ void row_spectrum_lds(float2* buf, int r, int ntp, const float2* twl) {
  __syncthreads();
  if constexpr (N > 0) {
    fft_tpl_to_pairs<N, false, NT>(buf, twl);
  } else {
    fft_lds<NT, kRowMaxN, false>(buf, ntp, 1, ntp, twl);
    natural_to_pairs<NT>(buf, ntp);
  }
  if (r == 0) row0_separate<N, NT>(buf, ntp);
}

// Row 0 holds the kx = 0 and Nyquist spectra packed as M(0) + i M(N):
// separate them in place so the pair reading gives the two halves.
template <int N, int NT>
__device__ __forceinline__ void row0_separate(float2* buf, int ntp) {
  {
    float4* P = reinterpret_cast<float4*>(buf);
    for (int k = 1 + threadIdx.x; k < ntp / 2; k += NT) {
      const float4 q = P[k];
      const float2 a = make_float2(q.x, q.y);
      const float2 b = make_float2(q.z, -q.w);
      const float2 m0 = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y + b.y));
      const float2 m1 = make_float2(0.5f * (a.y - b.y), -0.5f * (a.x - b.x));
      P[k] = make_float4(m0.x, m0.y, m1.x, -m1.y);
    }
    __syncthreads();
  }
}

template <int N, int NT>
__device__ __forceinline__ void row_inverse(float2* buf, int ntp, const float2* twl) {
  if constexpr (N > 0) fft_tpl<N, N, true, NT>(buf, 1, fft_padlen(N), twl);
  else fft_lds<NT, kRowMaxN, true>(buf, ntp, 1, ntp, twl);
}

// Inverse time FFT of a spectrum held in the pair layout (bins 0 and ntp/2
// zero); the output is in the transform's usual layout.
template <int N, int NT>
__device__ __forceinline__ void row_inverse_from_pairs(float2* buf, int ntp, const float2* twl) {
  if constexpr (N > 0) {
    fft_tpl_from_pairs<N, true, NT>(buf, twl);
  } else {
    pairs_to_natural<NT>(buf, ntp);
    fft_lds<NT, kRowMaxN, true>(buf, ntp, 1, ntp, twl);
  }
}

// ------------------------------------------------------------ forward rows
//
// LDS: twiddles [ntp], row spectrum [ntp], accumulators D(+l), D(-l) [2 nband].
template <int N, int RC, int NT>
__device__ __forceinline__ void rows_fwd_item(const RowsArgs& A, const WorkItem& w, const GatherDev& G,
                                              float2* lds, const float* ctab, const float* stab) {
  const int R = RC > 0 ? RC : A.R;
  const int r = w.a, chunk = w.b;
  const int nt = G.nt, ntp = N > 0 ? N : G.ntp, nrows = G.nrows, P = G.npanel;
  const int jlo = G.jlo, jhi = G.jhi, nband = jhi - jlo + 1;
  // chunk c takes panels c, c + nchunk, ... (interleaved, so chunks of one
  // row see a similar mix of slow and fast panels); panels whose live rows
  // end at or below r are skipped
  const int S = G.nchunk;
  const int hmax = ntp / 2 - 1;
  const int plen = N > 0 ? fft_padlen(N) : ntp;
  // compile-time lengths: kMapGuardSlots zero slots in front of the
  // spectrum, and the FFT's pair output leaves pair 0 and the pairs N/2 ..
  // N/2 + 3 zero, so taps k = -3 .. 0 and past N/2 - 1 read zeros and the
  // map needs no bounds test
  float2* twl = lds;
  float2* buf = lds + fft_tw_slots(N, ntp) + (N > 0 ? kMapGuardSlots : 0);
  float2* acc = buf + plen;
  // row spectrum, pair layout (16-byte aligned: the twiddle and guard slot
  // counts are even)
  const float4* P4 = reinterpret_cast<const float4*>(buf);
  stage_twiddles<N, NT>(twl, A.tw, G.tw_t_off, G.twp_t_off, ntp);
  for (int i = threadIdx.x; i < 2 * nband; i += NT) acc[i] = make_float2(0.f, 0.f);
  if constexpr (N > 0) {
    if ((int)threadIdx.x < kMapGuardSlots) buf[(int)threadIdx.x - kMapGuardSlots] = make_float2(0.f, 0.f);
  }
  const int lu = (r == 0) ? 0 : r;
  const int ll = (r == 0) ? nrows : r;
  const double lup2 = (double)lu * (double)lu;
  const double llo2 = (double)ll * (double)ll;

  const float2* __restrict__ xrow = A.X + G.X_off + (long long)r * nt;  // panel p's row at + p nrows nt
  const long long pstride = (long long)nrows * nt;
  // compile-time lengths: the next panel's row is loaded while this panel
  // is transformed and mapped (the first FFT pass takes it straight from
  // registers), and the panel constants one panel further ahead, so that the
  // liveness of the row to load is known without a wait
  FftRegsIn<(N > 0 ? N : kRowMaxN), NT> pf;
  PanelDev pdc, pdn;  // constants of the panel whose row is in pf, and of the one after
  if constexpr (N > 0) {
    if (chunk < P) {
      pdc = A.panels[G.panel_off + chunk];
      if (r < pdc.rlive) pf.load(xrow + chunk * pstride, nt);
      if (chunk + S < P) pdn = A.panels[G.panel_off + chunk + S];
    }
  }

  for (int p = chunk; p < P; p += S) {
    PanelDev PD;
    if constexpr (N > 0) {
      PD = pdc;
      const bool live = r < PD.rlive;
      if (live) fft_tpl_regs_pass0<N, false, NT>(buf, pf);
      if (p + S < P) {
        pdc = pdn;
        if (r < pdc.rlive) pf.load(xrow + (p + S) * pstride, nt);
        if (p + 2 * S < P) pdn = A.panels[G.panel_off + p + 2 * S];
      }
      if (!live) continue;
      fft_tpl_rest_to_pairs<N, false, NT>(buf, twl);
      if (r == 0) row0_separate<N, NT>(buf, ntp);
    } else {
      PD = A.panels[G.panel_off + p];
      if (r >= PD.rlive) continue;
      row_spectrum<N, NT>(buf, xrow + p * pstride, r, nt, ntp, twl);
    }
    const bool plain = (PD.n0 == 0) && (G.wav_off < 0);
    // rows >= 1 map only bins inside the cone (the rest add zero); row 0's
    // l = 0 half covers the whole band
    const int jstart = (r != 0) ? max(jlo, cone_first_bin(PD.c2 * lup2)) : jlo;
    if constexpr (RC > 0) {
      static_assert(RC == 4, "compile-time row kernels use the half-width-4 weight polynomials");
      const RowA2 aup = split_a2(PD.c2 * lup2);
      const RowA2 alo = split_a2(PD.c2 * llo2);
      const int jcone_lo = (r == 0) ? cone_first_bin(PD.c2 * llo2) : 0;
      auto put = [&](int j, float2 au, float2 al) {
        float2* du = acc + (j - jlo);
        float2* dl = acc + nband + (j - jlo);
        if (plain) {
          *du = cfma(PD.scale, au, *du);
          *dl = cfma(PD.scale, al, *dl);
        } else {
          const float2 cj = bin_factor(G, PD, A.tw, A.wav, j);
          *du = cadd(*du, cmul(cj, au));
          *dl = cadd(*dl, cmul(cj, al));
        }
      };
      // rows >= 1 and row 0 run separate loops, so that no tap load is
      // shared between them: the rows >= 1 loop then reads each 16-byte
      // pair with one ds_read_b128 at an immediate offset
      if (r != 0) {
#pragma unroll 1
        for (int j = jstart + (int)threadIdx.x; j <= jhi; j += NT) {
          float2 au = make_float2(0.f, 0.f), al = make_float2(0.f, 0.f);
          const Taps4 tu = taps4(j, aup);
          const float4* qu = P4 + (tu.k0 - 3);
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const float4 q = qu[t];
            au = cfma(tu.w[t], make_float2(q.x, q.y), au);
            al = cfma(tu.w[t], make_float2(q.z, -q.w), al);
          }
          put(j, au, al);
        }
      } else {
#pragma unroll 1
        for (int j = jstart + (int)threadIdx.x; j <= jhi; j += NT) {
          float2 au = make_float2(0.f, 0.f), al = make_float2(0.f, 0.f);
          const Taps4 tu = taps4(j, aup);
          const float4* qu = P4 + (tu.k0 - 3);
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const float4 q = qu[t];
            au = cfma(tu.w[t], make_float2(q.x, q.y), au);
          }
          if (j >= jcone_lo) {
            const Taps4 tl = taps4(j, alo);
            const float4* ql = P4 + (tl.k0 - 3);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              const float4 q = ql[t];
              al = cfma(tl.w[t], make_float2(q.z, -q.w), al);
            }
          }
          put(j, au, al);
        }
      }
      __syncthreads();
      continue;
    }
#pragma unroll 1
    for (int j = jstart + (int)threadIdx.x; j <= jhi; j += NT) {
      const Taps tu = taps_of<RC>(j, PD.c2 * lup2, R);
      float2 au = make_float2(0.f, 0.f), al = make_float2(0.f, 0.f);
      if (r != 0) {
        if (tu.k0 != kNoTap) {
#pragma unroll
          for (int t = -R + 1; t <= R; ++t) {
            const int k = tu.k0 + t;
            const bool ok = (k >= 1) && (k <= hmax);
            const int kc = ok ? k : 1;
            float wt = tap_weight(tu.trig, t, ctab[t + R - 1], stab[t + R - 1]);
            wt = ok ? wt : 0.f;
            const float4 q = P4[kc];
            au = cfma(wt, make_float2(q.x, q.y), au);
            al = cfma(wt, make_float2(q.z, -q.w), al);
          }
        }
      } else {
        const Taps tl = taps_of<RC>(j, PD.c2 * llo2, R);
        if (tu.k0 != kNoTap) {
#pragma unroll
          for (int t = -R + 1; t <= R; ++t) {
            const int k = tu.k0 + t;
            if (k >= 1 && k <= hmax) {
              const float4 q = P4[k];
              au = cfma(tap_weight(tu.trig, t, ctab[t + R - 1], stab[t + R - 1]), make_float2(q.x, q.y), au);
            }
          }
        }
        if (tl.k0 != kNoTap) {
#pragma unroll
          for (int t = -R + 1; t <= R; ++t) {
            const int k = tl.k0 + t;
            if (k >= 1 && k <= hmax) {
              const float4 q = P4[k];
              al = cfma(tap_weight(tl.trig, t, ctab[t + R - 1], stab[t + R - 1]), make_float2(q.z, -q.w), al);
            }
          }
        }
      }
      float2* du = acc + (j - jlo);
      float2* dl = acc + nband + (j - jlo);
      if (plain) {
        *du = cfma(PD.scale, au, *du);
        *dl = cfma(PD.scale, al, *dl);
      } else {
        const float2 cj = bin_factor(G, PD, A.tw, A.wav, j);
        *du = cadd(*du, cmul(cj, au));
        *dl = cadd(*dl, cmul(cj, al));
      }
    }
    __syncthreads();
  }
  float2* __restrict__ dp = A.Dp + G.Dp_off + ((long long)chunk * nrows + r) * 2 * nband;
  for (int i = threadIdx.x; i < 2 * nband; i += NT) dp[i] = acc[i];
  __syncthreads();
}

template <int N, int RC>
__global__ __launch_bounds__(row_threads(N)) __attribute__((amdgpu_waves_per_eu(row_waves_per_eu(N)))) void k_rows_fwd(RowsArgs A) {
  extern __shared__ float4 lds_raw[];  // 16-byte aligned: the map reads 16-byte pairs
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  __shared__ float ctab[2 * kMaxHalfWidth], stab[2 * kMaxHalfWidth];
  init_tap_trig(ctab, stab, RC > 0 ? RC : A.R);
  __syncthreads();
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const WorkItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    rows_fwd_item<N, RC, row_threads(N)>(A, w, G, lds, ctab, stab);
  }
}

// Sum the panel-chunk partials of row r, complete the Hermitian time
// spectrum (rows >= 1: Q[j] = D(+l,j), Q[ntp-j] = conj D(-l,j); row 0:
// Q[j] = D(0,j) + i D(N,j), Q[ntp-j] = conj D(0,j) + i conj D(N,j)), inverse
// time FFT, scale 1/ntp, keep t < nt.
template <int N, int NT>
__device__ __forceinline__ void rows_fin_item(const RowsArgs& A, const WorkItem& w, const GatherDev& G,
                                              float2* lds) {
  const int r = w.a;
  const int nt = G.nt, ntp = N > 0 ? N : G.ntp, nrows = G.nrows;
  const int jlo = G.jlo, jhi = G.jhi, nband = jhi - jlo + 1;
  float2* twl = lds;
  float2* buf = lds + fft_tw_slots(N, ntp);
  stage_twiddles<N, NT>(twl, A.tw, G.tw_t_off, G.twp_t_off, ntp);
  // time-spectrum bin k of the row: the chunk sums, Hermitian completion.
  // Branch-free (bins outside the band read the band's first entry and are
  // zeroed by a select), so the loads of all of a thread's bins can be in
  // flight together.
  const float2* __restrict__ dp0 = A.Dp + uniform64(G.Dp_off + (long long)r * 2 * nband);
  const long long cstride = uniform64((long long)nrows * 2 * nband);
  auto bin = [&](int k) {
    const bool up = k >= jlo && k <= jhi;
    const bool dn = !up && ntp - k >= jlo && ntp - k <= jhi;
    const int jj = (up ? k : (dn ? ntp - k : jlo)) - jlo;
    float2 su = make_float2(0.f, 0.f), sl = make_float2(0.f, 0.f);
    for (int c = 0; c < G.nchunk; ++c) {
      su = cadd(su, dp0[c * cstride + jj]);
      sl = cadd(sl, dp0[c * cstride + nband + jj]);
    }
    const float2 vu = (r == 0) ? make_float2(su.x - sl.y, su.y + sl.x) : su;
    const float2 vd = (r == 0) ? make_float2(su.x + sl.y, -su.y + sl.x) : cconj(sl);
    return up ? vu : (dn ? vd : make_float2(0.f, 0.f));
  };
  const float inv = 1.0f / (float)ntp;
  float2* __restrict__ dst = A.H + G.H_off + (long long)r * nt;
  if constexpr (N > 0) {
    // first pass from registers, last pass to global memory
    // the chunk loop outside, the thread's bins inside: all of a chunk's
    // loads are issued together
    using I = FftRegsIn<N, NT>;
    I in;
    float2 sl[I::MAXB][I::R];
    int jj[I::MAXB][I::R];
#pragma unroll
    for (int i = 0; i < I::MAXB; ++i) {
#pragma unroll
      for (int q = 0; q < I::R; ++q) {
        const int k = min((int)threadIdx.x + i * NT, I::B - 1) + q * I::B;
        const bool up = k >= jlo && k <= jhi;
        const bool dn = !up && ntp - k >= jlo && ntp - k <= jhi;
        jj[i][q] = 8 * ((up ? k : (dn ? ntp - k : jlo)) - jlo);  // byte offset
        in.v[i][q] = make_float2(0.f, 0.f);
        sl[i][q] = make_float2(0.f, 0.f);
      }
    }
    for (int c = 0; c < G.nchunk; ++c) {
      const float2* __restrict__ dpc = dp0 + c * cstride;
      float2 lu[I::MAXB][I::R], ld[I::MAXB][I::R];
#pragma unroll
      for (int i = 0; i < I::MAXB; ++i) {
#pragma unroll
        for (int q = 0; q < I::R; ++q) {
          lu[i][q] = at_byte<float2>(dpc, (unsigned)jj[i][q]);
          ld[i][q] = at_byte<float2>(dpc + nband, (unsigned)jj[i][q]);
        }
      }
#pragma unroll
      for (int i = 0; i < I::MAXB; ++i) {
#pragma unroll
        for (int q = 0; q < I::R; ++q) {
          in.v[i][q] = cadd(in.v[i][q], lu[i][q]);
          sl[i][q] = cadd(sl[i][q], ld[i][q]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < I::MAXB; ++i) {
      const int id = (int)threadIdx.x + i * NT;
#pragma unroll
      for (int q = 0; q < I::R; ++q) {
        const int k = id + q * I::B;
        const bool up = k >= jlo && k <= jhi;
        const bool dn = !up && ntp - k >= jlo && ntp - k <= jhi;
        const float2 su = in.v[i][q], sd = sl[i][q];
        const float2 vu = (r == 0) ? make_float2(su.x - sd.y, su.y + sd.x) : su;
        const float2 vd = (r == 0) ? make_float2(su.x + sd.y, -su.y + sd.x) : cconj(sd);
        in.v[i][q] = (id < I::B && up) ? vu : ((id < I::B && dn) ? vd : make_float2(0.f, 0.f));
      }
    }
    fft_tpl_regs_pass0<N, true, NT>(buf, in);
    using O = FftRegsOut<N, NT>;
    O o;
    fft_tpl_passes_to_regs<N, true, NT, 1, false>(buf, twl, o);
#pragma unroll
    for (int i = 0; i < O::MAXB; ++i) {
      const int id = (int)threadIdx.x + i * NT;
#pragma unroll
      for (int q = 0; q < O::R; ++q) {
        const int t = id + q * O::B;
        if (id < O::B && t < nt) dst[t] = cscale(o.v[i][q], inv);
      }
    }
  } else {
    for (int k = threadIdx.x; k < ntp; k += NT) buf[px<N>(k)] = bin(k);
    __syncthreads();
    row_inverse<N, NT>(buf, ntp, twl);
    for (int t = threadIdx.x; t < nt; t += NT) dst[t] = cscale(buf[px<N>(t)], inv);
  }
  __syncthreads();
}

template <int N>
// one workgroup per row and a few hundred rows: occupancy is low anyway, so the
// register budget goes to loads in flight
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_rows_fwd_fin(RowsArgs A) {
  extern __shared__ float2 lds[];
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const WorkItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    rows_fin_item<N, kThreads>(A, w, G, lds);
  }
}

// ------------------------------------------------------------ adjoint rows
//
// The transpose of the forward gather, as a scatter: data bin j adds
// h(u_j - k) times its ramped, scaled value to the 2R model bins
// k = floor(u_j) - R + 1 .. floor(u_j) + R, with the weights the forward
// uses.  floor(u_j) is strictly increasing in j inside the cone
// (u_{j+1} - u_j = (2j+1) / (u_{j+1} + u_j) >= 1), so:
//
// * for one tap, different bins j write different k: the lanes of a wave,
//   taking the taps in order, never collide within a tap, and the LDS
//   operations of one wave complete in issue order, so the read-modify-write
//   of tap t+1 sees that of tap t (a wave barrier keeps the compiler from
//   reordering them); the model spectrum is kept in the pair layout, so
//   one 16-byte read-modify-write updates bins k and ntp - k together;
// * a wave owns a 64-bin segment of the band; two segments with a full
//   segment between them (64 >= 2R - 1 bins) touch disjoint model bins, so
//   even segments run first, then a barrier, then odd ones.
//
// No atomics: each model bin sums its contributions in a fixed order.
//
// LDS: twiddles [ntp], data row spectrum bufD and model spectrum bufM
// (padded lengths).
// One data bin of the adjoint scatter: its taps and the two values it adds
// (k0 = kNoTap when j is past jmax or outside the cone).  The tap adds
// wgt * e1 at k and wgt * e2 at ntp - k of the model spectrum:
//   rows >= 1: Q[k] = M(+l), Q[ntp-k] = conj M(-l)
//   row 0:     Q[k] = M(0) + i M(N), Q[ntp-k] = conj M(0) + i conj M(N)
struct ScatterBin {
  int k0;
  float4 trig;
  float2 e1, e2;
};

template <int RC>
__device__ __forceinline__ ScatterBin scatter_bin(const RowsArgs& A, const GatherDev& G, const PanelDev& PD,
                                                  bool plain, const float2* bufD, int r, int pass, double a2, int R,
                                                  int j, int jmax) {
  ScatterBin b;
  b.k0 = kNoTap;
  b.trig = make_float4(0.f, 0.f, 1.f, 0.f);
  b.e1 = b.e2 = make_float2(0.f, 0.f);
  if (j > jmax) return b;
  const Taps T = taps_of<RC>(j, a2, R);
  if (T.k0 == kNoTap) return b;
  b.k0 = T.k0;
  b.trig = T.trig;
  // spectrum values of bin j, ramped and scaled
  const float4 dq = reinterpret_cast<const float4*>(bufD)[j];
  float2 du = make_float2(dq.x, dq.y);
  float2 dl = make_float2(dq.z, -dq.w);
  if (plain) {
    du = cscale(du, PD.scale);
    dl = cscale(dl, PD.scale);
  } else {
    const float2 c = bin_factor(G, PD, A.tw, A.wav, j);
    du = cmulconj(du, c);
    dl = cmulconj(dl, c);
  }
  if (r != 0) {
    b.e1 = du;
    b.e2 = cconj(dl);
  } else if (pass == 0) {
    b.e1 = du;
    b.e2 = cconj(du);
  } else {
    b.e1 = make_float2(-dl.y, dl.x);
    b.e2 = make_float2(dl.y, dl.x);
  }
  return b;
}

// Half-width-4 form: the eight weights instead of the trig terms.
struct ScatterBin4 {
  int k0;
  float w[8];
  float2 e1, e2;
};

// MODE 0: a row r >= 1; 1: row 0's l = 0 half (pass 0); 2: its Nyquist half
// (pass 1).  A compile-time mode keeps the per-bin selection of the two
// scattered values out of the bin loop.
template <int MODE>
__device__ __forceinline__ ScatterBin4 scatter_bin4(const RowsArgs& A, const GatherDev& G, const PanelDev& PD,
                                                    bool plain, const float2* bufD, RowA2 a, int j, int jmax) {
  ScatterBin4 b;
  b.k0 = kNoTap;
  b.e1 = b.e2 = make_float2(0.f, 0.f);
#pragma unroll
  for (int t = 0; t < 8; ++t) b.w[t] = 0.f;
  if (j > jmax) return b;
  const Taps4 T = taps4(j, a);
  b.k0 = T.k0;
#pragma unroll
  for (int t = 0; t < 8; ++t) b.w[t] = T.w[t];
  const float4 dq = reinterpret_cast<const float4*>(bufD)[j];
  float2 du = make_float2(dq.x, dq.y);
  float2 dl = make_float2(dq.z, -dq.w);
  if (plain) {
    du = cscale(du, PD.scale);
    dl = cscale(dl, PD.scale);
  } else {
    const float2 c = bin_factor(G, PD, A.tw, A.wav, j);
    du = cmulconj(du, c);
    dl = cmulconj(dl, c);
  }
  if constexpr (MODE == 0) {
    b.e1 = du;
    b.e2 = cconj(dl);
  } else if constexpr (MODE == 1) {
    b.e1 = du;
    b.e2 = cconj(du);
  } else {
    b.e1 = make_float2(-dl.y, dl.x);
    b.e2 = make_float2(dl.y, dl.x);
  }
  return b;
}

template <int N, int RC, int NT>
__device__ __forceinline__ void rows_adj_item(const RowsArgs& A, const WorkItem& w, const GatherDev& G,
                                              float2* lds, const float* ctab, const float* stab) {
  constexpr int NW = NT / 64;
  const int R = RC > 0 ? RC : A.R;
  const int r = w.a, chunk = w.b;
  const int nt = G.nt, ntp = N > 0 ? N : G.ntp, nrows = G.nrows, P = G.npanel;
  const int jlo = G.jlo, jhi = G.jhi;
  const int hmax = ntp / 2 - 1;
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int plen = N > 0 ? fft_padlen(N) : ntp;
  float2* twl = lds;
  float2* bufD = lds + fft_tw_slots(N, ntp);
  float2* bufM = bufD + plen;
  stage_twiddles<N, NT>(twl, A.tw, G.tw_t_off, G.twp_t_off, ntp);

  row_spectrum<N, NT>(bufD, A.H + G.H_off + (long long)r * nt, r, nt, ntp, twl);

  // window rotations cos/sin(pi t / R) in registers (the wave barriers below
  // would otherwise reload them from LDS at every tap)
  constexpr int RT = RC > 0 ? RC : 1;
  float cr[2 * RT], sr[2 * RT];
  if constexpr (RC > 0) {
#pragma unroll
    for (int i = 0; i < 2 * RC; ++i) {
      cr[i] = ctab[i];
      sr[i] = stab[i];
    }
  }

  const int npass = (r == 0) ? 2 : 1;
  // panels chunk, chunk + nchunk, ... as in the forward; rows at or above a
  // panel's live-row count get no taps and their x-spectra are not written
  for (int p = chunk; p < P; p += G.nchunk) {
    const PanelDev PD = A.panels[G.panel_off + p];
    if (r >= PD.rlive) continue;
    const bool plain = (PD.n0 == 0) && (G.wav_off < 0);
    for (int k = threadIdx.x; k < ntp / 2; k += NT) reinterpret_cast<float4*>(bufM)[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    for (int pass = 0; pass < npass; ++pass) {
      const int l = (r == 0) ? (pass == 0 ? 0 : nrows) : r;
      const double a2 = PD.c2 * (double)l * (double)l;
      // segments start at the cone edge (bins below it have no taps)
      const int jb = max(jlo, cone_first_bin(a2));
      const int nseg = jb <= jhi ? (jhi - jb + 64) >> 6 : 0;
      if constexpr (RC > 0) {
        static_assert(RC == 4, "compile-time row kernels use the half-width-4 weight polynomials");
        const RowA2 a = split_a2(a2);
        // Lanes without taps (bins past jhi) scatter zeros into the last
        // eight 16-byte slots of bufD's padding (never read after its
        // transform, N / 16 >= 32 slots), so every lane of a segment runs the
        // same branch-free read-modify-write sequence.
        float4* const sink = reinterpret_cast<float4*>(bufM) - 8;
        auto add = [](float4 v, const ScatterBin4& b, int t) {
          v.x = fmaf(b.w[t], b.e1.x, v.x);
          v.y = fmaf(b.w[t], b.e1.y, v.y);
          v.z = fmaf(b.w[t], b.e2.x, v.z);
          v.w = fmaf(b.w[t], b.e2.y, v.w);
          return v;
        };
        auto scatter = [&](auto mode) {
          constexpr int MODE = decltype(mode)::value;
          for (int ph = 0; ph < 2; ++ph) {
            // a wave takes its segments two at a time (sg and sg + 2 NW, far
            // apart in the band, so their model bins are disjoint): the two
            // read-modify-write chains overlap their LDS latencies
#pragma unroll 1
            for (int sg = 2 * wave + ph; sg < nseg; sg += 4 * NW) {
              // taps below bin 1 land in the padding that ends bufD (never
              // read after its transform), taps past N/2-1 in bufM's own
              // padding (overwritten by its transform), and pair 0 is never
              // read by the inverse transform
              const ScatterBin4 sa = scatter_bin4<MODE>(A, G, PD, plain, bufD, a, jb + sg * 64 + lane, jhi);
              float4* qa = sa.k0 != kNoTap ? reinterpret_cast<float4*>(bufM) + (sa.k0 - 3) : sink;
              const int sg2 = sg + 2 * NW;
              if (sg2 < nseg) {
                const ScatterBin4 sb = scatter_bin4<MODE>(A, G, PD, plain, bufD, a, jb + sg2 * 64 + lane, jhi);
                float4* qb = sb.k0 != kNoTap ? reinterpret_cast<float4*>(bufM) + (sb.k0 - 3) : sink;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                  // both reads before either write (the compiler cannot tell
                  // that qa and qb never alias)
                  const float4 va = qa[t], vb = qb[t];
                  qa[t] = add(va, sa, t);
                  qb[t] = add(vb, sb, t);
                  __builtin_amdgcn_wave_barrier();
                }
              } else {
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                  qa[t] = add(qa[t], sa, t);
                  __builtin_amdgcn_wave_barrier();
                }
              }
            }
            __syncthreads();
          }
        };
        if (r != 0) scatter(std::integral_constant<int, 0>{});
        else if (pass == 0) scatter(std::integral_constant<int, 1>{});
        else scatter(std::integral_constant<int, 2>{});
        continue;
      }
      for (int ph = 0; ph < 2; ++ph) {
#pragma unroll 1
        for (int sg = 2 * wave + ph; sg < nseg; sg += 2 * NW) {
          const ScatterBin sb = scatter_bin<RC>(A, G, PD, plain, bufD, r, pass, a2, R, jb + sg * 64 + lane, jhi);
          if (sb.k0 != kNoTap) {
#pragma unroll
            for (int t = -R + 1; t <= R; ++t) {
              const int k = sb.k0 + t;
              // compile-time lengths skip the test: taps below bin 1 land in
              // the padding that ends bufD (never read after its transform),
              // taps past N/2-1 in bufM's own padding (overwritten by its
              // transform), and pair 0 is never read by the inverse transform
              if (N > 0 || (k >= 1 && k <= hmax)) {
                const float wt = RC > 0 ? tap_weight(sb.trig, t, cr[(t + R - 1) % (2 * RT)], sr[(t + R - 1) % (2 * RT)])
                                        : tap_weight(sb.trig, t, ctab[t + R - 1], stab[t + R - 1]);
                float4* q = reinterpret_cast<float4*>(bufM) + k;
                float4 v = *q;
                v.x = fmaf(wt, sb.e1.x, v.x);
                v.y = fmaf(wt, sb.e1.y, v.y);
                v.z = fmaf(wt, sb.e2.x, v.z);
                v.w = fmaf(wt, sb.e2.y, v.w);
                *q = v;
              }
              __builtin_amdgcn_wave_barrier();
            }
          }
        }
        __syncthreads();
      }
    }
    const float inv_n = 1.0f / (float)ntp;
    float2* __restrict__ dst = A.X + G.X_off + ((long long)p * nrows + r) * nt;
    if constexpr (N > 0) {
      // the last pass's outputs go from registers to global memory
      using O = FftRegsOut<N, NT>;
      O o;
      fft_tpl_from_pairs_to_regs<N, true, NT>(bufM, twl, o);
#pragma unroll
      for (int i = 0; i < O::MAXB; ++i) {
        const int id = (int)threadIdx.x + i * NT;
#pragma unroll
        for (int rr = 0; rr < O::R; ++rr) {
          const int t = id + rr * O::B;
          if (id < O::B && t < nt) dst[t] = cscale(o.v[i][rr], inv_n);
        }
      }
    } else {
      row_inverse_from_pairs<N, NT>(bufM, ntp, twl);
      for (int t = threadIdx.x; t < nt; t += NT) dst[t] = cscale(bufM[px<N>(t)], inv_n);
    }
    __syncthreads();
  }
}

template <int N, int RC>
__global__ __launch_bounds__(row_threads(N)) __attribute__((amdgpu_waves_per_eu(row_waves_per_eu(N)))) void k_rows_adj(RowsArgs A) {
  extern __shared__ float4 lds_raw[];  // 16-byte aligned: the map reads 16-byte pairs
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  __shared__ float ctab[2 * kMaxHalfWidth], stab[2 * kMaxHalfWidth];
  init_tap_trig(ctab, stab, RC > 0 ? RC : A.R);
  __syncthreads();
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const WorkItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    rows_adj_item<N, RC, row_threads(N)>(A, w, G, lds, ctab, stab);
  }
}

// ------------------------------------------------------------ launchers
//
// One instantiation per compile-time FFT length (time: ASHRT_ROW_SIZES with
// R = 4; x: ASHRT_X_SIZES); every other length or half-width runs the
// generic kernels (runtime FFT, runtime R).  The host groups work items by
// the length class so each launch uses one instantiation.
#define ASHRT_ROW_SIZES(X) X(512) X(768) X(1024) X(1536) X(2048) X(3072) X(4096)
#define ASHRT_X_SIZES(X) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

bool rows_size_is_tpl(int n, int R) {
  if (R != 4) return false;
#define C_(S) if (n == S) return true;
  ASHRT_ROW_SIZES(C_)
#undef C_
  return false;
}
bool x_size_is_tpl(int n) {
#define C_(S) if (n == S) return true;
  ASHRT_X_SIZES(C_)
#undef C_
  return false;
}

template <class F>
static void set_lds(F* k, size_t b, hipError_t& e) {
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
}

// Allow every operator kernel the dynamic LDS a plan may request (the
// actual amount is given per launch; occupancy follows the launch value).
hipError_t op_kernels_init(size_t max_lds) {
  hipError_t e = hipSuccess;
#define X_(S) set_lds(k_xfft_fwd<S>, max_lds, e); set_lds(k_xfft_inv<S>, max_lds, e);
  ASHRT_X_SIZES(X_)
#undef X_
  set_lds(k_xfft_fwd<0>, max_lds, e);
  set_lds(k_xfft_inv<0>, max_lds, e);
#define R_(S) set_lds(k_rows_fwd<S, 4>, max_lds, e); set_lds(k_rows_adj<S, 4>, max_lds, e); set_lds(k_rows_fwd_fin<S>, max_lds, e);
  ASHRT_ROW_SIZES(R_)
#undef R_
  set_lds(k_rows_fwd<0, 0>, max_lds, e);
  set_lds(k_rows_adj<0, 0>, max_lds, e);
  set_lds(k_rows_fwd_fin<0>, max_lds, e);
  return e;
}

hipError_t launch_xfft_fwd(int key, const XfwdArgs& a, size_t lds, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  switch (key) {
#define L_(S)                                                                               \
  case S:                                                                                   \
    hipLaunchKernelGGL(k_xfft_fwd<S>, dim3(a.nitems), dim3(kThreads), lds, s, a); \
    break;
    ASHRT_X_SIZES(L_)
#undef L_
    default:
      hipLaunchKernelGGL(k_xfft_fwd<0>, dim3(a.nitems), dim3(kThreads), lds, s, a);
  }
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_xfft_inv(int key, const XinvArgs& a, size_t lds, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  switch (key) {
#define L_(S)                                                                               \
  case S:                                                                                   \
    hipLaunchKernelGGL(k_xfft_inv<S>, dim3(a.nitems), dim3(kThreads), lds, s, a); \
    break;
    ASHRT_X_SIZES(L_)
#undef L_
    default:
      hipLaunchKernelGGL(k_xfft_inv<0>, dim3(a.nitems), dim3(kThreads), lds, s, a);
  }
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_rows_fwd(int key, const RowsArgs& a, size_t lds, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  switch (key) {
#define L_(S)                                                                                  \
  case S:                                                                                      \
    hipLaunchKernelGGL((k_rows_fwd<S, 4>), dim3(a.nitems), dim3(row_threads(S)), lds, s, a); \
    break;
    ASHRT_ROW_SIZES(L_)
#undef L_
    default:
      hipLaunchKernelGGL((k_rows_fwd<0, 0>), dim3(a.nitems), dim3(kRowThreads), lds, s, a);
  }
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_rows_fwd_fin(int key, const RowsArgs& a, size_t lds, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  switch (key) {
#define L_(S)                                                                               \
  case S:                                                                                   \
    hipLaunchKernelGGL(k_rows_fwd_fin<S>, dim3(a.nitems), dim3(kThreads), lds, s, a); \
    break;
    ASHRT_ROW_SIZES(L_)
#undef L_
    default:
      hipLaunchKernelGGL(k_rows_fwd_fin<0>, dim3(a.nitems), dim3(kThreads), lds, s, a);
  }
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_rows_adj(int key, const RowsArgs& a, size_t lds, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  switch (key) {
#define L_(S)                                                                                  \
  case S:                                                                                      \
    hipLaunchKernelGGL((k_rows_adj<S, 4>), dim3(a.nitems), dim3(row_threads(S)), lds, s, a); \
    break;
    ASHRT_ROW_SIZES(L_)
#undef L_
    default:
      hipLaunchKernelGGL((k_rows_adj<0, 0>), dim3(a.nitems), dim3(kRowThreads), lds, s, a);
  }
  return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace ashrt
