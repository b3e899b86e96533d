// HIP kernels of the Stolt (A)ASHRT operator pair for gfx950.
//
// Data flow (the same linear operator as F^-1 M F of the thesis' Chapter 5
// operator factorisation, with the two FFT axes taken in the order that lets
// the Stolt map run in LDS):
//
//   forward  m_p[x][t] --(x-RFFT, per time column)--> X_p[l][t]     (HBM)
//            per wavenumber row l (+ its mirror -l): time FFT of X_p[l][:]
//            in LDS, Stolt map (gather over 2R taps) + phase ramp + scale,
//            accumulated over the panels in registers --> partial D (HBM)
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
#include "kernels.h"
#include "fft_lds.h"

namespace ashrt {

// ------------------------------------------------------------ interpolation taps
//
// Hann-windowed sinc h(x) = sinc(x) (1/2 + 1/2 cos(pi x / R)), |x| < R, at
// x = delta - t for the 2R taps t = -R+1..R around floor(u).  Using
// sin(pi (delta - t)) = (-1)^t sin(pi delta) and the angle-difference formula,
// one sincos pair per output bin gives all 2R weights.
struct Taps {
  int k0;       // floor(u), or a large negative sentinel outside the cone
  float4 trig;  // (delta, sin(pi delta)/pi, cos(pi delta/R), sin(pi delta/R))
};

constexpr int kNoTap = -(1 << 28);

// u = sqrt(j^2 - a^2) in FP64 (the coordinate decides the phase of the
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
  float s1, c1, s2, c2;
  sincospif(dl, &s1, &c1);
  sincospif(dl * (1.0f / (float)R), &s2, &c2);
  T.trig = make_float4(dl, s1 * 0.31830988618379067154f, c2, s2);
  return T;
}

// Weight of tap t (k = k0 + t); ct/st = cos/sin(pi t / R).
__device__ __forceinline__ float tap_weight(float4 tr, int t, float ct, float st) {
  const float x = tr.x - (float)t;
  if (x == 0.0f) return 1.0f;
  const float sg = (t & 1) ? -tr.y : tr.y;
  const float win = 0.5f + 0.5f * (tr.z * ct + tr.w * st);
  return sg / x * win;
}

template <int R>
__device__ __forceinline__ void init_tap_trig(float* ct, float* st) {
  if (threadIdx.x < 2 * R) {
    const int t = (int)threadIdx.x - R + 1;
    ct[threadIdx.x] = (float)cospi((double)t / (double)R);
    st[threadIdx.x] = (float)sinpi((double)t / (double)R);
  }
}

// Per data bin j of panel p: W_j s_p exp(-2 pi i j n0 / ntp), from the exact
// FFT twiddle table (the ramp index is reduced with integer arithmetic).
__device__ __forceinline__ float2 bin_factor(const GatherDev& G, const PanelDev& P,
                                             const float2* __restrict__ twt,
                                             const float* __restrict__ wav, int j) {
  float2 e = make_float2(1.0f, 0.0f);
  if (P.n0 != 0) e = twt[(int)(((long long)j * P.n0) % G.ntp)];
  float s = P.scale;
  if (G.wav_off >= 0) s *= wav[G.wav_off + j];
  return cscale(e, s);
}

// ------------------------------------------------------------ x-direction RFFT

__global__ __launch_bounds__(kThreads) void k_xfft_fwd(XfwdArgs A) {
  extern __shared__ float2 lds[];
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const WorkItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    const int p = w.a;
    const int nx = G.nx, nt = G.nt, nxp = G.nxp, nrows = G.nrows;
    const int T = G.tileT, half = T >> 1, bs = nxp + 1;
    const int t0 = w.b * T;
    const long long fbase = A.is_model ? (G.m_off + (long long)p * nx * nt) : G.d_off;
    const float* __restrict__ src = A.src + fbase;
    const float* __restrict__ mul = A.mul ? A.mul + fbase : nullptr;
    const uint8_t* __restrict__ tm = A.tmask ? A.tmask + G.mask_off : nullptr;

    for (int idx = threadIdx.x; idx < nx * half; idx += kThreads) {
      const int x = idx / half;
      const int i = idx - x * half;
      const int t = t0 + 2 * i;
      const long long o = (long long)x * nt + t;
      float a = 0.f, b = 0.f;
      if (t < nt) {
        a = src[o];
        if (mul) a *= mul[o];
      }
      if (t + 1 < nt) {
        b = src[o + 1];
        if (mul) b *= mul[o + 1];
      }
      if (tm && tm[x] == 0) {
        a = 0.f;
        b = 0.f;
      }
      lds[i * bs + x] = make_float2(a, b);
    }
    for (int idx = threadIdx.x; idx < (nxp - nx) * half; idx += kThreads) {
      const int xx = idx / half;
      const int i = idx - xx * half;
      lds[i * bs + nx + xx] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    fft_lds<kThreads, kXfftMaxTotal, false>(lds, nxp, half, bs, A.tw + G.tw_x_off);

    float2* __restrict__ dst = A.dst + (A.is_model ? G.X_off + (long long)p * nrows * nt : G.H_off);
    for (int idx = threadIdx.x; idx < nrows * T; idx += kThreads) {
      const int r = idx / T;
      const int c = idx - r * T;
      const int t = t0 + c;
      if (t >= nt) continue;
      const float2* Z = lds + (c >> 1) * bs;
      float2 out;
      if (r == 0) {
        const float2 z0 = Z[0], zn = Z[nrows];
        out = (c & 1) ? make_float2(z0.y, zn.y) : make_float2(z0.x, zn.x);
      } else {
        const float2 a = Z[r];
        const float2 b = cconj(Z[nxp - r]);
        out = (c & 1) ? make_float2(0.5f * (a.y - b.y), -0.5f * (a.x - b.x))
                      : make_float2(0.5f * (a.x + b.x), 0.5f * (a.y + b.y));
      }
      dst[(long long)r * nt + t] = out;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ x-direction C2R

__global__ __launch_bounds__(kThreads) void k_xfft_inv(XinvArgs A) {
  extern __shared__ float2 lds[];
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const WorkItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    const int p = w.a;
    const int nx = G.nx, nt = G.nt, nxp = G.nxp, nrows = G.nrows;
    const int T = G.tileT, half = T >> 1, bs = nxp + 1;
    const int t0 = w.b * T;
    const float2* __restrict__ src = A.src + (A.is_model ? G.X_off + (long long)p * nrows * nt : G.H_off);

    for (int idx = threadIdx.x; idx < nrows * half; idx += kThreads) {
      const int l = idx / half;
      const int i = idx - l * half;
      const int t = t0 + 2 * i;
      float2 h1 = make_float2(0.f, 0.f), h2 = make_float2(0.f, 0.f);
      if (t < nt) h1 = src[(long long)l * nt + t];
      if (t + 1 < nt) h2 = src[(long long)l * nt + t + 1];
      float2* Z = lds + i * bs;
      if (l == 0) {
        Z[0] = make_float2(h1.x, h2.x);
        Z[nrows] = make_float2(h1.y, h2.y);
      } else {
        Z[l] = make_float2(h1.x - h2.y, h1.y + h2.x);
        Z[nxp - l] = make_float2(h1.x + h2.y, -h1.y + h2.x);
      }
    }
    __syncthreads();
    fft_lds<kThreads, kXfftMaxTotal, true>(lds, nxp, half, bs, A.tw + G.tw_x_off);

    const float inv = 1.0f / (float)nxp;
    const long long fbase = A.is_model ? (G.m_off + (long long)p * nx * nt) : G.d_off;
    const uint8_t* __restrict__ tm = A.tmask ? A.tmask + G.mask_off : nullptr;
    for (int idx = threadIdx.x; idx < nx * T; idx += kThreads) {
      const int x = idx / T;
      const int c = idx - x * T;
      const int t = t0 + c;
      if (t >= nt) continue;
      const float2 z = lds[(c >> 1) * bs + x];
      float v = ((c & 1) ? z.y : z.x) * inv;
      const long long o = fbase + (long long)x * nt + t;
      if (A.raw_out) A.raw_out[o] = v;
      if (A.sub) v = A.sub[o] - v;
      if (tm && tm[x] == 0) v = 0.f;
      if (A.wmul) v *= A.wmul[o];
      A.out[o] = v;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ forward rows

// Load row r of a [nrows][nt] complex field into buf[0..nt), zero to ntp,
// forward time FFT, and for row 0 separate the packed kx = 0 / Nyquist
// spectra: slot k gets the kx = 0 spectrum, slot ntp-k the conjugate of the
// Nyquist one, so that both rows read "up = buf[k], lo = conj(buf[ntp-k])".
__device__ __forceinline__ void row_spectrum(float2* buf, const float2* __restrict__ src, int r,
                                             int nt, int ntp, const float2* __restrict__ twt) {
  for (int t = threadIdx.x; t < ntp; t += kThreads) buf[t] = (t < nt) ? src[t] : make_float2(0.f, 0.f);
  __syncthreads();
  fft_lds<kThreads, kRowMaxN, false>(buf, ntp, 1, ntp, twt);
  if (r == 0) {
    for (int k = 1 + threadIdx.x; k < ntp / 2; k += kThreads) {
      const float2 a = buf[k];
      const float2 b = cconj(buf[ntp - k]);
      const float2 m0 = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y + b.y));
      const float2 m1 = make_float2(0.5f * (a.y - b.y), -0.5f * (a.x - b.x));
      buf[k] = m0;
      buf[ntp - k] = cconj(m1);
    }
    __syncthreads();
  }
}

template <int R>
__global__ __launch_bounds__(kThreads) void k_rows_fwd(RowsArgs A) {
  extern __shared__ float2 lds[];
  __shared__ float ctab[2 * R], stab[2 * R];
  init_tap_trig<R>(ctab, stab);
  __syncthreads();
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const WorkItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    const int r = w.a, chunk = w.b;
    const int nt = G.nt, ntp = G.ntp, nrows = G.nrows, P = G.npanel;
    const int jlo = G.jlo, jhi = G.jhi, nband = jhi - jlo + 1;
    const int p0 = (int)((long long)chunk * P / G.nchunk);
    const int p1 = (int)((long long)(chunk + 1) * P / G.nchunk);
    const int hmax = ntp / 2 - 1;
    const float2* __restrict__ twt = A.tw + G.tw_t_off;
    const double lup2 = (double)(r == 0 ? 0 : r) * (double)(r == 0 ? 0 : r);
    const double llo2 = (double)(r == 0 ? nrows : r) * (double)(r == 0 ? nrows : r);

    float2 dup[kMaxSlots], dlo[kMaxSlots];
#pragma unroll
    for (int s = 0; s < kMaxSlots; ++s) {
      dup[s] = make_float2(0.f, 0.f);
      dlo[s] = make_float2(0.f, 0.f);
    }
    for (int p = p0; p < p1; ++p) {
      row_spectrum(lds, A.X + G.X_off + ((long long)p * nrows + r) * nt, r, nt, ntp, twt);
      const PanelDev PD = A.panels[G.panel_off + p];
#pragma unroll
      for (int s = 0; s < kMaxSlots; ++s) {
        const int j = jlo + (int)threadIdx.x + s * kThreads;
        if (j > jhi) break;
        const float2 cj = bin_factor(G, PD, twt, A.wav, j);
        const Taps tu = make_taps<R>(j, PD.c2 * lup2);
        const Taps tl = (r == 0) ? make_taps<R>(j, PD.c2 * llo2) : tu;
        float2 au = make_float2(0.f, 0.f), al = make_float2(0.f, 0.f);
        if (tu.k0 != kNoTap) {
#pragma unroll
          for (int t = -R + 1; t <= R; ++t) {
            const int k = tu.k0 + t;
            if (k >= 1 && k <= hmax) au = cfma(tap_weight(tu.trig, t, ctab[t + R - 1], stab[t + R - 1]), lds[k], au);
          }
        }
        if (tl.k0 != kNoTap) {
#pragma unroll
          for (int t = -R + 1; t <= R; ++t) {
            const int k = tl.k0 + t;
            if (k >= 1 && k <= hmax)
              al = cfma(tap_weight(tl.trig, t, ctab[t + R - 1], stab[t + R - 1]), cconj(lds[ntp - k]), al);
          }
        }
        dup[s] = cadd(dup[s], cmul(cj, au));
        dlo[s] = cadd(dlo[s], cmul(cj, al));
      }
      __syncthreads();
    }
    float2* __restrict__ dp = A.Dp + G.Dp_off + ((long long)chunk * nrows + r) * 2 * nband;
#pragma unroll
    for (int s = 0; s < kMaxSlots; ++s) {
      const int j = jlo + (int)threadIdx.x + s * kThreads;
      if (j > jhi) break;
      dp[j - jlo] = dup[s];
      dp[nband + j - jlo] = dlo[s];
    }
  }
}

// Sum the panel-chunk partials of row r, complete the Hermitian time
// spectrum (rows >= 1: Q[j] = D(+l,j), Q[ntp-j] = conj D(-l,j); row 0:
// Q[j] = D(0,j) + i D(N,j), Q[ntp-j] = conj D(0,j) + i conj D(N,j)), inverse
// time FFT, scale 1/ntp, keep t < nt.
__global__ __launch_bounds__(kThreads) void k_rows_fwd_fin(RowsArgs A) {
  extern __shared__ float2 lds[];
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const WorkItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    const int r = w.a;
    const int nt = G.nt, ntp = G.ntp, nrows = G.nrows;
    const int jlo = G.jlo, jhi = G.jhi, nband = jhi - jlo + 1;
    for (int k = threadIdx.x; k < ntp; k += kThreads) {
      float2 v = make_float2(0.f, 0.f);
      const int j = (k >= jlo && k <= jhi) ? k : ((ntp - k >= jlo && ntp - k <= jhi) ? ntp - k : -1);
      if (j >= 0) {
        float2 su = make_float2(0.f, 0.f), sl = make_float2(0.f, 0.f);
        for (int c = 0; c < G.nchunk; ++c) {
          const float2* dp = A.Dp + G.Dp_off + ((long long)c * nrows + r) * 2 * nband;
          su = cadd(su, dp[j - jlo]);
          sl = cadd(sl, dp[nband + j - jlo]);
        }
        if (j == k) {
          v = (r == 0) ? make_float2(su.x - sl.y, su.y + sl.x) : su;
        } else {
          v = (r == 0) ? make_float2(su.x + sl.y, -su.y + sl.x) : cconj(sl);
        }
      }
      lds[k] = v;
    }
    __syncthreads();
    fft_lds<kThreads, kRowMaxN, true>(lds, ntp, 1, ntp, A.tw + G.tw_t_off);
    const float inv = 1.0f / (float)ntp;
    float2* __restrict__ dst = A.H + G.H_off + (long long)r * nt;
    for (int t = threadIdx.x; t < nt; t += kThreads) dst[t] = cscale(lds[t], inv);
    __syncthreads();
  }
}

// ------------------------------------------------------------ adjoint rows
//
// LDS: bufD[ntp] (data time spectrum of the row), bufM[ntp] (per panel: first
// the ramp-weighted data bins E(j) = conj(c_pj) D(j), then the model
// spectrum), and per-bin tap tables (k0, trig) over the band.
template <int R>
__global__ __launch_bounds__(kThreads) void k_rows_adj(RowsArgs A) {
  extern __shared__ float2 lds[];
  __shared__ float ctab[2 * R], stab[2 * R];
  init_tap_trig<R>(ctab, stab);
  __syncthreads();
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const WorkItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    const int r = w.a, chunk = w.b;
    const int nt = G.nt, ntp = G.ntp, nrows = G.nrows, P = G.npanel;
    const int jlo = G.jlo, jhi = G.jhi, nband = jhi - jlo + 1;
    const int kmax = G.kmax;
    const int p0 = (int)((long long)chunk * P / G.nchunk);
    const int p1 = (int)((long long)(chunk + 1) * P / G.nchunk);
    const float2* __restrict__ twt = A.tw + G.tw_t_off;
    float2* bufD = lds;
    float2* bufM = lds + ntp;
    float4* tab_tr = reinterpret_cast<float4*>(lds + 2 * ntp);
    int* tab_k0 = reinterpret_cast<int*>(tab_tr + nband);

    row_spectrum(bufD, A.H + G.H_off + (long long)r * nt, r, nt, ntp, twt);

    const int npass = (r == 0) ? 2 : 1;
    for (int p = p0; p < p1; ++p) {
      const PanelDev PD = A.panels[G.panel_off + p];
      float2 mup[kMaxSlots], mlo[kMaxSlots];
#pragma unroll
      for (int s = 0; s < kMaxSlots; ++s) {
        mup[s] = make_float2(0.f, 0.f);
        mlo[s] = make_float2(0.f, 0.f);
      }
      for (int pass = 0; pass < npass; ++pass) {
        const int l = (r == 0) ? (pass == 0 ? 0 : nrows) : r;
        const double a2 = PD.c2 * (double)l * (double)l;
        // phase 1: taps and ramp-weighted data per band bin
        for (int j = jlo + threadIdx.x; j <= jhi; j += kThreads) {
          const Taps T = make_taps<R>(j, a2);
          tab_k0[j - jlo] = T.k0;
          tab_tr[j - jlo] = T.trig;
          const float2 cj = bin_factor(G, PD, twt, A.wav, j);
          bufM[j] = cmulconj(bufD[j], cj);                   // E_up(j) = conj(c) D(+l, j)
          bufM[ntp - j] = cmulconj(cconj(bufD[ntp - j]), cj);  // E_lo(j) = conj(c) D(-l, j)
        }
        __syncthreads();
        // phase 2: gather, one model bin k per thread slot
        const float a2f = (float)a2;
#pragma unroll
        for (int s = 0; s < kMaxSlots; ++s) {
          const int k = 1 + (int)threadIdx.x + s * kThreads;
          if (k > kmax) break;
          const float lo = (float)max(k - R, 0);
          const float hi = (float)(k + R);
          int ja = (int)ceilf(sqrtf(lo * lo + a2f)) - 1;
          int jb = (int)ceilf(sqrtf(hi * hi + a2f)) + 1;
          ja = max(ja, jlo);
          jb = min(jb, jhi);
          float2 au = make_float2(0.f, 0.f), al = make_float2(0.f, 0.f);
          for (int j = ja; j <= jb; ++j) {
            const int t = k - tab_k0[j - jlo];
            if (t < -R + 1 || t > R) continue;
            const float wgt = tap_weight(tab_tr[j - jlo], t, ctab[t + R - 1], stab[t + R - 1]);
            if (r != 0 || pass == 0) au = cfma(wgt, bufM[j], au);
            if (r != 0 || pass == 1) al = cfma(wgt, bufM[ntp - j], al);
          }
          if (r != 0 || pass == 0) mup[s] = au;
          if (r != 0 || pass == 1) mlo[s] = al;
        }
        __syncthreads();
      }
      // model time spectrum of panel p, then inverse time FFT
      for (int k = threadIdx.x; k < ntp; k += kThreads) bufM[k] = make_float2(0.f, 0.f);
      __syncthreads();
#pragma unroll
      for (int s = 0; s < kMaxSlots; ++s) {
        const int k = 1 + (int)threadIdx.x + s * kThreads;
        if (k > kmax) break;
        const float2 u = mup[s], v = mlo[s];
        if (r == 0) {
          bufM[k] = make_float2(u.x - v.y, u.y + v.x);
          bufM[ntp - k] = make_float2(u.x + v.y, -u.y + v.x);
        } else {
          bufM[k] = u;
          bufM[ntp - k] = cconj(v);
        }
      }
      __syncthreads();
      fft_lds<kThreads, kRowMaxN, true>(bufM, ntp, 1, ntp, twt);
      const float inv = 1.0f / (float)ntp;
      float2* __restrict__ dst = A.X + G.X_off + ((long long)p * nrows + r) * nt;
      for (int t = threadIdx.x; t < nt; t += kThreads) dst[t] = cscale(bufM[t], inv);
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------ launchers
template <int R>
static void launch_rows_fwd_t(const RowsArgs& a, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_rows_fwd<R>, dim3(a.nitems), dim3(kThreads), lds, s, a);
}
template <int R>
static void launch_rows_adj_t(const RowsArgs& a, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_rows_adj<R>, dim3(a.nitems), dim3(kThreads), lds, s, a);
}

#define ASHRT_R_SWITCH(R, CALL) \
  switch (R) {                  \
    case 1: CALL(1); break;     \
    case 2: CALL(2); break;     \
    case 3: CALL(3); break;     \
    case 4: CALL(4); break;     \
    case 5: CALL(5); break;     \
    case 6: CALL(6); break;     \
    case 7: CALL(7); break;     \
    case 8: CALL(8); break;     \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_xfft_fwd(const XfwdArgs& a, size_t lds, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xfft_fwd, dim3(a.nitems), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}
hipError_t launch_xfft_inv(const XinvArgs& a, size_t lds, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xfft_inv, dim3(a.nitems), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}
hipError_t launch_rows_fwd(int R, const RowsArgs& a, size_t lds, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
#define CALLF(RR) launch_rows_fwd_t<RR>(a, lds, s)
  ASHRT_R_SWITCH(R, CALLF)
#undef CALLF
  return hipGetLastError();
}
hipError_t launch_rows_fwd_fin(const RowsArgs& a, size_t lds, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_fwd_fin, dim3(a.nitems), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}
hipError_t launch_rows_adj(int R, const RowsArgs& a, size_t lds, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
#define CALLA(RR) launch_rows_adj_t<RR>(a, lds, s)
  ASHRT_R_SWITCH(R, CALLA)
#undef CALLA
  return hipGetLastError();
}

// Raise the dynamic-LDS limit of every operator kernel (gfx950 has 160 KB per CU).
hipError_t op_kernels_set_lds(size_t xfft, size_t rows_fwd, size_t rows_adj) {
  hipError_t e = hipSuccess;
#define SETA(K, B) \
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)(K), hipFuncAttributeMaxDynamicSharedMemorySize, (int)(B))
  SETA(k_xfft_fwd, xfft);
  SETA(k_xfft_inv, xfft);
  SETA(k_rows_fwd_fin, rows_fwd);
  SETA(k_rows_fwd<1>, rows_fwd); SETA(k_rows_fwd<2>, rows_fwd); SETA(k_rows_fwd<3>, rows_fwd);
  SETA(k_rows_fwd<4>, rows_fwd); SETA(k_rows_fwd<5>, rows_fwd); SETA(k_rows_fwd<6>, rows_fwd);
  SETA(k_rows_fwd<7>, rows_fwd); SETA(k_rows_fwd<8>, rows_fwd);
  SETA(k_rows_adj<1>, rows_adj); SETA(k_rows_adj<2>, rows_adj); SETA(k_rows_adj<3>, rows_adj);
  SETA(k_rows_adj<4>, rows_adj); SETA(k_rows_adj<5>, rows_adj); SETA(k_rows_adj<6>, rows_adj);
  SETA(k_rows_adj<7>, rows_adj); SETA(k_rows_adj<8>, rows_adj);
#undef SETA
  return e;
}

}  // namespace ashrt
