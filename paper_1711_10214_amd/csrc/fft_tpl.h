// Compile-time-length Stockham FFT in LDS for 256-thread workgroups.
//
// N = 2^a or 3*2^a.  Passes: one radix-3 pass if 3 | N, then radix-8 passes,
// then one radix-4 or radix-2 pass for the leftover power of two.  Pass i
// with radix R and span Ns (product of the earlier radices) maps
//   v_r = x[j + r N/R] * w^(r (j mod Ns)),  w = exp(-+2 pi i / (Ns R)),
//   y[(j div Ns) Ns R + (j mod Ns) + r Ns] = DFT_R(v)_r .
// Elements live at padded LDS positions fft_pad(i) = i + i/16 (one 8-byte
// gap every 128 bytes), which makes the strided writes of the first passes
// hit distinct banks; a padded transform occupies fft_padlen(N) slots.
// Its twiddles w^(r jm), r = 1..R-1, jm = 0..Ns-1, come from one tabulated
// w^jm per butterfly (FftPlan<N>::twoff(i) + jm in a per-length "pass
// table" built in FP64 on the host) by complex multiplication.  Each pass
// reads its butterflies into registers, waits at a barrier, and writes the
// outputs in place.
#pragma once

#include <hip/hip_runtime.h>

#include "ashrt_internal.h"
#include "fft_lds.h"

namespace ashrt {

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

__host__ __device__ constexpr int fft_pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int fft_padlen(int n) { return n + (n >> 4); }

// True when fft_pad(x + r S) == fft_pad(x) + fft_pad(r S) for every r < R
// and every x congruent mod 16 to q QS + m (q >= 0, 0 <= m < M): no step r S
// carries out of x's low four bits.  A butterfly's R padded addresses are
// then one base plus compile-time offsets, which the LDS instructions take
// as immediates instead of a shift and two adds per element.
constexpr bool pad_linear(int S, int R, int QS, int M) {
  for (int q = 0; q < 16; ++q)
    for (int m = 0; m < M && m < 16; ++m)
      for (int r = 0; r < R; ++r)
        if (((q * QS + m) & 15) + ((r * S) & 15) >= 16) return false;
  return true;
}

// fft_pad(x + c) for a constant c >= 0 from p = fft_pad(x) and lo = x & 15:
// the step adds c + c/16 slots, and one more when x's low four bits carry
// (a compare against a constant instead of a shift and two adds).
__device__ __forceinline__ int pad_step(int p, int lo, int c) {
  return p + c + (c >> 4) + ((c & 15) != 0 && lo >= 16 - (c & 15) ? 1 : 0);
}

// Index of logical element i of a buffer written by an FFT of compile-time
// length N (padded) or by the generic runtime FFT (N == 0, unpadded).
template <int N>
__device__ __forceinline__ int px(int i) {
  if constexpr (N > 0) return fft_pad(i);
  else return i;
}

// The thread index as a fresh value that the compiler cannot relate to any
// other use of threadIdx.x.  Every pass derives its LDS indices from its own
// copy.  With the plain index, the compiler built the address of element
// j + 384 once, as (j | 384), inside the 96-lane guard of pass 1 of the
// 768-point transform (where the bits are disjoint), and reused it in the
// 192-lane radix-4 pass, where lanes 128..191 then read the wrong element.
__device__ __forceinline__ int pass_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

template <int N>
struct FftPlan {
  static constexpr bool three = (N % 3) == 0;
  static constexpr int M = three ? N / 3 : N;
  static constexpr int L = ilog2c(M);
  static constexpr int n8 = L / 3;
  static constexpr int rem = L % 3;
  static constexpr int npass = (three ? 1 : 0) + n8 + (rem ? 1 : 0);
  static constexpr int radix(int i) {
    return (three && i == 0) ? 3 : (i < (three ? 1 : 0) + n8 ? 8 : (rem == 1 ? 2 : 4));
  }
  static constexpr int ns(int i) {
    int s = 1;
    for (int k = 0; k < i; ++k) s *= radix(k);
    return s;
  }
  static constexpr int twoff(int i) {
    int o = 0;
    for (int k = 0; k < i; ++k) o += ns(k);
    return o;
  }
  static constexpr int twsize() { return twoff(npass); }
};

// LDS slots of the staged twiddles in front of an FFT buffer: the pass
// table rounded up to an even count (what follows stays 16-byte aligned), or
// the plain n-entry table of the generic runtime FFT (key 0).
inline __host__ __device__ int fft_tw_slots(int key, int n);

// Host and device: pass-table length for a runtime N of a supported size
// (0 for lengths handled by the generic runtime FFT).
// Lengths with a compile-time FFT (others use the runtime-generic fft_lds).
#define ASHRT_TPL_SIZES(X) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048) X(3072) X(4096)

inline __host__ __device__ int fft_tpl_twsize(int n) {
#define ASHRT_TW_CASE(S) \
  if (n == S) return FftPlan<S>::twsize();
  ASHRT_TPL_SIZES(ASHRT_TW_CASE)
#undef ASHRT_TW_CASE
  return 0;
}

inline __host__ __device__ int fft_tw_slots(int key, int n) { return key > 0 ? (fft_tpl_twsize(key) + 1) & ~1 : n; }


template <bool INV>
__device__ __forceinline__ void dft8(float2 (&v)[8]) {
  constexpr float h = 0.70710678118654752440f;
  float2 b[4], c[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    b[n] = cadd(v[n], v[n + 4]);
    c[n] = csub(v[n], v[n + 4]);
  }
  // c_n *= W^n, W = exp(-+2 pi i / 8)
  {
    const float2 x = c[1];
    c[1] = INV ? make_float2(h * (x.x - x.y), h * (x.x + x.y)) : make_float2(h * (x.x + x.y), h * (x.y - x.x));
    const float2 y = c[2];
    c[2] = INV ? make_float2(-y.y, y.x) : make_float2(y.y, -y.x);
    const float2 z = c[3];
    c[3] = INV ? make_float2(-h * (z.x + z.y), h * (z.x - z.y)) : make_float2(h * (z.y - z.x), -h * (z.x + z.y));
  }
  float2 B[4] = {b[0], b[1], b[2], b[3]};
  float2 C[4] = {c[0], c[1], c[2], c[3]};
  butterfly<4, INV>(B);
  butterfly<4, INV>(C);
  v[0] = B[0];
  v[2] = B[1];
  v[4] = B[2];
  v[6] = B[3];
  v[1] = C[0];
  v[3] = C[1];
  v[5] = C[2];
  v[7] = C[3];
}

template <int R, bool INV>
__device__ __forceinline__ void dft_r(float2 (&v)[R]) {
  if constexpr (R == 8) dft8<INV>(v);
  else butterfly<R, INV>(v);
}

// Pair layout of a length-N spectrum whose bins 0 and N/2 are not needed:
// pair k (1 <= k < N/2) holds bin k at float2 slot 2k and bin N-k at slot
// 2k+1, so a map that touches both mirror bins of k reads 16 bytes at once.
// The pairs occupy the first N float2 slots of the transform's buffer.
template <int N>
__device__ __forceinline__ float2 pair_get(const float2* buf, int i) {
  if (i == 0 || i == N / 2) return make_float2(0.f, 0.f);
  return i < N / 2 ? buf[2 * i] : buf[2 * (N - i) + 1];
}

template <int N>
__device__ __forceinline__ void pair_put(float2* buf, int o, float2 v) {
  if (o == 0 || o == N / 2) return;
  if (o < N / 2) buf[2 * o] = v;
  else buf[2 * (N - o) + 1] = v;
}

// One pass of a batch of nb transforms (nb * N <= NBN) at buf + b*bstride,
// run by a workgroup of NT threads.  IO = 1: this pass reads its input from
// the pair layout; IO = 2: it writes its output in the pair layout (bins 0
// and N/2 dropped; one transform: pair 0 and slots N .. N+7 are zeroed); IO = 3: inputs at index >= nvalid are taken as zero (and
// never read); IO = 4: outputs at index >= nvalid are dropped; IO = 0:
// padded layout both ways.  Reads complete before the barrier and writes
// follow it, so the layouts may share memory.
template <int N, int PASS, int NBN, bool INV, int NT = kThreads, int IO = 0>
__device__ __forceinline__ void tpl_pass(float2* buf, int nb, int bstride, const float2* twp, int nvalid = N) {
  using P = FftPlan<N>;
  constexpr int R = P::radix(PASS);
  constexpr int Ns = P::ns(PASS);
  constexpr int B = N / R;
  constexpr int TW = P::twoff(PASS);
  constexpr int MAXB = (NBN / R + NT - 1) / NT;
  // reads x[j + r B], j < B; writes y[jq Ns R + jm + r Ns], jm < Ns
  constexpr bool RLIN = IO != 1 && pad_linear(B, R, 0, B);
  constexpr bool WLIN = IO != 2 && IO != 4 && pad_linear(Ns, R, Ns * R, Ns);
  // one transform whose butterflies split evenly over the NT threads of the
  // workgroup: every id below is a butterfly, so no lane test is needed
  constexpr bool FULL = NBN == N && B % NT == 0;
  float2 v[MAXB][R];
  int dst[MAXB], bq[MAXB];
  const int total = B * nb;
  const int tid = pass_tid();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int id = tid + i * NT;
    dst[i] = -1;
    if (FULL || id < total) {
      // one transform (NBN == N) has b = 0; indices are non-negative, so
      // unsigned division by the compile-time B and Ns is a shift or mul_hi
      const int b = NBN == N ? 0 : (int)((unsigned)id / (unsigned)B);
      const int j = id - b * B;
      const int jq = (int)((unsigned)j / (unsigned)Ns);
      const int jm = j - jq * Ns;
      const float2* src = buf + b * bstride;
      const float2* s0 = src + fft_pad(j);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (IO == 1 && R % 2 == 0) {
          // B R = N and j < B: element j + r B lies below N/2 exactly when
          // r < R/2, so each read is one of two bases plus a constant
          // (elements 0 and N/2, for j = 0, read a valid slot and are zeroed)
          if (r < R / 2) {
            const float2 x = src[2 * j + 2 * r * B];
            v[i][r] = (r == 0 && j == 0) ? make_float2(0.f, 0.f) : x;
          } else {
            const float2 x = src[2 * (N - j) + 1 - 2 * r * B];
            v[i][r] = (r == R / 2 && j == 0) ? make_float2(0.f, 0.f) : x;
          }
        } else if constexpr (IO == 1) v[i][r] = pair_get<N>(src, j + r * B);
        else if constexpr (IO == 3 && RLIN) v[i][r] = (j + r * B < nvalid) ? s0[fft_pad(r * B)] : make_float2(0.f, 0.f);
        else if constexpr (IO == 3) v[i][r] = (j + r * B < nvalid) ? src[fft_pad(j + r * B)] : make_float2(0.f, 0.f);
        else if constexpr (RLIN) v[i][r] = s0[fft_pad(r * B)];
        else v[i][r] = src[fft_pad(j + r * B)];
      }
      if constexpr (Ns > 1) {
        // w^r by recurrence from the tabulated w = exp(-+2 pi i jm / (Ns R))
        float2 w1 = twp[TW + jm];
        if (INV) w1.y = -w1.y;
        float2 w = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[i][r] = cmul(v[i][r], w);
          if (r + 1 < R) w = cmul(w, w1);
        }
      }
      dft_r<R, INV>(v[i]);
      bq[i] = jq * Ns * R + jm;
      // padded layout: dst is the padded address of bq, and bq keeps only
      // its low four bits when the steps r Ns need them
      if constexpr (IO == 2 || IO == 4) {
        dst[i] = b * bstride;
      } else {
        dst[i] = b * bstride + fft_pad(bq[i]);
        bq[i] &= 15;
      }
    }
  }
  __syncthreads();
  if constexpr (IO == 2) {
    // pair 0 (bins 0 and N) and pairs N/2 .. N/2 + 3 (slots N .. N + 7, in
    // the padding) are left zero: a map reading taps there gets zeros
    static_assert(N >= 128, "pair output needs eight padding slots");
    if (tid < 10) buf[tid < 2 ? tid : N + tid - 2] = make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    if (FULL || dst[i] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (IO == 2 && R % 2 == 0 && Ns * R == N) {
          // last pass: bq = jm < Ns, so output jm + r Ns lies below N/2
          // exactly when r < R/2 (outputs 0 and N/2, for jm = 0, are dropped)
          if (r < R / 2) {
            if (r != 0 || bq[i] != 0) buf[dst[i] + 2 * bq[i] + 2 * r * Ns] = v[i][r];
          } else {
            if (r != R / 2 || bq[i] != 0) buf[dst[i] + 2 * (N - bq[i]) + 1 - 2 * r * Ns] = v[i][r];
          }
        } else if constexpr (IO == 2) {
          pair_put<N>(buf + dst[i], bq[i] + r * Ns, v[i][r]);
        } else if constexpr (IO == 4) {
          if (bq[i] + r * Ns < nvalid) buf[dst[i] + fft_pad(bq[i] + r * Ns)] = v[i][r];
        } else if constexpr (WLIN) {
          buf[dst[i] + fft_pad(r * Ns)] = v[i][r];
        } else {
          buf[pad_step(dst[i], bq[i], r * Ns)] = v[i][r];
        }
      }
    }
  }
  __syncthreads();
}

// PAIRS_IN: the first pass reads the pair layout; PAIRS_OUT: the last pass
// writes it.
// Passes PASS .. END-1 (END defaults to all of them).  MASK_IN: the first
// pass reads only indices < nvalid (the rest is zero); MASK_OUT: the last
// pass writes only indices < nvalid.
template <int N, int PASS, int NBN, bool INV, int NT, bool PAIRS_IN = false, bool PAIRS_OUT = false,
          int END = FftPlan<N>::npass, bool MASK_IN = false, bool MASK_OUT = false>
__device__ __forceinline__ void tpl_passes(float2* buf, int nb, int bstride, const float2* twp, int nvalid = N) {
  if constexpr (PASS < END) {
    constexpr bool last = PASS == FftPlan<N>::npass - 1;
    constexpr int IO = (PAIRS_IN && PASS == 0)   ? 1
                       : (PAIRS_OUT && last)     ? 2
                       : (MASK_IN && PASS == 0)  ? 3
                       : (MASK_OUT && last)      ? 4
                                                 : 0;
    static_assert(!(PAIRS_IN && PAIRS_OUT && FftPlan<N>::npass == 1), "pair input and output need two passes");
    static_assert(!(MASK_IN && MASK_OUT && FftPlan<N>::npass == 1), "masked input and output need two passes");
    tpl_pass<N, PASS, NBN, INV, NT, IO>(buf, nb, bstride, twp, nvalid);
    tpl_passes<N, PASS + 1, NBN, INV, NT, PAIRS_IN, PAIRS_OUT, END, MASK_IN, MASK_OUT>(buf, nb, bstride, twp, nvalid);
  }
}

// Full transform(s); the caller places a barrier after filling buf.
template <int N, int NBN, bool INV, int NT = kThreads>
__device__ __forceinline__ void fft_tpl(float2* buf, int nb, int bstride, const float2* twp) {
  tpl_passes<N, 0, NBN, INV, NT>(buf, nb, bstride, twp);
}

// Full transform(s) of inputs that are zero at index >= nvalid (MASK_IN:
// those slots are never read, so they need not be filled) or of which only
// outputs < nvalid are wanted (MASK_OUT: the others are not written).
template <int N, int NBN, bool INV, bool MASK_IN, bool MASK_OUT, int NT = kThreads>
__device__ __forceinline__ void fft_tpl_masked(float2* buf, int nb, int bstride, const float2* twp, int nvalid) {
  tpl_passes<N, 0, NBN, INV, NT, false, false, FftPlan<N>::npass, MASK_IN, MASK_OUT>(buf, nb, bstride, twp, nvalid);
}

// One transform of length N whose output is left in the pair layout.
template <int N, bool INV, int NT>
__device__ __forceinline__ void fft_tpl_to_pairs(float2* buf, const float2* twp) {
  tpl_passes<N, 0, N, INV, NT, false, true>(buf, 1, fft_padlen(N), twp);
}

// First-pass inputs of a length-N transform held in registers: the
// butterfly with id = threadIdx.x + i NT takes x[id + r N/R0], r < R0 (R0 the
// first radix), so a caller can load them straight from global memory.
template <int N, int NT>
struct FftRegsIn {
  static constexpr int R = FftPlan<N>::radix(0);
  static constexpr int B = N / R;
  static constexpr int MAXB = (B + NT - 1) / NT;
  static_assert(FftPlan<N>::npass >= 2, "register input needs a later pass to write the pair layout");
  float2 v[MAXB][R];
  // x[t] = src[t] for t < nt, zero after
  __device__ __forceinline__ void load(const float2* __restrict__ src, int nt) {
    const int tid = pass_tid();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      const int id = tid + i * NT;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int t = id + r * B;
        v[i][r] = ((B % NT == 0 || id < B) && t < nt) ? src[t] : make_float2(0.f, 0.f);
      }
    }
  }
};

// Transform whose first pass takes its inputs from registers (no twiddles
// there: its span is 1) and whose output is left in the pair layout, in two
// calls: regs_pass0 (the caller must have finished every read of buf; the
// registers are free again when it returns) and rest_to_pairs.
template <int N, bool INV, int NT>
__device__ __forceinline__ void fft_tpl_regs_pass0(float2* buf, FftRegsIn<N, NT>& in) {
  using I = FftRegsIn<N, NT>;
  const int tid = pass_tid();
#pragma unroll
  for (int i = 0; i < I::MAXB; ++i) {
    const int id = tid + i * NT;
    if (I::B % NT == 0 || id < I::B) {
      dft_r<I::R, INV>(in.v[i]);
      constexpr bool LIN = pad_linear(1, I::R, I::R, 1);
      const int p0 = fft_pad(id * I::R), lo = (id * I::R) & 15;
#pragma unroll
      for (int r = 0; r < I::R; ++r) {
        if constexpr (LIN) buf[p0 + r] = in.v[i][r];
        else buf[pad_step(p0, lo, r)] = in.v[i][r];
      }
    }
  }
  __syncthreads();
}

template <int N, bool INV, int NT>
__device__ __forceinline__ void fft_tpl_rest_to_pairs(float2* buf, const float2* twp) {
  tpl_passes<N, 1, N, INV, NT, false, true>(buf, 1, fft_padlen(N), twp);
}

// Outputs of a length-N transform's last pass held in registers: the
// butterfly with id = threadIdx.x + i NT (id < N/RL, RL the last radix) holds
// output element id + r N/RL in v[i][r], so a caller can store them
// straight to global memory.
template <int N, int NT>
struct FftRegsOut {
  static constexpr int L = FftPlan<N>::npass - 1;
  static constexpr int R = FftPlan<N>::radix(L);
  static constexpr int B = N / R;
  static constexpr int MAXB = (B + NT - 1) / NT;
  static_assert(L >= 1 && FftPlan<N>::ns(L) == B, "the last pass spans N/R");
  float2 v[MAXB][R];
};

// Passes FIRST .. last of a transform (FIRST reading the pair layout when
// PAIRS_IN, for FIRST == 0) whose last pass leaves its outputs in
// registers; buf may be reused once every thread has passed a barrier after
// this returns.
template <int N, bool INV, int NT, int FIRST, bool PAIRS_IN>
__device__ __forceinline__ void fft_tpl_passes_to_regs(float2* buf, const float2* twp, FftRegsOut<N, NT>& out) {
  using O = FftRegsOut<N, NT>;
  using P = FftPlan<N>;
  static_assert(!PAIRS_IN || FIRST == 0, "only the first pass reads pairs");
  tpl_passes<N, FIRST, N, INV, NT, PAIRS_IN, false, O::L>(buf, 1, fft_padlen(N), twp);
  constexpr int TW = P::twoff(O::L);
  const int tid = pass_tid();
#pragma unroll
  for (int i = 0; i < O::MAXB; ++i) {
    const int id = tid + i * NT;
    if (O::B % NT == 0 || id < O::B) {
      constexpr bool LIN = pad_linear(O::B, O::R, 0, O::B);
      const float2* s0 = buf + fft_pad(id);
#pragma unroll
      for (int r = 0; r < O::R; ++r) out.v[i][r] = LIN ? s0[fft_pad(r * O::B)] : buf[fft_pad(id + r * O::B)];
      float2 w1 = twp[TW + id];
      if (INV) w1.y = -w1.y;
      float2 w = w1;
#pragma unroll
      for (int r = 1; r < O::R; ++r) {
        out.v[i][r] = cmul(out.v[i][r], w);
        if (r + 1 < O::R) w = cmul(w, w1);
      }
      dft_r<O::R, INV>(out.v[i]);
    }
  }
}

// Transform whose input is read from the pair layout (bins 0 and N/2 taken
// as zero) and whose last pass leaves its outputs in registers.
template <int N, bool INV, int NT>
__device__ __forceinline__ void fft_tpl_from_pairs_to_regs(float2* buf, const float2* twp, FftRegsOut<N, NT>& out) {
  fft_tpl_passes_to_regs<N, INV, NT, 0, true>(buf, twp, out);
}

// One transform of length N whose input is read from the pair layout (bins
// 0 and N/2 taken as zero); the output is in the padded layout.
template <int N, bool INV, int NT>
__device__ __forceinline__ void fft_tpl_from_pairs(float2* buf, const float2* twp) {
  tpl_passes<N, 0, N, INV, NT, true, false>(buf, 1, fft_padlen(N), twp);
}

}  // namespace ashrt
