// HIP kernels of the warm-start U-Net for gfx950.
//
// 3x3 convolutions (forward and input-gradient) and their weight gradients
// run on the BF16 matrix cores, v_mfma_f32_16x16x32_bf16: a wave multiplies
// a 16 x 32 BF16 tile A by a 32 x 16 tile B into a 16 x 16 FP32 tile.
// Lane l supplies A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16]
// (i = 0..7, eight consecutive BF16 values = 16 bytes) and receives
// D[4 (l / 16) + i][l % 16] (i = 0..3).
//
// Forward convolution: A = packed weights (rows = output channels, k =
// (tap, input channel)), B = the input tile staged in LDS as [row][col][ci]
// (so eight consecutive channels of one tap are one 16-byte read), D =
// output channels x pixels, written as four consecutive channels of one
// pixel (NHWC).  The input-gradient is the same kernel on the gradient of
// the output's pre-activation with the transposed, tap-flipped weights; its
// epilogue routes the result to the tensors the forward input was built
// from (ConvRoute).  Launches with few workgroups split the channel chunks
// over workgroups and finish in k_conv_finish.
// Weight gradient: A = output gradient, B = input, k = pixels, both staged
// [pixel][channel] and read with the LDS transpose read; workgroups split
// the pixels and write FP32 partials that one kernel for all layers sums in
// a fixed order.
#include "unet_internal.h"

namespace unet {

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint32_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ uint4 pack8(const float v[8]) {
  uint4 r;
  r.x = f2bf(v[0]) | (f2bf(v[1]) << 16);
  r.y = f2bf(v[2]) | (f2bf(v[3]) << 16);
  r.z = f2bf(v[4]) | (f2bf(v[5]) << 16);
  r.w = f2bf(v[6]) | (f2bf(v[7]) << 16);
  return r;
}

__device__ __forceinline__ void unpack8(uint4 q, float v[8]) {
  v[0] = bf2f(q.x & 0xFFFFu);
  v[1] = bf2f(q.x >> 16);
  v[2] = bf2f(q.y & 0xFFFFu);
  v[3] = bf2f(q.y >> 16);
  v[4] = bf2f(q.z & 0xFFFFu);
  v[5] = bf2f(q.z >> 16);
  v[6] = bf2f(q.w & 0xFFFFu);
  v[7] = bf2f(q.w >> 16);
}

// ReLU derivative from the stored (post-ReLU) BF16 output: 1 where it is > 0.
__device__ __forceinline__ bool relu_on(uint32_t h) { return (h & 0x8000u) == 0 && (h & 0x7FFFu) != 0; }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Channels [c, c + 8) of conv-input pixel (b, y, x); zero outside the image
// and beyond the real channels.  c is a multiple of 8, and so are Ca and Cb
// unless Ca == 1 (the FP32 network input).
template <bool AF32>
__device__ __forceinline__ void load_in8(const ConvIn& I, int b, int y, int x, int c, float v[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = 0.f;
  if (y < 0 || y >= I.H || x < 0 || x >= I.W) return;
  if (c < I.Ca) {
    if constexpr (AF32) {
      const float* A = static_cast<const float*>(I.A);
      if (I.Ca == 1) {
        v[0] = A[((long long)b * I.H + y) * I.W + x];
      } else {
        const long long o = (((long long)b * I.H + y) * I.W + x) * I.Ca + c;
        const float4 p = *reinterpret_cast<const float4*>(A + o);
        const float4 q = *reinterpret_cast<const float4*>(A + o + 4);
        v[0] = p.x; v[1] = p.y; v[2] = p.z; v[3] = p.w;
        v[4] = q.x; v[5] = q.y; v[6] = q.z; v[7] = q.w;
      }
    } else {
      const uint16_t* A = static_cast<const uint16_t*>(I.A);
      if (I.modeA == 0) {
        unpack8(*reinterpret_cast<const uint4*>(A + (((long long)b * I.H + y) * I.W + x) * I.Ca + c), v);
      } else if (I.modeA == 1) {
        const int Ha = I.H >> 1, Wa = I.W >> 1;
        unpack8(*reinterpret_cast<const uint4*>(A + (((long long)b * Ha + (y >> 1)) * Wa + (x >> 1)) * I.Ca + c),
                v);
      } else {
        const int Ha = I.H * 2, Wa = I.W * 2;
        float t[8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ya = 2 * y + (q >> 1), xa = 2 * x + (q & 1);
          unpack8(*reinterpret_cast<const uint4*>(A + (((long long)b * Ha + ya) * Wa + xa) * I.Ca + c), t);
#pragma unroll
          for (int i = 0; i < 8; ++i) v[i] += t[i];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] *= 0.25f;
      }
    }
  } else if (c < I.Ca + I.Cb) {
    unpack8(*reinterpret_cast<const uint4*>(I.Bs + (((long long)b * I.H + y) * I.W + x) * I.Cb + (c - I.Ca)), v);
  }
}

// Source of channels [c, c + 8) of conv-input pixel (b, y, x) for a BF16
// loader without pooling (A at the same or at half resolution, and the
// skip): one 16-byte load, or null where the channels are zero.
__device__ __forceinline__ const uint4* in8_src(const ConvIn& I, int b, int y, int x, int c) {
  if (y < 0 || y >= I.H || x < 0 || x >= I.W) return nullptr;
  if (c < I.Ca) {
    const uint16_t* A = static_cast<const uint16_t*>(I.A);
    if (I.modeA == 0) return reinterpret_cast<const uint4*>(A + (((long long)b * I.H + y) * I.W + x) * I.Ca + c);
    const int Ha = I.H >> 1, Wa = I.W >> 1;
    return reinterpret_cast<const uint4*>(A + (((long long)b * Ha + (y >> 1)) * Wa + (x >> 1)) * I.Ca + c);
  }
  if (c < I.Ca + I.Cb)
    return reinterpret_cast<const uint4*>(I.Bs + (((long long)b * I.H + y) * I.W + x) * I.Cb + (c - I.Ca));
  return nullptr;
}

// Stage the (rows x cols) input tile of channel chunk [c0, c0 + 8 ng) into
// LDS as [pixel][channel] with pixel stride PS, pixel (r, q) of the tile
// being input pixel (y0 + r, x0 + q).  Loaders without pooling (BF16
// activations, the FP32 gradient) issue the loads of several tasks before
// storing any, so that a thread waits on one memory latency per group of
// tasks rather than per task.
template <bool AF32>
__device__ __forceinline__ void stage_tile(const ConvIn& I, int b, int y0, int x0, int rows, int cols, int c0,
                                           int ng, uint16_t* dst, int PS) {
  const int ntask = rows * cols * ng;
  if (!AF32 && I.modeA != 2) {
    constexpr int U = 4;
    for (int t0 = threadIdx.x; t0 < ntask; t0 += U * 256) {
      uint4 q[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int task = t0 + u * 256;
        q[u] = make_uint4(0u, 0u, 0u, 0u);
        if (task < ntask) {
          const int g = task % ng, pix = task / ng;
          const int r = pix / cols, x = pix - r * cols;
          const uint4* src = in8_src(I, b, y0 + r, x0 + x, c0 + g * 8);
          if (src) q[u] = *src;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int task = t0 + u * 256;
        if (task < ntask) *reinterpret_cast<uint4*>(dst + (task / ng) * PS + (task % ng) * 8) = q[u];
      }
    }
  } else if (AF32 && I.Ca > 1 && I.Cb == 0 && I.modeA == 0) {
    constexpr int U = 4;
    const float* A = static_cast<const float*>(I.A);
    for (int t0 = threadIdx.x; t0 < ntask; t0 += U * 256) {
      float4 p[U], q[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int task = t0 + u * 256;
        p[u] = q[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (task < ntask) {
          const int g = task % ng, pix = task / ng;
          const int r = pix / cols, x = pix - r * cols;
          const int y = y0 + r, xx = x0 + x, c = c0 + g * 8;
          if (y >= 0 && y < I.H && xx >= 0 && xx < I.W && c < I.Ca) {
            const long long o = (((long long)b * I.H + y) * I.W + xx) * I.Ca + c;
            p[u] = *reinterpret_cast<const float4*>(A + o);
            q[u] = *reinterpret_cast<const float4*>(A + o + 4);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int task = t0 + u * 256;
        if (task < ntask) {
          const float v[8] = {p[u].x, p[u].y, p[u].z, p[u].w, q[u].x, q[u].y, q[u].z, q[u].w};
          *reinterpret_cast<uint4*>(dst + (task / ng) * PS + (task % ng) * 8) = pack8(v);
        }
      }
    }
  } else {
    for (int task = threadIdx.x; task < ntask; task += 256) {
      const int g = task % ng, pix = task / ng;
      const int r = pix / cols, x = pix - r * cols;
      float v[8];
      load_in8<AF32>(I, b, y0 + r, x0 + x, c0 + g * 8, v);
      *reinterpret_cast<uint4*>(dst + pix * PS + g * 8) = pack8(v);
    }
  }
}

// ------------------------------------------------------------ routed epilogue
// float4 store or accumulate of four consecutive channels, each zeroed where
// the activation m (four BF16 values, or null: none) is not positive.
__device__ __forceinline__ void put4(float* p, const uint16_t* m, float v0, float v1, float v2, float v3, bool add) {
  if (m) {
    const uint2 h = *reinterpret_cast<const uint2*>(m);
    if (!relu_on(h.x & 0xFFFFu)) v0 = 0.f;
    if (!relu_on(h.x >> 16)) v1 = 0.f;
    if (!relu_on(h.y & 0xFFFFu)) v2 = 0.f;
    if (!relu_on(h.y >> 16)) v3 = 0.f;
  }
  float4 o = make_float4(v0, v1, v2, v3);
  if (add) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    o.x += q.x;
    o.y += q.y;
    o.z += q.z;
    o.w += q.w;
  }
  *reinterpret_cast<float4*>(p) = o;
}

// The value held by lane l ^ 1 (DPP quad permutation 1, 0, 3, 2).
__device__ __forceinline__ float lane_pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// Epilogue of an input-gradient convolution (see ConvRoute): lane (sub, n16)
// of wave w holds channels co0 + 16 mi + 4 sub + [0, 4) of pixel (ty0 + w,
// tx0 + 16 ni + n16).  An upsampled A (UP, mode 1) sums each 2 x 2 pixel
// block: the two columns by a lane exchange, then the two rows (waves 2k and
// 2k + 1) through LDS, (g00 + g01) + (g10 + g11); every wave reaches that
// barrier.  UP is a template parameter so that the other input gradients do
// not carry its registers.
template <int MT, int NTL, bool UP>
__device__ __forceinline__ void route_store(const ConvArgs& a, f32x4 (&acc)[MT][NTL], int b, int ty0, int tx0,
                                            int co0, int MI, float* red) {
  const ConvRoute& R = a.rt;
  const int H = a.in.H, W = a.in.W;
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int sub = lane >> 4, n16 = lane & 15;
  const int y = ty0 + wave;
  if constexpr (UP) {
    // column-pair sums (DPP lane swap) of the A tiles, written by the even
    // lanes of every wave to LDS as [row][A column][channel of the tile]
    // (16-channel tiles lie wholly in A or in B, Ca being a multiple of 16);
    // then every thread adds the two rows of an A pixel and stores four of
    // its channels, consecutive threads taking consecutive channels, then
    // A columns, so that the stores are contiguous
    constexpr int XA = 8 * NTL;        // A columns of the tile
    constexpr int CS = 16 * MT + 4;    // LDS floats per A column of a row
    const int MA = max(0, min(MI, (R.Ca - co0) >> 4));  // A tiles of this workgroup
#pragma unroll
    for (int mi = 0; mi < MT; ++mi) {
      if (mi >= MA) continue;
#pragma unroll
      for (int ni = 0; ni < NTL; ++ni) {
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[mi][ni][i] += lane_pair_swap(acc[mi][ni][i]);
        if (!(n16 & 1))
          *reinterpret_cast<float4*>(red + (wave * XA + ((ni * 16 + n16) >> 1)) * CS + mi * 16 + sub * 4) =
              make_float4(acc[mi][ni][0], acc[mi][ni][1], acc[mi][ni][2], acc[mi][ni][3]);
      }
    }
    __syncthreads();
    const int ng = MA * 4, Hh = H >> 1, Wh = W >> 1;
    for (int idx = (int)threadIdx.x; idx < 2 * XA * ng; idx += 256) {
      const int g = idx % ng, rest = idx / ng;
      const int xa = rest % XA, ya = rest / XA;
      const int yh = (ty0 >> 1) + ya, xh = (tx0 >> 1) + xa;
      if (yh >= Hh || xh >= Wh) continue;
      // (g00 + g01) + (g10 + g11): row 2 ya, then row 2 ya + 1
      const float4 r0 = *reinterpret_cast<const float4*>(red + ((2 * ya) * XA + xa) * CS + 4 * g);
      const float4 r1 = *reinterpret_cast<const float4*>(red + ((2 * ya + 1) * XA + xa) * CS + 4 * g);
      const long long oa = (((long long)b * Hh + yh) * Wh + xh) * R.Ca + co0 + 4 * g;
      put4(R.gA + oa, R.mA ? R.mA + oa : nullptr, r0.x + r1.x, r0.y + r1.y, r0.z + r1.z, r0.w + r1.w,
           R.accA != 0);
    }
  }
  if (y >= H) return;
#pragma unroll
  for (int mi = 0; mi < MT; ++mi) {
    const int co = co0 + mi * 16 + sub * 4;
    if (mi >= MI || co >= R.Ca + R.Cb) continue;
    if (UP && co < R.Ca) continue;  // stored above
#pragma unroll
    for (int ni = 0; ni < NTL; ++ni) {
      const int x = tx0 + ni * 16 + n16;
      if (x >= W) continue;
      const f32x4 o = acc[mi][ni];
      if (co >= R.Ca) {
        const long long ob = (((long long)b * H + y) * W + x) * R.Cb + (co - R.Ca);
        put4(R.gB + ob, R.mB ? R.mB + ob : nullptr, o[0], o[1], o[2], o[3], R.accB != 0);
      } else if (R.modeA == 0) {
        const long long oa = (((long long)b * H + y) * W + x) * R.Ca + co;
        put4(R.gA + oa, R.mA ? R.mA + oa : nullptr, o[0], o[1], o[2], o[3], R.accA != 0);
      } else {
        // mode 2 (pooled A): an upsampled A (mode 1) always launches with UP
        // set, or split with the route left to k_conv_finish
        const int H2 = 2 * H, W2 = 2 * W;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const long long oa = (((long long)b * H2 + 2 * y + (q >> 1)) * W2 + 2 * x + (q & 1)) * R.Ca + co;
          put4(R.gA + oa, R.mA ? R.mA + oa : nullptr, 0.25f * o[0], 0.25f * o[1], 0.25f * o[2], 0.25f * o[3],
               R.accA != 0);
        }
      }
    }
  }
}

// ------------------------------------------------------------ 3x3 convolution
// Grid: (row tiles x column tiles, output-channel tiles of 16 MT, batch x
// ksplit).  Wave w computes output row w of the tile: up to MT x NTL MFMA tiles
// (16 MT channels x 16 NTL columns).  MT = 4, NTL = 2 in general; layers
// with at most 16 output channels take MT = 1, NTL = 4 (64 columns).
template <bool AF32, bool OUTF32, int MT = 4, int NTL = 2, bool UP = false>
__global__ __launch_bounds__(256) void k_conv3(ConvArgs a) {
  static_assert((MT == 4 && NTL == 2) || (MT == 1 && NTL == 4), "4 x 2 or 1 x 4 accumulator tiles per wave");
  constexpr int TW = 16 * NTL;
  constexpr int TW2 = TW + 2;
  // input tile [row][col][channel], (kConvTH + 2) x TW2 pixels of CC + 8
  // channel slots (dynamic: conv3_launch)
  extern __shared__ __attribute__((aligned(16))) uint16_t sX[];
  const int H = a.in.H, W = a.in.W;
  const int tiles_x = (W + TW - 1) / TW;
  const int ty0 = ((int)blockIdx.x / tiles_x) * kConvTH;
  const int tx0 = ((int)blockIdx.x % tiles_x) * TW;
  const int co0 = (int)blockIdx.y * 16 * MT, b = (int)blockIdx.z % a.B, ks = (int)blockIdx.z / a.B;
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int sub = lane >> 4, n16 = lane & 15;
  const ConvPack& P = a.pk;
  const int MI = min(MT, (P.Coutp - co0) >> 4);
  const int CC = P.CC, PS = CC + 8, ng = CC >> 3;
  const int kl = sub * 8, tap_l = kl / CC, coff = kl - tap_l * CC;
  const int nkc = P.KKp / P.TPK;

  f32x4 acc[MT][NTL];
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
#pragma unroll
    for (int ni = 0; ni < NTL; ++ni) acc[mi][ni] = f32x4{0.f, 0.f, 0.f, 0.f};

  // packed weights of output channel co0 + mi 16 + n16, k-step s of the
  // whole reduction (s = cc nkc + kc): consecutive k-steps are consecutive
  // KKp-CC blocks, 32 BF16 apart
  const uint16_t* wrow[MT];
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
    wrow[mi] = a.Wp + ((long long)min(co0 + mi * 16 + n16, P.Coutp - 1) * P.ncc * P.KKp + tap_l) * CC + coff;
  // the A fragments of the next two k-steps are in flight while this one
  // multiplies (wq: step s + 1, wq2: step s + 2)
  uint4 wq[MT], wq2[MT];
  // this split's channel chunks (all of them without a split)
  const int cc_lo = ks * P.ncc / a.ksplit, cc_hi = (ks + 1) * P.ncc / a.ksplit;
  const int nks = cc_hi * nkc, sb = cc_lo * nkc;
#pragma unroll
  for (int mi = 0; mi < MT; ++mi) {
    wq[mi] = mi < MI ? *reinterpret_cast<const uint4*>(wrow[mi] + (long long)sb * P.TPK * CC) : make_uint4(0u, 0u, 0u, 0u);
    wq2[mi] = (mi < MI && sb + 1 < nks) ? *reinterpret_cast<const uint4*>(wrow[mi] + (long long)(sb + 1) * P.TPK * CC)
                                          : make_uint4(0u, 0u, 0u, 0u);
  }

  for (int cc = cc_lo; cc < cc_hi; ++cc) {
    stage_tile<AF32>(a.in, b, ty0 - 1, tx0 - 1, kConvTH + 2, TW2, cc * CC, ng, sX, PS);
    __syncthreads();
    for (int kc = 0; kc < nkc; ++kc) {
      const int kk = kc * P.TPK + tap_l;
      const bool valid = kk < 9;
      const int dy = valid ? kk / 3 : 0, dx = valid ? kk - (kk / 3) * 3 : 0;
      bf16x8 bfrag[NTL];
#pragma unroll
      for (int ni = 0; ni < NTL; ++ni) {
        const int px = ni * 16 + n16;
        uint4 q = *reinterpret_cast<const uint4*>(sX + ((wave + dy) * TW2 + px + dx) * PS + coff);
        if (!valid) q = make_uint4(0u, 0u, 0u, 0u);
        bfrag[ni] = __builtin_bit_cast(bf16x8, q);
      }
      bf16x8 afrag[MT];
#pragma unroll
      for (int mi = 0; mi < MT; ++mi) {
        afrag[mi] = __builtin_bit_cast(bf16x8, wq[mi]);
        wq[mi] = wq2[mi];
      }
      const int sn = cc * nkc + kc + 2;
      if (sn < nks) {
#pragma unroll
        for (int mi = 0; mi < MT; ++mi)
          if (mi < MI) wq2[mi] = *reinterpret_cast<const uint4*>(wrow[mi] + (long long)sn * P.TPK * CC);
      }
#pragma unroll
      for (int mi = 0; mi < MT; ++mi) {
        if (mi < MI) {
#pragma unroll
          for (int ni = 0; ni < NTL; ++ni) acc[mi][ni] = mfma(afrag[mi], bfrag[ni], acc[mi][ni]);
        }
      }
    }
    __syncthreads();
  }

  const int y = ty0 + wave;
  if (!UP && a.ksplit > 1) {  // the upsampled route is launched unsplit
    // raw partial sums of this split; the finishing kernel applies the epilogue
    if (y >= H) return;
#pragma unroll
    for (int mi = 0; mi < MT; ++mi) {
      if (mi >= MI) continue;
      const int co = co0 + mi * 16 + sub * 4;
#pragma unroll
      for (int ni = 0; ni < NTL; ++ni) {
        const int x = tx0 + ni * 16 + n16;
        if (x >= W) continue;
        const long long off = ((((long long)ks * a.B + b) * H + y) * W + x) * P.Coutp + co;
        *reinterpret_cast<float4*>(a.kpart + off) =
            make_float4(acc[mi][ni][0], acc[mi][ni][1], acc[mi][ni][2], acc[mi][ni][3]);
      }
    }
    return;
  }
  if constexpr (OUTF32) {
    if (a.rt.gA) {
      route_store<MT, NTL, UP>(a, acc, b, ty0, tx0, co0, MI, reinterpret_cast<float*>(sX));
      return;
    }
  }
  if (y >= H) return;
#pragma unroll
  for (int mi = 0; mi < MT; ++mi) {
    if (mi >= MI) continue;
    const int co = co0 + mi * 16 + sub * 4;
    if (co >= P.Cout) continue;
#pragma unroll
    for (int ni = 0; ni < NTL; ++ni) {
      const int x = tx0 + ni * 16 + n16;
      if (x >= W) continue;
      float o[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        o[i] = acc[mi][ni][i] + (a.bias ? a.bias[co + i] : 0.f);
        if (a.relu) o[i] = fmaxf(o[i], 0.f);
      }
      const long long off = (((long long)b * H + y) * W + x) * P.Cout + co;
      if constexpr (OUTF32) {
        *reinterpret_cast<float4*>(static_cast<float*>(a.out) + off) = make_float4(o[0], o[1], o[2], o[3]);
      } else {
        *reinterpret_cast<uint2*>(static_cast<uint16_t*>(a.out) + off) =
            make_uint2(f2bf(o[0]) | (f2bf(o[1]) << 16), f2bf(o[2]) | (f2bf(o[3]) << 16));
      }
    }
  }
}

// Finish a convolution split over its channel chunks: S(pixel, co) = the
// ksplit partials added in split order, then the epilogue of k_conv3 for
// that value: bias, ReLU and a BF16 (or FP32) store, or the route to A and
// the skip (see ConvRoute).  Four channels a thread.  An upsampled A takes
// its 2 x 2 block sums as (S00 + S01) + (S10 + S11) in a second index range
// over A's pixels.
__device__ __forceinline__ float4 ksum4(const ConvArgs& a, long long pix, int co) {
  const long long stride = (long long)a.B * a.in.H * a.in.W * a.pk.Coutp;
  float4 t = *reinterpret_cast<const float4*>(a.kpart + pix * a.pk.Coutp + co);
  for (int k = 1; k < a.ksplit; ++k) {
    const float4 q = *reinterpret_cast<const float4*>(a.kpart + k * stride + pix * a.pk.Coutp + co);
    t.x += q.x;
    t.y += q.y;
    t.z += q.z;
    t.w += q.w;
  }
  return t;
}

template <bool OUTF32>
__global__ __launch_bounds__(256) void k_conv_finish(ConvArgs a) {
  const int H = a.in.H, W = a.in.W;
  const long long npix = (long long)a.B * H * W;
  const ConvRoute& R = a.rt;
  const bool routed = OUTF32 && R.gA;
  const bool up = routed && R.modeA == 1;
  // range 1: every output pixel's channel groups (without the A channels of
  // an upsampled route); range 2: the A pixels of an upsampled route
  const int c_lo = up ? R.Ca : 0, ng1 = (a.pk.Cout - c_lo) >> 2;
  const long long n1 = npix * ng1;
  const long long n2 = up ? npix / 4 * (R.Ca >> 2) : 0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n1 + n2; i += (long long)gridDim.x * 256) {
    if (i < n1) {
      const long long pix = i / ng1;
      const int co = c_lo + 4 * (int)(i - pix * ng1);
      const float4 t = ksum4(a, pix, co);
      if (!routed) {
        float o[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (a.bias) o[k] += a.bias[co + k];
          if (a.relu) o[k] = fmaxf(o[k], 0.f);
        }
        const long long off = pix * a.pk.Cout + co;
        if constexpr (OUTF32) {
          *reinterpret_cast<float4*>(static_cast<float*>(a.out) + off) = make_float4(o[0], o[1], o[2], o[3]);
        } else {
          *reinterpret_cast<uint2*>(static_cast<uint16_t*>(a.out) + off) =
              make_uint2(f2bf(o[0]) | (f2bf(o[1]) << 16), f2bf(o[2]) | (f2bf(o[3]) << 16));
        }
      } else if (co >= R.Ca) {
        const long long ob = pix * R.Cb + (co - R.Ca);
        put4(R.gB + ob, R.mB ? R.mB + ob : nullptr, t.x, t.y, t.z, t.w, R.accB != 0);
      } else if (R.modeA == 0) {
        const long long oa = pix * R.Ca + co;
        put4(R.gA + oa, R.mA ? R.mA + oa : nullptr, t.x, t.y, t.z, t.w, R.accA != 0);
      } else {
        const long long b = pix / ((long long)H * W);
        const int rem = (int)(pix - b * H * W), y = rem / W, x = rem - y * W;
        const int H2 = 2 * H, W2 = 2 * W;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const long long oa = ((b * H2 + 2 * y + (q >> 1)) * W2 + 2 * x + (q & 1)) * R.Ca + co;
          put4(R.gA + oa, R.mA ? R.mA + oa : nullptr, 0.25f * t.x, 0.25f * t.y, 0.25f * t.z, 0.25f * t.w,
               R.accA != 0);
        }
      }
    } else {
      const long long j = i - n1;
      const int ngA = R.Ca >> 2;
      const long long ph = j / ngA;  // A pixel (b, yh, xh)
      const int co = 4 * (int)(j - ph * ngA);
      const int Hh = H >> 1, Wh = W >> 1;
      const long long b = ph / ((long long)Hh * Wh);
      const int rem = (int)(ph - b * Hh * Wh), yh = rem / Wh, xh = rem - yh * Wh;
      const long long p00 = (b * H + 2 * yh) * W + 2 * xh;
      const float4 s00 = ksum4(a, p00, co), s01 = ksum4(a, p00 + 1, co);
      const float4 s10 = ksum4(a, p00 + W, co), s11 = ksum4(a, p00 + W + 1, co);
      put4(R.gA + ph * R.Ca + co, R.mA ? R.mA + ph * R.Ca + co : nullptr, (s00.x + s01.x) + (s10.x + s11.x),
           (s00.y + s01.y) + (s10.y + s11.y), (s00.z + s01.z) + (s10.z + s11.z), (s00.w + s01.w) + (s10.w + s11.w),
           R.accA != 0);
    }
  }
}

// ------------------------------------------------------------ weight gradient
// Grid: (input-channel chunks, output-channel tiles of COT (16, 32 or 64), pixel splits).
// Wave w accumulates the taps kk = w, w + 4, w + 8.  Both operands are
// staged in LDS pixel-major with channels contiguous (one 16-byte store per
// 8 channels of a pixel, the tap shift being a per-lane address offset) and
// read as MFMA fragments with the gfx950 LDS transpose read: for each group
// of 16 lanes, lane 4 r + q loads four consecutive channels 4 q + [0, 4) of
// pixel r, and lane c receives channel c of pixels 0..3.  Two such reads
// (pixels 8 s + [0, 4) and 8 s + [4, 8)) give lane (s, c) the eight
// consecutive pixels of k-group s of channel c.
typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef short v8i16 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) v4i16 lds_v4i16;

__device__ __forceinline__ bf16x8 tr_frag(const uint16_t* p, int step) {
  const v4i16 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4i16*)((__attribute__((address_space(3))) uint16_t*)p));
  const v4i16 hi =
      __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4i16*)((__attribute__((address_space(3))) uint16_t*)(p + step)));
  return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

template <bool AF32, int COT>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
  constexpr int MT = COT / 16;
  constexpr int NG = COT / 8;            // 8-channel groups of the output gradient
  constexpr int ZP = COT + 8;            // LDS pixel stride of the output gradient
  constexpr int XW = kWgTW + 2, XR = kWgTH + 2;
  constexpr int XP = 32 + 8;             // LDS pixel stride of the input (chunks of up to 32 channels)
  __shared__ __attribute__((aligned(16))) uint16_t sZ[kWgTH * kWgTW * ZP];
  __shared__ __attribute__((aligned(16))) uint16_t sX[XR * XW * XP];
  const int H = a.in.H, W = a.in.W;
  const int cc = (int)blockIdx.x, co0 = (int)blockIdx.y * COT, split = (int)blockIdx.z;
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int sub = lane >> 4, n16 = lane & 15;
  const int MI = min(MT, (a.Cout - co0 + 15) >> 4);
  // 16-channel input tiles of this chunk holding real channels (the last
  // chunk of a padded count stages and multiplies only those)
  const int NI = min(a.CCw, a.Cin - cc * a.CCw + 15) >> 4;
  const int ngx = 2 * NI;
  const int tiles_x = (W + kWgTW - 1) / kWgTW, tiles_y = (H + kWgTH - 1) / kWgTH;
  const int T = a.B * tiles_x * tiles_y;
  // this lane's transpose-read offsets: pixel n16 / 4 of its k-group, channel quad n16 % 4
  const int kp = 8 * sub + (n16 >> 2), cq = 4 * (n16 & 3);

  f32x4 acc[3][MT][2];
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int mi = 0; mi < MT; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) acc[s][mi][ni] = f32x4{0.f, 0.f, 0.f, 0.f};
  // bias partial: thread t always stages channel group t % NG
  float bsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

  // the MFMA work of the tile staged in sZ and sX
  auto tile_mfma = [&]() {
    for (int row = 0; row < kWgTH; ++row) {
      bf16x8 af[MT];
#pragma unroll
      for (int mi = 0; mi < MT; ++mi)
        af[mi] = mi < MI ? tr_frag(sZ + (row * kWgTW + kp) * ZP + mi * 16 + cq, 4 * ZP) : bf16x8{};
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int kk = wave + 4 * s;
        if (kk >= 9) continue;
        const int dy = kk / 3, dx = kk - dy * 3;
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
          if (ni >= NI) continue;
          const bf16x8 bf = tr_frag(sX + ((row + dy) * XW + kp + dx) * XP + ni * 16 + cq, 4 * XP);
#pragma unroll
          for (int mi = 0; mi < MT; ++mi)
            if (mi < MI) acc[s][mi][ni] = mfma(af[mi], bf, acc[s][mi][ni]);
        }
      }
    }
  };

  // Light loaders (BF16 without pooling) and 16-channel output tiles: the
  // next tile's loads are issued before this tile's multiplies, so a
  // workgroup walking many tiles waits on one memory latency per tile less
  // (wider tiles measured slower with the extra registers).
  constexpr int UZ = kWgTH * kWgTW * NG / 256;  // output-gradient tasks per thread
  constexpr int UX = 4;                           // input tasks per thread (XR XW ngx <= 816)
  if (COT == 16 && !AF32 && a.in.modeA != 2) {
    const int ntx = XR * XW * ngx;
    float4 zp[UZ], zq[UZ];
    uint4 xq[UX];
    auto fetch = [&](int t) {
      const int b = t / (tiles_x * tiles_y);
      const int rem = t - b * tiles_x * tiles_y;
      const int ty0 = (rem / tiles_x) * kWgTH, tx0 = (rem % tiles_x) * kWgTW;
#pragma unroll
      for (int u = 0; u < UZ; ++u) {
        const int task = (int)threadIdx.x + u * 256;
        const int g = task % NG, pix = task / NG;
        const int row = pix / kWgTW, px = pix - row * kWgTW;
        const int y = ty0 + row, x = tx0 + px, co = co0 + g * 8;
        zp[u] = zq[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (y < H && x < W && co < a.Cout) {
          const long long o = (((long long)b * H + y) * W + x) * a.Cout + co;
          zp[u] = *reinterpret_cast<const float4*>(a.gY + o);
          zq[u] = *reinterpret_cast<const float4*>(a.gY + o + 4);
        }
      }
#pragma unroll
      for (int u = 0; u < UX; ++u) {
        const int task = (int)threadIdx.x + u * 256;
        xq[u] = make_uint4(0u, 0u, 0u, 0u);
        if (task < ntx) {
          const int g = task % ngx, pix = task / ngx;
          const int r = pix / XW, xx = pix - r * XW;
          const uint4* src = in8_src(a.in, b, ty0 - 1 + r, tx0 - 1 + xx, cc * a.CCw + g * 8);
          if (src) xq[u] = *src;
        }
      }
    };
    fetch(split);  // split < T: the host takes at most T splits
    for (int t = split; t < T; t += a.nsplit) {
#pragma unroll
      for (int u = 0; u < UZ; ++u) {
        const int task = (int)threadIdx.x + u * 256;
        const float v[8] = {zp[u].x, zp[u].y, zp[u].z, zp[u].w, zq[u].x, zq[u].y, zq[u].z, zq[u].w};
#pragma unroll
        for (int i = 0; i < 8; ++i) bsum[i] += v[i];
        *reinterpret_cast<uint4*>(sZ + (task / NG) * ZP + (task % NG) * 8) = pack8(v);
      }
#pragma unroll
      for (int u = 0; u < UX; ++u) {
        const int task = (int)threadIdx.x + u * 256;
        if (task < ntx) *reinterpret_cast<uint4*>(sX + (task / ngx) * XP + (task % ngx) * 8) = xq[u];
      }
      __syncthreads();
      if (t + a.nsplit < T) fetch(t + a.nsplit);
      tile_mfma();
      __syncthreads();
    }
  } else {
    for (int t = split; t < T; t += a.nsplit) {
      const int b = t / (tiles_x * tiles_y);
      const int rem = t - b * tiles_x * tiles_y;
      const int ty0 = (rem / tiles_x) * kWgTH, tx0 = (rem % tiles_x) * kWgTW;
      // output gradient (of the pre-activation), [pixel][co]; the loads of
      // U tasks are issued before any is stored
      {
        constexpr int U = 4;
        constexpr int NTASK = kWgTH * kWgTW * NG;
        for (int t0 = threadIdx.x; t0 < NTASK; t0 += U * 256) {
          float4 p[U], q[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int task = t0 + u * 256;
            p[u] = q[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            const int g = task % NG, pix = task / NG;
            const int row = pix / kWgTW, px = pix - row * kWgTW;
            const int y = ty0 + row, x = tx0 + px, co = co0 + g * 8;
            if (task < NTASK && y < H && x < W && co < a.Cout) {
              const long long o = (((long long)b * H + y) * W + x) * a.Cout + co;
              p[u] = *reinterpret_cast<const float4*>(a.gY + o);
              q[u] = *reinterpret_cast<const float4*>(a.gY + o + 4);
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int task = t0 + u * 256;
            if (task < NTASK) {
              const float v[8] = {p[u].x, p[u].y, p[u].z, p[u].w, q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
              for (int i = 0; i < 8; ++i) bsum[i] += v[i];
              *reinterpret_cast<uint4*>(sZ + (task / NG) * ZP + (task % NG) * 8) = pack8(v);
            }
          }
        }
      }
      // input tile with a one-pixel halo, [pixel][ci]
      stage_tile<AF32>(a.in, b, ty0 - 1, tx0 - 1, XR, XW, cc * a.CCw, ngx, sX, XP);
      __syncthreads();
      tile_mfma();
      __syncthreads();
    }
  }

#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int kk = wave + 4 * s;
    if (kk >= 9) continue;
#pragma unroll
    for (int mi = 0; mi < MT; ++mi) {
      if (mi >= MI) continue;
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        if (ni >= NI) continue;
        const int ci = cc * a.CCw + ni * 16 + n16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int co = co0 + mi * 16 + sub * 4 + i;
          if (co < a.Cout && ci < a.Cipw)
            a.part[(((long long)split * a.Cout + co) * 9 + kk) * a.Cipw + ci] = acc[s][mi][ni][i];
        }
      }
    }
  }
  // bias partial of this split (channel chunk 0 only): the threads of one
  // channel group are added in thread order
  if (a.bpart && cc == 0) {
    float* red = reinterpret_cast<float*>(sX);  // the loop ended with a barrier
#pragma unroll
    for (int i = 0; i < 8; ++i) red[threadIdx.x * 8 + i] = bsum[i];
    __syncthreads();
    const int c = (int)threadIdx.x;
    if (c < COT && co0 + c < a.Cout) {
      float sum = 0.f;
      for (int k = c >> 3; k < 256; k += NG) sum += red[k * 8 + (c & 7)];
      a.bpart[(long long)split * a.Cout + co0 + c] = sum;
    }
  }
}

// Sum the pixel-split partials of every layer (see RedAll) into the
// canonical weight gradients [Cout][Cin][3][3] and the bias gradients.  A
// workgroup takes E consecutive elements of one layer (E = 64: each wave
// load is 64 consecutive floats; E = 16 for layers with many splits, so that
// no thread walks a long chain of them) and 256 / E thread groups over the
// splits (split sp -> group sp mod G); the G partial sums of an element are
// added in group order, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_wgrad_reduce(RedAll a) {
  __shared__ float s[16 * 17 > 4 * 65 ? 16 * 17 : 4 * 65];
  const int b = (int)blockIdx.x;
  int l = 0;
  while (b >= a.wg[l + 1]) ++l;
  const RedLayer& L = a.L[l];
  const int E = L.e, G = 256 / E;
  const int te = (int)threadIdx.x % E, g = (int)threadIdx.x / E;
  const int nw = L.Cout * L.Cin * 9, n = nw + L.Cout;
  const int jl = (b - a.wg[l]) * E + te;
  float acc = 0.f;
  int co = 0, kk = 0, ci = 0;
  if (jl < nw) {
    // neighbouring elements are neighbouring ci: coalesced partial reads
    co = jl / (9 * L.Cin);
    const int r = jl - co * 9 * L.Cin;
    kk = r / L.Cin;
    ci = r - kk * L.Cin;
    const long long stride = (long long)L.Cout * 9 * L.Cipw;
    const float* p = L.part + ((long long)co * 9 + kk) * L.Cipw + ci;
#pragma unroll 8
    for (int sp = g; sp < L.nsplit; sp += G) acc += p[sp * stride];
  } else if (jl < n) {
#pragma unroll 8
    for (int sp = g; sp < L.nsplit; sp += G) acc += L.bpart[(long long)sp * L.Cout + (jl - nw)];
  }
  s[g * (E + 1) + te] = acc;
  __syncthreads();
  if (g == 0 && jl < n) {
    float t = 0.f;
    for (int q = 0; q < G; ++q) t += s[q * (E + 1) + te];
    if (jl < nw) L.grad[((long long)co * L.Cin + ci) * 9 + kk] = t;
    else L.gb[jl - nw] = t;
  }
}

// out[seg ne + e] = sum over the rows k of segment seg (rows seg R ..
// min(seg R + R, nblk) - 1) of part[k ne + e]: 64 consecutive elements per
// workgroup (one per lane: each wave load is 64 consecutive floats) and
// the four waves over the segment's rows (row k -> wave (k - seg R) mod 4),
// the waves' sums added in wave order (deterministic).
__global__ __launch_bounds__(256) void k_sum_rows(const float* __restrict__ part, int nblk, int ne, int R,
                                                 float* __restrict__ out) {
  __shared__ float s[4][65];
  const int te = (int)threadIdx.x & 63, g = (int)threadIdx.x >> 6;
  const int seg = (int)blockIdx.y, e = (int)blockIdx.x * 64 + te;
  const int k0 = seg * R, k1 = min(k0 + R, nblk);
  float acc = 0.f;
  if (e < ne)
    for (int k = k0 + g; k < k1; k += 4) acc += part[(long long)k * ne + e];
  s[g][te] = acc;
  __syncthreads();
  if (g == 0 && e < ne) out[(long long)seg * ne + e] = ((s[0][te] + s[1][te]) + s[2][te]) + s[3][te];
}

// out[e] = sum over k < nblk of part[k ne + e], in two fixed-order stages:
// segments of kSumRowsSeg rows into scratch (ceil(nblk / kSumRowsSeg) rows
// of ne), then those rows.
constexpr int kSumRowsSeg = 64;
static void sum_parts(const float* part, int nblk, int ne, float* scratch, float* out, hipStream_t s) {
  const unsigned gx = (unsigned)((ne + 63) / 64);
  const int nseg = (nblk + kSumRowsSeg - 1) / kSumRowsSeg;
  hipLaunchKernelGGL(k_sum_rows, dim3(gx, (unsigned)nseg), dim3(256), 0, s, part, nblk, ne, kSumRowsSeg, scratch);
  hipLaunchKernelGGL(k_sum_rows, dim3(gx, 1), dim3(256), 0, s, (const float*)scratch, nseg, ne, nseg, out);
}

// ------------------------------------------------------------ heads
constexpr int kHeadRowTiles = 5;  // 16-row tiles of the P + 1 <= 65 head-gradient rows

// One pixel per thread: y_m = Wm h + bm (P channels, planar output), y_w =
// sigmoid(Ww h + bw).  FP32 weights in LDS.
// C1 (8, 16 or 32) at compile time: the head input stays in registers and
// every weight row is read as C1 / 4 16-byte LDS broadcasts.
template <int C1>
__global__ __launch_bounds__(256) void k_head_fwd(HeadArgs a) {
  extern __shared__ __attribute__((aligned(16))) float shw[];
  const int P = a.P;
  float* sWm = shw;                 // [P][C1], then bm [P]
  float* sWw = shw + P * C1 + P;    // [C1], then bw
  for (int i = threadIdx.x; i < P * C1 + P; i += blockDim.x) sWm[i] = a.Wm[i];
  for (int i = threadIdx.x; i < C1 + 1; i += blockDim.x) sWw[i] = a.Ww[i];
  __syncthreads();
  const long long HW = (long long)a.H * a.W, npix = a.B * HW;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  float h[C1];
  const uint16_t* hp = a.h + p * C1;
#pragma unroll
  for (int c = 0; c < C1; c += 8) {
    float v[8];
    unpack8(*reinterpret_cast<const uint4*>(hp + c), v);
#pragma unroll
    for (int i = 0; i < 8; ++i) h[c + i] = v[i];
  }
  const long long b = p / HW, yx = p - b * HW;
  float* ym = a.y_m + b * P * HW + yx;
#pragma unroll 2
  for (int co = 0; co < P; ++co) {
    float s = sWm[P * C1 + co];
    const float4* w = reinterpret_cast<const float4*>(sWm + co * C1);
#pragma unroll
    for (int c = 0; c < C1 / 4; ++c) {
      const float4 q = w[c];
      s = fmaf(q.x, h[4 * c], s);
      s = fmaf(q.y, h[4 * c + 1], s);
      s = fmaf(q.z, h[4 * c + 2], s);
      s = fmaf(q.w, h[4 * c + 3], s);
    }
    ym[co * HW] = s;
  }
  float z = sWw[C1];
#pragma unroll
  for (int c = 0; c < C1; ++c) z = fmaf(sWw[c], h[c], z);
  a.y_w[p] = 1.0f / (1.0f + __expf(-z));
}

// Loss terms, gradient of the head input's pre-activation (FP32 NHWC: the
// head input is a ReLU output) and per-block partial sums of the
// head-parameter gradient and of the two squared errors.
// One 256-pixel block per workgroup.  Dynamic LDS: gy [256][P+1] (column
// P: the gradient gz of the weight head's logit), h [256][C1+1] (column C1:
// 1), Wm [P][C1], Ww [C1]; the waves' partials of the parameter gradient
// reuse it from the start once those are read.  Every head parameter's
// block gradient is one entry of sum_t gy[t] h[t]^T, a (P+1) x (C1+1)
// outer-product sum (Wm, bm; Ww, bw), computed on the FP32 matrix cores,
// each wave over a quarter of the block's pixels, and added over the waves
// in wave order.
template <int C1>
__global__ __launch_bounds__(256) void k_head_bwd(LossArgs a) {
  extern __shared__ __attribute__((aligned(16))) float sh[];
  __shared__ double sred[2][4];
  const HeadArgs& d = a.hd;
  const int P = d.P, tid = (int)threadIdx.x;
  const int GP = P + 1, HC = C1 + 1;
  float* sgy = sh;
  float* shh = sgy + 256 * GP;
  float* sWm = shh + 256 * HC;
  float* sWw = sWm + P * C1;
  for (int i = tid; i < P * C1; i += 256) sWm[i] = d.Wm[i];
  for (int i = tid; i < C1; i += 256) sWw[i] = d.Ww[i];
  const long long HW = (long long)d.H * d.W, npix = d.B * HW;
  const float inv_m = 1.0f / (float)((double)npix * P), inv_w = 1.0f / (float)npix;
  // parameter-gradient block sums on the FP32 matrix cores
  // (v_mfma_f32_16x16x4_f32: lane l supplies A[l % 16][l / 16] and
  // B[l / 16][l % 16] and receives D[4 (l / 16) + i][l % 16]):
  // D[r][c] = sum_t gy[t][r] h[t][c], r < P + 1, c < C1 + 1, in 16 x 16
  // tiles; wave w takes pixels 64 w .. 64 w + 63 (16 k-steps of 4)
  constexpr int TC = (C1 + 1 + 15) / 16;
  const int TR = (GP + 15) / 16;  // <= kHeadRowTiles: checked by the launcher
  const int wave = tid >> 6, lane = tid & 63, kq = lane >> 4, l16 = lane & 15;
  f32x4 acc[kHeadRowTiles][TC];
#pragma unroll
  for (int i = 0; i < kHeadRowTiles; ++i)
#pragma unroll
    for (int j = 0; j < TC; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  double lm = 0.0, lw = 0.0;
  const long long p = (long long)blockIdx.x * 256 + tid;
  if (p < npix) {
    const uint16_t* hp = d.h + p * C1;
    for (int c = 0; c < C1; c += 8) {
      float v[8];
      unpack8(*reinterpret_cast<const uint4*>(hp + c), v);
#pragma unroll
      for (int i = 0; i < 8; ++i) shh[tid * HC + c + i] = v[i];
    }
    shh[tid * HC + C1] = 1.f;
    const long long b = p / HW, yx = p - b * HW;
    for (int co = 0; co < P; ++co) {
      const long long o = (b * P + co) * HW + yx;
      const float df = d.y_m[o] - a.t_m[o];
      lm += (double)df * (double)df;
      sgy[tid * GP + co] = 2.0f * df * inv_m;
    }
    const float yw = d.y_w[p], dw = yw - a.t_w[p];
    lw = (double)dw * (double)dw;
    sgy[tid * GP + P] = 2.0f * a.lam_w * dw * inv_w * yw * (1.0f - yw);
  } else {
    for (int co = 0; co < GP; ++co) sgy[tid * GP + co] = 0.f;
    for (int c = 0; c < HC; ++c) shh[tid * HC + c] = 0.f;
  }
  __syncthreads();
  if (p < npix) {
    // g_h[c] = Ww[c] gz + sum over co of Wm[co][c] gy[co], co ascending; all
    // C1 sums in registers, each gy read once, each Wm row as C1 / 4
    // 16-byte LDS broadcasts
    const float gz = sgy[tid * GP + P];
    float s[C1];
#pragma unroll
    for (int c = 0; c < C1; ++c) s[c] = sWw[c] * gz;
    for (int co = 0; co < P; ++co) {
      const float gy = sgy[tid * GP + co];
      const float4* w = reinterpret_cast<const float4*>(sWm + co * C1);
#pragma unroll
      for (int c = 0; c < C1 / 4; ++c) {
        const float4 q = w[c];
        s[4 * c] = fmaf(q.x, gy, s[4 * c]);
        s[4 * c + 1] = fmaf(q.y, gy, s[4 * c + 1]);
        s[4 * c + 2] = fmaf(q.z, gy, s[4 * c + 2]);
        s[4 * c + 3] = fmaf(q.w, gy, s[4 * c + 3]);
      }
    }
    // the head input is a ReLU output: store the gradient of its pre-activation
#pragma unroll
    for (int c = 0; c < C1; ++c)
      if (!(shh[tid * HC + c] > 0.f)) s[c] = 0.f;
#pragma unroll
    for (int c = 0; c < C1; c += 4)
      *reinterpret_cast<float4*>(a.g_h + p * C1 + c) = make_float4(s[c], s[c + 1], s[c + 2], s[c + 3]);
  }
  for (int ks = 0; ks < 16; ++ks) {
    const int t = 64 * wave + 4 * ks + kq;
    float hb[TC];
#pragma unroll
    for (int ct = 0; ct < TC; ++ct) hb[ct] = 16 * ct + l16 < HC ? shh[t * HC + 16 * ct + l16] : 0.f;
#pragma unroll
    for (int rt = 0; rt < kHeadRowTiles; ++rt) {
      if (rt >= TR) continue;
      const float ga = 16 * rt + l16 < GP ? sgy[t * GP + 16 * rt + l16] : 0.f;
#pragma unroll
      for (int ct = 0; ct < TC; ++ct) acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga, hb[ct], acc[rt][ct], 0, 0, 0);
    }
  }
  __syncthreads();  // gy and h are read: their space takes the wave partials
  float* red = sh;   // [wave][TR][TC][16 x 16]
#pragma unroll
  for (int rt = 0; rt < kHeadRowTiles; ++rt) {
    if (rt >= TR) continue;
#pragma unroll
    for (int ct = 0; ct < TC; ++ct)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        red[((wave * TR + rt) * TC + ct) * 256 + (4 * kq + i) * 16 + l16] = acc[rt][ct][i];
  }
  __syncthreads();
  // entry e of the partial layout [Wm P x C1][bm P][Ww C1][bw] -> (r, c),
  // the four waves' sums added in wave order
  for (int e = tid; e < a.ne; e += 256) {
    int r, c;
    if (e < P * C1) {
      r = e / C1;
      c = e - r * C1;
    } else if (e < P * C1 + P) {
      r = e - P * C1;
      c = C1;
    } else {
      r = P;
      c = e - P * C1 - P;  // C1 for bw
    }
    const int o = ((r >> 4) * TC + (c >> 4)) * 256 + (r & 15) * 16 + (c & 15);
    float sum = 0.f;
    for (int w = 0; w < 4; ++w) sum += red[w * TR * TC * 256 + o];
    a.hpart[(long long)blockIdx.x * a.ne + e] = sum;
  }
  // block sums of the squared errors (fixed order)
  for (int off = 32; off > 0; off >>= 1) {
    lm += __shfl_down(lm, off);
    lw += __shfl_down(lw, off);
  }
  if ((tid & 63) == 0) {
    sred[0][tid >> 6] = lm;
    sred[1][tid >> 6] = lw;
  }
  __syncthreads();
  if (tid == 0) {
    a.lpart[2 * blockIdx.x] = sred[0][0] + sred[0][1] + sred[0][2] + sred[0][3];
    a.lpart[2 * blockIdx.x + 1] = sred[1][0] + sred[1][1] + sred[1][2] + sred[1][3];
  }
}

// loss = sum_m / Nm + lam_w sum_w / Nw over the block partials (one block).
__global__ __launch_bounds__(256) void k_loss_reduce(const double* __restrict__ lpart, int nblk, double Nm,
                                                    double Nw, double lam_w, double* loss) {
  __shared__ double s[2][256];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nblk; k += 256) {
    a += lpart[2 * k];
    b += lpart[2 * k + 1];
  }
  s[0][threadIdx.x] = a;
  s[1][threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int k = 0; k < 256; ++k) {
      ta += s[0][k];
      tb += s[1][k];
    }
    *loss = ta / Nm + lam_w * tb / Nw;
  }
}

// ------------------------------------------------------------ parameters
__global__ __launch_bounds__(256) void k_pack(PackAll a) {
  for (int e = (int)(blockIdx.x * blockDim.x + threadIdx.x); e < a.start[a.n]; e += (int)(gridDim.x * blockDim.x)) {
    int l = 0;
    while (e >= a.start[l + 1]) ++l;
    const PackArgs& L = a.L[l];
    const int nf = L.f.Coutp * L.f.ncc * L.f.KKp * L.f.CC;
    const bool fw = e - a.start[l] < nf;
    const ConvPack& P = fw ? L.f : L.t;
    const int i = fw ? e - a.start[l] : e - a.start[l] - nf;
    int r = i;
    const int c = r % P.CC;
    r /= P.CC;
    const int kk = r % P.KKp;
    r /= P.KKp;
    const int cc = r % P.ncc;
    const int co = r / P.ncc;
    const int ci = cc * P.CC + c;
    float v = 0.f;
    if (co < P.Cout && ci < P.Cin && kk < 9) {
      // forward: W[co][ci][kk]; transposed: output = forward input channel
      // co, input = forward output channel ci, taps flipped
      v = fw ? L.W[((long long)co * P.Cin + ci) * 9 + kk] : L.W[((long long)ci * P.Cout + co) * 9 + (8 - kk)];
    }
    (fw ? L.Wp : L.Wtp)[i] = (uint16_t)f2bf(v);
  }
}

__global__ __launch_bounds__(256) void k_adamw(float* __restrict__ th, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, long long n, float lr,
                                              float b1, float b2, float eps, float wd, float bc1, float bc2) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    th[i] = th[i] * (1.f - lr * wd) - lr * mh / (sqrtf(vh) + eps);
  }
}


// ------------------------------------------------------------ launchers
static inline unsigned grid_for(long long n, int per = 256, int cap = 8192) {
  long long g = (n + per - 1) / per;
  return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

// Workgroups below which a convolution launch splits its channel chunks
// (such launches leave CUs idle while each workgroup walks every chunk).
constexpr long long kConvSplitGroups = 512;

// MFMA tile of a launch: MT 16-channel output tiles by NTL 16-column tiles
// per wave.  4 x 2 in general and for the upsampled route; 16-channel
// outputs take 1 x 4 (64 columns: wider tiles' input staging, 37-62 KB of
// LDS, held a CU to two to four workgroups and measured slower).
static void conv_tile(const ConvPack& pk, bool up, int& MT, int& NTL) {
  MT = 4;
  NTL = 2;
  if (!up && pk.Coutp <= 16) {
    MT = 1;
    NTL = 4;
  }
}

// Channel-chunk split of a launch (1: none); the host sizes the partial
// buffer with this same function.
int conv_ksplit(const ConvPack& pk, int B, int H, int W, bool up) {
  int MT, NTL;
  conv_tile(pk, up, MT, NTL);
  const long long groups = (long long)((H + kConvTH - 1) / kConvTH) * ((W + 16 * NTL - 1) / (16 * NTL)) *
                           ((pk.Coutp + 16 * MT - 1) / (16 * MT)) * B;
  if (groups >= kConvSplitGroups) return 1;
  return (int)std::min<long long>(pk.ncc, (kConvSplitGroups + groups - 1) / groups);
}

template <int MT, int NTL>
static void conv3_launch(const ConvArgs& a, bool af32, bool outf32, hipStream_t s) {
  const int tiles = ((a.in.H + kConvTH - 1) / kConvTH) * ((a.in.W + 16 * NTL - 1) / (16 * NTL));
  const int ks = a.ksplit;
  const dim3 grid(tiles, (a.pk.Coutp + 16 * MT - 1) / (16 * MT), a.B * ks);
  size_t lds = (size_t)(kConvTH + 2) * (16 * NTL + 2) * (a.pk.CC + 8) * sizeof(uint16_t);
  if constexpr (MT == 4) {
    if (ks == 1 && outf32 && a.rt.gA && a.rt.modeA == 1) {
      // an upsampled route stages every wave's column-pair sums of its A tiles
      lds = std::max(lds, (size_t)4 * (8 * NTL) * (16 * MT + 4) * sizeof(float));
      hipLaunchKernelGGL((k_conv3<true, true, MT, NTL, true>), grid, dim3(256), lds, s, a);
      return;
    }
  }
  if (af32 && outf32) hipLaunchKernelGGL((k_conv3<true, true, MT, NTL>), grid, dim3(256), lds, s, a);
  else if (af32) hipLaunchKernelGGL((k_conv3<true, false, MT, NTL>), grid, dim3(256), lds, s, a);
  else hipLaunchKernelGGL((k_conv3<false, false, MT, NTL>), grid, dim3(256), lds, s, a);
}

hipError_t launch_conv3(const ConvArgs& args, bool af32, bool outf32, hipStream_t s) {
  ConvArgs a = args;
  a.ksplit = std::max(1, a.ksplit);  // the kernel divides by it
  const bool up = outf32 && a.rt.gA && a.rt.modeA == 1;
  // FP32 outputs are input gradients: FP32 input, routed or not
  if (outf32 && !af32) return hipErrorInvalidValue;
  if (a.ksplit > 1 && (!a.kpart || a.ksplit > a.pk.ncc)) return hipErrorInvalidValue;
  int MT, NTL;
  conv_tile(a.pk, up, MT, NTL);
  if (MT == 1) conv3_launch<1, 4>(a, af32, outf32, s);
  else conv3_launch<4, 2>(a, af32, outf32, s);
  if (a.ksplit > 1) {
    const long long npix = (long long)a.B * a.in.H * a.in.W;
    const long long n = npix * (a.pk.Cout >> 2);  // an upper bound of both index ranges
    if (outf32) hipLaunchKernelGGL(k_conv_finish<true>, dim3(grid_for(n)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_conv_finish<false>, dim3(grid_for(n)), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

// output-channel tile of the weight gradient: 16, 32 or 64 (no idle tiles
// for 16- and 32-channel layers)
int wgrad_cot(int Cout) { return Cout <= 16 ? 16 : (Cout <= 32 ? 32 : 64); }

hipError_t launch_wgrad(const WgradArgs& a, bool af32, hipStream_t s) {
  const int cot = wgrad_cot(a.Cout);
  const dim3 grid(a.nccw, (a.Cout + cot - 1) / cot, a.nsplit);
  if (cot == 16) {
    if (af32) hipLaunchKernelGGL((k_wgrad<true, 16>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_wgrad<false, 16>), grid, dim3(256), 0, s, a);
  } else if (cot == 32) {
    if (af32) hipLaunchKernelGGL((k_wgrad<true, 32>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_wgrad<false, 32>), grid, dim3(256), 0, s, a);
  } else {
    if (af32) hipLaunchKernelGGL((k_wgrad<true, 64>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_wgrad<false, 64>), grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_wgrad_reduce(const RedAll& a, hipStream_t s) {
  if (a.wg[a.n] < 1) return hipSuccess;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)a.wg[a.n]), dim3(256), 0, s, a);
  return hipGetLastError();
}

size_t head_fwd_lds(int P, int C1) { return (size_t)(P * C1 + P + C1 + 1) * 4; }
size_t head_bwd_lds(int P, int C1) {
  // the four waves' 16 x 16 tiles of the (P + 1) x (C1 + 1) entries
  const size_t red = (size_t)4 * ((P + 16) / 16) * ((C1 + 16) / 16) * 256;
  return std::max((size_t)(256 * (P + 1) + 256 * (C1 + 1) + P * C1 + C1), red) * 4;
}

hipError_t launch_head_fwd(const HeadArgs& a, hipStream_t s) {
  const long long npix = (long long)a.B * a.H * a.W;
  const dim3 grid((unsigned)((npix + 255) / 256));
  const size_t lds = head_fwd_lds(a.P, a.C1);
  if (a.C1 == 8) hipLaunchKernelGGL(k_head_fwd<8>, grid, dim3(256), lds, s, a);
  else if (a.C1 == 16) hipLaunchKernelGGL(k_head_fwd<16>, grid, dim3(256), lds, s, a);
  else if (a.C1 == 32) hipLaunchKernelGGL(k_head_fwd<32>, grid, dim3(256), lds, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_head_bwd(const LossArgs& a, int nblk, float* ghead, double* loss, double lam_w, hipStream_t s) {
  const long long npix = (long long)a.hd.B * a.hd.H * a.hd.W;
  if ((a.hd.P + 1 + 15) / 16 > kHeadRowTiles) return hipErrorInvalidValue;
  const size_t lds = head_bwd_lds(a.hd.P, a.hd.C1);
  if (a.hd.C1 == 8) hipLaunchKernelGGL(k_head_bwd<8>, dim3(nblk), dim3(256), lds, s, a);
  else if (a.hd.C1 == 16) hipLaunchKernelGGL(k_head_bwd<16>, dim3(nblk), dim3(256), lds, s, a);
  else if (a.hd.C1 == 32) hipLaunchKernelGGL(k_head_bwd<32>, dim3(nblk), dim3(256), lds, s, a);
  else return hipErrorInvalidValue;
  sum_parts((const float*)a.hpart, nblk, a.ne, a.hpart + (long long)nblk * a.ne, ghead, s);
  hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(256), 0, s, (const double*)a.lpart, nblk,
                     (double)npix * a.hd.P, (double)npix, lam_w, loss);
  return hipGetLastError();
}

hipError_t launch_pack(const PackAll& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(grid_for(a.start[a.n])), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adamw(float* th, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                        float eps, float wd, float bc1, float bc2, hipStream_t s) {
  hipLaunchKernelGGL(k_adamw, dim3(grid_for(n)), dim3(256), 0, s, th, g, m, v, n, lr, b1, b2, eps, wd, bc1, bc2);
  return hipGetLastError();
}


hipError_t unet_kernels_init() {
  hipError_t e = hipSuccess;
  const void* fns[3] = {reinterpret_cast<const void*>(&k_head_bwd<8>), reinterpret_cast<const void*>(&k_head_bwd<16>),
                        reinterpret_cast<const void*>(&k_head_bwd<32>)};
  for (const void* f : fns) {
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
  }
  return e;
}

}  // namespace unet
