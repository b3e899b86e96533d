// Internal types shared by the U-Net host code and its HIP kernels.
//
// Activations are BF16 (stored as raw uint16_t bit patterns) in NHWC layout
// [B][H][W][C]; activation gradients are FP32 NHWC.  A 3x3 convolution is an
// implicit GEMM on the BF16 matrix cores: out[co][pixel] = sum over
// k = (tap, ci) of Wp[co][k] * in[pixel + tap][ci].  The reduction index is
// split into channel chunks of CC channels (8, 16 or 32), and one 32-wide
// MFMA k-step covers TPK = 32 / CC taps of one chunk; taps are padded to KKp
// (a multiple of TPK) with zero weights.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace unet {

constexpr int kConvTH = 4;    // output rows per conv workgroup (one per wave)
constexpr int kWgTH = 4;      // pixel tile of the weight-gradient kernel (rows)
constexpr int kWgTW = 32;     //                                      (columns)

// Input of a convolution as its loader sees it: channels [0, Ca) come from
// tensor A (mode 0: same resolution; 1: A at half resolution, nearest 2x
// upsample; 2: A at double resolution, 2x2 mean), channels [Ca, Ca + Cb)
// from tensor Bs at the same resolution (the concatenated skip), and the
// rest up to the padded count are zero.
struct ConvIn {
  const void* A;            // BF16 NHWC, or FP32 NHWC when the kernel's AF32 is set
  const uint16_t* Bs;       // BF16 NHWC skip, or null
  int Ca, Cb, modeA;
  int H, W;                 // conv (output) resolution
};

// Packed-weight geometry of one convolution (forward or transposed).
struct ConvPack {
  int Cin, Cout;            // real channel counts
  int Cip;                  // padded input channels: 8, 16 or a multiple of 32
  int CC, ncc, TPK, KKp;    // channel chunk, chunk count, taps per k-step, padded taps
  int Coutp;                // Cout rounded up to 16
};

// Where an input-gradient convolution stores its result: the gradient of a
// forward convolution's input goes straight to the tensors that input was
// built from.  Channels [0, Ca) belong to A (mode 0: same resolution; 1: A at
// half resolution, so a 2 x 2 block of gradient pixels sums into one A pixel;
// 2: A at double resolution, each gradient pixel gives a quarter to its four
// A pixels), channels [Ca, Ca + Cb) to the skip B at the same resolution.  A
// tensor's first contribution is written, later ones are added (accA, accB).
// A and B are ReLU outputs: the stored gradient is that of their
// pre-activations, each value zeroed where the activation (mA, mB) is not
// positive, which is what every consumer of the gradient needs.
struct ConvRoute {
  float* gA;                // FP32 NHWC gradient of A, or null: plain output to ConvArgs::out
  float* gB;                // FP32 NHWC gradient of the skip, or null
  const uint16_t* mA;       // BF16 activation A (ReLU mask), or null
  const uint16_t* mB;       // BF16 skip activation (ReLU mask), or null
  int Ca, Cb, modeA, accA, accB;
};
struct ConvArgs {
  ConvIn in;
  ConvPack pk;
  const uint16_t* Wp;       // BF16 [Coutp][ncc][KKp][CC]
  const float* bias;        // [Cout] or null
  int relu;
  void* out;                // BF16 or FP32 NHWC [B][H][W][Cout]
  int B;
  ConvRoute rt;             // FP32 outputs only
  // split over the channel chunks: with ksplit > 1, grid.z = ksplit B and
  // split ks sums chunks [ks ncc / ksplit, (ks + 1) ncc / ksplit) into
  // kpart [ksplit][B][H][W][Coutp] (FP32); k_conv_finish adds the splits in
  // order and applies the epilogue (bias, ReLU and store, or the route)
  int ksplit;
  float* kpart;
};

struct WgradArgs {
  ConvIn in;                // the convolution's input (forward view)
  const float* gY;          // FP32 NHWC [B][H][W][Cout]: gradient of the conv output before its ReLU
  int Cout, Cin;            // real counts
  int CCw, nccw, Cipw;      // channel chunk of the reduction tile (16 or 32), chunks, padded count
  float* part;              // [nsplit][Cout][9][Cipw]
  float* bpart;             // [nsplit][Cout] bias partials (from channel chunk 0)
  int nsplit, B;
};

struct PackArgs {
  const float* W;           // canonical [Cout][Cin][3][3]
  uint16_t* Wp;             // forward packing
  uint16_t* Wtp;            // transposed packing (input = Cout channels, output = Cin), or null
  ConvPack f, t;
};
// The weight and bias gradients of every convolution summed from their
// pixel-split partials in one launch.  Layer l's elements (weights in the
// partials' (co, kk, ci) order, then the Cout biases) go to workgroups
// wg[l] <= b < wg[l + 1], e of them per workgroup (64, or 16 with more
// thread groups over the splits where a layer has many splits).
constexpr int kRedMax = 20;
struct RedLayer {
  const float* part;        // [nsplit][Cout][9][Cipw]
  const float* bpart;       // [nsplit][Cout]
  float* grad;              // [Cout][Cin][3][3]
  float* gb;                // [Cout]
  int nsplit, Cout, Cin, Cipw;
  int e;                    // elements per workgroup: 16 or 64
};
struct RedAll {
  int n;
  int wg[kRedMax + 1];
  RedLayer L[kRedMax];
};
// Every convolution's packings in one launch: packed element e belongs to
// layer l with start[l] <= e < start[l + 1] (forward packing first).
constexpr int kPackMax = 20;
struct PackAll {
  int n;
  int start[kPackMax + 1];
  PackArgs L[kPackMax];
};



struct HeadArgs {
  const uint16_t* h;        // BF16 NHWC [B][H][W][C1]
  const float* Wm;          // [P][C1], then bias [P]
  const float* Ww;          // [1][C1], then bias [1]
  float* y_m;               // [B][P][H][W]
  float* y_w;               // [B][H][W]
  int C1, P, B, H, W;
};

struct LossArgs {
  HeadArgs hd;
  const float* t_m;
  const float* t_w;
  float lam_w;
  float* g_h;               // FP32 NHWC [B][H][W][C1] gradient of the head input's pre-activation (ReLU)
  float* hpart;             // [nblk][ne] head parameter-gradient partials, then [ceil(nblk / 64)][ne] scratch
  double* lpart;            // [nblk][2]
  int ne;                   // entries per head partial: P*C1 + P + C1 + 1
};

}  // namespace unet
