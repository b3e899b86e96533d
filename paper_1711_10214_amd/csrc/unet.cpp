// Host side of the warm-start U-Net behind include/unet.h: parameter
// storage, workspace layout and the forward / backward launch sequences.
//
// The network is a fixed graph of 14 3x3 convolutions and two 1x1 heads.
// Each convolution reads its input through a loader that fuses the 2x2 mean
// pool (encoder), the nearest 2x upsample and the skip concatenation
// (decoder), so pooled, upsampled and concatenated tensors never exist in
// memory.  The backward pass walks the graph in reverse: bias gradient,
// weight gradient (split over pixels, fixed-order reduction) and input
// gradient (the same convolution kernel with transposed, tap-flipped
// weights), whose result is routed back to the tensors the loader read.
#include "ashrt.h"
#include "unet.h"
#include "unet_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace ashrt {
int set_error(int code, const std::string& msg);
}

namespace unet {
hipError_t launch_conv3(const ConvArgs& a, bool af32, bool outf32, hipStream_t s);
int conv_ksplit(const ConvPack& pk, int B, int H, int W, bool up);
hipError_t launch_wgrad(const WgradArgs& a, bool af32, hipStream_t s);
hipError_t launch_wgrad_reduce(const RedAll& a, hipStream_t s);
int wgrad_cot(int Cout);
hipError_t launch_head_fwd(const HeadArgs& a, hipStream_t s);
hipError_t launch_head_bwd(const LossArgs& a, int nblk, float* ghead, double* loss, double lam_w, hipStream_t s);
hipError_t launch_pack(const PackAll& a, hipStream_t s);
hipError_t launch_adamw(float* th, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                        float eps, float wd, float bc1, float bc2, hipStream_t s);
hipError_t unet_kernels_init();
}  // namespace unet

using namespace unet;

namespace {

int fail(int code, const std::string& m) { return ashrt::set_error(code, m); }

#define U_TRY(expr)                                                                \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ASHRT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kNConv = 18;
// Pixel splits of a weight gradient: at most kWgradTargetGroups workgroups,
// and no more splits than balance the FP32 partials each split writes (and
// the reduction reads back) against the tiles each workgroup walks in
// sequence: with P partial bytes per split and T pixel tiles, about
// sqrt(T kWgradTileBytes / P) splits, kWgradTileBytes being the partial
// traffic that costs about as long as one tile's load latency.
constexpr int kWgradTargetGroups = 1024;
constexpr double kWgradTileBytes = 6e6;

ConvPack make_pack(int Cin, int Cout) {
  ConvPack p{};
  p.Cin = Cin;
  p.Cout = Cout;
  p.Cip = Cin <= 8 ? 8 : (Cin <= 16 ? 16 : (Cin + 31) / 32 * 32);
  p.CC = std::min(p.Cip, 32);
  p.ncc = p.Cip / p.CC;
  p.TPK = 32 / p.CC;
  p.KKp = (9 + p.TPK - 1) / p.TPK * p.TPK;
  p.Coutp = (Cout + 15) / 16 * 16;
  return p;
}

long long pack_elems(const ConvPack& p) { return (long long)p.Coutp * p.ncc * p.KKp * p.CC; }

struct Layer {
  int ci = 0, co = 0, k = 3;
  long long woff = 0, boff = 0;
  int level = 0;
  int srcA = -1, modeA = 0, srcB = -1;  // srcA -1: the network input
  int Ca = 0, Cb = 0;
  ConvPack f{}, t{};
  long long wp_off = 0, wtp_off = 0;
};

long long align_up(long long v, long long a) { return (v + a - 1) / a * a; }

}  // namespace

struct unet_net {
  int device = 0, cin = 1, pout = 0, base = 16;
  std::vector<Layer> L;  // kNConv convolutions, then head_m, head_w
  long long nparam = 0, npk = 0;
  void* dev = nullptr;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* wpk = nullptr;
  long long step = 0;
};

namespace {

void build_graph(unet_net& n) {
  // four 2x down-samplings (levels 0..4), channels c1..c4 and a c4-wide bottleneck
  const int c1 = n.base, c2 = 2 * n.base, c3 = 4 * n.base, c4 = 8 * n.base, c5 = 8 * n.base;
  struct Spec {
    int ci, co, level, srcA, modeA, srcB;
  };
  const Spec S[kNConv] = {
      {n.cin, c1, 0, -1, 0, -1},    // enc1a
      {c1, c1, 0, 0, 0, -1},        // enc1b
      {c1, c2, 1, 1, 2, -1},        // enc2a (pool)
      {c2, c2, 1, 2, 0, -1},        // enc2b
      {c2, c3, 2, 3, 2, -1},        // enc3a
      {c3, c3, 2, 4, 0, -1},        // enc3b
      {c3, c4, 3, 5, 2, -1},        // enc4a
      {c4, c4, 3, 6, 0, -1},        // enc4b
      {c4, c5, 4, 7, 2, -1},        // bota
      {c5, c5, 4, 8, 0, -1},        // botb
      {c5 + c4, c4, 3, 9, 1, 7},    // dec4a [up(botb), enc4b]
      {c4, c4, 3, 10, 0, -1},       // dec4b
      {c4 + c3, c3, 2, 11, 1, 5},   // dec3a [up(dec4b), enc3b]
      {c3, c3, 2, 12, 0, -1},       // dec3b
      {c3 + c2, c2, 1, 13, 1, 3},   // dec2a [up(dec3b), enc2b]
      {c2, c2, 1, 14, 0, -1},       // dec2b
      {c2 + c1, c1, 0, 15, 1, 1},   // dec1a [up(dec2b), enc1b]
      {c1, c1, 0, 16, 0, -1},       // dec1b
  };
  long long off = 0, pk = 0;
  n.L.clear();
  for (int i = 0; i < kNConv; ++i) {
    Layer l;
    l.ci = S[i].ci;
    l.co = S[i].co;
    l.k = 3;
    l.level = S[i].level;
    l.srcA = S[i].srcA;
    l.modeA = S[i].modeA;
    l.srcB = S[i].srcB;
    l.Cb = l.srcB >= 0 ? S[l.srcB].co : 0;
    l.Ca = l.ci - l.Cb;
    l.woff = off;
    l.boff = off + (long long)l.co * l.ci * 9;
    off = l.boff + l.co;
    l.f = make_pack(l.ci, l.co);
    l.t = make_pack(l.co, l.ci);
    l.wp_off = pk;
    pk += align_up(pack_elems(l.f), 8);
    l.wtp_off = pk;
    pk += align_up(pack_elems(l.t), 8);
    n.L.push_back(l);
  }
  for (int h = 0; h < 2; ++h) {
    Layer l;
    l.ci = c1;
    l.co = h == 0 ? n.pout : 1;
    l.k = 1;
    l.woff = off;
    l.boff = off + (long long)l.co * l.ci;
    off = l.boff + l.co;
    n.L.push_back(l);
  }
  n.nparam = off;
  n.npk = pk;
}

struct WsLayout {
  std::vector<size_t> act, gact;
  std::vector<size_t> wpart, bpart;  // per layer: its weight-gradient partials stay until the reduction
  size_t y_m = 0, y_w = 0, hpart = 0, lpart = 0, kpart = 0, total = 0;
  std::vector<int> ks_f, ks_d;  // channel-chunk splits of the forward and input-gradient convolutions
  std::vector<int> nsplit;
  int nblk_h = 0;
};

int wgrad_cipw(const Layer& l) { return std::max(16, l.f.Cip); }
int wgrad_ccw(const Layer& l) { return std::min(wgrad_cipw(l), 32); }

WsLayout layout(const unet_net& n, int B, int H, int W, bool train) {
  WsLayout w;
  size_t off = 0;
  auto take = [&](long long bytes) {
    const size_t o = off;
    off = (size_t)align_up((long long)off + std::max(bytes, 0LL), 256);
    return o;
  };
  const long long npix0 = (long long)B * H * W;
  w.act.resize(kNConv);
  for (int i = 0; i < kNConv; ++i) {
    const Layer& l = n.L[i];
    w.act[i] = take((long long)B * (H >> l.level) * (W >> l.level) * l.co * 2);
  }
  w.y_m = take(npix0 * n.pout * 4);
  w.y_w = take(npix0 * 4);
  // FP32 partials of the convolutions split over their channel chunks
  long long kp = 0;
  w.ks_f.resize(kNConv);
  w.ks_d.resize(kNConv);
  for (int i = 0; i < kNConv; ++i) {
    const Layer& l = n.L[i];
    const int Hl = H >> l.level, Wl = W >> l.level;
    w.ks_f[i] = conv_ksplit(l.f, B, Hl, Wl, false);
    kp = std::max(kp, (long long)w.ks_f[i] * B * Hl * Wl * l.f.Coutp);
    w.ks_d[i] = train && i > 0 ? conv_ksplit(l.t, B, Hl, Wl, l.modeA == 1) : 1;
    if (w.ks_d[i] > 1) kp = std::max(kp, (long long)w.ks_d[i] * B * Hl * Wl * l.t.Coutp);
  }
  w.kpart = take(kp * 4);
  if (train) {
    w.gact.resize(kNConv);
    w.nsplit.resize(kNConv);
    for (int i = 0; i < kNConv; ++i) {
      const Layer& l = n.L[i];
      const int Hl = H >> l.level, Wl = W >> l.level;
      w.gact[i] = take((long long)B * Hl * Wl * l.co * 4);
      const int cipw = wgrad_cipw(l), ccw = wgrad_ccw(l);
      const long long T = (long long)B * ((Hl + kWgTH - 1) / kWgTH) * ((Wl + kWgTW - 1) / kWgTW);
      const int cot = wgrad_cot(l.co);
      const long long groups = (long long)(cipw / ccw) * ((l.co + cot - 1) / cot);
      const double pbytes = (double)l.co * 9 * cipw * 4;
      const long long nbal = std::max(1LL, (long long)std::sqrt((double)T * kWgradTileBytes / pbytes));
      const int ns = (int)std::max(
          1LL, std::min({T, (long long)kWgradTargetGroups / std::max(1LL, groups), nbal}));
      w.nsplit[i] = ns;
      w.wpart.push_back(take((long long)ns * l.co * 9 * cipw * 4));
      w.bpart.push_back(take((long long)ns * l.co * 4));
    }
    w.nblk_h = (int)((npix0 + 255) / 256);  // head-backward workgroups, one per 256 pixels
    const int ne = n.pout * n.base + n.pout + n.base + 1;
    // the head partials, then the rows of their first summation stage
    w.hpart = take(((long long)w.nblk_h + (w.nblk_h + 63) / 64) * ne * 4);
    w.lpart = take((long long)w.nblk_h * 2 * 8);
  }
  w.total = off;
  return w;
}

int check_shape(const unet_net* n, int B, int H, int W) {
  if (!n) return fail(ASHRT_E_INVALID_ARG, "net is NULL");
  if (B < 1 || H < 16 || W < 16 || (H % 16) || (W % 16))
    return fail(ASHRT_E_INVALID_ARG, "B >= 1 and H, W positive multiples of 16 required");
  return ASHRT_OK;
}

struct DevGuard {
  int prev = -1;
  bool ok = false;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess) ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
  }
  ~DevGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

ConvIn conv_input(const unet_net& n, const WsLayout& w, unsigned char* ws, const float* x, int i, int H, int W) {
  const Layer& l = n.L[i];
  ConvIn in{};
  in.A = l.srcA < 0 ? (const void*)x : (const void*)(ws + w.act[l.srcA]);
  in.Bs = l.srcB >= 0 ? (const uint16_t*)(ws + w.act[l.srcB]) : nullptr;
  in.Ca = l.Ca;
  in.Cb = l.Cb;
  in.modeA = l.modeA;
  in.H = H >> l.level;
  in.W = W >> l.level;
  return in;
}

int run_forward(const unet_net& n, const WsLayout& w, unsigned char* ws, const float* x, int B, int H, int W,
                float* y_m, float* y_w, hipStream_t s) {
  for (int i = 0; i < kNConv; ++i) {
    const Layer& l = n.L[i];
    ConvArgs a{};
    a.in = conv_input(n, w, ws, x, i, H, W);
    a.pk = l.f;
    a.Wp = n.wpk + l.wp_off;
    a.bias = n.theta + l.boff;
    a.relu = 1;
    a.out = ws + w.act[i];
    a.B = B;
    a.ksplit = w.ks_f[i];
    a.kpart = (float*)(ws + w.kpart);
    U_TRY(launch_conv3(a, l.srcA < 0, false, s));
  }
  HeadArgs h{};
  h.h = (const uint16_t*)(ws + w.act[kNConv - 1]);
  h.Wm = n.theta + n.L[kNConv].woff;
  h.Ww = n.theta + n.L[kNConv + 1].woff;
  h.y_m = y_m;
  h.y_w = y_w;
  h.C1 = n.base;
  h.P = n.pout;
  h.B = B;
  h.H = H;
  h.W = W;
  U_TRY(launch_head_fwd(h, s));
  return ASHRT_OK;
}

// Loss and gradient into g (nparam floats) after run_forward.
int run_backward(const unet_net& n, const WsLayout& w, unsigned char* ws, const float* x, const float* t_m,
                 const float* t_w, int B, int H, int W, double lam_w, double* loss, float* g, hipStream_t s) {
  // every activation gradient is written by its first contribution (the
  // head, or the input gradient of the first consumer in backward order)
  // and added to by the later ones
  std::vector<char> written(kNConv, 0);
  written[kNConv - 1] = 1;
  LossArgs la{};
  la.hd.h = (const uint16_t*)(ws + w.act[kNConv - 1]);
  la.hd.Wm = n.theta + n.L[kNConv].woff;
  la.hd.Ww = n.theta + n.L[kNConv + 1].woff;
  la.hd.y_m = (float*)(ws + w.y_m);
  la.hd.y_w = (float*)(ws + w.y_w);
  la.hd.C1 = n.base;
  la.hd.P = n.pout;
  la.hd.B = B;
  la.hd.H = H;
  la.hd.W = W;
  la.t_m = t_m;
  la.t_w = t_w;
  la.lam_w = (float)lam_w;
  la.g_h = (float*)(ws + w.gact[kNConv - 1]);
  la.hpart = (float*)(ws + w.hpart);
  la.lpart = (double*)(ws + w.lpart);
  la.ne = n.pout * n.base + n.pout + n.base + 1;
  U_TRY(launch_head_bwd(la, w.nblk_h, g + n.L[kNConv].woff, loss, lam_w, s));

  static_assert(kNConv <= kRedMax, "reduction table too small");
  RedAll red{};
  red.n = kNConv;
  for (int i = kNConv - 1; i >= 0; --i) {
    const Layer& l = n.L[i];
    const int Hl = H >> l.level, Wl = W >> l.level;
    const float* gY = (const float*)(ws + w.gact[i]);
    WgradArgs wa{};
    wa.in = conv_input(n, w, ws, x, i, H, W);
    wa.gY = gY;
    wa.Cout = l.co;
    wa.Cin = l.ci;
    wa.Cipw = wgrad_cipw(l);
    wa.CCw = wgrad_ccw(l);
    wa.nccw = wa.Cipw / wa.CCw;
    wa.part = (float*)(ws + w.wpart[i]);
    wa.bpart = (float*)(ws + w.bpart[i]);
    wa.nsplit = w.nsplit[i];
    wa.B = B;
    U_TRY(launch_wgrad(wa, l.srcA < 0, s));
    RedLayer& rl = red.L[i];
    rl.part = wa.part;
    rl.bpart = wa.bpart;
    rl.grad = g + l.woff;
    rl.gb = g + l.boff;
    rl.nsplit = wa.nsplit;
    rl.Cout = l.co;
    rl.Cin = l.ci;
    rl.Cipw = wa.Cipw;

    if (i == 0) continue;
    ConvArgs da{};
    da.in.A = gY;
    da.in.Bs = nullptr;
    da.in.Ca = l.co;
    da.in.Cb = 0;
    da.in.modeA = 0;
    da.in.H = Hl;
    da.in.W = Wl;
    da.pk = l.t;
    da.Wp = n.wpk + l.wtp_off;
    da.bias = nullptr;
    da.relu = 0;
    da.out = nullptr;
    da.B = B;
    da.rt.gA = (float*)(ws + w.gact[l.srcA]);
    da.rt.gB = l.srcB >= 0 ? (float*)(ws + w.gact[l.srcB]) : nullptr;
    da.rt.mA = (const uint16_t*)(ws + w.act[l.srcA]);
    da.rt.mB = l.srcB >= 0 ? (const uint16_t*)(ws + w.act[l.srcB]) : nullptr;
    da.rt.Ca = l.Ca;
    da.rt.Cb = l.srcB >= 0 ? l.Cb : 0;
    da.rt.modeA = l.modeA;
    da.rt.accA = written[l.srcA];
    da.rt.accB = l.srcB >= 0 ? written[l.srcB] : 0;
    written[l.srcA] = 1;
    if (l.srcB >= 0) written[l.srcB] = 1;
    da.ksplit = w.ks_d[i];
    da.kpart = (float*)(ws + w.kpart);
    U_TRY(launch_conv3(da, true, true, s));
  }
  // 16 elements a workgroup (16 thread groups over the splits) where a
  // layer has at least 256 splits, else 64 (4 groups)
  red.wg[0] = 0;
  for (int i = 0; i < kNConv; ++i) {
    RedLayer& rl = red.L[i];
    rl.e = rl.nsplit >= 256 ? 16 : 64;
    red.wg[i + 1] = red.wg[i] + (rl.Cout * (rl.Cin * 9 + 1) + rl.e - 1) / rl.e;
  }
  U_TRY(launch_wgrad_reduce(red, s));
  return ASHRT_OK;
}

int refresh_packed(const unet_net& n, hipStream_t s) {
  static_assert(kNConv <= kPackMax, "pack table too small");
  PackAll p{};
  p.n = kNConv;
  p.start[0] = 0;
  for (int i = 0; i < kNConv; ++i) {
    const Layer& l = n.L[i];
    PackArgs& a = p.L[i];
    a.W = n.theta + l.woff;
    a.Wp = n.wpk + l.wp_off;
    a.Wtp = i > 0 ? n.wpk + l.wtp_off : nullptr;
    a.f = l.f;
    a.t = l.t;
    const long long ne = (long long)l.f.Coutp * l.f.ncc * l.f.KKp * l.f.CC +
                         (a.Wtp ? (long long)l.t.Coutp * l.t.ncc * l.t.KKp * l.t.CC : 0);
    p.start[i + 1] = p.start[i] + (int)ne;
  }
  U_TRY(launch_pack(p, s));
  return ASHRT_OK;
}

std::once_flag g_init_once;
hipError_t g_init_err = hipSuccess;

}  // namespace

extern "C" int unet_create(const unet_desc* d, int device, unet_net** out) {
  if (!out) return fail(ASHRT_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!d) return fail(ASHRT_E_INVALID_ARG, "desc is NULL");
  if (d->cin != 1) return fail(ASHRT_E_UNSUPPORTED_SIZE, "cin must be 1");
  if (d->pout < 1 || d->pout > 64) return fail(ASHRT_E_UNSUPPORTED_SIZE, "pout must be in [1, 64]");
  if (d->base != 8 && d->base != 16 && d->base != 32) return fail(ASHRT_E_UNSUPPORTED_SIZE, "base must be 8, 16 or 32");
  unet_net* n = new (std::nothrow) unet_net();
  if (!n) return fail(ASHRT_E_OOM, "host allocation failed");
  n->device = device;
  n->cin = d->cin;
  n->pout = d->pout;
  n->base = d->base;
  build_graph(*n);
  DevGuard dg(device);
  if (!dg.ok) {
    delete n;
    return fail(ASHRT_E_HIP, "cannot select the device");
  }
  std::call_once(g_init_once, [] { g_init_err = unet_kernels_init(); });
  if (g_init_err != hipSuccess) {
    delete n;
    return fail(ASHRT_E_HIP, std::string("U-Net kernel set-up: ") + hipGetErrorString(g_init_err));
  }
  const size_t pb = (size_t)align_up(n->nparam * 4, 256);
  const size_t bytes = 4 * pb + (size_t)align_up(n->npk * 2, 256);
  if (hipMalloc(&n->dev, bytes) != hipSuccess) {
    delete n;
    return fail(ASHRT_E_OOM, "device allocation of the network failed");
  }
  unsigned char* p = (unsigned char*)n->dev;
  n->theta = (float*)p;
  n->grad = (float*)(p + pb);
  n->m = (float*)(p + 2 * pb);
  n->v = (float*)(p + 3 * pb);
  n->wpk = (uint16_t*)(p + 4 * pb);
  if (hipMemset(n->dev, 0, bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(n->dev);
    delete n;
    return fail(ASHRT_E_HIP, "clearing the network storage failed");
  }
  *out = n;
  return ASHRT_OK;
}

extern "C" void unet_destroy(unet_net* n) {
  if (!n) return;
  if (n->dev) {
    DevGuard dg(n->device);
    (void)hipFree(n->dev);
  }
  delete n;
}

extern "C" int64_t unet_param_count(const unet_net* n) { return n ? n->nparam : -1; }

extern "C" int unet_set_params(unet_net* n, const float* host, int64_t cnt) {
  if (!n || !host) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  if (cnt != n->nparam) return fail(ASHRT_E_INVALID_ARG, "parameter count mismatch");
  DevGuard dg(n->device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the device");
  U_TRY(hipMemcpy(n->theta, host, (size_t)cnt * 4, hipMemcpyHostToDevice));
  U_TRY(hipMemset(n->m, 0, (size_t)cnt * 4));
  U_TRY(hipMemset(n->v, 0, (size_t)cnt * 4));
  n->step = 0;
  int st = refresh_packed(*n, nullptr);
  if (st) return st;
  U_TRY(hipDeviceSynchronize());
  return ASHRT_OK;
}

extern "C" int unet_get_params(const unet_net* n, float* host, int64_t cnt) {
  if (!n || !host) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  if (cnt != n->nparam) return fail(ASHRT_E_INVALID_ARG, "parameter count mismatch");
  DevGuard dg(n->device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the device");
  U_TRY(hipDeviceSynchronize());
  U_TRY(hipMemcpy(host, n->theta, (size_t)cnt * 4, hipMemcpyDeviceToHost));
  return ASHRT_OK;
}

extern "C" int unet_workspace_bytes(const unet_net* n, int32_t B, int32_t H, int32_t W, int32_t train,
                                    size_t* bytes) {
  int st = check_shape(n, B, H, W);
  if (st) return st;
  if (!bytes) return fail(ASHRT_E_INVALID_ARG, "bytes is NULL");
  *bytes = layout(*n, B, H, W, train != 0).total;
  return ASHRT_OK;
}

static int check_ws(const WsLayout& w, void* ws, size_t wsb) {
  if (!ws || ((uintptr_t)ws & 255u)) return fail(ASHRT_E_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (wsb < w.total)
    return fail(ASHRT_E_WORKSPACE, "workspace has " + std::to_string(wsb) + " bytes, needs " + std::to_string(w.total));
  return ASHRT_OK;
}

extern "C" int unet_forward(const unet_net* n, const float* x, int32_t B, int32_t H, int32_t W, float* y_m,
                            float* y_w, void* ws, size_t wsb, void* stream) {
  int st = check_shape(n, B, H, W);
  if (st) return st;
  if (!x || !y_m || !y_w) return fail(ASHRT_E_INVALID_ARG, "x, y_model and y_w must be non-NULL");
  const WsLayout w = layout(*n, B, H, W, false);
  st = check_ws(w, ws, wsb);
  if (st) return st;
  DevGuard dg(n->device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the device");
  return run_forward(*n, w, (unsigned char*)ws, x, B, H, W, y_m, y_w, (hipStream_t)stream);
}

static int loss_grad_impl(unet_net* n, const float* x, const float* t_m, const float* t_w, int B, int H, int W,
                          double lam_w, double* loss, float* grad, void* ws, size_t wsb, hipStream_t s) {
  int st = check_shape(n, B, H, W);
  if (st) return st;
  if (!x || !t_m || !t_w || !loss || !grad) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  const WsLayout w = layout(*n, B, H, W, true);
  st = check_ws(w, ws, wsb);
  if (st) return st;
  unsigned char* W8 = (unsigned char*)ws;
  st = run_forward(*n, w, W8, x, B, H, W, (float*)(W8 + w.y_m), (float*)(W8 + w.y_w), s);
  if (st) return st;
  return run_backward(*n, w, W8, x, t_m, t_w, B, H, W, lam_w, loss, grad, s);
}

extern "C" int unet_loss_grad(unet_net* n, const float* x, const float* t_m, const float* t_w, int32_t B,
                              int32_t H, int32_t W, double lam_w, double* loss, float* grad, void* ws,
                              size_t wsb, void* stream) {
  if (!n) return fail(ASHRT_E_INVALID_ARG, "net is NULL");
  DevGuard dg(n->device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the device");
  return loss_grad_impl(n, x, t_m, t_w, B, H, W, lam_w, loss, grad, ws, wsb, (hipStream_t)stream);
}

extern "C" int unet_train_step(unet_net* n, const unet_train_params* tp, const float* x, const float* t_m,
                               const float* t_w, int32_t B, int32_t H, int32_t W, double* loss, void* ws,
                               size_t wsb, void* stream) {
  if (!n || !tp) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  if (!(tp->lr > 0.0) || !(tp->beta1 >= 0.0 && tp->beta1 < 1.0) || !(tp->beta2 >= 0.0 && tp->beta2 < 1.0) ||
      !(tp->eps > 0.0) || !(tp->weight_decay >= 0.0))
    return fail(ASHRT_E_INVALID_ARG, "invalid optimiser settings");
  DevGuard dg(n->device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the device");
  const hipStream_t s = (hipStream_t)stream;
  int st = loss_grad_impl(n, x, t_m, t_w, B, H, W, tp->lam_w, loss, n->grad, ws, wsb, s);
  if (st) return st;
  n->step += 1;
  const double bc1 = 1.0 - std::pow(tp->beta1, (double)n->step);
  const double bc2 = 1.0 - std::pow(tp->beta2, (double)n->step);
  U_TRY(launch_adamw(n->theta, n->grad, n->m, n->v, n->nparam, (float)tp->lr, (float)tp->beta1, (float)tp->beta2,
                     (float)tp->eps, (float)tp->weight_decay, (float)bc1, (float)bc2, s));
  return refresh_packed(*n, s);
}
