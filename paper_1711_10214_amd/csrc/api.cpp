// Host runtime of libashrt: argument validation, plans (small device tables
// and work lists), workspace layout, the operator pipelines and the IRLS-CG
// solver loop, behind the C ABI declared in include/ashrt.h.
//
// Nothing here allocates large buffers: the caller's workspace holds every
// intermediate spectrum and solver vector.  All launches go to the caller's
// stream; solver step lengths stay on the device, so a solve needs no host
// round trip unless a report or an early-stopping tolerance is requested.
#include "ashrt.h"
#include "fft_tpl.h"
#include "kernels.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace ashrt;

// ------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// Shared with the other C-ABI sources of the library (unet.cpp).
namespace ashrt {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace ashrt

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ASHRT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------ sizes
static bool is_fft_len(int n) {
  if (n < 2) return false;
  while ((n & 1) == 0) n >>= 1;
  return n == 1 || n == 3;
}

static int auto_fft_len(int n) {
  const long long target = 2LL * n;
  long long best = -1;
  for (long long p = 1; p < 4 * target + 8; p *= 2) {
    for (long long c : {p, 3 * p})
      if (c >= target && (best < 0 || c < best)) best = c;
  }
  return (int)best;
}

static long long align_up(long long v, long long a) { return (v + a - 1) / a * a; }

// Dynamic LDS a kernel may request (gfx950: 160 KB per workgroup, minus a
// margin for the kernels' static LDS).
static constexpr size_t kMaxDynLds = 150 * 1024;
// Largest sum over gathers of (per-tile partials)^2 that the consuming
// transform reduces in every workgroup (8 M doubles of cached reads per launch).
static constexpr double kInKernelSumLimit = 8.0 * 1024 * 1024;

// ------------------------------------------------------------ C ABI: defaults/validation
extern "C" void ashrt_desc_default(ashrt_desc* d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->half_width = 4;
}

extern "C" void irls_params_default(irls_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->p = 1;
  p->q = 2;
  p->n_outer = 10;
  p->n_inner = 20;
  p->b_r = 1.345;
  p->b_m = 1.0;
  p->tol = 0.0;
  p->eps_floor_rel = 1e-6;
  p->freeze_eps = 0;
  p->cg_graph = 1;
}

struct Resolved {
  int nt, nx, ntp, nxp, P, R, jlo, jhi, kmax;
};

static int resolve_desc(const ashrt_desc* d, Resolved* out) {
  if (!d) return fail(ASHRT_E_INVALID_ARG, "desc is NULL");
  if (d->nt < 2 || d->nx < 2) return fail(ASHRT_E_INVALID_ARG, "nt and nx must be >= 2");
  if (!(d->dt > 0.0) || !(d->dx > 0.0) || !std::isfinite(d->dt) || !std::isfinite(d->dx))
    return fail(ASHRT_E_INVALID_ARG, "dt and dx must be finite and > 0");
  if (d->npanel < 1) return fail(ASHRT_E_INVALID_ARG, "npanel must be >= 1");
  if (!d->vel) return fail(ASHRT_E_INVALID_ARG, "vel is NULL");
  for (int p = 0; p < d->npanel; ++p) {
    if (!(d->vel[p] >= 0.0) || !std::isfinite(d->vel[p]))
      return fail(ASHRT_E_INVALID_ARG, "velocities must be finite and >= 0");
    if (d->tau0_samples && d->tau0_samples[p] < 0)
      return fail(ASHRT_E_INVALID_ARG, "tau0_samples must be >= 0");
    if (d->panel_scale && !std::isfinite(d->panel_scale[p]))
      return fail(ASHRT_E_INVALID_ARG, "panel_scale must be finite");
  }
  const int R = d->half_width == 0 ? 4 : d->half_width;
  if (R < 1 || R > kMaxHalfWidth) return fail(ASHRT_E_INVALID_ARG, "half_width must be 1..8");
  const int ntp = d->ntp ? d->ntp : auto_fft_len(d->nt);
  const int nxp = d->nxp ? d->nxp : auto_fft_len(d->nx);
  if (!is_fft_len(ntp) || !is_fft_len(nxp))
    return fail(ASHRT_E_UNSUPPORTED_SIZE, "ntp and nxp must be 2^a or 3*2^a");
  if (ntp < d->nt || nxp < d->nx) return fail(ASHRT_E_INVALID_ARG, "ntp >= nt and nxp >= nx required");
  if (ntp < 8 || ntp > kRowMaxN) return fail(ASHRT_E_UNSUPPORTED_SIZE, "ntp must be in [8, 4096]");
  if (nxp < 4 || nxp > 4096) return fail(ASHRT_E_UNSUPPORTED_SIZE, "nxp must be in [4, 4096]");
  if (!std::isfinite(d->fmin_hz) || !std::isfinite(d->fmax_hz) || d->fmin_hz < 0.0)
    return fail(ASHRT_E_INVALID_ARG, "fmin_hz must be >= 0 and both band edges finite");
  int jlo = (int)std::ceil(d->fmin_hz * ntp * d->dt);
  jlo = std::max(1, jlo);
  int jhi = ntp / 2 - 1;
  if (d->fmax_hz > 0.0) jhi = std::min(jhi, (int)std::floor(d->fmax_hz * ntp * d->dt));
  if (jhi < jlo) return fail(ASHRT_E_INVALID_ARG, "the mapped band is empty");
  if (d->wavelet_amp) {
    for (int j = 0; j <= ntp / 2; ++j)
      if (!std::isfinite(d->wavelet_amp[j])) return fail(ASHRT_E_INVALID_ARG, "wavelet_amp must be finite");
  }
  if (out) {
    out->nt = d->nt;
    out->nx = d->nx;
    out->ntp = ntp;
    out->nxp = nxp;
    out->P = d->npanel;
    out->R = R;
    out->jlo = jlo;
    out->jhi = jhi;
    out->kmax = std::min(ntp / 2 - 1, jhi + R);
  }
  return ASHRT_OK;
}

extern "C" int ashrt_desc_validate(const ashrt_desc* d) { return resolve_desc(d, nullptr); }

extern "C" int irls_params_validate(const irls_params* p) {
  if (!p) return fail(ASHRT_E_INVALID_ARG, "params is NULL");
  if (p->p != 1 && p->p != 2) return fail(ASHRT_E_INVALID_ARG, "p must be 1 or 2");
  if (p->q != 1 && p->q != 2) return fail(ASHRT_E_INVALID_ARG, "q must be 1 or 2");
  if (p->n_outer < 1 || p->n_outer > 64) return fail(ASHRT_E_INVALID_ARG, "n_outer must be 1..64");
  if (p->n_inner < 1 || p->n_inner > 100000) return fail(ASHRT_E_INVALID_ARG, "n_inner must be >= 1");
  if (!(p->b_r > 0.0) || !std::isfinite(p->b_r)) return fail(ASHRT_E_INVALID_ARG, "b_r must be > 0");
  if (!(p->b_m > 0.0) || !std::isfinite(p->b_m)) return fail(ASHRT_E_INVALID_ARG, "b_m must be > 0");
  if (!(p->tol >= 0.0) || !std::isfinite(p->tol)) return fail(ASHRT_E_INVALID_ARG, "tol must be >= 0");
  if (!(p->eps_floor_rel >= 0.0) || !std::isfinite(p->eps_floor_rel))
    return fail(ASHRT_E_INVALID_ARG, "eps_floor_rel must be >= 0");
  return ASHRT_OK;
}

extern "C" const char* ashrt_status_string(int s) {
  switch (s) {
    case ASHRT_OK: return "ok";
    case ASHRT_E_INVALID_ARG: return "invalid argument";
    case ASHRT_E_UNSUPPORTED_SIZE: return "unsupported size";
    case ASHRT_E_HIP: return "HIP runtime error";
    case ASHRT_E_NONFINITE: return "non-finite result";
    case ASHRT_E_OOM: return "out of memory";
    case ASHRT_E_NOT_IMPLEMENTED: return "not implemented";
    case ASHRT_E_WORKSPACE: return "workspace too small or misaligned";
    default: return "unknown status";
  }
}

extern "C" const char* ashrt_last_error(void) { return g_last_error.c_str(); }
extern "C" int ashrt_abi_version(void) { return ASHRT_ABI_VERSION; }

// ------------------------------------------------------------ plans
struct GatherHost {
  Resolved z;
  int nrows, tileT, ntiles, tileTd, ntilesd, nchunk;
  std::vector<PanelDev> panels;
  std::vector<float> wav;
  std::vector<double> xpos;  // irregular data-trace positions (m), empty = regular
  long long d_off, m_off, mask_off, X_off, H_off, Dp_off;
  long long nd() const { return (long long)z.nx * z.nt; }
  long long nm() const { return (long long)z.P * z.nx * z.nt; }
};

struct WsLayout {
  size_t X, H, Dp;                                  // operator scratch
  size_t r, s, q, Wr, pdir, g, u, Wminv;            // solver vectors
  size_t part, pdel, pgam, sc, sel, hist, rep;
  size_t total;
};

struct PlanImpl {
  int device = 0;
  int R = 4;
  int ngather = 0;
  std::vector<GatherHost> g;
  void* dev = nullptr;  // one allocation holding every device table
  GatherDev* d_gd = nullptr;
  PanelDev* d_pan = nullptr;
  float2* d_tw = nullptr;
  float* d_wav = nullptr;
  WorkItem *d_xm = nullptr, *d_xd = nullptr, *d_rf = nullptr, *d_rfin = nullptr, *d_ra = nullptr;
  int n_xm = 0, n_xd = 0, n_rf = 0, n_rfin = 0, n_ra = 0;
  // CG reductions of per-tile partials: summed by every consuming workgroup
  // (no extra launch) while that costs little (sum over gathers of items^2
  // below kInKernelSumLimit), else once per gather by k_sum_items
  bool sum_model_in_kernel = false, sum_data_in_kernel = false;
  // Work-list segments: items [first, first + count) share one kernel
  // instantiation (FFT length class `key`, 0 = generic) and LDS size.
  struct Seg {
    int key, first, count;
    size_t lds;
  };
  std::vector<Seg> s_xm, s_xd, s_rf, s_rfin, s_ra;
  VecItem *d_vm = nullptr, *d_vd = nullptr;
  int n_vm = 0, n_vd = 0;
  // Executable graphs of a CG iteration pair, keyed by the buffers their
  // launches read and write (everything else comes from the plan).
  struct CgGraph {
    const void* ws;
    const float* m;
    const uint8_t* mask;
    int q;
    hipGraphExec_t exec;
  };
  mutable std::mutex graph_mu;
  mutable std::vector<CgGraph> graphs;
  long long tot_d = 0, tot_m = 0, tot_mask = 0, tot_X = 0, tot_H = 0, tot_Dp = 0;

  WsLayout layout(int op, int q) const {
    WsLayout L{};
    long long off = 0;
    auto take = [&](long long bytes) {
      const long long o = off;
      off = align_up(off + std::max(bytes, 0LL), 256);
      return (size_t)o;
    };
    L.X = take(tot_X * 8);
    L.H = take(tot_H * 8);
    L.Dp = take(tot_Dp * 8);
    if (op == ASHRT_OP_INVERT) {
      L.r = take(tot_d * 4);
      L.s = take(tot_d * 4);
      L.q = take(tot_d * 4);
      L.Wr = take(tot_d * 4);
      L.pdir = take(tot_m * 4);
      L.g = take(tot_m * 4);
      if (q == 1) {
        L.u = take(tot_m * 4);
        L.Wminv = take(tot_m * 4);
      }
      L.part = take((long long)2 * std::max(n_vm, n_vd) * 8);
      L.pdel = take((long long)n_xd * 8);
      L.pgam = take((long long)n_xm * 8);
      L.sc = take((long long)ngather * kNScal * 8);
      L.sel = take((long long)ngather * sizeof(SelState));
      L.hist = take((long long)ngather * 2 * kSelBins * 4);
      L.rep = take((long long)ngather * sizeof(RepDev));
    }
    L.total = (size_t)off;
    return L;
  }
};

struct ashrt_plan {
  PlanImpl impl;
};
struct ashrt_batch_plan {
  PlanImpl impl;
};

static int build_gather(const ashrt_desc* d, const ashrt_tuning* tn, GatherHost* gh) {
  int st = resolve_desc(d, &gh->z);
  if (st) return st;
  const Resolved& z = gh->z;
  gh->nrows = z.nxp / 2;
  if (tn && ((tn->tile_model < 0 || (tn->tile_model & 1)) || (tn->tile_data < 0 || (tn->tile_data & 1)) ||
             tn->nchunk < 0))
    return fail(ASHRT_E_INVALID_ARG, "tile sizes must be even (or 0) and nchunk >= 0");
  int T = std::min(64, 2 * (kXfftTilePoints / z.nxp));
  T = std::max(2, T & ~1);
  if (tn && tn->tile_model > 0) T = tn->tile_model;
  gh->tileT = T;
  gh->ntiles = (z.nt + T - 1) / T;
  // the data transform is one panel: narrower tiles give it ~256 workgroups
  int Td = 2 * ((z.nt + 511) / 512);
  Td = std::max(2, std::min(T, Td));
  if (tn && tn->tile_data > 0) Td = tn->tile_data;
  gh->tileTd = Td;
  gh->ntilesd = (z.nt + Td - 1) / Td;
  gh->panels.resize(z.P);
  const double bin = (double)z.ntp * d->dt / ((double)z.nxp * d->dx);
  for (int p = 0; p < z.P; ++p) {
    const double c = d->vel[p] * bin;
    gh->panels[p].c2 = c * c;
    gh->panels[p].scale = d->panel_scale ? (float)d->panel_scale[p] : 1.0f;
    gh->panels[p].n0 = d->tau0_samples ? d->tau0_samples[p] : 0;
    // live rows: row 0 (its l = 0 half covers the band) and every row whose
    // cone edge c2 r^2 is at most jhi^2 (with a relative margin, so that a
    // row declared dead has no tap whichever way its a^2 is rounded)
    int rl = gh->nrows;
    if (z.jhi >= z.jlo && c * c > 0.0) {
      const double lim = (double)z.jhi * (double)z.jhi * (1.0 + 1e-9);
      rl = 1;
      while (rl < gh->nrows && c * c * (double)rl * (double)rl <= lim) ++rl;
    }
    gh->panels[p].rlive = rl;
    gh->panels[p].pad_ = 0;
  }
  gh->xpos.clear();
  if (d->x_pos) {
    for (int i = 0; i < z.nx; ++i)
      if (!std::isfinite(d->x_pos[i])) return fail(ASHRT_E_INVALID_ARG, "x_pos must be finite");
    gh->xpos.assign(d->x_pos, d->x_pos + z.nx);
  }
  gh->wav.clear();
  if (d->wavelet_amp) {
    gh->wav.resize(z.ntp / 2 + 1);
    for (int j = 0; j <= z.ntp / 2; ++j) gh->wav[j] = (float)d->wavelet_amp[j];
  }
  return ASHRT_OK;
}

static void destroy_impl(PlanImpl& P) {
  if (P.dev) {
    // hipFree waits for the device, so no cached graph is still running
    // when it is destroyed
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != P.device) {
      (void)hipSetDevice(P.device);
      (void)hipFree(P.dev);
      for (auto& gr : P.graphs) (void)hipGraphExecDestroy(gr.exec);
      (void)hipSetDevice(cur);
    } else {
      (void)hipFree(P.dev);
      for (auto& gr : P.graphs) (void)hipGraphExecDestroy(gr.exec);
    }
    P.graphs.clear();
    P.dev = nullptr;
  }
}

// ------------------------------------------------------------ static scratch
// Workspace of the allocation-free forward (ashrt_forward_noalloc): a
// file-scope device array, one copy per GPU the library runs on, held until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// a device address: kernels get the address from hipGetSymbolAddress,
// resolved once per device (with that device current) when a plan is
// created there, and kept in g_scratch.
constexpr size_t kStaticScratchBytes = (size_t)96 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch;  // device -> that device's copy of scratch

// The calling thread's current device must be `device`.
static int static_scratch_setup(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(device);
  if (it == g_scratch.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ASHRT_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = g_scratch.emplace(device, p).first;
  }
  if (out) *out = it->second;
  return ASHRT_OK;
}

// Build work lists and device tables for a set of gathers.
static int create_impl(const ashrt_desc* descs, int ngather, int device, PlanImpl& P,
                       const ashrt_tuning* tn = nullptr) {
  if (!descs || ngather < 1) return fail(ASHRT_E_INVALID_ARG, "no gathers");
  P.device = device;
  P.ngather = ngather;
  P.g.resize(ngather);
  for (int i = 0; i < ngather; ++i) {
    int st = build_gather(&descs[i], tn, &P.g[i]);
    if (st) return st;
  }
  P.R = P.g[0].z.R;
  for (auto& gh : P.g)
    if (gh.z.R != P.R) return fail(ASHRT_E_INVALID_ARG, "all gathers of a batch must share half_width");

  // panel chunks so that the row passes have enough workgroups
  long long total_rows = 0;
  for (auto& gh : P.g) total_rows += gh.nrows;
  for (auto& gh : P.g) {
    long long want = (1024 + total_rows - 1) / total_rows;
    if (tn && tn->nchunk > 0) want = tn->nchunk;
    gh.nchunk = (int)std::max(1LL, std::min<long long>(want, gh.z.P));
  }

  // packed offsets
  long long od = 0, om = 0, omask = 0, oX = 0, oH = 0, oDp = 0;
  for (auto& gh : P.g) {
    gh.d_off = od;
    gh.m_off = om;
    gh.mask_off = omask;
    gh.X_off = oX;
    gh.H_off = oH;
    gh.Dp_off = oDp;
    od += gh.nd();
    om += gh.nm();
    omask += gh.z.nx;
    oX += (long long)gh.z.P * gh.nrows * gh.z.nt;
    oH += (long long)gh.nrows * gh.z.nt;
    oDp += (long long)gh.nchunk * gh.nrows * 2 * (gh.z.jhi - gh.z.jlo + 1);
  }
  P.tot_d = od;
  P.tot_m = om;
  P.tot_mask = omask;
  P.tot_X = oX;
  P.tot_H = oH;
  P.tot_Dp = oDp;

  // twiddle pool (one table per distinct length)
  std::vector<int> lens;
  for (auto& gh : P.g) {
    lens.push_back(gh.z.ntp);
    lens.push_back(gh.z.nxp);
  }
  std::sort(lens.begin(), lens.end());
  lens.erase(std::unique(lens.begin(), lens.end()), lens.end());
  std::vector<float2> tw;
  std::vector<int> tw_off(lens.size()), twp_off(lens.size());
  for (size_t i = 0; i < lens.size(); ++i) {
    const int N = lens[i];
    tw_off[i] = (int)tw.size();
    for (int m = 0; m < N; ++m) {
      const double a = -2.0 * M_PI * (double)m / (double)N;
      tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
    }
    // pass table of the compile-time FFT: per pass (radix R, span Ns) the
    // base twiddles exp(-2 pi i jm / (Ns R)), jm = 0..Ns-1 (the kernels take
    // the powers r = 2..R-1 by recurrence)
    twp_off[i] = (int)tw.size();
    const int want = fft_tpl_twsize(N);
    if (want > 0) {
      std::vector<int> radices;
      int M = N;
      if (M % 3 == 0) {
        radices.push_back(3);
        M /= 3;
      }
      int L2 = 0;
      while ((1 << L2) < M) ++L2;
      for (int k = 0; k < L2 / 3; ++k) radices.push_back(8);
      if (L2 % 3 == 1) radices.push_back(2);
      if (L2 % 3 == 2) radices.push_back(4);
      int Ns = 1;
      const size_t start = tw.size();
      for (int R : radices) {
        for (int jm = 0; jm < Ns; ++jm) {
          const double a = -2.0 * M_PI * (double)jm / ((double)Ns * (double)R);
          tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
        }
        Ns *= R;
      }
      if ((int)(tw.size() - start) != want || Ns != N)
        return fail(ASHRT_E_UNSUPPORTED_SIZE, "internal: FFT pass table mismatch");
    }
  }
  auto idx_of = [&](int N) { return std::lower_bound(lens.begin(), lens.end(), N) - lens.begin(); };
  auto tw_of = [&](int N) { return tw_off[idx_of(N)]; };
  auto twp_of = [&](int N) { return twp_off[idx_of(N)]; };

  std::vector<PanelDev> pan;
  std::vector<float> wav;
  std::vector<GatherDev> gd(ngather);
  std::vector<WorkItem> xm, xd, rf, rfin, ra;
  std::vector<VecItem> vm, vd;
  std::vector<int> key_x(ngather), key_t(ngather);
  for (int gi = 0; gi < ngather; ++gi) {
    GatherHost& gh = P.g[gi];
    key_x[gi] = x_size_is_tpl(gh.z.nxp) ? gh.z.nxp : 0;
    key_t[gi] = rows_size_is_tpl(gh.z.ntp, gh.z.R) ? gh.z.ntp : 0;
    GatherDev& G = gd[gi];
    std::memset(&G, 0, sizeof(G));
    G.nt = gh.z.nt;
    G.nx = gh.z.nx;
    G.ntp = gh.z.ntp;
    G.nxp = gh.z.nxp;
    G.nrows = gh.nrows;
    G.jlo = gh.z.jlo;
    G.jhi = gh.z.jhi;
    G.kmax = gh.z.kmax;
    G.npanel = gh.z.P;
    G.panel_off = (int)pan.size();
    pan.insert(pan.end(), gh.panels.begin(), gh.panels.end());
    G.tw_t_off = tw_of(gh.z.ntp);
    G.tw_x_off = tw_of(gh.z.nxp);
    G.twp_t_off = twp_of(gh.z.ntp);
    G.twp_x_off = twp_of(gh.z.nxp);
    if (!gh.wav.empty()) {
      G.wav_off = (int)wav.size();
      wav.insert(wav.end(), gh.wav.begin(), gh.wav.end());
    } else {
      G.wav_off = -1;
    }
    G.nudft_off = -1;
    if (!gh.xpos.empty()) {
      // exp(-2 pi i r x / (nxp dx)), r = 0..nrows-1; the phase in turns is
      // reduced in FP64 before the FP32 rounding
      if (tw.size() + (size_t)gh.nrows * gh.z.nx > (size_t)INT32_MAX)
        return fail(ASHRT_E_UNSUPPORTED_SIZE, "irregular-trace tables too large");
      G.nudft_off = (int)tw.size();
      const double period = (double)gh.z.nxp * descs[gi].dx;
      for (int r = 0; r < gh.nrows; ++r)
        for (int x = 0; x < gh.z.nx; ++x) {
          double turns = std::fmod((double)r * gh.xpos[x] / period, 1.0);
          const double a = -2.0 * M_PI * turns;
          tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
        }
    }
    G.tileT = gh.tileT;
    G.ntiles = gh.ntiles;
    G.tileTd = gh.tileTd;
    G.ntilesd = gh.ntilesd;
    G.nchunk = gh.nchunk;
    G.d_off = gh.d_off;
    G.m_off = gh.m_off;
    G.mask_off = gh.mask_off;
    G.X_off = gh.X_off;
    G.H_off = gh.H_off;
    G.Dp_off = gh.Dp_off;
    G.mit_lo = (int)vm.size();
    for (long long s0 = 0; s0 < gh.nm(); s0 += kVecChunk)
      vm.push_back(VecItem{gi, 0, gh.m_off + s0, std::min(kVecChunk, gh.nm() - s0)});
    G.mit_hi = (int)vm.size();
    G.dit_lo = (int)vd.size();
    for (long long s0 = 0; s0 < gh.nd(); s0 += kDataVecChunk)
      vd.push_back(VecItem{gi, 0, gh.d_off + s0, std::min(kDataVecChunk, gh.nd() - s0)});
    G.dit_hi = (int)vd.size();
  }
  // LDS bytes of each kernel family for one gather
  // (padded FFT buffers: fft_padlen slots; x columns at an odd slot stride)
  auto xstride = [](const GatherHost& gh) { return (size_t)(fft_padlen(gh.z.nxp) | 1); };
  auto twx_of = [](const GatherHost& gh) {
    return (size_t)fft_tw_slots(x_size_is_tpl(gh.z.nxp) ? gh.z.nxp : 0, gh.z.nxp);
  };
  auto twt_of = [](const GatherHost& gh) {
    return (size_t)fft_tw_slots(rows_size_is_tpl(gh.z.ntp, gh.z.R) ? gh.z.ntp : 0, gh.z.ntp);
  };
  auto lds_x_of = [&](const GatherHost& gh) {
    return twx_of(gh) * 8 + (size_t)(gh.tileT / 2) * xstride(gh) * 8;
  };
  auto lds_xd_of = [&](const GatherHost& gh) {
    return twx_of(gh) * 8 + (size_t)(gh.tileTd / 2) * xstride(gh) * 8;
  };
  auto nband_of = [](const GatherHost& gh) { return (size_t)(gh.z.jhi - gh.z.jlo + 1); };
  auto plen_of = [](const GatherHost& gh) { return (size_t)fft_padlen(gh.z.ntp); };
  auto lds_rf_of = [&](const GatherHost& gh) {
    return (twt_of(gh) + kMapGuardSlots + plen_of(gh)) * 8 + nband_of(gh) * 16;
  };
  auto lds_fin_of = [&](const GatherHost& gh) { return (twt_of(gh) + plen_of(gh)) * 8; };
  auto lds_ra_of = [&](const GatherHost& gh) { return (twt_of(gh) + 2 * plen_of(gh)) * 8; };
  // work lists grouped by kernel instantiation; a gather's items stay contiguous
  auto build_segments = [&](const std::vector<int>& keys, std::vector<PlanImpl::Seg>& segs,
                            std::vector<WorkItem>& items, auto&& add_items, auto&& lds_of) {
    std::map<int, std::vector<int>> by_key;
    for (int gi = 0; gi < ngather; ++gi) by_key[keys[gi]].push_back(gi);
    for (auto& kv : by_key) {
      PlanImpl::Seg sg{kv.first, (int)items.size(), 0, 0};
      for (int gi : kv.second) {
        add_items(gi);
        sg.lds = std::max(sg.lds, (size_t)lds_of(P.g[gi]));
      }
      sg.count = (int)items.size() - sg.first;
      if (sg.count > 0) segs.push_back(sg);
    }
  };
  build_segments(key_x, P.s_xm, xm, [&](int gi) {
    gd[gi].xm_lo = (int)xm.size();
    for (int p = 0; p < P.g[gi].z.P; ++p)
      for (int t = 0; t < P.g[gi].ntiles; ++t) xm.push_back(WorkItem{gi, p, t, 0});
    gd[gi].xm_hi = (int)xm.size();
  }, lds_x_of);
  build_segments(key_x, P.s_xd, xd, [&](int gi) {
    gd[gi].xd_lo = (int)xd.size();
    for (int t = 0; t < P.g[gi].ntilesd; ++t) xd.push_back(WorkItem{gi, 0, t, 0});
    gd[gi].xd_hi = (int)xd.size();
  }, lds_xd_of);
  build_segments(key_t, P.s_rf, rf, [&](int gi) {
    for (int r = 0; r < P.g[gi].nrows; ++r)
      for (int c = 0; c < P.g[gi].nchunk; ++c) rf.push_back(WorkItem{gi, r, c, 0});
  }, lds_rf_of);
  build_segments(key_t, P.s_ra, ra, [&](int gi) {
    for (int r = 0; r < P.g[gi].nrows; ++r)
      for (int c = 0; c < P.g[gi].nchunk; ++c) ra.push_back(WorkItem{gi, r, c, 0});
  }, lds_ra_of);
  build_segments(key_t, P.s_rfin, rfin, [&](int gi) {
    for (int r = 0; r < P.g[gi].nrows; ++r) rfin.push_back(WorkItem{gi, r, 0, 0});
  }, lds_fin_of);
  if (wav.empty()) wav.push_back(0.f);

  for (auto* segs : {&P.s_xm, &P.s_xd, &P.s_rf, &P.s_rfin, &P.s_ra})
    for (auto& sg : *segs)
      if (sg.lds > kMaxDynLds) return fail(ASHRT_E_UNSUPPORTED_SIZE, "LDS requirement exceeds the per-workgroup limit");

  // one device allocation for all tables
  struct Part {
    const void* src;
    size_t bytes;
    void** dst;
  };
  P.n_xm = (int)xm.size();
  P.n_xd = (int)xd.size();
  {
    double cm = 0.0, cd = 0.0;
    for (const auto& G : gd) {
      cm += (double)(G.xm_hi - G.xm_lo) * (double)(G.xm_hi - G.xm_lo);
      cd += (double)(G.xd_hi - G.xd_lo) * (double)(G.xd_hi - G.xd_lo);
    }
    P.sum_model_in_kernel = cm <= kInKernelSumLimit;
    P.sum_data_in_kernel = cd <= kInKernelSumLimit;
  }
  P.n_rf = (int)rf.size();
  P.n_rfin = (int)rfin.size();
  P.n_ra = (int)ra.size();
  P.n_vm = (int)vm.size();
  P.n_vd = (int)vd.size();
  std::vector<Part> parts = {
      {gd.data(), gd.size() * sizeof(GatherDev), (void**)&P.d_gd},
      {pan.data(), pan.size() * sizeof(PanelDev), (void**)&P.d_pan},
      {tw.data(), tw.size() * sizeof(float2), (void**)&P.d_tw},
      {wav.data(), wav.size() * sizeof(float), (void**)&P.d_wav},
      {xm.data(), xm.size() * sizeof(WorkItem), (void**)&P.d_xm},
      {xd.data(), xd.size() * sizeof(WorkItem), (void**)&P.d_xd},
      {rf.data(), rf.size() * sizeof(WorkItem), (void**)&P.d_rf},
      {rfin.data(), rfin.size() * sizeof(WorkItem), (void**)&P.d_rfin},
      {ra.data(), ra.size() * sizeof(WorkItem), (void**)&P.d_ra},
      {vm.data(), vm.size() * sizeof(VecItem), (void**)&P.d_vm},
      {vd.data(), vd.size() * sizeof(VecItem), (void**)&P.d_vd},
  };
  size_t total = 0;
  std::vector<size_t> offs;
  for (auto& pt : parts) {
    offs.push_back(total);
    total = (size_t)align_up((long long)(total + pt.bytes), 256);
  }
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  HIP_TRY(hipSetDevice(device));
  std::vector<unsigned char> host(total, 0);
  for (size_t i = 0; i < parts.size(); ++i)
    if (parts[i].bytes) std::memcpy(host.data() + offs[i], parts[i].src, parts[i].bytes);
  hipError_t e = hipMalloc(&P.dev, total);
  if (e != hipSuccess) {
    (void)hipSetDevice(prev);
    P.dev = nullptr;
    return fail(ASHRT_E_OOM, std::string("hipMalloc of plan tables: ") + hipGetErrorString(e));
  }
  e = hipMemcpy(P.dev, host.data(), total, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    static std::once_flag once;
    static hipError_t init_err = hipSuccess;
    std::call_once(once, [] { init_err = op_kernels_init(kMaxDynLds); });
    e = init_err;
  }
  if (e == hipSuccess && static_scratch_setup(device, nullptr) != ASHRT_OK) {
    (void)hipSetDevice(prev);
    destroy_impl(P);
    return ASHRT_E_HIP;  // the message is already set
  }
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    destroy_impl(P);
    return fail(ASHRT_E_HIP, std::string("plan upload: ") + hipGetErrorString(e));
  }
  for (size_t i = 0; i < parts.size(); ++i) *parts[i].dst = (unsigned char*)P.dev + offs[i];
  return ASHRT_OK;
}

extern "C" int ashrt_plan_create(const ashrt_desc* desc, int device, ashrt_plan** out) {
  return ashrt_plan_create_tuned(desc, nullptr, device, out);
}

extern "C" int ashrt_plan_create_tuned(const ashrt_desc* desc, const ashrt_tuning* tuning, int device,
                                       ashrt_plan** out) {
  if (!out) return fail(ASHRT_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ashrt_plan* p = new (std::nothrow) ashrt_plan();
  if (!p) return fail(ASHRT_E_OOM, "host allocation failed");
  int st = create_impl(desc, 1, device, p->impl, tuning);
  if (st) {
    destroy_impl(p->impl);
    delete p;
    return st;
  }
  *out = p;
  return ASHRT_OK;
}

extern "C" void ashrt_plan_destroy(ashrt_plan* p) {
  if (!p) return;
  destroy_impl(p->impl);
  delete p;
}

extern "C" int ashrt_batch_plan_create(const ashrt_desc* descs, int32_t ngather, int device,
                                       ashrt_batch_plan** out) {
  return ashrt_batch_plan_create_tuned(descs, ngather, nullptr, device, out);
}

extern "C" int ashrt_batch_plan_create_tuned(const ashrt_desc* descs, int32_t ngather, const ashrt_tuning* tuning,
                                             int device, ashrt_batch_plan** out) {
  if (!out) return fail(ASHRT_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ashrt_batch_plan* p = new (std::nothrow) ashrt_batch_plan();
  if (!p) return fail(ASHRT_E_OOM, "host allocation failed");
  int st = create_impl(descs, ngather, device, p->impl, tuning);
  if (st) {
    destroy_impl(p->impl);
    delete p;
    return st;
  }
  *out = p;
  return ASHRT_OK;
}

extern "C" void ashrt_batch_plan_destroy(ashrt_batch_plan* p) {
  if (!p) return;
  destroy_impl(p->impl);
  delete p;
}

extern "C" int ashrt_plan_get_info(const ashrt_plan* plan, ashrt_plan_info* info) {
  if (!plan || !info) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  const PlanImpl& P = plan->impl;
  const GatherHost& g = P.g[0];
  std::memset(info, 0, sizeof(*info));
  info->nt = g.z.nt;
  info->nx = g.z.nx;
  info->ntp = g.z.ntp;
  info->nxp = g.z.nxp;
  info->npanel = g.z.P;
  info->half_width = g.z.R;
  info->jlo = g.z.jlo;
  info->jhi = g.z.jhi;
  info->kmax = g.z.kmax;
  info->nchunk = g.nchunk;
  info->tile_model = g.tileT;
  info->tile_data = g.tileTd;
  info->ws_forward = P.layout(ASHRT_OP_FORWARD, 2).total;
  info->ws_adjoint = P.layout(ASHRT_OP_ADJOINT, 2).total;
  info->ws_invert_q2 = P.layout(ASHRT_OP_INVERT, 2).total;
  info->ws_invert_q1 = P.layout(ASHRT_OP_INVERT, 1).total;
  return ASHRT_OK;
}

static int ws_bytes_impl(const PlanImpl& P, int op, const irls_params* prm, size_t* bytes) {
  if (!bytes) return fail(ASHRT_E_INVALID_ARG, "bytes is NULL");
  if (op < ASHRT_OP_FORWARD || op > ASHRT_OP_FISTA) return fail(ASHRT_E_INVALID_ARG, "unknown op");
  if (op == ASHRT_OP_FISTA) {  // the solver layout with four model-sized vectors
    *bytes = P.layout(ASHRT_OP_INVERT, 1).total;
    return ASHRT_OK;
  }
  int q = 2;
  if (op == ASHRT_OP_INVERT) {
    if (!prm) return fail(ASHRT_E_INVALID_ARG, "params needed for ASHRT_OP_INVERT");
    int st = irls_params_validate(prm);
    if (st) return st;
    q = prm->q;
  }
  *bytes = P.layout(op, q).total;
  return ASHRT_OK;
}

extern "C" int ashrt_workspace_bytes(const ashrt_plan* plan, int op, const irls_params* prm, size_t* bytes) {
  if (!plan) return fail(ASHRT_E_INVALID_ARG, "plan is NULL");
  return ws_bytes_impl(plan->impl, op, prm, bytes);
}

extern "C" int ashrt_batch_workspace_bytes(const ashrt_batch_plan* plan, int op, const irls_params* prm,
                                           size_t* bytes) {
  if (!plan) return fail(ASHRT_E_INVALID_ARG, "plan is NULL");
  return ws_bytes_impl(plan->impl, op, prm, bytes);
}

extern "C" int ashrt_batch_layout(const ashrt_batch_plan* plan, int64_t* data_off, int64_t* model_off,
                                  int64_t* mask_off, int64_t* data_total, int64_t* model_total,
                                  int64_t* mask_total) {
  if (!plan) return fail(ASHRT_E_INVALID_ARG, "plan is NULL");
  const PlanImpl& P = plan->impl;
  for (int i = 0; i < P.ngather; ++i) {
    if (data_off) data_off[i] = P.g[i].d_off;
    if (model_off) model_off[i] = P.g[i].m_off;
    if (mask_off) mask_off[i] = P.g[i].mask_off;
  }
  if (data_total) *data_total = P.tot_d;
  if (model_total) *model_total = P.tot_m;
  if (mask_total) *mask_total = P.tot_mask;
  return ASHRT_OK;
}

// ------------------------------------------------------------ profiling
namespace {

struct Prof {
  unsigned mask = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> rec[ASHRT_K_COUNT];
  std::vector<hipEvent_t> pool;
};
Prof g_prof;

hipEvent_t prof_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run `launch` (returning hipError_t) between two recorded events when the
// family is enabled.
template <class F>
hipError_t timed(int kid, hipStream_t s, F&& launch) {
  if (!(g_prof.mask & (1u << kid))) return launch();
  hipEvent_t a = prof_event(), b = prof_event();
  if (!a || !b) return launch();
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  if (e != hipSuccess) return e;
  g_prof.rec[kid].push_back({a, b});
  return hipSuccess;
}

}  // namespace

extern "C" int ashrt_profile_enable(uint32_t mask) {
  g_prof.mask = mask;
  return ASHRT_OK;
}

extern "C" int ashrt_profile_read(int kid, double* total_ms, int64_t* launches, int reset) {
  if (kid < 0 || kid >= ASHRT_K_COUNT) return fail(ASHRT_E_INVALID_ARG, "unknown kernel id");
  double tot = 0.0;
  auto& v = g_prof.rec[kid];
  for (auto& pr : v) {
    HIP_TRY(hipEventSynchronize(pr.second));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (int64_t)v.size();
  if (reset) {
    for (auto& pr : v) {
      g_prof.pool.push_back(pr.first);
      g_prof.pool.push_back(pr.second);
    }
    v.clear();
  }
  return ASHRT_OK;
}

extern "C" const char* ashrt_kernel_name(int kid) {
  static const char* names[ASHRT_K_COUNT] = {"k_xfft_fwd(model)", "k_xfft_fwd(data)", "k_rows_fwd",
                                             "k_rows_fwd_fin",    "k_xfft_inv(data)", "k_rows_adj",
                                             "k_xfft_inv(model)", "k_elementwise",    "k_reduce",
                                             "k_sel"};
  if (kid < 0 || kid >= ASHRT_K_COUNT) return "unknown";
  return names[kid];
}

// ------------------------------------------------------------ operator pipelines
namespace {

struct Ctx {
  const PlanImpl* P;
  unsigned char* ws;
  WsLayout L;
  hipStream_t s;
  float2* X() const { return (float2*)(ws + L.X); }
  float2* H() const { return (float2*)(ws + L.H); }
  float2* Dp() const { return (float2*)(ws + L.Dp); }
};

RowsArgs rows_args(const Ctx& c, const WorkItem* items, int n) {
  RowsArgs a{};
  a.gd = c.P->d_gd;
  a.items = items;
  a.nitems = n;
  a.panels = c.P->d_pan;
  a.tw = c.P->d_tw;
  a.wav = c.P->d_wav;
  a.X = c.X();
  a.H = c.H();
  a.Dp = c.Dp();
  a.R = c.P->R;
  return a;
}

// The previous CG iteration's vector update, fused into the next forward's
// model transform (which then reads pdir after the update).
struct CgUpd {
  float* u = nullptr;
  float* pdir = nullptr;
  const float* g = nullptr;
  const double* part_gamma = nullptr;  // the adjoint's per-tile partials of |g|^2
  double* sc = nullptr;
  int par = 0;  // gamma slot of the previous iteration
};

// d_out = epilogue(L (mul_m * m)); the epilogue is: raw_out = y; y = sub - y;
// y *= mask; y *= wmul.
// part: per-tile partials of sum y^2 over the data tiles; with sc they are
// also summed per gather into sc[SC_DELTA].
hipError_t run_forward(const Ctx& c, const float* m, const float* mul_m, float* d_out, const float* sub,
                       const float* wmul, float* raw_out, const uint8_t* tmask, double* part = nullptr,
                       const CgUpd* upd = nullptr, double* sc = nullptr) {
  const PlanImpl& P = *c.P;
  hipError_t e = hipSuccess;
  for (const auto& sg : P.s_xm) {
    XfwdArgs xa{};
    xa.gd = P.d_gd;
    xa.items = P.d_xm + sg.first;
    xa.nitems = sg.count;
    xa.item_base = sg.first;
    xa.is_model = 1;
    xa.src = m;
    xa.mul = mul_m;
    xa.dst = c.X();
    xa.tw = P.d_tw;
    xa.panels = P.d_pan;
    if (upd) {
      xa.cg_upd = 1;
      xa.cg_par = upd->par;
      xa.cg_p = upd->pdir;
      xa.cg_u = upd->u;
      xa.cg_g = upd->g;
      xa.part_red = P.sum_model_in_kernel ? upd->part_gamma : nullptr;
      xa.sc = upd->sc;
    }
    e = timed(ASHRT_K_XFFT_MODEL, c.s, [&] { return launch_xfft_fwd(sg.key, xa, sg.lds, c.s); });
    if (e != hipSuccess) return e;
  }
  for (const auto& sg : P.s_rf) {
    e = timed(ASHRT_K_ROWS_FWD, c.s,
              [&] { return launch_rows_fwd(sg.key, rows_args(c, P.d_rf + sg.first, sg.count), sg.lds, c.s); });
    if (e != hipSuccess) return e;
  }
  for (const auto& sg : P.s_rfin) {
    e = timed(ASHRT_K_ROWS_FIN, c.s, [&] {
      return launch_rows_fwd_fin(sg.key, rows_args(c, P.d_rfin + sg.first, sg.count), sg.lds, c.s);
    });
    if (e != hipSuccess) return e;
  }
  for (const auto& sg : P.s_xd) {
    XinvArgs ia{};
    ia.gd = P.d_gd;
    ia.items = P.d_xd + sg.first;
    ia.nitems = sg.count;
    ia.item_base = sg.first;
    ia.is_model = 0;
    ia.src = c.H();
    ia.out = d_out;
    ia.sub = sub;
    ia.wmul = wmul;
    ia.raw_out = raw_out;
    ia.tmask = tmask;
    ia.tw = P.d_tw;
    ia.panels = P.d_pan;
    ia.part = part;
    e = timed(ASHRT_K_XINV_DATA, c.s, [&] { return launch_xfft_inv(sg.key, ia, sg.lds, c.s); });
    if (e != hipSuccess) return e;
  }
  if (part && sc && !P.sum_data_in_kernel)
    return timed(ASHRT_K_REDUCE, c.s, [&] { return launch_sum_items(P.d_gd, P.ngather, part, 0, sc, SC_DELTA, c.s); });
  return hipSuccess;
}

// CG step folded into the adjoint's first pass (s -= alpha q first).
struct CgStep {
  float* s_inout = nullptr;
  const float* qv = nullptr;
  const double* part_delta = nullptr;  // the forward's per-tile partials of |q|^2
  double* sc = nullptr;
  int par = 0;
};

// m_out = wmul * L' (mask * mul_d * d); part: per-tile sums of m_out^2,
// with sc also summed per gather into sc[SC_GNEW].  wmul_sq: m_out gets
// wmul^2 * L'(...) and the partials sum (wmul * L'(...))^2.
hipError_t run_adjoint(const Ctx& c, const float* d, const float* mul_d, const uint8_t* tmask, float* m_out,
                       const float* wmul, double* part = nullptr, const CgStep* cg = nullptr,
                       double* sc = nullptr, bool wmul_sq = false) {
  const PlanImpl& P = *c.P;
  hipError_t e = hipSuccess;
  for (const auto& sg : P.s_xd) {
    XfwdArgs xa{};
    xa.gd = P.d_gd;
    xa.items = P.d_xd + sg.first;
    xa.nitems = sg.count;
    xa.item_base = sg.first;
    xa.is_model = 0;
    xa.src = d;
    xa.mul = mul_d;
    xa.tmask = tmask;
    xa.dst = c.H();
    xa.tw = P.d_tw;
    xa.panels = P.d_pan;
    if (cg) {
      xa.s_inout = cg->s_inout;
      xa.qv = cg->qv;
      xa.part_red = P.sum_data_in_kernel ? cg->part_delta : nullptr;
      xa.sc = cg->sc;
      xa.par = cg->par;
    }
    e = timed(ASHRT_K_XFFT_DATA, c.s, [&] { return launch_xfft_fwd(sg.key, xa, sg.lds, c.s); });
    if (e != hipSuccess) return e;
  }
  for (const auto& sg : P.s_ra) {
    e = timed(ASHRT_K_ROWS_ADJ, c.s,
              [&] { return launch_rows_adj(sg.key, rows_args(c, P.d_ra + sg.first, sg.count), sg.lds, c.s); });
    if (e != hipSuccess) return e;
  }
  for (const auto& sg : P.s_xm) {
    XinvArgs ia{};
    ia.gd = P.d_gd;
    ia.items = P.d_xm + sg.first;
    ia.nitems = sg.count;
    ia.item_base = sg.first;
    ia.is_model = 1;
    ia.src = c.X();
    ia.out = m_out;
    ia.wmul = wmul;
    ia.wmul_sq = wmul_sq ? 1 : 0;
    ia.tw = P.d_tw;
    ia.panels = P.d_pan;
    ia.part = part;
    e = timed(ASHRT_K_XINV_MODEL, c.s, [&] { return launch_xfft_inv(sg.key, ia, sg.lds, c.s); });
    if (e != hipSuccess) return e;
  }
  if (part && sc && !P.sum_model_in_kernel)
    return timed(ASHRT_K_REDUCE, c.s, [&] { return launch_sum_items(P.d_gd, P.ngather, part, 1, sc, SC_GNEW, c.s); });
  return hipSuccess;
}

int check_ws(const PlanImpl& P, int op, int q, void* ws, size_t ws_bytes, Ctx* c, void* stream) {
  c->P = &P;
  c->L = P.layout(op, q);
  if (!ws || ((uintptr_t)ws & 255u) != 0) return fail(ASHRT_E_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (ws_bytes < c->L.total)
    return fail(ASHRT_E_WORKSPACE, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                                       std::to_string(c->L.total));
  c->ws = (unsigned char*)ws;
  c->s = (hipStream_t)stream;
  return ASHRT_OK;
}

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess) ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int forward_impl(const PlanImpl& P, const float* m, float* d, const uint8_t* mask, void* ws, size_t wsb,
                 void* stream) {
  if (!m || !d) return fail(ASHRT_E_INVALID_ARG, "m and d must be non-NULL");
  Ctx c;
  int st = check_ws(P, ASHRT_OP_FORWARD, 2, ws, wsb, &c, stream);
  if (st) return st;
  DeviceGuard dg(P.device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the plan's device");
  HIP_TRY(run_forward(c, m, nullptr, d, nullptr, nullptr, nullptr, mask));
  return ASHRT_OK;
}

int adjoint_impl(const PlanImpl& P, const float* d, float* m, const uint8_t* mask, void* ws, size_t wsb,
                 void* stream) {
  if (!m || !d) return fail(ASHRT_E_INVALID_ARG, "m and d must be non-NULL");
  Ctx c;
  int st = check_ws(P, ASHRT_OP_ADJOINT, 2, ws, wsb, &c, stream);
  if (st) return st;
  DeviceGuard dg(P.device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the plan's device");
  HIP_TRY(run_adjoint(c, d, nullptr, mask, m, nullptr));
  return ASHRT_OK;
}

// ------------------------------------------------------------ IRLS-CG solver loop
struct Solver {
  Ctx c;
  const PlanImpl& P;
  const irls_params& prm;
  float* r;
  float* s;
  float* q;
  float* Wr;
  float* pdir;
  float* g;
  float* u;
  float* Wminv;
  double* part;
  double* pdel;
  double* pgam;
  double* sc;
  SelState* sel;
  unsigned* hist;
  RepDev* rep;

  EwArgs ew(int op, bool model) const {
    EwArgs a{};
    a.gd = P.d_gd;
    a.items = model ? P.d_vm : P.d_vd;
    a.nitems = model ? P.n_vm : P.n_vd;
    a.op = op;
    a.sc = sc;
    a.sign = 1.f;
    return a;
  }
  hipError_t reduce(int op, bool model, const float* x, const uint8_t* tmask, int dst0, int dst1, bool is_max,
                    RepDev* rp, int outer) const {
    RedArgs a{};
    a.gd = P.d_gd;
    a.items = model ? P.d_vm : P.d_vd;
    a.nitems = model ? P.n_vm : P.n_vd;
    a.op = op;
    a.is_model = model;
    a.x = x;
    a.tmask = tmask;
    a.sc = sc;
    a.p = prm.p;
    a.part = part;
    hipError_t e = timed(ASHRT_K_REDUCE, c.s, [&] { return launch_reduce_part(a, c.s); });
    if (e != hipSuccess) return e;
    FinArgs f{};
    f.gd = P.d_gd;
    f.ngather = P.ngather;
    f.is_model = model;
    f.is_max = is_max;
    f.part = part;
    f.sc = sc;
    f.dst0 = dst0;
    f.dst1 = dst1;
    f.rep = rp;
    f.outer = outer;
    return timed(ASHRT_K_REDUCE, c.s, [&] { return launch_reduce_fin(f, c.s); });
  }
  hipError_t scalar(int step, int outer) const {
    ScalArgs a{};
    a.ngather = P.ngather;
    a.step = step;
    a.sc = sc;
    a.rep = rep;
    a.outer = outer;
    a.b_r = prm.b_r;
    a.b_m = prm.b_m;
    a.floor_rel = prm.eps_floor_rel;
    a.freeze = prm.freeze_eps;
    return launch_scalar(a, c.s);
  }
  hipError_t cg(int init, int par) const {
    CgArgs a{};
    a.gd = P.d_gd;
    a.items = P.d_vm;
    a.nitems = P.n_vm;
    a.init = init;
    a.par = par;
    a.u = u;
    a.pdir = pdir;
    a.g = g;
    a.part_gamma = P.sum_model_in_kernel ? pgam : nullptr;
    a.sc = sc;
    return timed(ASHRT_K_VECTOR, c.s, [&] { return launch_cg(a, c.s); });
  }
  hipError_t median(const float* x, const uint8_t* tmask, int stage, int dst) const {
    SelArgs a{};
    a.gd = P.d_gd;
    a.items = P.d_vd;
    a.nitems = P.n_vd;
    a.ngather = P.ngather;
    a.x = x;
    a.tmask = tmask;
    a.sc = sc;
    a.st = sel;
    a.hist = hist;
    a.stage = stage;
    return timed(ASHRT_K_SELECT, c.s, [&] { return launch_select_median(a, sc, dst, c.s); });
  }
};

#define E_TRY(expr)                                                                  \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return fail(ASHRT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// One CG iteration on A = W_r S L W_m^-1, all on S.c.s, with its vectors
// kept in model space (u = m, pdir and g scaled by W_m^-1, so the forward
// needs no weight; the q = 2 case has W_m = 1):
//   q = W_r S L pdir (per-tile partials of |q|^2); alpha = gamma / |q|^2;
//   s -= alpha q; g = W_m^-2 L' S W_r s, gamma = |W_m^-1 L' S W_r s|^2.  Its
//   vector update (beta, m += alpha pdir, pdir = g + beta pdir) runs inside
//   the next iteration's model transform (fused: this iteration applies the
//   previous one's), or as k_cg after the last iteration.  par selects the
//   gamma slot pair.
hipError_t cg_iteration(const Solver& S, const uint8_t* mask, int par, bool fused) {
  CgUpd up;
  up.u = S.u;
  up.pdir = S.pdir;
  up.g = S.g;
  up.part_gamma = S.pgam;
  up.sc = S.sc;
  up.par = par ^ 1;
  hipError_t e = run_forward(S.c, S.pdir, nullptr, S.q, nullptr, S.Wr, nullptr, mask, S.pdel,
                             fused ? &up : nullptr, S.sc);
  if (e != hipSuccess) return e;
  CgStep st;
  st.s_inout = S.s;
  st.qv = S.q;
  st.part_delta = S.pdel;
  st.sc = S.sc;
  st.par = par;
  return run_adjoint(S.c, S.s, S.Wr, mask, S.g, S.Wminv, S.pgam, &st, S.sc, S.Wminv != nullptr);
}

constexpr size_t kMaxCgGraphs = 8;

// The executable graph of two fused CG iterations (parities 1 then 0, each
// applying the other's update) for these buffers: captured on a private
// stream the first time, then cached.
int cg_graph_get(const PlanImpl& P, const Solver& S, const uint8_t* mask, int q, hipGraphExec_t* out) {
  std::lock_guard<std::mutex> lk(P.graph_mu);
  const float* mkey = S.u;
  for (const auto& gr : P.graphs)
    if (gr.ws == (const void*)S.c.ws && gr.m == mkey && gr.mask == mask && gr.q == q) {
      *out = gr.exec;
      return ASHRT_OK;
    }
  if (P.graphs.size() >= kMaxCgGraphs) {
    // the oldest graph may still be running on some stream
    E_TRY(hipDeviceSynchronize());
    (void)hipGraphExecDestroy(P.graphs.front().exec);
    P.graphs.erase(P.graphs.begin());
  }
  hipStream_t cs = nullptr;
  E_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  Solver S2 = S;
  S2.c.s = cs;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    e = cg_iteration(S2, mask, 1, true);
    if (e == hipSuccess) e = cg_iteration(S2, mask, 0, true);
    hipGraph_t graph = nullptr;
    const hipError_t e_end = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = e_end;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e == hipSuccess) {
      P.graphs.push_back(PlanImpl::CgGraph{S.c.ws, mkey, mask, q, exec});
      *out = exec;
    }
  }
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) return fail(ASHRT_E_HIP, std::string("CG graph capture: ") + hipGetErrorString(e));
  return ASHRT_OK;
}

int invert_impl(const PlanImpl& P, const irls_params* prm, const float* d, const uint8_t* mask, float* m,
                const float* w0, float* d_rec, irls_report* reps, void* ws, size_t wsb, void* stream,
                bool batched) {
  if (!d || !m) return fail(ASHRT_E_INVALID_ARG, "d and m must be non-NULL");
  int st = irls_params_validate(prm);
  if (st) return st;
  if (batched && prm->tol > 0.0)
    return fail(ASHRT_E_INVALID_ARG, "batched solves run fixed iteration counts (tol must be 0)");
  Ctx c;
  st = check_ws(P, ASHRT_OP_INVERT, prm->q, ws, wsb, &c, stream);
  if (st) return st;
  DeviceGuard dg(P.device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the plan's device");
  const WsLayout& L = c.L;
  unsigned char* W = c.ws;
  Solver S{c, P, *prm,
           (float*)(W + L.r), (float*)(W + L.s), (float*)(W + L.q), (float*)(W + L.Wr),
           (float*)(W + L.pdir), (float*)(W + L.g), m,
           prm->q == 1 ? (float*)(W + L.Wminv) : nullptr,
           (double*)(W + L.part), (double*)(W + L.pdel), (double*)(W + L.pgam), (double*)(W + L.sc), (SelState*)(W + L.sel), (unsigned*)(W + L.hist),
           (RepDev*)(W + L.rep)};
  const hipStream_t s = c.s;
  const bool q1 = prm->q == 1, p1 = prm->p == 1;
  hipGraphExec_t cg_exec = nullptr;
  if (prm->cg_graph && prm->n_inner >= 3 && g_prof.mask == 0) {
    st = cg_graph_get(P, S, mask, prm->q, &cg_exec);
    if (st) return st;
  }

  // clear scalars, selection histograms and the report
  E_TRY(launch_zero_words(S.sc, (long long)P.ngather * kNScal * 2, s));
  E_TRY(launch_zero_words(S.hist, (long long)P.ngather * 2 * kSelBins, s));
  E_TRY(launch_zero_words(S.rep, (long long)P.ngather * sizeof(RepDev) / 4, s));
  E_TRY(launch_count_live(P.d_gd, P.ngather, mask, S.sc, s));
  E_TRY(S.reduce(RED_ABSMAX_LIVE, false, d, mask, SC_DMAX, -1, true, nullptr, 0));
  // r = S (d - L m)
  E_TRY(run_forward(c, m, nullptr, S.r, d, nullptr, nullptr, mask));

  std::vector<RepDev> host_rep;
  int outer_done = 0;
  for (int k = 0; k < prm->n_outer; ++k) {
    // weights of this outer iteration
    if (k == 0) {
      EwArgs a = S.ew(EW_WR_INIT, false);
      a.y = S.Wr;
      a.x = w0;
      a.tmask = mask;
      E_TRY(timed(ASHRT_K_VECTOR, s, [&] { return launch_elementwise(a, s); }));
      if (q1) {
        EwArgs f = S.ew(EW_FILL, true);
        f.y = S.Wminv;
        f.value = 1.0f;
        E_TRY(timed(ASHRT_K_VECTOR, s, [&] { return launch_elementwise(f, s); }));
      }
    } else {
      EwArgs a = S.ew(p1 ? EW_WR_UPDATE : EW_WR_MASK, false);
      a.y = S.Wr;
      a.x = S.r;
      a.coef = SC_EPS_R;
      a.tmask = mask;
      E_TRY(timed(ASHRT_K_VECTOR, s, [&] { return launch_elementwise(a, s); }));
      if (q1) {
        E_TRY(S.reduce(RED_ABSMAX, true, m, nullptr, SC_MMAX, -1, true, nullptr, 0));
        E_TRY(S.scalar(ST_EPS_M, k));
        // W_m^-1 from m (its z_out = W_m m is not needed: pdir, overwritten
        // by the CG initialisation below, takes it)
        EwArgs w = S.ew(EW_WM_UPDATE, true);
        w.y = S.Wminv;
        w.x = m;
        w.z_out = S.pdir;
        w.coef = SC_EPS_M;
        E_TRY(timed(ASHRT_K_VECTOR, s, [&] { return launch_elementwise(w, s); }));
      }
    }
    // CGLS on A = W_r S L W_m^-1 from u = W_m m (in model space, see
    // cg_iteration):  s = W_r r ; g = W_m^-2 L' S s ; pdir = g
    {
      EwArgs a = S.ew(EW_MUL, false);
      a.y = S.s;
      a.x = S.Wr;
      a.z = S.r;
      E_TRY(timed(ASHRT_K_VECTOR, s, [&] { return launch_elementwise(a, s); }));
    }
    E_TRY(run_adjoint(c, S.s, S.Wr, mask, S.g, S.Wminv, S.pgam, nullptr, S.sc, q1));
    E_TRY(S.cg(1, 0));
    if (prm->n_inner > 0) {
      // iteration 0 starts from pdir = g; iterations 1.. apply their
      // predecessor's update in their model transform; k_cg applies the last
      E_TRY(cg_iteration(S, mask, 0, false));
      int i = 1;
      if (cg_exec)
        for (; i + 1 < prm->n_inner; i += 2) E_TRY(hipGraphLaunch(cg_exec, s));
      for (; i < prm->n_inner; ++i) E_TRY(cg_iteration(S, mask, i & 1, true));
      E_TRY(S.cg(0, (prm->n_inner - 1) & 1));
    }
    E_TRY(S.scalar(ST_REPORT_INNER, k));
    // residual, separated gather, clip and misfit
    E_TRY(run_forward(c, m, nullptr, S.r, d, nullptr, d_rec, mask));
    if (p1) {
      E_TRY(S.median(S.r, mask, 0, SC_MED));
      E_TRY(S.median(S.r, mask, 1, SC_MAD));
      E_TRY(S.scalar(ST_EPS_R, k));
    }
    E_TRY(S.reduce(RED_MISFIT, false, S.r, mask, SC_MISFIT, SC_HUBER, false, S.rep, k));
    outer_done = k + 1;
    if (prm->tol > 0.0 && k >= 1) {
      host_rep.resize(P.ngather);
      E_TRY(hipMemcpyAsync(host_rep.data(), S.rep, sizeof(RepDev) * P.ngather, hipMemcpyDeviceToHost, s));
      E_TRY(hipStreamSynchronize(s));
      const double a = host_rep[0].misfit[k - 1], b = host_rep[0].misfit[k];
      if (a > 0.0 && std::fabs(b - a) / a < prm->tol) break;
    }
  }

  if (reps || prm->tol > 0.0) {
    host_rep.resize(P.ngather);
    std::vector<double> hsc((size_t)P.ngather * kNScal);
    E_TRY(hipMemcpyAsync(host_rep.data(), S.rep, sizeof(RepDev) * P.ngather, hipMemcpyDeviceToHost, s));
    E_TRY(hipMemcpyAsync(hsc.data(), S.sc, hsc.size() * 8, hipMemcpyDeviceToHost, s));
    E_TRY(hipStreamSynchronize(s));
    bool nonfinite = false;
    for (int gi = 0; gi < P.ngather; ++gi) {
      const bool bad = hsc[(size_t)gi * kNScal + SC_NONFINITE] != 0.0;
      nonfinite |= bad;
      if (reps) {
        irls_report& R = reps[gi];
        std::memset(&R, 0, sizeof(R));
        R.status = bad ? ASHRT_E_NONFINITE : ASHRT_OK;
        R.outer_done = outer_done;
        for (int k = 0; k < outer_done; ++k) {
          R.inner[k] = (int32_t)host_rep[gi].inner[k];
          R.misfit[k] = host_rep[gi].misfit[k];
          R.huber[k] = host_rep[gi].huber[k];
          R.eps_r[k] = host_rep[gi].eps_r[k];
          R.eps_m[k] = host_rep[gi].eps_m[k];
        }
      }
    }
    if (nonfinite) return fail(ASHRT_E_NONFINITE, "the solve produced a non-finite misfit");
  }
  return ASHRT_OK;
}

// ------------------------------------------------------------ FISTA solver loop
// Workspace: the solver layout with q = 1 (vectors r: residual; pdir: y;
// g: gradient; u: power-method vector).
int fista_impl(const PlanImpl& P, const fista_params* prm, const float* d, const uint8_t* mask, float* m,
               float* d_rec, fista_report* rep, void* ws, size_t wsb, void* stream) {
  if (!prm || !d || !m) return fail(ASHRT_E_INVALID_ARG, "params, d and m must be non-NULL");
  if (prm->n_iter < 1 || prm->n_power < 1) return fail(ASHRT_E_INVALID_ARG, "n_iter and n_power must be >= 1");
  if (!(prm->mu > 0.0) && !(prm->mu_rel > 0.0))
    return fail(ASHRT_E_INVALID_ARG, "mu > 0 or mu_rel > 0 required");
  if (!(prm->lip_safety >= 1.0)) return fail(ASHRT_E_INVALID_ARG, "lip_safety must be >= 1");
  Ctx c;
  int st = check_ws(P, ASHRT_OP_INVERT, 1, ws, wsb, &c, stream);
  if (st) return st;
  DeviceGuard dg(P.device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the plan's device");
  const WsLayout& L = c.L;
  unsigned char* W = c.ws;
  irls_params dummy{};
  Solver S{c, P, dummy,
           (float*)(W + L.r), (float*)(W + L.s), (float*)(W + L.q), (float*)(W + L.Wr),
           (float*)(W + L.pdir), (float*)(W + L.g), (float*)(W + L.u), (float*)(W + L.Wminv),
           (double*)(W + L.part), (double*)(W + L.pdel), (double*)(W + L.pgam), (double*)(W + L.sc),
           (SelState*)(W + L.sel), (unsigned*)(W + L.hist), (RepDev*)(W + L.rep)};
  const hipStream_t s = c.s;
  float* y = S.pdir;
  float* g = S.g;
  float* x = S.u;
  E_TRY(launch_zero_words(S.sc, (long long)P.ngather * kNScal * 2, s));
  // power method on L' S L from the all-ones model, normalised
  {
    EwArgs f = S.ew(EW_FILL, true);
    f.y = x;
    f.value = (float)(1.0 / std::sqrt((double)P.tot_m / P.ngather));
    E_TRY(timed(ASHRT_K_VECTOR, s, [&] { return launch_elementwise(f, s); }));
  }
  for (int it = 0; it < prm->n_power; ++it) {
    E_TRY(run_forward(c, x, nullptr, S.r, nullptr, nullptr, nullptr, mask));
    E_TRY(run_adjoint(c, S.r, nullptr, mask, g, nullptr));
    E_TRY(S.reduce(RED_SUMSQ, true, g, nullptr, SC_POW_SS, -1, false, nullptr, 0));
    EwArgs a = S.ew(EW_SCALE_RSQRT, true);
    a.y = x;
    a.x = g;
    a.coef = SC_POW_SS;
    E_TRY(timed(ASHRT_K_VECTOR, s, [&] { return launch_elementwise(a, s); }));
  }
  // mu from max|L' S d|, then Lf, step and threshold
  E_TRY(run_adjoint(c, d, nullptr, mask, g, nullptr));
  E_TRY(S.reduce(RED_ABSMAX, true, g, nullptr, SC_MMAX, -1, true, nullptr, 0));
  {
    ScalArgs a{};
    a.ngather = P.ngather;
    a.step = ST_FISTA;
    a.sc = S.sc;
    a.safety = prm->lip_safety;
    a.mu_abs = prm->mu;
    a.mu_rel = prm->mu_rel;
    E_TRY(launch_scalar(a, s));
  }
  {
    EwArgs cp = S.ew(EW_COPY, true);
    cp.y = y;
    cp.x = m;
    E_TRY(timed(ASHRT_K_VECTOR, s, [&] { return launch_elementwise(cp, s); }));
  }
  double t = 1.0;
  for (int k = 0; k < prm->n_iter; ++k) {
    // r = S (d - L y); g = L' S r; then the shrinkage and momentum step
    E_TRY(run_forward(c, y, nullptr, S.r, d, nullptr, nullptr, mask));
    E_TRY(run_adjoint(c, S.r, nullptr, mask, g, nullptr));
    const double t_new = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    EwArgs a = S.ew(EW_FISTA, true);
    a.y = y;
    a.x = g;
    a.z_out = m;
    a.coef = SC_FSTEP;
    a.value = (float)((t - 1.0) / t_new);
    E_TRY(timed(ASHRT_K_VECTOR, s, [&] { return launch_elementwise(a, s); }));
    t = t_new;
  }
  // residual, separated / reconstructed gather, objective terms
  E_TRY(run_forward(c, m, nullptr, S.r, d, nullptr, d_rec, mask));
  E_TRY(S.reduce(RED_SUMSQ, false, S.r, mask, SC_MISFIT, -1, false, nullptr, 0));
  E_TRY(S.reduce(RED_ABSSUM, true, m, nullptr, SC_HUBER, -1, false, nullptr, 0));
  if (rep) {
    std::vector<double> hsc((size_t)P.ngather * kNScal);
    E_TRY(hipMemcpyAsync(hsc.data(), S.sc, hsc.size() * 8, hipMemcpyDeviceToHost, s));
    E_TRY(hipStreamSynchronize(s));
    std::memset(rep, 0, sizeof(*rep));
    rep->iters = prm->n_iter;
    rep->lipschitz = hsc[SC_LIP];
    rep->mu = hsc[SC_MU];
    rep->misfit = hsc[SC_MISFIT];
    rep->l1 = hsc[SC_HUBER];
    rep->objective = rep->misfit + rep->mu * rep->l1;
    rep->status = std::isfinite(rep->objective) ? ASHRT_OK : ASHRT_E_NONFINITE;
    if (rep->status) return fail(ASHRT_E_NONFINITE, "FISTA produced a non-finite objective");
  }
  return ASHRT_OK;
}

}  // namespace

extern "C" void fista_params_default(fista_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n_iter = 50;
  p->n_power = 20;
  p->mu = 0.0;
  p->mu_rel = 0.05;
  p->lip_safety = 1.05;
}

extern "C" int fista_invert(const ashrt_plan* plan, const fista_params* prm, const float* d, const uint8_t* mask,
                            float* m, float* d_rec, fista_report* rep, void* ws, size_t wsb, void* stream) {
  if (!plan) return fail(ASHRT_E_INVALID_ARG, "plan is NULL");
  return fista_impl(plan->impl, prm, d, mask, m, d_rec, rep, ws, wsb, stream);
}

extern "C" int ashrt_forward(const ashrt_plan* plan, const float* m, float* d, const uint8_t* mask, void* ws,
                             size_t wsb, void* stream) {
  if (!plan) return fail(ASHRT_E_INVALID_ARG, "plan is NULL");
  return forward_impl(plan->impl, m, d, mask, ws, wsb, stream);
}

extern "C" int ashrt_forward_noalloc(const ashrt_plan* plan, const float* m, float* d, const uint8_t* mask,
                                     void* stream) {
  if (!plan) return fail(ASHRT_E_INVALID_ARG, "plan is NULL");
  const PlanImpl& P = plan->impl;
  const size_t need = P.layout(ASHRT_OP_FORWARD, 2).total;
  if (need > kStaticScratchBytes)
    return fail(ASHRT_E_WORKSPACE, "the plan's forward needs " + std::to_string(need) +
                                       " bytes of scratch; the allocation-free entry point has " +
                                       std::to_string(kStaticScratchBytes) + " (use ashrt_forward with a workspace)");
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(P.device);
    if (it != g_scratch.end()) ws = it->second;
  }
  if (!ws) return fail(ASHRT_E_HIP, "no static scratch address for the plan's device");
  return forward_impl(P, m, d, mask, ws, kStaticScratchBytes, stream);
}

extern "C" int ashrt_adjoint(const ashrt_plan* plan, const float* d, float* m, const uint8_t* mask, void* ws,
                             size_t wsb, void* stream) {
  if (!plan) return fail(ASHRT_E_INVALID_ARG, "plan is NULL");
  return adjoint_impl(plan->impl, d, m, mask, ws, wsb, stream);
}

extern "C" int ashrt_td_forward(const ashrt_plan* plan, const float* m, float* d, const uint8_t* mask, void* stream) {
  if (!plan || !m || !d) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  const PlanImpl& P = plan->impl;
  if (!P.g[0].xpos.empty())
    return fail(ASHRT_E_NOT_IMPLEMENTED, "the time-domain pair takes regular traces only (plan has x_pos)");
  DeviceGuard dg(P.device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the plan's device");
  TdArgs a{P.d_gd, P.d_pan, const_cast<float*>(m), d, mask, (long long)P.g[0].nd()};
  HIP_TRY(launch_td(a, true, (hipStream_t)stream));
  return ASHRT_OK;
}

extern "C" int ashrt_td_adjoint(const ashrt_plan* plan, const float* d, float* m, const uint8_t* mask, void* stream) {
  if (!plan || !m || !d) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  const PlanImpl& P = plan->impl;
  if (!P.g[0].xpos.empty())
    return fail(ASHRT_E_NOT_IMPLEMENTED, "the time-domain pair takes regular traces only (plan has x_pos)");
  DeviceGuard dg(P.device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the plan's device");
  TdArgs a{P.d_gd, P.d_pan, m, const_cast<float*>(d), mask, (long long)P.g[0].nm()};
  HIP_TRY(launch_td(a, false, (hipStream_t)stream));
  return ASHRT_OK;
}

extern "C" int ashrt_forward_batched(const ashrt_batch_plan* plan, const float* m, float* d,
                                     const uint8_t* mask, void* ws, size_t wsb, void* stream) {
  if (!plan) return fail(ASHRT_E_INVALID_ARG, "plan is NULL");
  return forward_impl(plan->impl, m, d, mask, ws, wsb, stream);
}

extern "C" int ashrt_adjoint_batched(const ashrt_batch_plan* plan, const float* d, float* m,
                                     const uint8_t* mask, void* ws, size_t wsb, void* stream) {
  if (!plan) return fail(ASHRT_E_INVALID_ARG, "plan is NULL");
  return adjoint_impl(plan->impl, d, m, mask, ws, wsb, stream);
}

extern "C" int robust_invert(const ashrt_plan* plan, const irls_params* prm, const float* d,
                             const uint8_t* mask, float* m, const float* w0, float* d_rec, irls_report* rep,
                             void* ws, size_t wsb, void* stream) {
  if (!plan) return fail(ASHRT_E_INVALID_ARG, "plan is NULL");
  return invert_impl(plan->impl, prm, d, mask, m, w0, d_rec, rep, ws, wsb, stream, false);
}

extern "C" int robust_invert_batched(const ashrt_batch_plan* plan, const irls_params* prm, const float* d,
                                     const uint8_t* mask, float* m, const float* w0, float* d_rec,
                                     irls_report* reps, void* ws, size_t wsb, void* stream) {
  if (!plan) return fail(ASHRT_E_INVALID_ARG, "plan is NULL");
  return invert_impl(plan->impl, prm, d, mask, m, w0, d_rec, reps, ws, wsb, stream, true);
}

// ------------------------------------------------------------ autotuner
namespace {
std::mutex g_tune_mu;
std::map<std::string, std::pair<ashrt_tuning, double>> g_tune_cache;

// Optional on-disk cache of tuned tilings: when ASHRT_TUNE_CACHE names a
// file, a result is looked up there (lines "<arch>|<geometry key> tm td
// chunks ms") before timing, and new results are appended.  Keyed by the
// device's architecture name, since tile timings do not carry across GPUs.
static std::string tune_file() {
  const char* p = std::getenv("ASHRT_TUNE_CACHE");
  return (p && *p) ? std::string(p) : std::string();
}

static bool tune_file_lookup(const std::string& fkey, ashrt_tuning* t, double* ms) {
  const std::string path = tune_file();
  if (path.empty()) return false;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    char k[384];
    int tm, td, ch;
    double v;
    if (std::sscanf(line, "%383s %d %d %d %lf", k, &tm, &td, &ch, &v) == 5 && fkey == k) {
      *t = ashrt_tuning{tm, td, ch};
      *ms = v;
      found = true;  // the last entry for a key wins
    }
  }
  std::fclose(f);
  return found;
}

static void tune_file_append(const std::string& fkey, const ashrt_tuning& t, double ms) {
  const std::string path = tune_file();
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %.6f\n", fkey.c_str(), t.tile_model, t.tile_data, t.nchunk, ms);
  std::fclose(f);
}
}  // namespace

extern "C" int ashrt_autotune(const ashrt_desc* desc, int device, int32_t repeats, ashrt_tuning* best,
                              double* best_ms) {
  if (!desc || !best) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  if (repeats < 1) return fail(ASHRT_E_INVALID_ARG, "repeats must be >= 1");
  Resolved z;
  int st = resolve_desc(desc, &z);
  if (st) return st;
  // cost depends on the geometry, the band, R and whether the panels carry
  // phase ramps or bin weights -- not on the velocity values beyond that
  char key[192];
  std::snprintf(key, sizeof key, "%d:%d,%d,%d,%d,%d,%d,%d,%d,%d", device, z.nt, z.nx, z.ntp, z.nxp, z.P, z.R, z.jlo,
                z.jhi, ((desc->tau0_samples || desc->wavelet_amp) ? 1 : 0) + (desc->x_pos ? 2 : 0));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *best = it->second.first;
      if (best_ms) *best_ms = it->second.second;
      return ASHRT_OK;
    }
  }
  DeviceGuard dg(device);
  if (!dg.ok) return fail(ASHRT_E_HIP, "cannot select the device");
  std::string fkey;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(ASHRT_E_HIP, "cannot query the device");
    std::string arch = prop.gcnArchName;
    for (char& ch : arch)
      if (ch == ' ' || ch == '|') ch = '_';
    fkey = arch + "|" + std::string(std::strchr(key, ':') + 1);
    ashrt_tuning ft;
    double fms = 0.0;
    if (tune_file_lookup(fkey, &ft, &fms)) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[key] = {ft, fms};
      *best = ft;
      if (best_ms) *best_ms = fms;
      return ASHRT_OK;
    }
  }
  const size_t nm = (size_t)z.P * z.nx * z.nt, nd = (size_t)z.nx * z.nt;
  float *m = nullptr, *d = nullptr, *m2 = nullptr;
  double *part = nullptr, *scal = nullptr;  // CG partial sums and scalar block (see below)
  size_t part_cap = 0;
  void* ws = nullptr;
  size_t ws_cap = 0;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&] {
    if (s) (void)hipStreamSynchronize(s);
    if (m) (void)hipFree(m);
    if (d) (void)hipFree(d);
    if (m2) (void)hipFree(m2);
    if (part) (void)hipFree(part);
    if (scal) (void)hipFree(scal);
    if (ws) (void)hipFree(ws);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
  };
  if (hipMalloc(&m, nm * 4) != hipSuccess || hipMalloc(&d, nd * 4) != hipSuccess ||
      hipMalloc(&m2, nm * 4) != hipSuccess || hipMalloc(&scal, kNScal * sizeof(double)) != hipSuccess) {
    cleanup();
    return fail(ASHRT_E_OOM, "autotune scratch allocation failed");
  }
  if (hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      hipMemsetAsync(m, 0, nm * 4, s) != hipSuccess || hipMemsetAsync(d, 0, nd * 4, s) != hipSuccess) {
    cleanup();
    return fail(ASHRT_E_HIP, "autotune set-up failed");
  }
  double best_t = 1e300;
  ashrt_tuning bt{0, 0, 0};
  for (int tm : {8, 16, 32})
    for (int td : {2, 4, 8})
      for (int ch : {1, 2, 4, 8}) {
        if (ch > z.P) continue;
        const ashrt_tuning tn{tm, td, ch};
        PlanImpl P;
        if (create_impl(desc, 1, device, P, &tn) != ASHRT_OK) {  // e.g. the tile does not fit in LDS
          destroy_impl(P);
          continue;
        }
        const size_t need = std::max(P.layout(ASHRT_OP_FORWARD, 2).total, P.layout(ASHRT_OP_ADJOINT, 2).total);
        if (need > ws_cap) {
          if (ws) (void)hipFree(ws);
          ws = nullptr;
          ws_cap = 0;
          if (hipMalloc(&ws, need) != hipSuccess) {
            destroy_impl(P);
            cleanup();
            return fail(ASHRT_E_OOM, "autotune workspace allocation failed");
          }
          ws_cap = need;
        }
        // A CG iteration also sums the per-tile partials of |q|^2 and |g|^2:
        // inside the consuming transform for small plans, else by one
        // k_sum_items launch each (sum_*_in_kernel).  Those launches are
        // timed with the pair, on zeroed partials, so that a tiling whose
        // tile count moves the sums out of the transforms pays for them.
        const size_t npart = (size_t)std::max(P.n_xm, P.n_xd);
        if (npart > part_cap) {
          if (part) (void)hipFree(part);
          part = nullptr;
          part_cap = 0;
          if (hipMalloc(&part, npart * sizeof(double)) != hipSuccess ||
              hipMemsetAsync(part, 0, npart * sizeof(double), s) != hipSuccess) {
            destroy_impl(P);
            cleanup();
            return fail(ASHRT_E_OOM, "autotune partial-sum allocation failed");
          }
          part_cap = npart;
        }
        auto sums = [&]() {
          hipError_t e = hipSuccess;
          if (!P.sum_data_in_kernel) e = launch_sum_items(P.d_gd, 1, part, 0, scal, SC_DELTA, s);
          if (e == hipSuccess && !P.sum_model_in_kernel) e = launch_sum_items(P.d_gd, 1, part, 1, scal, SC_GNEW, s);
          return e == hipSuccess;
        };
        bool ok = forward_impl(P, m, d, nullptr, ws, ws_cap, s) == ASHRT_OK &&
                  adjoint_impl(P, d, m2, nullptr, ws, ws_cap, s) == ASHRT_OK && sums();
        std::vector<float> ts;
        for (int r = 0; ok && r < repeats; ++r) {
          ok = hipEventRecord(e0, s) == hipSuccess && forward_impl(P, m, d, nullptr, ws, ws_cap, s) == ASHRT_OK &&
               adjoint_impl(P, d, m2, nullptr, ws, ws_cap, s) == ASHRT_OK && sums() &&
               hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
          float ms = 0.f;
          if (ok) ok = hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
          ts.push_back(ms);
        }
        (void)hipStreamSynchronize(s);
        destroy_impl(P);
        if (!ok) continue;
        std::sort(ts.begin(), ts.end());
        const double med = ts[ts.size() / 2];
        if (med < best_t) {
          best_t = med;
          bt = tn;
        }
      }
  cleanup();
  if (best_t >= 1e300) return fail(ASHRT_E_UNSUPPORTED_SIZE, "no candidate tiling could run");
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {bt, best_t};
    tune_file_append(fkey, bt, best_t);
  }
  *best = bt;
  if (best_ms) *best_ms = best_t;
  return ASHRT_OK;
}

// ------------------------------------------------------------ warm-start support
extern "C" int ashrt_vec_stats(const float* a, const float* b, int64_t n, double alpha, int32_t p, double* out,
                               void* stream) {
  if (!a || !out) return fail(ASHRT_E_INVALID_ARG, "a and out must be non-NULL");
  if (n < 0) return fail(ASHRT_E_INVALID_ARG, "n must be >= 0");
  if (p != 1 && p != 2) return fail(ASHRT_E_INVALID_ARG, "p must be 1 or 2");
  if (!std::isfinite(alpha)) return fail(ASHRT_E_INVALID_ARG, "alpha must be finite");
  HIP_TRY(launch_vec_stats(a, b, n, alpha, p, out, (hipStream_t)stream));
  return ASHRT_OK;
}

extern "C" int ashrt_weight_target(const float* d, const float* d_rec, int64_t n, double eps, float* w,
                                   void* stream) {
  if (!d || !d_rec || !w) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  if (n < 0) return fail(ASHRT_E_INVALID_ARG, "n must be >= 0");
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(ASHRT_E_INVALID_ARG, "eps must be finite and > 0");
  if (n == 0) return ASHRT_OK;
  HIP_TRY(launch_weight_target(d, d_rec, n, (float)eps, w, (hipStream_t)stream));
  return ASHRT_OK;
}

extern "C" int ashrt_vec_scale(const float* x, int64_t n, double s, float* y, void* stream) {
  if (!x || !y) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  if (n < 0) return fail(ASHRT_E_INVALID_ARG, "n must be >= 0");
  if (!std::isfinite(s)) return fail(ASHRT_E_INVALID_ARG, "s must be finite");
  if (n == 0) return ASHRT_OK;
  HIP_TRY(launch_vec_scale(x, n, (float)s, y, (hipStream_t)stream));
  return ASHRT_OK;
}

// ------------------------------------------------------------ survey cubes
extern "C" int ashrt_blend(const float* D, int32_t ns, int32_t nr, int32_t nt, const int32_t* fire, float* b,
                           int32_t nrec, void* stream) {
  if (!D || !fire || !b) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  if (ns < 1 || nr < 1 || nt < 1 || nrec < 1) return fail(ASHRT_E_INVALID_ARG, "sizes must be >= 1");
  HIP_TRY(launch_blend(D, ns, nr, nt, fire, b, nrec, (hipStream_t)stream));
  return ASHRT_OK;
}

extern "C" int ashrt_deblend(const float* b, int32_t ns, int32_t nr, int32_t nt, const int32_t* fire, int32_t nrec,
                             float* out, int32_t receiver_major, void* stream) {
  if (!b || !fire || !out) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  if (ns < 1 || nr < 1 || nt < 1 || nrec < 1) return fail(ASHRT_E_INVALID_ARG, "sizes must be >= 1");
  HIP_TRY(launch_deblend(b, ns, nr, nt, fire, nrec, out, receiver_major ? 1 : 0, (hipStream_t)stream));
  return ASHRT_OK;
}

extern "C" int ashrt_resort(const float* in, int32_t na, int32_t nb, int32_t nt, float* out, void* stream) {
  if (!in || !out) return fail(ASHRT_E_INVALID_ARG, "NULL argument");
  if (in == out) return fail(ASHRT_E_INVALID_ARG, "in and out must not alias");
  if (na < 1 || nb < 1 || nt < 1) return fail(ASHRT_E_INVALID_ARG, "sizes must be >= 1");
  HIP_TRY(launch_resort(in, na, nb, nt, out, (hipStream_t)stream));
  return ASHRT_OK;
}
