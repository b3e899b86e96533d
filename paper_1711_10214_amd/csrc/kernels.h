// Kernel argument blocks and launchers of libashrt (shared by the HIP
// kernel sources and the host runtime).
#pragma once

#include "ashrt_internal.h"

namespace ashrt {

struct XfwdArgs {
  const GatherDev* gd;
  const WorkItem* items;  // (g, panel, tile)
  int nitems;
  int is_model;           // 1: model panels -> X ; 0: data -> H
  const float* src;
  const float* mul;       // optional element-wise factor, same layout as src
  const uint8_t* tmask;   // optional trace mask (data only)
  float2* dst;
  const float2* tw;
  const PanelDev* panels; // live-row counts of the model panels
  // CG step (data input only): before the transform, s -= alpha q with
  // alpha = gamma[par] / delta; delta is the sum of the forward's per-tile
  // partials, reduced here from part_red (every workgroup in the same
  // order) when set, else read from sc[SC_DELTA] (summed by k_sum_items);
  // the gather's first item stores alpha.
  float* s_inout;
  const float* qv;
  const double* part_red;
  double* sc;
  int par;
  int item_base;          // index of items[0] in the plan's full list (partials, first-item checks)
  // Model input with the previous CG iteration's update fused in (cg_upd):
  // beta = gamma_new / gamma[cg_par] (gamma_new reduced from part_red as
  // above when set, else sc[SC_GNEW]),
  // alpha = sc[SC_ALPHA] (both 0 once done); u += alpha pdir,
  // pdir = g + beta pdir (cg_p, updated in place), and the new pdir is the
  // transform's input; the gather's first item stores gamma[cg_par ^ 1].
  int cg_upd;
  int cg_par;
  float* cg_p;
  float* cg_u;
  const float* cg_g;
};

struct XinvArgs {
  const GatherDev* gd;
  const WorkItem* items;  // (g, panel, tile)
  int nitems;
  int is_model;           // 1: G_p (X region) -> model ; 0: H -> data
  const float2* src;
  float* out;             // result (after the epilogue)
  const float* sub;       // data: out = sub - y (residual) when set
  const float* wmul;      // out *= wmul (element-wise) when set
  int wmul_sq;            // with wmul: out = y wmul^2, and part sums (y wmul)^2
  float* raw_out;         // data: y before the epilogue when set
  const uint8_t* tmask;   // data: out *= mask
  const float2* tw;
  const PanelDev* panels; // live-row counts of the model panels
  double* part;           // per work item: sum of out^2 (or of (y wmul)^2, see wmul_sq)
  int item_base;          // index of items[0] in the plan's full list
};

struct RowsArgs {
  const GatherDev* gd;
  const WorkItem* items;  // (g, row, chunk)
  int nitems;
  const PanelDev* panels;
  const float2* tw;
  const float* wav;
  float2* X;              // model-side x-spectra / adjoint output G
  float2* H;              // data-side x-spectrum
  float2* Dp;             // forward partials
  int R;                  // interpolation half-width (generic kernels)
};

enum RedOp { RED_SUMSQ = 0, RED_ABSMAX_LIVE = 1, RED_ABSMAX = 2, RED_MISFIT = 3, RED_ABSSUM = 4 };

struct RedArgs {
  const GatherDev* gd;
  const VecItem* items;
  int nitems;
  int op;
  int is_model;
  const float* x;
  const uint8_t* tmask;   // data ops: skip dead traces
  const double* sc;       // per-gather scalars (RED_MISFIT reads eps_r)
  int p;                  // misfit exponent
  double* part;           // [nitems][2]
};

struct FinArgs {
  const GatherDev* gd;
  int ngather;
  int is_model;
  int is_max;
  const double* part;
  double* sc;
  int dst0, dst1;
  RepDev* rep;       // optional: also store into the report at outer index `outer`
  int outer;
};

enum EwOp {
  EW_AXPY = 0,        // y += sign * sc[g][coef] * x
  EW_XPBY = 1,        // y = x + sc[g][coef] * y
  EW_MUL = 2,         // y = x * z
  EW_COPY = 3,        // y = x
  EW_FILL = 4,        // y = value
  EW_WR_INIT = 5,     // y = live ? (x ? x : 1) : 0           (x = w0 or null)
  EW_WR_UPDATE = 6,   // y = live ? (eps > 0 ? max(|x|, eps)^-1/2 : 1) : 0   (p = 1)
  EW_WM_UPDATE = 7,   // y = max(|x|, eps_m)^1/2 (or 1), z_out = x / y        (q = 1)
  EW_WR_MASK = 8,     // y = live ? 1 : 0                     (p = 2)
  EW_SCALE_RSQRT = 9, // y = x / sqrt(sc[g][coef])            (power-method normalisation)
  EW_FISTA = 10       // v = y + sc[coef] x; m' = soft(v, sc[coef + 1]); y = m' + value (m' - m); m = m'
                      //   (m is z_out, in and out)
};

struct EwArgs {
  const GatherDev* gd;
  const VecItem* items;
  int nitems;
  int op;
  float* y;
  const float* x;
  const float* z;
  float* z_out;
  const double* sc;
  int coef;
  float sign;
  float value;
  const uint8_t* tmask;
};

enum ScalStep {
  ST_EPS_M = 3,        // eps_m = b_m * mmax / 100
  ST_EPS_R = 4,        // eps_r = max(b_r * MAD / 0.6745, floor * dmax) (or frozen)
  ST_REPORT_INNER = 5, // report.inner[outer] = ninner
  ST_FISTA = 6         // Lf = 2 safety sqrt(pow_ss); mu; step = 2 / Lf; thr = mu / Lf
};

struct ScalArgs {
  int ngather;
  int step;
  double* sc;
  RepDev* rep;
  int outer;
  double b_r, b_m, floor_rel;
  int freeze;
  double safety, mu_abs, mu_rel;  // ST_FISTA
};

struct SelArgs {
  const GatherDev* gd;
  const VecItem* items;
  int nitems;
  int ngather;
  const float* x;
  const uint8_t* tmask;
  const double* sc;        // SC_MED for stage 1
  SelState* st;
  unsigned* hist;          // [ngather][2][kSelBins]
  int stage;               // 0: r ; 1: |r - med|
  int shift, width;        // digit = (key >> shift) & ((1 << width) - 1)
};

// CG initialisation and update over model-vector items; gamma_new = |g|^2 of
// the latest adjoint is reduced from its per-tile partials part_gamma when
// set (every workgroup in the same order), else read from sc[SC_GNEW].
//   init:   pdir = g ; gamma[0] = gamma_new, done = 0, ninner = 0
//   update: beta = gamma_new / gamma[par] ; u += alpha pdir ; pdir = g + beta pdir ;
//           gamma[par ^ 1] = gamma_new
struct CgArgs {
  const GatherDev* gd;
  const VecItem* items;
  int nitems;
  int init;
  int par;
  float* u;
  float* pdir;
  const float* g;
  const double* part_gamma;
  double* sc;
};

// operator kernels; `key` is the FFT length class (see rows_size_is_tpl /
// x_size_is_tpl; 0 = generic)
bool rows_size_is_tpl(int n, int R);

// Time-domain ASHRT pair (one gather, gd[0]): forward m -> d, adjoint d -> m.
struct TdArgs {
  const GatherDev* gd;
  const PanelDev* panels;
  float* m;                // [P][nx][nt]
  float* d;                // [nx][nt]
  const uint8_t* tmask;    // [nx] or null
  long long n_out;         // output samples of the launch
};
hipError_t launch_td(const TdArgs& a, bool forward, hipStream_t s);

// vec_kernels.hip
hipError_t launch_vec_stats(const float* a, const float* b, long long n, double alpha, int p, double* out,
                            hipStream_t s);
hipError_t launch_weight_target(const float* d, const float* drec, long long n, float eps, float* w, hipStream_t s);
hipError_t launch_vec_scale(const float* x, long long n, float sc, float* y, hipStream_t s);

// Blending / pseudo-deblending / re-sort of survey cubes (survey_kernels.hip).
hipError_t launch_blend(const float* D, int ns, int nr, int nt, const int* fire, float* b, int nrec, hipStream_t s);
hipError_t launch_deblend(const float* b, int ns, int nr, int nt, const int* fire, int nrec, float* out, int rmaj,
                          hipStream_t s);
hipError_t launch_resort(const float* in, int na, int nb, int nt, float* out, hipStream_t s);
bool x_size_is_tpl(int n);
hipError_t launch_xfft_fwd(int key, const XfwdArgs& a, size_t lds, hipStream_t s);
hipError_t launch_xfft_inv(int key, const XinvArgs& a, size_t lds, hipStream_t s);
hipError_t launch_rows_fwd(int key, const RowsArgs& a, size_t lds, hipStream_t s);
hipError_t launch_rows_fwd_fin(int key, const RowsArgs& a, size_t lds, hipStream_t s);
hipError_t launch_rows_adj(int key, const RowsArgs& a, size_t lds, hipStream_t s);
hipError_t op_kernels_init(size_t max_lds);

// solver kernels
hipError_t launch_reduce_part(const RedArgs& a, hipStream_t s);
hipError_t launch_reduce_fin(const FinArgs& a, hipStream_t s);
hipError_t launch_elementwise(const EwArgs& a, hipStream_t s);
hipError_t launch_scalar(const ScalArgs& a, hipStream_t s);
hipError_t launch_zero_words(void* p, long long n, hipStream_t s);
hipError_t launch_count_live(const GatherDev* gd, int ngather, const uint8_t* tmask, double* sc,
                             hipStream_t s);
hipError_t launch_select_median(SelArgs a, double* sc, int dst, hipStream_t s);
hipError_t launch_cg(const CgArgs& a, hipStream_t s);
// sc[g][dst] = sum of the per-tile partials of gather g's model (xm) or data
// (xd) x-transform items, in a fixed order (one workgroup per gather).
hipError_t launch_sum_items(const GatherDev* gd, int ngather, const double* part, int is_model, double* sc,
                            int dst, hipStream_t s);

}  // namespace ashrt
