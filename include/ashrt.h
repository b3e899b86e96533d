/*
 * ashrt.h -- C ABI of libashrt: the Stolt-based apex-shifted hyperbolic Radon
 * transform (ASHRT) and its asymptote-shifted extension (AASHRT), and the
 * robust IRLS-CG inversion that separates blended sources in common receiver
 * gathers, on AMD Instinct MI355X (gfx950).
 *
 * Method (Ibrahim, "Separating simultaneous seismic sources using robust
 * inversion of Radon and migration operators", thesis, 2015):
 *   - Chapter 5, "Stolt-based Radon Transform", equations ch5_Stolt_adj,
 *     ch5_Stolt_forward, ch5_adj_operator, ch5_forward_operator: the operator
 *     pair L = S F^-1 M F (forward, demigration) and L' = F^-1 M' F S'
 *     (adjoint, migration), one Stolt map per scanned velocity, summed over
 *     velocities in the forward and sprayed in the adjoint.
 *   - Chapter 6, "Stolt-based AASHRT", equations ch6_adj_operator and
 *     ch6_forward_operator: the asymptote shift tau0 as a frequency-domain
 *     phase ramp T and the trace-sampling operator S.
 *   - Chapter 4, "Robust Radon transform": the l_p-l_q cost (equation
 *     ch4_cost_fn), IRLS weights clipped at eps_r = b_r MAD / 0.6745
 *     (equation ch4_epcilon_r) and eps_m = b_m max|m| / 100, the change of
 *     variables u = W_m m (equation equ:11), inner CG and outer reweighting.
 *
 * Discrete operator (all conventions are fixed here, and the library
 * computes exactly this up to FP32 rounding):
 *   ntp, nxp   FFT lengths (smallest 2^a or 3*2^a >= 2n by default).
 *   F          zero-pad [nx][nt] to [nxp][ntp]; unnormalised FFT along t
 *              (real to half spectrum) and along x.
 *   F^-1       inverse along x first, then the inverse real FFT along t,
 *              each carrying 1/N; truncate to [nx][nt].
 *   Bins       data frequency j, model frequency k (both 1..ntp/2-1: DC and
 *              Nyquist never take part), wavenumber l with signed index l'.
 *   a_{p,l}    = v_p |l'| ntp dt / (nxp dx)          (v |kx| in bins)
 *   u          = sqrt(j^2 - a^2) for j >= a (signal cone), else no output.
 *   forward    D[l,j] = W_j sum_p s_p e^{-2 pi i j n0_p / ntp}
 *                        sum_{t=-R+1..R} h(u - k) M_p[l,k],  k = floor(u)+t,
 *              for j in the band [jlo, jhi]; h(x) = sinc(x)(1/2 + 1/2 cos(pi x/R))
 *              on |x| < R (Hann-windowed sinc).
 *   adjoint    the exact transpose of the above (conjugate ramp); it
 *              reproduces the change-of-variables factor w_tau / w.
 *   band       jlo = max(1, ceil((fmin*ntp)*dt)), jhi = min(ntp/2-1,
 *              floor((fmax*ntp)*dt)); fmax <= 0 means ntp/2-1.
 *
 * Memory: every array argument is a device pointer owned by the caller
 * (e.g. a PyTorch tensor's storage), contiguous, 16-byte aligned, on the
 * plan's device.  Layouts are row-major with time contiguous:
 *   data  d[nx][nt]          float32
 *   model m[P][nx][nt]       float32  (panel p, apex x_a on the receiver grid, tau)
 *   mask  trace_mask[nx]     uint8    (1 = live trace, 0 = missing) or NULL (all live)
 * The library never allocates the large buffers: the caller passes a
 * workspace `ws` of at least ashrt_workspace_bytes() bytes (256-byte
 * aligned).  Plans own only small device tables (twiddles, panel constants,
 * work lists).  `stream` is a hipStream_t (NULL = the null stream); every
 * call is stream-ordered and asynchronous unless stated otherwise.  Input and
 * output arrays must not alias.
 *
 * Errors: every function returns an int status (0 = ASHRT_OK, negative on
 * error) and never aborts or throws; ashrt_last_error() gives a message for
 * the calling thread's last failure.  A plan is not thread-safe: calls that
 * share a plan must be serialised by the caller.
 */
#ifndef ASHRT_H
#define ASHRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASHRT_ABI_VERSION 5

enum ashrt_status {
  ASHRT_OK = 0,
  ASHRT_E_INVALID_ARG = -1,      /* a NULL pointer, non-positive size or out-of-range parameter  */
  ASHRT_E_UNSUPPORTED_SIZE = -2, /* an FFT length or band the kernels do not handle              */
  ASHRT_E_HIP = -3,              /* a HIP runtime call failed (message in ashrt_last_error)      */
  ASHRT_E_NONFINITE = -4,        /* the solve produced a NaN or Inf                              */
  ASHRT_E_OOM = -5,              /* allocating a plan's small tables failed                      */
  ASHRT_E_NOT_IMPLEMENTED = -6,
  ASHRT_E_WORKSPACE = -7         /* ws is NULL, misaligned or smaller than required              */
};

enum ashrt_op { ASHRT_OP_FORWARD = 0, ASHRT_OP_ADJOINT = 1, ASHRT_OP_INVERT = 2, ASHRT_OP_FISTA = 3 };

/* Operator description (host memory; copied at plan creation). */
typedef struct ashrt_desc {
  int32_t nt, nx;              /* samples per trace (>= 2), traces (>= 2)                          */
  int32_t ntp, nxp;            /* FFT lengths; 0 = auto. Supported: 2^a or 3*2^a, ntp in [8, 4096]
                                  with ntp >= nt, nxp in [4, 4096] with nxp >= nx                    */
  double dt, dx;               /* sample interval (s) and trace spacing (m), > 0                    */
  int32_t npanel;              /* P >= 1 model panels                                                */
  const double *vel;           /* [P] panel velocity (m/s), >= 0; v = 0 makes that panel a band-pass */
  const int32_t *tau0_samples; /* [P] asymptote shift n0 >= 0 (tau0 = n0*dt), or NULL (all 0)       */
  const double *panel_scale;   /* [P] real panel scale s_p, or NULL (all 1)                          */
  double fmin_hz, fmax_hz;     /* mapped band; fmax_hz <= 0 means up to ntp/2-1                      */
  int32_t half_width;          /* R, interpolation half-width in bins, 1..8 (0 = default 4)          */
  const double *wavelet_amp;   /* [ntp/2+1] real per-bin weight W_j (zero-phase wavelet), or NULL    */
  const double *x_pos;         /* [nx] data trace positions (m, finite), or NULL = regular i*dx.  With
                                  positions, the data-side x transforms are non-uniform DFTs at them
                                  (no Nyquist wavenumber); the model (apex) grid stays i*dx.  Thesis
                                  Chapters 5 and 7 name non-uniform transforms for irregular traces. */
} ashrt_desc;

/* Inversion settings (thesis Chapter 4). */
typedef struct irls_params {
  int32_t p, q;                /* misfit and model norms, each 1 or 2                                */
  int32_t n_outer, n_inner;    /* outer (reweighting) iterations 1..64, CG iterations >= 1           */
  double b_r;                  /* residual clip tuning constant (1.345)                              */
  double b_m;                  /* model clip tuning constant (1.0), used when q = 1                  */
  double tol;                  /* stop when the relative change of sum|r|^p < tol; 0 = fixed counts */
  double eps_floor_rel;        /* eps_r >= eps_floor_rel * max|d_live| (1e-6)                        */
  int32_t freeze_eps;          /* nonzero: eps_r computed once (after outer 1) and kept             */
  int32_t cg_graph;            /* nonzero (default): CG iterations replayed two at a time from a
                                  hipGraph captured on first use and cached in the plan per
                                  (workspace, m, mask, q); 0 = launched one by one.  Results are
                                  identical either way.  Ignored while kernel timing is enabled. */
} irls_params;

/* Per-solve report (host memory).  Entry k describes outer iteration k+1,
 * after its CG run: misfit = sum_live |r|^p, r = S(d - L m); eps_r = the
 * residual clip computed from that r (0 when p = 2); huber = the Huber
 * objective of r at eps_r (p = 1) or sum r^2 / 2 (p = 2); inner = CG
 * iterations run (fewer than n_inner only on an exact breakdown). */
typedef struct irls_report {
  int32_t status, outer_done;
  int32_t inner[64];
  double misfit[64], huber[64], eps_r[64], eps_m[64];
} irls_report;

/* Plan facts (host memory). */
typedef struct ashrt_plan_info {
  int32_t nt, nx, ntp, nxp, npanel, half_width;
  int32_t jlo, jhi;            /* mapped data band (inclusive)                                       */
  int32_t kmax;                /* highest model frequency bin the map touches                        */
  int32_t nchunk;              /* panel chunks of the row passes                                     */
  int32_t tile_model, tile_data;  /* x-FFT time columns per workgroup (model panels, data)           */
  size_t ws_forward, ws_adjoint, ws_invert_q2, ws_invert_q1;   /* workspace bytes per operation    */
} ashrt_plan_info;

/* Tile shapes of the pipeline; 0 selects the built-in rule.
 *   tile_model: time columns per model-panel x-FFT workgroup (even, >= 2)
 *   tile_data:  time columns per data x-FFT workgroup (even, >= 2)
 *   nchunk:     panel chunks of the row passes (1..npanel)
 * Any setting gives the same results up to FP32 rounding order; it only
 * changes the work decomposition.  Tiles whose LDS exceeds the
 * per-workgroup limit make plan creation fail with ASHRT_E_UNSUPPORTED_SIZE. */
typedef struct ashrt_tuning {
  int32_t tile_model, tile_data, nchunk;
} ashrt_tuning;

typedef struct ashrt_plan ashrt_plan;

/* Fill defaults: desc -> all zero except half_width 4; params -> p=1, q=2,
 * 10 x 20, b_r 1.345, b_m 1, tol 0, floor 1e-6, cg_graph 1. */
void ashrt_desc_default(ashrt_desc *desc);
void irls_params_default(irls_params *params);

/* Host-only checks, no GPU needed.  Return ASHRT_OK or the reason. */
int ashrt_desc_validate(const ashrt_desc *desc);
int irls_params_validate(const irls_params *params);

/* Create a plan on HIP device `device`; uploads twiddle tables, panel
 * constants and work lists (a few hundred KB).  *out is NULL on failure. */
int ashrt_plan_create(const ashrt_desc *desc, int device, ashrt_plan **out);
/* As ashrt_plan_create with explicit tile shapes (tuning may be NULL). */
int ashrt_plan_create_tuned(const ashrt_desc *desc, const ashrt_tuning *tuning, int device, ashrt_plan **plan);

/* Autotuner: times one forward + adjoint pair (median of `repeats`, >= 1)
 * for every candidate tiling -- model tiles {8, 16, 32}, data tiles
 * {2, 4, 8}, chunks {1, 2, 4, 8} within 1..npanel -- on zero-filled scratch
 * inputs of the descriptor's geometry, and returns the fastest in *best
 * (and its time in *best_ms, may be NULL).  Allocates and frees its own
 * scratch device memory and synchronises `device`; results are cached per
 * geometry for the life of the process.  The time includes the per-gather
 * sums of the CG partials that a tiling with many model tiles moves into
 * their own launches.  When the environment variable ASHRT_TUNE_CACHE names
 * a file, results are also looked up in and appended to it, keyed by the
 * device's architecture name (gcnArchName) and the geometry; an unreadable
 * or unwritable file is ignored. */
int ashrt_autotune(const ashrt_desc *desc, int device, int32_t repeats, ashrt_tuning *best, double *best_ms);

void ashrt_plan_destroy(ashrt_plan *plan);
int ashrt_plan_get_info(const ashrt_plan *plan, ashrt_plan_info *info);

/* Workspace needed by `op` (ASHRT_OP_*); for ASHRT_OP_INVERT pass the params
 * (q = 1 needs two more model-sized vectors), else params may be NULL
 * (ASHRT_OP_FISTA: the workspace of fista_invert). */
int ashrt_workspace_bytes(const ashrt_plan *plan, int op, const irls_params *params, size_t *bytes);

/* d = S L m  (Chapter 5 equation ch5_forward_operator; with tau0 and the mask,
 * Chapter 6 equation ch6_forward_operator).  m: [P][nx][nt], d: [nx][nt]. */
int ashrt_forward(const ashrt_plan *plan, const float *m, float *d, const uint8_t *trace_mask,
                  void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operator as ashrt_forward, with the same kernels and results, but its
 * workspace is a library-owned static device array of 96 MiB (one per GPU,
 * held until the process ends; its address is resolved when a plan is
 * created on that GPU).  Calls no hipMalloc/hipFree.  Returns
 * ASHRT_E_WORKSPACE when the plan's forward workspace
 * (ashrt_workspace_bytes(plan, ASHRT_OP_FORWARD, ...)) exceeds 96 MiB.
 * Nothing in the array needs to start at zero.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (on different
 * streams, or from different threads) race and must be serialised by the
 * caller. */
int ashrt_forward_noalloc(const ashrt_plan *plan, const float *m, float *d, const uint8_t *trace_mask,
                          void *stream);

/* Learned warm start support (an initial model m0 and initial residual
 * weights w0 for robust_invert, predicted by the U-Net of unet.h).  All
 * pointers are device pointers; calls are stream-ordered; nothing is
 * allocated.
 *
 * ashrt_vec_stats: out[0] = sum_i |a_i - alpha b_i|^p (p = 1 or 2),
 * out[1] = sum_i a_i b_i, out[2] = sum_i b_i^2, over n elements, summed in
 * FP64 in a fixed order (deterministic); b may be NULL (a zero vector).
 * out: 3 doubles.  Serves the gather's RMS scale (alpha = 0, p = 2), the
 * least-squares step length of a predicted model along L m0 (out[1] /
 * out[2] with b = L m0) and the l_p misfit that decides whether the
 * prediction replaces the zero start (Chapter 4's misfit, equation
 * ch4_cost_fn with mu = 0).  One workgroup does the sums (that is what
 * makes the order fixed), which suits a gather's data; over a buffer of
 * model labels (~10^9 elements, once per training run) it is slow. */
int ashrt_vec_stats(const float *a, const float *b, int64_t n, double alpha, int32_t p, double *out, void *stream);

/* w_i = sqrt(eps / max(|d_i - d_rec_i|, eps)) over n elements, eps > 0: the
 * final l1 IRLS residual weight of a solve (Chapter 4, W_r with p = 1),
 * scaled into (0, 1] -- the training label of the predicted weights. */
int ashrt_weight_target(const float *d, const float *d_rec, int64_t n, double eps, float *w, void *stream);

/* y = s x over n elements (y may be x). */
int ashrt_vec_scale(const float *x, int64_t n, double s, float *y, void *stream);

/* m = L' S d  (Chapter 5 equation ch5_adj_operator; Chapter 6 equation
 * ch6_adj_operator), the exact transpose of ashrt_forward. */
int ashrt_adjoint(const ashrt_plan *plan, const float *d, float *m, const uint8_t *trace_mask,
                  void *ws, size_t ws_bytes, void *stream);

/* Robust inversion (Chapter 4 "Robust Radon transform"): minimise
 * ||d - S L m||_p^p (+ the q-norm of m through W_m) by IRLS with CGLS inner
 * solves on A = W_r S L W_m^-1.  Outer iteration 1 is unweighted unless w0
 * is given (then W_r = w0 on live samples); each CG run starts from the
 * current model.
 *   d     [nx][nt] observed (blended or decimated) gather
 *   m     [P][nx][nt] in: starting model (zeros for a cold start); out: model
 *   w0    [nx][nt] initial residual weights or NULL
 *   d_rec [nx][nt] out: L m without the mask (the separated gather) or NULL
 *   rep   host report or NULL.  When rep != NULL or tol > 0 the call waits on
 *         the stream (once per outer iteration with tol > 0, once at the end
 *         for the report); otherwise it is asynchronous.
 * When the call waits (rep != NULL or tol > 0) it returns ASHRT_E_NONFINITE
 * if a misfit came out NaN or Inf; asynchronous calls report that only
 * through a later report. */
int robust_invert(const ashrt_plan *plan, const irls_params *params, const float *d,
                  const uint8_t *trace_mask, float *m, const float *w0, float *d_rec,
                  irls_report *rep, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- batched
 * Many gathers of uneven size in one plan: every pipeline stage is one
 * launch over a flattened work list covering all gathers.  Arrays are packed:
 * gather g's data starts at float offset data_off[g] (= sum of nx*nt before
 * it), its model at model_off[g] (= sum of P*nx*nt), its mask at
 * mask_off[g] (= sum of nx).  Reports are an array of ngather entries. */
typedef struct ashrt_batch_plan ashrt_batch_plan;

int ashrt_batch_plan_create(const ashrt_desc *descs, int32_t ngather, int device,
                            ashrt_batch_plan **out);
/* As ashrt_batch_plan_create with one tiling for every gather (NULL = rule). */
int ashrt_batch_plan_create_tuned(const ashrt_desc *descs, int32_t ngather, const ashrt_tuning *tuning, int device,
                                  ashrt_batch_plan **plan);
void ashrt_batch_plan_destroy(ashrt_batch_plan *plan);
/* Offsets (host arrays of ngather entries, may be NULL) and totals. */
int ashrt_batch_layout(const ashrt_batch_plan *plan, int64_t *data_off, int64_t *model_off,
                       int64_t *mask_off, int64_t *data_total, int64_t *model_total,
                       int64_t *mask_total);
int ashrt_batch_workspace_bytes(const ashrt_batch_plan *plan, int op, const irls_params *params,
                                size_t *bytes);
/* l2-l1 sparse inversion by FISTA (thesis Chapter 6, section "Sparse
 * inversion", equation cost_fn with p = 2, q = 1): minimise
 * J(m) = ||d - S L m||_2^2 + mu ||m||_1.  The step uses Lf = 2 lambda
 * lip_safety, lambda the largest eigenvalue of L' S L estimated by n_power
 * power-method iterations from the all-ones model; mu = the given value if
 * mu > 0, else mu_rel * max|2 L' S d| (the smallest mu with m = 0 optimal,
 * scaled).  Iteration (Beck and Teboulle):
 *   m_k = soft(y_k + (2 / Lf) L' S (d - L y_k), mu / Lf),
 *   t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
 *   y_{k+1} = m_k + (t_k - 1) / t_{k+1} (m_k - m_{k-1}),   y_1 = m_0, t_1 = 1.
 * m: in, the start m_0; out, the model.  d_rec (optional) = L m (unmasked).
 * Stream-ordered; synchronises once at the end only when rep is non-NULL.
 * Workspace: ashrt_workspace_bytes(plan, ASHRT_OP_FISTA, NULL, ...). */
typedef struct fista_params {
  int32_t n_iter, n_power;   /* FISTA and power-method iterations (>= 1, >= 1)        */
  double mu;                 /* > 0: the trade-off parameter itself                    */
  double mu_rel;             /* else mu = mu_rel * max|2 L' S d| (0 < mu_rel)          */
  double lip_safety;         /* >= 1 (1.05): Lf = 2 * lambda * lip_safety              */
} fista_params;

typedef struct fista_report {
  int32_t status, iters;
  double lipschitz, mu;      /* Lf and mu used                                         */
  double misfit, l1, objective;  /* ||S(d - L m)||^2, ||m||_1, misfit + mu l1          */
} fista_report;

void fista_params_default(fista_params *params);
int fista_invert(const ashrt_plan *plan, const fista_params *params, const float *d, const uint8_t *trace_mask,
                 float *m, float *d_rec, fista_report *rep, void *ws, size_t ws_bytes, void *stream);

/* Survey cubes (thesis Chapter 2, equations ch2_blending and
 * pseudodeblending_equ).  All arrays are device memory; fire holds the
 * firing time of each source in samples (>= 0).
 *   ashrt_blend:   b[r][tau] = sum_s D[s][r][tau - fire[s]] over 0 <= tau -
 *                  fire[s] < nt; D: [ns][nr][nt], b: [nr][nrec].
 *   ashrt_deblend: the adjoint, D~[s][r][t] = b[r][fire[s] + t] (0 outside
 *                  the record), written [ns][nr][nt], or [nr][ns][nt] (the
 *                  batch of common receiver gathers) when receiver_major.
 *   ashrt_resort:  out[b][a][t] = in[a][b][t] (in [na][nb][nt]); in and out
 *                  must not alias. */
int ashrt_blend(const float *D, int32_t ns, int32_t nr, int32_t nt, const int32_t *fire, float *b, int32_t nrec,
                void *stream);
int ashrt_deblend(const float *b, int32_t ns, int32_t nr, int32_t nt, const int32_t *fire, int32_t nrec, float *out,
                  int32_t receiver_major, void *stream);
int ashrt_resort(const float *in, int32_t na, int32_t nb, int32_t nt, float *out, void *stream);

/* Time-domain (classical) ASHRT / AASHRT pair on the plan's single gather
 * (thesis Chapter 3, the hyperbolic Radon-operator table; Chapter 6,
 * equations ch6_AASHRT_forward and ch6_AASHRT_adjoint): a model sample at
 * apex time tau, apex trace xa and panel p lies on
 * t = tau0_p + sqrt(tau^2 + (x - xa)^2 dx^2 / v_p^2), read (adjoint) or
 * spread (forward, the exact transpose) with linear interpolation in time;
 * the apex grid is the receiver grid; samples outside the record dropped.
 * Cost O(P nx^2 nt): the operator the Stolt pair is compared against.  No
 * padding, band or wavelet; panel_scale is not applied.  Same layouts and
 * mask semantics as ashrt_forward / ashrt_adjoint; no workspace. */
int ashrt_td_forward(const ashrt_plan *plan, const float *m, float *d, const uint8_t *trace_mask, void *stream);
int ashrt_td_adjoint(const ashrt_plan *plan, const float *d, float *m, const uint8_t *trace_mask, void *stream);

int ashrt_forward_batched(const ashrt_batch_plan *plan, const float *m_packed, float *d_packed,
                          const uint8_t *mask_packed, void *ws, size_t ws_bytes, void *stream);
int ashrt_adjoint_batched(const ashrt_batch_plan *plan, const float *d_packed, float *m_packed,
                          const uint8_t *mask_packed, void *ws, size_t ws_bytes, void *stream);
int robust_invert_batched(const ashrt_batch_plan *plan, const irls_params *params,
                          const float *d_packed, const uint8_t *mask_packed, float *m_packed,
                          const float *w0_packed, float *drec_packed, irls_report *reps,
                          void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- profiling
 * Optional HIP-event timing of individual kernel families, for measurement
 * tools (not for production paths).  ashrt_profile_enable(mask) makes every
 * later launch of a family whose bit (1u << ASHRT_K_*) is set record a
 * start/end event pair on the launch stream (0 disables; pairs already
 * recorded are kept).  ashrt_profile_read() waits for the recorded events of
 * one family and returns the summed kernel time and launch count, optionally
 * clearing them.  Process-wide; not thread-safe with concurrent solves. */
enum ashrt_kernel_id {
  ASHRT_K_XFFT_MODEL = 0,   /* x-axis real FFT of model panels (forward input)          */
  ASHRT_K_XFFT_DATA = 1,    /* x-axis real FFT of the data (adjoint input)              */
  ASHRT_K_ROWS_FWD = 2,     /* time FFT + Stolt map + panel sum per wavenumber row     */
  ASHRT_K_ROWS_FIN = 3,     /* chunk sum + inverse time FFT per row (forward)          */
  ASHRT_K_XINV_DATA = 4,    /* x-axis inverse real FFT to the data (+ epilogue)        */
  ASHRT_K_ROWS_ADJ = 5,     /* time FFT + transposed Stolt map + inverse FFT per panel */
  ASHRT_K_XINV_MODEL = 6,   /* x-axis inverse real FFT to the model panels             */
  ASHRT_K_VECTOR = 7,       /* CG vector updates and weights                            */
  ASHRT_K_REDUCE = 8,       /* FP64 reductions                                          */
  ASHRT_K_SELECT = 9,       /* radix-select medians                                     */
  ASHRT_K_COUNT = 10
};
int ashrt_profile_enable(uint32_t kernel_mask);
int ashrt_profile_read(int kernel_id, double *total_ms, int64_t *launches, int reset);
const char *ashrt_kernel_name(int kernel_id);

/* Messages. */
const char *ashrt_status_string(int status);
const char *ashrt_last_error(void);
int ashrt_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ASHRT_H */
