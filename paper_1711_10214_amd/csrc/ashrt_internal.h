// Internal types shared by the host runtime and the HIP kernels of libashrt.
//
// Every pipeline stage is one launch over a flattened work list, so the same
// kernels serve one gather and a batch of gathers of uneven size: a work item
// names its gather and the tile / row / chunk it covers, and the gather's
// geometry and buffer offsets come from a small device table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ashrt {

constexpr int kThreads = 256;          // threads per workgroup (all kernels but the row passes)
constexpr int kRowThreads = 256;       // threads per workgroup of the forward/adjoint row passes
// Compile-time row lengths of 3072 and 4096 need 60-75 KB of LDS per
// workgroup (two per CU): they run 512 threads (8 waves) so that each SIMD
// still holds four waves; shorter lengths run kRowThreads.
constexpr int row_threads(int n) { return n >= 3072 ? 512 : kRowThreads; }
// Compile-time row kernels fit four waves per SIMD in LDS (four 256-thread or
// two 512-thread workgroups per CU); they are held to the 128 VGPRs that
// allows.  Generic lengths keep their registers.
constexpr int row_waves_per_eu(int n) { return n > 0 ? 4 : 1; }
constexpr int kMaxHalfWidth = 8;       // interpolation half-width R supported
constexpr int kMapGuardSlots = 6;      // zero float2 slots in front of the forward map's spectrum (taps k >= -3)
constexpr int kRowMaxN = 4096;         // longest time FFT (ntp) the row kernels take
constexpr int kXLoadBatch = 4;        // x kernels: tile-loop iterations whose global loads are issued together
constexpr int kXfftTilePoints = 4096;  // complex points of a model x-FFT tile (T = 2 * this / nxp columns)
constexpr int kXfftBatch = 2048;       // complex points per compile-time x-FFT call (register bound)
constexpr int kXfftGenericBatch = 4096;  // complex points per generic x-FFT call (nxp <= 4096)
constexpr int kMaxSlots = (kRowMaxN / 2 + kThreads - 1) / kThreads;  // per-thread bins
constexpr long long kVecChunk = 8192;  // elements per vector-kernel work item
constexpr long long kDataVecChunk = 2048;  // the same for data vectors (a gather's data is P times smaller)
constexpr int kSelBins = 2048;         // radix-select histogram bins (11 bits)

// One gather's geometry and its offsets into packed buffers.
struct GatherDev {
  int nt, nx, ntp, nxp;
  int nrows;        // nxp / 2: wavenumber rows (row 0 packs kx = 0 and kx = Nyquist)
  int jlo, jhi;     // mapped data band, inclusive
  int kmax;         // highest model bin the map reads or writes: min(ntp/2-1, jhi+R)
  int npanel;
  int panel_off;    // first panel in the panel table
  int tw_t_off;     // float2 offset of the plain ntp twiddles exp(-2 pi i m / ntp) in the pool
  int tw_x_off;     // float2 offset of the plain nxp twiddles
  int twp_t_off;    // float2 offset of the ntp pass table (compile-time FFT lengths)
  int twp_x_off;    // float2 offset of the nxp pass table
  int wav_off;      // float offset of the W_j table, -1 = none
  int tileT;        // time columns per x-FFT tile of a model panel (even)
  int ntiles;       // ceil(nt / tileT)
  int tileTd;       // time columns per x-FFT tile of the data (even, smaller: more workgroups)
  int ntilesd;      // ceil(nt / tileTd)
  int nchunk;       // panel chunks of the forward row pass
  int mit_lo, mit_hi;   // model-vector work items of this gather
  int dit_lo, dit_hi;   // data-vector work items of this gather
  int xm_lo, xm_hi;     // model x-FFT tile items of this gather (partial sums)
  int xd_lo, xd_hi;     // data x-FFT tile items of this gather
  int nudft_off;        // float2 offset of the irregular-trace table exp(-2 pi i r x_pos / (nxp dx)),
                        // [nrows][nx], in the twiddle pool; -1 = regular traces
  long long d_off;      // float offset of the gather in packed data arrays
  long long m_off;      // float offset in packed model arrays
  long long mask_off;   // byte offset in packed trace masks
  long long X_off;      // float2 offset of the model-side x-spectra [P][nrows][nt]
  long long H_off;      // float2 offset of the data-side x-spectrum [nrows][nt]
  long long Dp_off;     // float2 offset of forward partials [nchunk][nrows][2][nband]
};

// One model panel: velocity as the squared bin scale, asymptote shift, scale.
struct PanelDev {
  double c2;     // (v * ntp * dt / (nxp * dx))^2, so a^2 = c2 * l'^2
  float scale;   // s_p
  int n0;        // asymptote shift in samples
  int rlive;     // rows r < rlive can reach the band (c2 r^2 <= jhi^2); rows at and above it have
                 // no in-cone bin, so their x-spectra are neither written nor read
  int pad_;
};

// Work item: gather g plus up to three stage-specific indices.
struct WorkItem {
  int g, a, b, c;
};

// Vector work item for model/data-sized element-wise kernels and reductions.
struct VecItem {
  int g;
  int pad_;
  long long start;  // absolute element offset in the packed array
  long long len;
};

// Device-side solver scalars, one block of kNScal doubles per gather.
enum ScalIdx {
  SC_GAMMA0 = 0, SC_GAMMA1, SC_DELTA, SC_ALPHA, SC_BETA, SC_DONE, SC_NINNER,
  SC_DMAX, SC_MMAX, SC_EPS_R, SC_EPS_M, SC_EPS_FROZEN, SC_FROZEN_SET, SC_MED, SC_MAD,
  SC_NLIVE, SC_MISFIT, SC_HUBER, SC_NONFINITE,
  // FISTA: power-method sum of squares, Lipschitz constant, mu, step 2 / Lf,
  // threshold mu / Lf (misfit and ||m||_1 reuse SC_MISFIT and SC_HUBER)
  SC_POW_SS, SC_LIP, SC_MU, SC_FSTEP, SC_FTHR,
  // CG: |g|^2 of the latest adjoint (its per-tile partials summed once per gather)
  SC_GNEW,
  kNScal = 25
};

// Radix-select state per gather: two order statistics (the two middle ranks).
struct SelState {
  unsigned prefix[2];
  unsigned kk[2];
};

// Device-side report accumulated per gather (copied to irls_report on the host).
struct RepDev {
  double misfit[64];
  double huber[64];
  double eps_r[64];
  double eps_m[64];
  double inner[64];
};

}  // namespace ashrt
