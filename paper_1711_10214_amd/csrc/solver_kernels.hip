// HIP kernels of the robust inversion (thesis Chapter 4, "Robust Radon
// transform"): CGLS vector updates in FP32 with FP64 inner products and step
// scalars kept on the device, the IRLS residual and model weights, and the
// median absolute deviation by radix selection on float bit patterns.
//
// All kernels take per-gather work lists so one launch serves a whole batch.
// Reductions are deterministic: each work item writes one partial, and the
// partials of a gather are summed in a fixed tree order.
#include "block_reduce.h"
#include "kernels.h"

namespace ashrt {

// ------------------------------------------------------------ partial reductions


__global__ __launch_bounds__(kThreads) void k_reduce_part(RedArgs A) {
  __shared__ double sh[kThreads / 64];
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const VecItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    const uint8_t* tm = A.tmask ? A.tmask + G.mask_off : nullptr;
    double a = 0.0, b = 0.0;
    const double eps = A.sc ? A.sc[w.g * kNScal + SC_EPS_R] : 0.0;
    long long i0 = threadIdx.x;
    if ((A.op == RED_SUMSQ || A.op == RED_ABSMAX) && ((w.start | w.len) & 3) == 0) {
      const float4* x4 = reinterpret_cast<const float4*>(A.x + w.start);
      for (long long i = threadIdx.x; i < (w.len >> 2); i += kThreads) {
        const float4 v = x4[i];
        if (A.op == RED_SUMSQ) {
          a += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
        } else {
          a = fmax(a, (double)fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
      }
      i0 = w.len;  // done
    }
    for (long long i = i0; i < w.len; i += kThreads) {
      const long long o = w.start + i;
      const double v = (double)A.x[o];
      if (A.op == RED_SUMSQ) {
        a += v * v;
      } else if (A.op == RED_ABSMAX) {
        a = fmax(a, fabs(v));
      } else if (A.op == RED_ABSSUM) {
        a += fabs(v);
      } else {
        bool live = true;
        if (tm) {
          const unsigned x = (unsigned)(o - G.d_off) / (unsigned)G.nt;  // nx nt < 2^31
          live = tm[x] != 0;
        }
        if (!live) continue;
        if (A.op == RED_ABSMAX_LIVE) {
          a = fmax(a, fabs(v));
        } else {  // RED_MISFIT: sum |r|^p and the Huber (p = 1) or LS (p = 2) objective
          const double av = fabs(v);
          if (A.p == 1) {
            a += av;
            b += (eps > 0.0) ? ((av <= eps) ? av * av / (2.0 * eps) : av - 0.5 * eps) : av;
          } else {
            a += v * v;
            b += 0.5 * v * v;
          }
        }
      }
    }
    double ra, rb = 0.0;
    if (A.op == RED_ABSMAX || A.op == RED_ABSMAX_LIVE) {
      ra = block_max(a, sh);
    } else {
      ra = block_sum(a, sh);
      if (A.op == RED_MISFIT) rb = block_sum(b, sh);
    }
    if (threadIdx.x == 0) {
      A.part[2 * it] = ra;
      A.part[2 * it + 1] = rb;
    }
  }
}

// One workgroup per gather: combine the partials of its items in a fixed order
// and store into the scalar slots (dst0, dst1; -1 = skip).  is_max selects max.

__global__ __launch_bounds__(kThreads) void k_reduce_fin(FinArgs A) {
  __shared__ double sh[kThreads / 64];
  const int g = blockIdx.x;
  if (g >= A.ngather) return;
  const GatherDev G = A.gd[g];
  const int lo = A.is_model ? G.mit_lo : G.dit_lo;
  const int hi = A.is_model ? G.mit_hi : G.dit_hi;
  double a = 0.0, b = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += kThreads) {
    if (A.is_max) {
      a = fmax(a, A.part[2 * i]);
    } else {
      a += A.part[2 * i];
      b += A.part[2 * i + 1];
    }
  }
  double ra, rb = 0.0;
  if (A.is_max) {
    ra = block_max(a, sh);
  } else {
    ra = block_sum(a, sh);
    rb = block_sum(b, sh);
  }
  if (threadIdx.x == 0) {
    if (A.dst0 >= 0) A.sc[g * kNScal + A.dst0] = ra;
    if (A.dst1 >= 0) A.sc[g * kNScal + A.dst1] = rb;
    if (A.rep) {
      A.rep[g].misfit[A.outer] = ra;
      A.rep[g].huber[A.outer] = rb;
      if (!isfinite(ra) || !isfinite(rb)) A.sc[g * kNScal + SC_NONFINITE] = 1.0;
    }
  }
}

// ------------------------------------------------------------ element-wise


__global__ __launch_bounds__(kThreads) void k_elementwise(EwArgs A) {
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const VecItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    float c = 0.f;
    float c2 = 0.f;
    if (A.op == EW_AXPY || A.op == EW_XPBY || A.op == EW_WR_UPDATE || A.op == EW_WM_UPDATE)
      c = (float)A.sc[w.g * kNScal + A.coef];
    if (A.op == EW_SCALE_RSQRT) {
      const double ss = A.sc[w.g * kNScal + A.coef];
      c = ss > 0.0 ? (float)(1.0 / sqrt(ss)) : 0.f;
    }
    if (A.op == EW_FISTA) {
      c = (float)A.sc[w.g * kNScal + A.coef];
      c2 = (float)A.sc[w.g * kNScal + A.coef + 1];
    }
    const uint8_t* tm = A.tmask ? A.tmask + G.mask_off : nullptr;
    long long i0 = threadIdx.x;
    if ((A.op <= EW_FILL) && ((w.start | w.len) & 3) == 0) {
      float4* y4 = reinterpret_cast<float4*>(A.y + w.start);
      const float4* x4 = reinterpret_cast<const float4*>(A.x + w.start);
      const float4* z4 = reinterpret_cast<const float4*>(A.z + w.start);
      const float sc_ = A.sign * c;
      for (long long i = threadIdx.x; i < (w.len >> 2); i += kThreads) {
        float4 r;
        if (A.op == EW_AXPY) {
          const float4 x = x4[i], y = y4[i];
          r = make_float4(fmaf(sc_, x.x, y.x), fmaf(sc_, x.y, y.y), fmaf(sc_, x.z, y.z), fmaf(sc_, x.w, y.w));
        } else if (A.op == EW_XPBY) {
          const float4 x = x4[i], y = y4[i];
          r = make_float4(fmaf(c, y.x, x.x), fmaf(c, y.y, x.y), fmaf(c, y.z, x.z), fmaf(c, y.w, x.w));
        } else if (A.op == EW_MUL) {
          const float4 x = x4[i], z = z4[i];
          r = make_float4(x.x * z.x, x.y * z.y, x.z * z.z, x.w * z.w);
        } else if (A.op == EW_COPY) {
          r = x4[i];
        } else {
          r = make_float4(A.value, A.value, A.value, A.value);
        }
        y4[i] = r;
      }
      i0 = w.len;
    }
    for (long long i = i0; i < w.len; i += kThreads) {
      const long long o = w.start + i;
      switch (A.op) {
        case EW_AXPY: A.y[o] = fmaf(A.sign * c, A.x[o], A.y[o]); break;
        case EW_XPBY: A.y[o] = fmaf(c, A.y[o], A.x[o]); break;
        case EW_MUL: A.y[o] = A.x[o] * A.z[o]; break;
        case EW_COPY: A.y[o] = A.x[o]; break;
        case EW_FILL: A.y[o] = A.value; break;
        case EW_WR_INIT:
        case EW_WR_UPDATE:
        case EW_WR_MASK: {
          const bool live = tm ? (tm[(unsigned)(o - G.d_off) / (unsigned)G.nt] != 0) : true;
          float v = 0.f;
          if (live) {
            if (A.op == EW_WR_INIT) v = A.x ? A.x[o] : 1.0f;
            else if (A.op == EW_WR_MASK) v = 1.0f;
            else v = (c > 0.f) ? 1.0f / sqrtf(fmaxf(fabsf(A.x[o]), c)) : 1.0f;
          }
          A.y[o] = v;
          break;
        }
        case EW_WM_UPDATE: {
          const float wi = (c > 0.f) ? sqrtf(fmaxf(fabsf(A.x[o]), c)) : 1.0f;
          A.y[o] = wi;
          A.z_out[o] = A.x[o] / wi;
          break;
        }
        case EW_SCALE_RSQRT: A.y[o] = A.x[o] * c; break;
        case EW_FISTA: {
          const float v = fmaf(c, A.x[o], A.y[o]);
          const float a = fabsf(v) - c2;
          const float mn = a > 0.f ? copysignf(a, v) : 0.f;
          const float mo = A.z_out[o];
          A.y[o] = fmaf(A.value, mn - mo, mn);
          A.z_out[o] = mn;
          break;
        }
        default: break;
      }
    }
  }
}

// ------------------------------------------------------------ per-gather scalar steps


__global__ void k_scalar(ScalArgs A) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= A.ngather) return;
  double* s = A.sc + g * kNScal;
  switch (A.step) {
    case ST_EPS_M:
      s[SC_EPS_M] = A.b_m * s[SC_MMAX] / 100.0;
      if (A.rep) A.rep[g].eps_m[A.outer] = s[SC_EPS_M];
      break;
    case ST_EPS_R: {
      double e;
      if (A.freeze && s[SC_FROZEN_SET] != 0.0) {
        e = s[SC_EPS_FROZEN];
      } else {
        e = fmax(A.b_r * s[SC_MAD] / 0.6745, A.floor_rel * s[SC_DMAX]);
        if (A.freeze) {
          s[SC_EPS_FROZEN] = e;
          s[SC_FROZEN_SET] = 1.0;
        }
      }
      s[SC_EPS_R] = e;
      if (A.rep) A.rep[g].eps_r[A.outer] = e;
      break;
    }
    case ST_REPORT_INNER:
      if (A.rep) A.rep[g].inner[A.outer] = s[SC_NINNER];
      break;
    case ST_FISTA: {
      const double lf = 2.0 * A.safety * sqrt(fmax(s[SC_POW_SS], 0.0));
      const double mu = A.mu_abs > 0.0 ? A.mu_abs : A.mu_rel * 2.0 * s[SC_MMAX];
      s[SC_LIP] = lf;
      s[SC_MU] = mu;
      s[SC_FSTEP] = lf > 0.0 ? 2.0 / lf : 0.0;
      s[SC_FTHR] = lf > 0.0 ? mu / lf : 0.0;
      break;
    }
    default:
      break;
  }
}

// ------------------------------------------------------------ radix select
//
// Order statistics of the live residual samples by three histogram passes
// over the float bit pattern mapped to an order-preserving unsigned key
// (11, 11, 10 bits).  The two middle ranks floor((n-1)/2) and floor(n/2) are
// selected together so the median of an even count is the mean of the two
// middle values.  Stage 0 selects on r, stage 1 on |r - median(r)|.
__device__ __forceinline__ unsigned float_key(float f) {
  const unsigned b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_float(unsigned k) {
  const unsigned b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(b);
}


// kSelSplit workgroups per data-vector item; each thread issues the loads
// of four samples before it bins them.
constexpr int kSelSplit = 2;
__global__ __launch_bounds__(kThreads) void k_sel_hist(SelArgs A) {
  __shared__ unsigned h[2][kSelBins];
  for (int b = blockIdx.x; b < A.nitems * kSelSplit; b += gridDim.x) {
    for (int i = threadIdx.x; i < 2 * kSelBins; i += kThreads) (&h[0][0])[i] = 0u;
    __syncthreads();
    const int it = b / kSelSplit, part = b - it * kSelSplit;
    const VecItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    const SelState S = A.st[w.g];
    const unsigned hmask = (A.shift + A.width >= 32) ? 0u : (0xffffffffu << (A.shift + A.width));
    const unsigned dmask = (1u << A.width) - 1u;
    const uint8_t* tm = A.tmask ? A.tmask + G.mask_off : nullptr;
    const double med = A.stage ? A.sc[w.g * kNScal + SC_MED] : 0.0;
    const long long lo = w.start + w.len * part / kSelSplit;
    const int n = (int)(w.start + w.len * (part + 1) / kSelSplit - lo);
    const unsigned rel0 = (unsigned)(lo - G.d_off);  // sample index in the gather (nx nt < 2^31)
    for (int base = threadIdx.x; base < n; base += 4 * kThreads) {
      float v[4];
      int live[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = A.x[lo + min(base + u * kThreads, n - 1)];
      if (tm) {
#pragma unroll
        for (int u = 0; u < 4; ++u) live[u] = tm[(rel0 + (unsigned)min(base + u * kThreads, n - 1)) / (unsigned)G.nt];
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) live[u] = 1;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (base + u * kThreads >= n || live[u] == 0) continue;
        float x = v[u];
        if (A.stage) x = (float)fabs((double)x - med);
        const unsigned key = float_key(x);
        const unsigned dg = (key >> A.shift) & dmask;
        if ((key & hmask) == (S.prefix[0] & hmask)) atomicAdd(&h[0][dg], 1u);
        if ((key & hmask) == (S.prefix[1] & hmask)) atomicAdd(&h[1][dg], 1u);
      }
    }
    __syncthreads();
    unsigned* gh = A.hist + (long long)w.g * 2 * kSelBins;
    for (int i = threadIdx.x; i < 2 * kSelBins; i += kThreads) {
      const unsigned c = (&h[0][0])[i];
      if (c) atomicAdd(&gh[i], c);
    }
    __syncthreads();
  }
}

// One workgroup per gather: find the digit holding rank kk, fix it in the
// prefix, subtract the counts below, and clear the histogram for the next pass.
__global__ __launch_bounds__(kThreads) void k_sel_pick(SelArgs A) {
  __shared__ unsigned cnt[kThreads];
  const int g = blockIdx.x;
  if (g >= A.ngather) return;
  unsigned* gh = A.hist + (long long)g * 2 * kSelBins;
  const int nb = 1 << A.width;
  const int per = nb / kThreads;  // bins per thread (nb >= kThreads)
  for (int s = 0; s < 2; ++s) {
    unsigned* hh = gh + s * kSelBins;
    const unsigned kk = A.st[g].kk[s];  // read before the scan's barriers; one thread rewrites it below
    unsigned loc = 0;
    for (int i = 0; i < per; ++i) loc += hh[threadIdx.x * per + i];
    cnt[threadIdx.x] = loc;
    __syncthreads();
    // inclusive scan (Hillis-Steele)
    for (int off = 1; off < kThreads; off <<= 1) {
      const unsigned v = (threadIdx.x >= (unsigned)off) ? cnt[threadIdx.x - off] : 0u;
      __syncthreads();
      cnt[threadIdx.x] += v;
      __syncthreads();
    }
    const unsigned before = (threadIdx.x == 0) ? 0u : cnt[threadIdx.x - 1];
    if (kk >= before && kk < cnt[threadIdx.x]) {
      unsigned run = before;
      for (int i = 0; i < per; ++i) {
        const unsigned c = hh[threadIdx.x * per + i];
        if (kk < run + c) {
          const unsigned dg = (unsigned)(threadIdx.x * per + i);
          A.st[g].prefix[s] |= dg << A.shift;
          A.st[g].kk[s] = kk - run;
          break;
        }
        run += c;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins; i += kThreads) hh[i] = 0u;
    __syncthreads();
  }
}

// Start a selection: ranks from the live count, empty prefixes.
__global__ void k_sel_init(SelArgs A) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= A.ngather) return;
  const double n = A.sc[g * kNScal + SC_NLIVE];
  const unsigned nn = (unsigned)n;
  A.st[g].prefix[0] = 0u;
  A.st[g].prefix[1] = 0u;
  A.st[g].kk[0] = nn ? (nn - 1u) / 2u : 0u;
  A.st[g].kk[1] = nn ? nn / 2u : 0u;
}

// Finish: median = mean of the two selected values (in FP64).
__global__ void k_sel_final(SelArgs A, double* sc, int dst) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= A.ngather) return;
  const double v0 = (double)key_float(A.st[g].prefix[0]);
  const double v1 = (double)key_float(A.st[g].prefix[1]);
  sc[g * kNScal + dst] = (sc[g * kNScal + SC_NLIVE] > 0.0) ? 0.5 * (v0 + v1) : 0.0;
}

// Live sample count per gather: (# live traces) * nt.
__global__ __launch_bounds__(kThreads) void k_count_live(const GatherDev* gd, int ngather,
                                                         const uint8_t* tmask, double* sc) {
  __shared__ double sh[kThreads / 64];
  const int g = blockIdx.x;
  if (g >= ngather) return;
  const GatherDev G = gd[g];
  double c = 0.0;
  for (int x = threadIdx.x; x < G.nx; x += kThreads) c += (tmask ? (tmask[G.mask_off + x] != 0) : 1) ? 1.0 : 0.0;
  const double r = block_sum(c, sh);
  if (threadIdx.x == 0) sc[g * kNScal + SC_NLIVE] = r * (double)G.nt;
}

// CG initialisation / update over model-vector items (see CgArgs).
// Per-gather sum of per-tile partials in a fixed order: four interleaved
// thread-strided partial sums per thread (loads in flight), then block_sum.
constexpr int kSumThreads = 1024;
__global__ __launch_bounds__(kSumThreads) void k_sum_items(const GatherDev* gd, int ngather, const double* part,
                                                           int is_model, double* sc, int dst) {
  __shared__ double sh[kSumThreads / 64];
  const int g = blockIdx.x;
  if (g >= ngather) return;
  const GatherDev G = gd[g];
  const int lo = is_model ? G.xm_lo : G.xd_lo;
  const int hi = is_model ? G.xm_hi : G.xd_hi;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = lo + (int)threadIdx.x;
  for (; i + 3 * kSumThreads < hi; i += 4 * kSumThreads) {
    a0 += part[i];
    a1 += part[i + kSumThreads];
    a2 += part[i + 2 * kSumThreads];
    a3 += part[i + 3 * kSumThreads];
  }
  for (; i < hi; i += kSumThreads) a0 += part[i];
  const double r = block_sum((a0 + a1) + (a2 + a3), sh);
  if (threadIdx.x == 0) sc[(long long)g * kNScal + dst] = r;
}

__global__ __launch_bounds__(kThreads) void k_cg(CgArgs A) {
  __shared__ float s_ab[2];
  __shared__ double sh[kThreads / 64];
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const VecItem w = A.items[it];
    const GatherDev G = A.gd[w.g];
    double gsum = 0.0;
    if (A.part_gamma) {
      double part = 0.0;
      for (int i = G.xm_lo + (int)threadIdx.x; i < G.xm_hi; i += kThreads) part += A.part_gamma[i];
      gsum = block_sum(part, sh);
    }
    if (threadIdx.x == 0) {
      double* sc = A.sc + (long long)w.g * kNScal;
      const double gnew = A.part_gamma ? gsum : sc[SC_GNEW];
      if (A.init) {
        if (it == G.mit_lo) {
          sc[SC_GAMMA0] = gnew;
          sc[SC_DONE] = 0.0;
          sc[SC_NINNER] = 0.0;
        }
        s_ab[0] = 0.f;
        s_ab[1] = 0.f;
      } else {
        const bool done = sc[SC_DONE] != 0.0;
        const double gold = sc[SC_GAMMA0 + A.par];
        const double beta = (done || gold == 0.0) ? 0.0 : gnew / gold;
        s_ab[0] = done ? 0.f : (float)sc[SC_ALPHA];
        s_ab[1] = (float)beta;
        if (it == G.mit_lo) {
          sc[SC_GAMMA0 + (A.par ^ 1)] = gnew;
          sc[SC_BETA] = beta;
        }
      }
    }
    __syncthreads();
    const float alpha = s_ab[0], beta = s_ab[1];
    float* __restrict__ u = A.u + w.start;
    float* __restrict__ p = A.pdir + w.start;
    const float* __restrict__ g = A.g + w.start;
    if (((w.start | w.len) & 3) == 0 && w.len > 0) {
      float4* u4 = reinterpret_cast<float4*>(u);
      float4* p4 = reinterpret_cast<float4*>(p);
      const float4* g4 = reinterpret_cast<const float4*>(g);
      // the loads of kBatch loop iterations are issued before any is used
      // (indices past the item clamped for the loads, skipped for the stores)
      constexpr int kBatch = 4;
      const int n4 = (int)(w.len >> 2);
      for (int base = threadIdx.x; base < n4; base += kBatch * kThreads) {
        float4 gv[kBatch], pv[kBatch], uv[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int i = min(base + b * kThreads, n4 - 1);
          gv[b] = g4[i];
          if (!A.init) {
            pv[b] = p4[i];
            uv[b] = u4[i];
          }
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int i = base + b * kThreads;
          if (i >= n4) break;
          if (A.init) {
            p4[i] = gv[b];
          } else {
            u4[i] = make_float4(fmaf(alpha, pv[b].x, uv[b].x), fmaf(alpha, pv[b].y, uv[b].y),
                                fmaf(alpha, pv[b].z, uv[b].z), fmaf(alpha, pv[b].w, uv[b].w));
            p4[i] = make_float4(fmaf(beta, pv[b].x, gv[b].x), fmaf(beta, pv[b].y, gv[b].y),
                                fmaf(beta, pv[b].z, gv[b].z), fmaf(beta, pv[b].w, gv[b].w));
          }
        }
      }
    } else {
      for (long long i = threadIdx.x; i < w.len; i += kThreads) {
        if (A.init) {
          p[i] = g[i];
        } else {
          const float pv = p[i];
          u[i] = fmaf(alpha, pv, u[i]);
          p[i] = fmaf(beta, pv, g[i]);
        }
      }
    }
    __syncthreads();
  }
}

// Clear n 32-bit words (a fill kernel rather than a memset, so the call can
// sit inside a captured graph).
__global__ void k_zero_words(unsigned* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ------------------------------------------------------------ launchers
static inline int grid_of(int n) { return n < 1 ? 1 : n; }

hipError_t launch_reduce_part(const RedArgs& a, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_part, dim3(grid_of(a.nitems)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_reduce_fin(const FinArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_fin, dim3(grid_of(a.ngather)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_elementwise(const EwArgs& a, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_elementwise, dim3(grid_of(a.nitems)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_scalar(const ScalArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_scalar, dim3((a.ngather + 63) / 64), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_zero_words(void* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(kThreads), 0, s, (unsigned*)p, n);
  return hipGetLastError();
}
hipError_t launch_sum_items(const GatherDev* gd, int ngather, const double* part, int is_model, double* sc,
                            int dst, hipStream_t s) {
  if (ngather <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_items, dim3(ngather), dim3(kSumThreads), 0, s, gd, ngather, part, is_model, sc, dst);
  return hipGetLastError();
}

hipError_t launch_cg(const CgArgs& a, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg, dim3(grid_of(a.nitems)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_count_live(const GatherDev* gd, int ngather, const uint8_t* tmask, double* sc,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_count_live, dim3(grid_of(ngather)), dim3(kThreads), 0, s, gd, ngather, tmask, sc);
  return hipGetLastError();
}

// Median of the live samples of x (stage 0) or of |x - median| (stage 1),
// into sc[g][dst].  The histogram must be zero on entry and is left zero.
hipError_t launch_select_median(SelArgs a, double* sc, int dst, hipStream_t s) {
  hipLaunchKernelGGL(k_sel_init, dim3((a.ngather + 63) / 64), dim3(64), 0, s, a);
  const int shifts[3] = {21, 10, 0};
  const int widths[3] = {11, 11, 10};
  for (int pass = 0; pass < 3; ++pass) {
    a.shift = shifts[pass];
    a.width = widths[pass];
    if (a.nitems > 0) hipLaunchKernelGGL(k_sel_hist, dim3(grid_of(a.nitems * kSelSplit)), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_sel_pick, dim3(grid_of(a.ngather)), dim3(kThreads), 0, s, a);
  }
  hipLaunchKernelGGL(k_sel_final, dim3((a.ngather + 63) / 64), dim3(64), 0, s, a, sc, dst);
  return hipGetLastError();
}

}  // namespace ashrt
