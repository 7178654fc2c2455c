// Bounds read-off (Step 1 of Section 5.1, Def. 2) and the ReLU approximant
// (Step 2) on gfx950.
//
// A pre-activation polynomial of per-variable degree D arrives as power
// coefficients a_J in the box coordinate t, stored in the total-degree layout
// (simplex.hpp: only |J| <= D); they are scattered into the dense (D+1)^n
// tensor in LDS, whose other entries are zero. Its Bernstein coefficients at
// degree D follow from the identity t^j = sum_{k>=j} C(k,j)/C(D,j) B_{k,D}(t)
// applied along every variable: a triangular (D+1)x(D+1) contraction per
// axis, b_k = sum_{j<=k} C(k,j)/C(D,j) a_j. The range enclosure (Def. 2) then
// gives lo = min b(lower) and hi = max b(upper). The contraction always runs
// in FP64, whatever the tensor precision.
//
// Tensors that fit the LDS budget are converted by one block each, all axes
// in LDS. Larger tensors take two passes: the trailing axes that fit LDS are
// converted per slice into an FP64 staging buffer, then the leading axes are
// converted per column chunk and reduced to per-chunk extrema, which a last
// small kernel folds.
//
// The same kernels pick each hidden neuron's rule (stable neurons, Section 5.1
// readings; plan codes) and build the ReLU over-approximant of Step 2: Bernstein
// coefficients b_k = sigma(lo + (hi-lo) k/L) (eq. bernpolcoeff2) turned into
// the power series in u = (y-lo)/(hi-lo) by forward differences,
// c_j = C(L,j) Delta^j b_0, and its value e at y = 0 (Prop. 2).
#include "common.hpp"
#include "rules.hpp"
#include "simplex.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <type_traits>

namespace bern {

constexpr int kSmallLds = 16384;  // FP64 elements of a tensor converted in one block (128 KiB)
constexpr int kTileLds = 8192;    // FP64 elements per staged tile of the two-pass path

// Block-wide reductions over wave64 shuffles + LDS.
template <typename Op>
__device__ double block_reduce(double v, Op op, double *red) {
  for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = op(r, red[w]);
    red[0] = r;
  }
  __syncthreads();
  double r = red[0];
  __syncthreads();
  return r;
}

struct OpMin { __device__ double operator()(double a, double b) const { return fmin(a, b); } };
struct OpMax { __device__ double operator()(double a, double b) const { return fmax(a, b); } };
struct OpAdd { __device__ double operator()(double a, double b) const { return a + b; } };

// In-place per-axis basis change of a tensor held in LDS (`t`, C doubles),
// axes [ax0, n). Table tab[k*(D+1)+j] = C(k,j)/C(D,j).
__device__ void lds_basis_change(double *t, int64_t C, int n, int D, int ax0, int ax1, const double *tab) {
  const int D1 = D + 1;
  int64_t stride = 1;
  for (int ax = n - 1; ax >= ax0; --ax) {
    if (ax < ax1) {
      const int64_t fibres = C / D1;
      for (int64_t f = threadIdx.x; f < fibres; f += blockDim.x) {
        const int64_t base = (f / stride) * stride * D1 + (f % stride);
        // descending k keeps the inputs a_j (j < k) intact until they are used
        for (int k = D; k >= 0; --k) {
          double s = 0.0;
          for (int j = 0; j <= k; ++j) s = fma(tab[k * D1 + j], t[base + (int64_t)j * stride], s);
          t[base + (int64_t)k * stride] = s;
        }
      }
      __syncthreads();
    }
    stride *= D1;
  }
}

__device__ void fill_table(double *tab, int D) {
  const int D1 = D + 1;
  for (int i = threadIdx.x; i < D1 * D1; i += blockDim.x) {
    const int k = i / D1, j = i % D1;
    tab[i] = (j <= k) ? binom_d(k, j) / binom_d(D, j) : 0.0;
  }
  __syncthreads();
}

// Least-squares affine fit of the Bernstein control net {(K/D, b_K)} and the
// range of its remainders (linear fallback rule). Outputs beta[0] = mean,
// beta[1+a] = slope along axis a for l(t) = beta0 + sum beta_a (t_a - 1/2),
// and the largest and smallest b_K - l(K/D). On the tensor grid the centred
// coordinates are orthogonal, so the normal equations are diagonal.
__device__ void lds_affine_fit(const double *t, int64_t C, int n, int D, double *beta, double *rmax, double *rmin,
                               double *red) {
  const int D1 = D + 1;
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < C; i += blockDim.x) m += t[i];
  beta[0] = block_reduce(m, OpAdd(), red) / (double)C;
  // sum over one axis of (k/D - 1/2)^2, times the other axes' sizes
  double s1 = 0.0;
  for (int k = 0; k <= D; ++k) {
    const double s = (double)k / D - 0.5;
    s1 += s * s;
  }
  const double ss = s1 * (double)(C / D1);
  int64_t stride = C / D1;  // stride of axis 0
  for (int a = 0; a < n; ++a) {
    double p = 0.0;
    for (int64_t i = threadIdx.x; i < C; i += blockDim.x) {
      const int k = (int)((i / stride) % D1);
      p += t[i] * ((double)k / D - 0.5);
    }
    beta[1 + a] = block_reduce(p, OpAdd(), red) / ss;
    stride /= D1;
  }
  double hi = -INFINITY, lo = INFINITY;
  for (int64_t i = threadIdx.x; i < C; i += blockDim.x) {
    double l = beta[0];
    int64_t rem = i;
    for (int a = n - 1; a >= 0; --a) {
      const int k = (int)(rem % D1);
      rem /= D1;
      l += beta[1 + a] * ((double)k / D - 0.5);
    }
    const double r = t[i] - l;
    hi = fmax(hi, r);
    lo = fmin(lo, r);
  }
  *rmax = block_reduce(hi, OpMax(), red);
  *rmin = block_reduce(lo, OpMin(), red);
}

// FP32 mode: radii epsU, epsL of the stored pre-activation polynomials of
// neuron j, i.e. the exact pre-activation lies in [L~ - epsL, U~ + epsU].
//  * first layer: the stored FP32 coefficients against the closed form,
//    recomputed in FP64 (its own rounding bounded by gamma);
//  * later layers: the previous layer's post radii through W+ and W-, the
//    FP64 accumulation of the affine map, and the exact FP32 store roundings
//    the GEMM blocks reported.
// The sums below are split over `nt` cooperating threads (thread index tid)
// and folded by `reduce` in a fixed order, so every thread gets the result.
template <typename Reduce>
__device__ void pre_radii(const ConvertArgs &a, int64_t box, int j, const void *pre, int tid, int nt, Reduce reduce,
                          double &epsU, double &epsL) {
  if (a.layer == 0) {
    const double *lo = a.box_lo + box * a.n, *hi = a.box_hi + box * a.n;
    const double *w = a.W + (int64_t)j * a.n;
    const float *p = reinterpret_cast<const float *>(pre) + box * a.slot + (int64_t)j * 2 * a.S;
    double a0 = a.b[j], sabs = fabs(a.b[j]);
    for (int k = 0; k < a.n; ++k) {
      a0 = fma(w[k], lo[k], a0);
      sabs += fabs(w[k]) * (fabs(lo[k]) + fabs(hi[k] - lo[k]));
    }
    double r = fabs((double)p[0] - a0);
    for (int k = 0; k < a.n; ++k) {
      const double ak = w[k] * (hi[k] - lo[k]);
      r += fabs((double)p[1 + k] - ak);  // coefficient of t_k
    }
    epsU = epsL = (r + gamma64(a.n + 4) * sabs) * kPadSafety;
    return;
  }
  double sU = 0.0, sL = 0.0, g = 0.0;
  for (int k = tid; k < a.hin; k += nt) {
    const double wk = a.W[(int64_t)j * a.hin + k];
    const double *P = a.prad + (box * a.hin + k) * 4;  // padU, padL, pl1U, pl1L
    if (wk >= 0.0) {
      sU += wk * P[0];
      sL += wk * P[1];
    } else {
      sU -= wk * P[1];
      sL -= wk * P[0];
    }
    g += fabs(wk) * (P[2] + P[3]);
  }
  double rU = 0.0, rL = 0.0;
  const double *rp = a.rpart + box * a.rpart_slot + (int64_t)j * 2 * a.cblocks;
  for (int64_t cb = tid; cb < a.cblocks; cb += nt) {
    rU += rp[cb];
    rL += rp[a.cblocks + cb];
  }
  sU = reduce(sU);
  sL = reduce(sL);
  g = reduce(g) + fabs(a.b[j]);
  rU = reduce(rU);
  rL = reduce(rL);
  const double gg = a.gpre * g;
  epsU = (sU + gg + rU) * kPadSafety;
  epsL = (sL + gg + rL) * kPadSafety;
}

// The first share of a later FP32 layer's radius inputs (k = tid: the
// weight, the previous layer's radii and l1 norms; cb = tid: the GEMM's
// rounding partials), loaded by a caller before its coefficients so that
// both loads are in flight together.
struct RadiiIn {
  double w = 0.0, r0 = 0.0, r1 = 0.0;
  double4 P = {0.0, 0.0, 0.0, 0.0};
};
__device__ inline void radii_prefetch(const ConvertArgs &a, int64_t box, int j, int tid, RadiiIn &ri) {
  if (a.mode == 2 || a.fp64 || a.layer == 0) return;
  if (tid < a.hin) {
    ri.w = a.W[(int64_t)j * a.hin + tid];
    ri.P = *reinterpret_cast<const double4 *>(a.prad + (box * a.hin + tid) * 4);
  }
  if (tid < a.cblocks) {
    const double *rp = a.rpart + box * a.rpart_slot + (int64_t)j * 2 * a.cblocks;
    ri.r0 = rp[tid];
    ri.r1 = rp[a.cblocks + tid];
  }
}

// The radii and the two tensors' l1 norms (l1: the lane's shares in, the
// team's totals out), their sums reduced together. `ri`: the first share,
// already loaded (radii_prefetch).
template <class Team>
__device__ void radii_and_l1(const ConvertArgs &a, int64_t box, int j, const Team &tm, double (&l1)[2],
                             double &epsU, double &epsL, const RadiiIn *ri = nullptr) {
  epsU = epsL = 0.0;
  if (a.mode == 2) {  // linearisation: the radii of the stored post polynomials
    if (!a.fp64) {
      const NeuronRec &r = a.recs[box * a.h + j];
      epsU = r.padU;
      epsL = r.padL;
    }
    tm.reduce(l1, OpAdd());
    return;
  }
  if (a.fp64 || a.layer == 0) {
    if (!a.fp64) pre_radii(a, box, j, a.pre, tm.tid, tm.nt, [](double v) { return v; }, epsU, epsL);
    tm.reduce(l1, OpAdd());
    return;
  }
  double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, l1[0], l1[1]};  // sU, sL, g, rU, rL, l1U, l1L
  for (int k = tm.tid; k < a.hin; k += tm.nt) {
    const bool pre = ri && k == tm.tid;
    const double wk = pre ? ri->w : a.W[(int64_t)j * a.hin + k];
    const double4 P = pre ? ri->P : *reinterpret_cast<const double4 *>(a.prad + (box * a.hin + k) * 4);
    if (wk >= 0.0) {
      v[0] += wk * P.x;
      v[1] += wk * P.y;
    } else {
      v[0] -= wk * P.y;
      v[1] -= wk * P.x;
    }
    v[2] += fabs(wk) * (P.z + P.w);
  }
  const double *rp = a.rpart + box * a.rpart_slot + (int64_t)j * 2 * a.cblocks;
  for (int64_t cb = tm.tid; cb < a.cblocks; cb += tm.nt) {
    const bool pre = ri && cb == tm.tid;
    v[3] += pre ? ri->r0 : rp[cb];
    v[4] += pre ? ri->r1 : rp[a.cblocks + cb];
  }
  tm.reduce(v, OpAdd());
  l1[0] = v[5];
  l1[1] = v[6];
  const double gg = a.gpre * (v[2] + fabs(a.b[j]));
  epsU = (v[0] + gg + v[3]) * kPadSafety;
  epsL = (v[1] + gg + v[4]) * kPadSafety;
}

// Bounds from the Bernstein extrema: in FP32 mode widened by the FP64
// basis-change rounding (gamma * sum|a|, the table entries lie in [0,1]) and
// the radii, then rounded outward. Called by all `nt` cooperating threads.
template <typename Reduce>
__device__ void padded_bounds(const ConvertArgs &a, int64_t box, int j, double mn, double mx, double l1L, double l1U,
                              int tid, int nt, Reduce reduce, double &lo, double &hi, double &epsU, double &epsL) {
  lo = mn;
  hi = mx;
  epsU = epsL = 0.0;
  if (a.fp64) return;
  pre_radii(a, box, j, a.pre, tid, nt, reduce, epsU, epsL);
  const double g = a.gconv;
  lo = round_down(mn - g * l1L - epsL);
  hi = round_up(mx + g * l1U + epsU);
}

// An output neuron's bounds (thread 0 only) and, when the caller takes the
// output polynomials, the radii of its two stored tensors.
__device__ inline void write_output(const ConvertArgs &a, int64_t box, int j, double lo, double hi, double epsU,
                                    double epsL) {
  a.out_lo[box * a.ld_out + a.col0 + j] = lo;
  a.out_hi[box * a.ld_out + a.col0 + j] = hi;
  if (a.out_eps) {
    a.out_eps[(box * a.h + j) * 2 + 0] = epsU;
    a.out_eps[(box * a.h + j) * 2 + 1] = epsL;
  }
}

// Record of one hidden neuron after its read-off (thread 0 only), then its
// rule unless a predictor chooses it later. Fitted neurons' affine fits are
// already in the record; the others get zeros unless the caller skips them
// (fits_written: an unfitted neuron's fit fields are never read).
__device__ void record_neuron(const ConvertArgs &a, int64_t box, int j, double lo, double hi, double epsU,
                              double epsL, double l1U, double l1L, const double *ext, bool fitted,
                              bool fits_written = false) {
  NeuronRec &r = a.recs[box * a.h + j];
  r.lo = lo;
  r.hi = hi;
  r.epsU = epsU;
  r.epsL = epsL;
  r.l1U = l1U;
  r.l1L = l1L;
  r.fitted = fitted ? 1 : 0;
  r.dpre = a.D;
  if (!fitted && !fits_written) {
    for (int q = 0; q <= kMaxInputs; ++q) r.fitU[q] = r.fitL[q] = 0.0;
  }
  r.rmaxU = fitted ? ext[0] : 0.0;
  r.rminU = fitted ? ext[1] : 0.0;
  r.rmaxL = fitted ? ext[2] : 0.0;
  r.rminL = fitted ? ext[3] : 0.0;
  if (a.learned) return;
  const int code = a.plan ? a.plan[box * a.plan_ld + a.plan_col0 + j] : a.L;
  decide_neuron(r, code, a.plan == nullptr, a.L, a.n, a.D, a.cap, a.fp64);
  if (a.used) a.used[box * a.ld_out + a.col0 + j] = (int8_t)r.kind;
}

__device__ void finish_neuron(const ConvertArgs &a, int64_t box, int j, double lo, double hi, double epsU,
                              double epsL, double l1U, double l1L, const double (*fit)[kMaxInputs + 1],
                              const double *ext, bool fitted) {
  if (fitted) {
    NeuronRec &r = a.recs[box * a.h + j];
    for (int q = 0; q <= kMaxInputs; ++q) {
      r.fitU[q] = fit[0][q];
      r.fitL[q] = fit[1][q];
    }
  }
  record_neuron(a, box, j, lo, hi, epsU, epsL, l1U, l1L, ext, fitted);
}

// One block per (box, neuron): both bounds of the neuron, all axes in LDS.
template <typename T>
__global__ void __launch_bounds__(kBlock) convert_small_kernel(ConvertArgs a) {
  extern __shared__ double lds[];
  const int D1 = a.D + 1;
  double *t = lds;
  double *tab = lds + a.C;
  double *red = tab + D1 * D1;
  __shared__ double fit[2][kMaxInputs + 1];
  __shared__ double ext[4];  // rmaxU, rminU, rmaxL, rminL
  const int64_t item = blockIdx.x;  // launch box * h + j
  if (item >= launch_boxes(a) * a.h) return;
  const int64_t box = a.bids ? a.bids[item / a.h] : item / a.h;
  const int j = (int)(item % a.h);
  fill_table(tab, a.D);
  const bool want_fit = a.mode == 0 && a.D > 0 &&
                        (a.learned || a.fits || (a.plan && a.plan[box * a.plan_ld + a.plan_col0 + j] <= 0));
  if (threadIdx.x < 2 * (kMaxInputs + 1)) fit[threadIdx.x / (kMaxInputs + 1)][threadIdx.x % (kMaxInputs + 1)] = 0.0;
  if (threadIdx.x < 4) ext[threadIdx.x] = 0.0;
  double ext_lo = 0.0, ext_hi = 0.0, l1s[2] = {0.0, 0.0};
  for (int s = 1; s >= 0; --s) {  // lower first, then upper
    const T *p = reinterpret_cast<const T *>(a.pre) + box * a.slot + ((int64_t)j * 2 + s) * a.S;
    for (int64_t i = threadIdx.x; i < a.C; i += blockDim.x) t[i] = 0.0;
    __syncthreads();
    double l1 = 0.0;
    for (int64_t i = threadIdx.x; i < a.S; i += blockDim.x) {
      const double v = (double)p[i];
      t[a.didx[i]] = v;
      l1 += fabs(v);
    }
    l1s[s] = block_reduce(l1, OpAdd(), red);
    lds_basis_change(t, a.C, a.n, a.D, 0, a.n, tab);
    double v = s ? INFINITY : -INFINITY;
    for (int64_t i = threadIdx.x; i < a.C; i += blockDim.x) v = s ? fmin(v, t[i]) : fmax(v, t[i]);
    v = s ? block_reduce(v, OpMin(), red) : block_reduce(v, OpMax(), red);
    if (s) ext_lo = v; else ext_hi = v;
    if (want_fit) {
      double beta[kMaxInputs + 1];
      double rmax, rmin;
      lds_affine_fit(t, a.C, a.n, a.D, beta, &rmax, &rmin, red);
      if (threadIdx.x == 0) {
        for (int ax = 0; ax <= a.n; ++ax) fit[s][ax] = beta[ax];
        ext[2 * s] = rmax;
        ext[2 * s + 1] = rmin;
      }
    }
    __syncthreads();
  }
  double lo, hi, epsU, epsL;
  padded_bounds(a, box, j, ext_lo, ext_hi, l1s[1], l1s[0], (int)threadIdx.x, (int)blockDim.x,
                [&](double v) { return block_reduce(v, OpAdd(), red); }, lo, hi, epsU, epsL);
  if (threadIdx.x == 0) {
    if (a.mode == 1) {
      write_output(a, box, j, lo, hi, epsU, epsL);
    } else {
      if (a.out_lo) a.out_lo[box * a.ld_out + a.col0 + j] = lo;
      if (a.out_hi) a.out_hi[box * a.ld_out + a.col0 + j] = hi;
      finish_neuron(a, box, j, lo, hi, epsU, epsL, l1s[0], l1s[1], fit, ext, want_fit);
    }
  }
}

// --------------------------------------------------- one wave per neuron
// Tensors of at most kWaveC coefficients: each wave64 of a 256-thread block
// handles one (box, neuron) with both bound tensors in its own LDS slice, so
// every reduction is a wave shuffle and no block barrier follows the shared
// table fill. The affine fits are computed only where a rule or the feature
// export needs them (unstable neurons, or every neuron when exporting).
constexpr int kWaveC = 1024;

template <typename Op>
__device__ inline double wave_reduce(double v, Op op) {
  for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ void wave_basis_change(double *t, int C, int n, int D, const double *tab, int lane) {
  const int D1 = D + 1;
  int stride = 1;
  for (int ax = n - 1; ax >= 0; --ax) {
    const int fibres = C / D1;
    for (int f = lane; f < fibres; f += 64) {
      const int base = (f / stride) * stride * D1 + (f % stride);
      for (int k = D; k >= 0; --k) {
        double s = 0.0;
        for (int j = 0; j <= k; ++j) s = fma(tab[k * D1 + j], t[base + j * stride], s);
        t[base + k * stride] = s;
      }
    }
    wave_sync();
    stride *= D1;
  }
}

// Same fit as lds_affine_fit, reduced over one wave.
__device__ void wave_affine_fit(const double *t, int C, int n, int D, int lane, double *beta, double &rmax,
                                double &rmin) {
  const int D1 = D + 1;
  double m = 0.0;
  for (int i = lane; i < C; i += 64) m += t[i];
  beta[0] = wave_reduce(m, OpAdd()) / (double)C;
  double s1 = 0.0;
  for (int k = 0; k <= D; ++k) {
    const double q = (double)k / D - 0.5;
    s1 += q * q;
  }
  const double ss = s1 * (double)(C / D1);
  int stride = C / D1;
  for (int ax = 0; ax < n; ++ax) {
    double p = 0.0;
    for (int i = lane; i < C; i += 64) p += t[i] * ((double)((i / stride) % D1) / D - 0.5);
    beta[1 + ax] = wave_reduce(p, OpAdd()) / ss;
    stride /= D1;
  }
  double hi = -INFINITY, lo = INFINITY;
  for (int i = lane; i < C; i += 64) {
    double l = beta[0];
    int rem = i;
    for (int ax = n - 1; ax >= 0; --ax) {
      l += beta[1 + ax] * ((double)(rem % D1) / D - 0.5);
      rem /= D1;
    }
    hi = fmax(hi, t[i] - l);
    lo = fmin(lo, t[i] - l);
  }
  rmax = wave_reduce(hi, OpMax());
  rmin = wave_reduce(lo, OpMin());
}

template <typename T>
__global__ void __launch_bounds__(kBlock) convert_wave_kernel(ConvertArgs a) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int D1 = a.D + 1;
  const int C = (int)a.C;
  double *tab = lds;
  double *tw = lds + D1 * D1 + (int64_t)wv * 2 * C;  // [2][C]: lower, upper
  fill_table(tab, a.D);
  const int64_t item = (int64_t)blockIdx.x * (kBlock / 64) + wv;
  if (item >= launch_boxes(a) * a.h) return;
  const int64_t box = a.bids ? a.bids[item / a.h] : item / a.h;
  const int j = (int)(item % a.h);
  double ext[2], l1s[2];
  for (int s = 1; s >= 0; --s) {
    double *t = tw + (1 - s) * C;
    const T *p = reinterpret_cast<const T *>(a.pre) + box * a.slot + ((int64_t)j * 2 + s) * a.S;
    for (int i = lane; i < C; i += 64) t[i] = 0.0;
    wave_sync();
    double l1 = 0.0;
    for (int i = lane; i < (int)a.S; i += 64) {
      const double v = (double)p[i];
      t[a.didx[i]] = v;
      l1 += fabs(v);
    }
    l1s[s] = wave_reduce(l1, OpAdd());
    wave_sync();
    wave_basis_change(t, C, a.n, a.D, tab, lane);
    double v = s ? INFINITY : -INFINITY;
    for (int i = lane; i < C; i += 64) v = s ? fmin(v, t[i]) : fmax(v, t[i]);
    ext[s] = s ? wave_reduce(v, OpMin()) : wave_reduce(v, OpMax());
  }
  double lo, hi, epsU, epsL;
  padded_bounds(a, box, j, ext[1], ext[0], l1s[1], l1s[0], lane, 64,
                [](double v) { return wave_reduce(v, OpAdd()); }, lo, hi, epsU, epsL);
  bool want_fit = a.mode == 0 && a.D > 0 &&
                  (a.learned || a.fits || (a.plan && a.plan[box * a.plan_ld + a.plan_col0 + j] <= 0));
  if (!a.fits) want_fit = want_fit && lo < 0.0 && hi > 0.0;  // only unstable neurons take a fitted rule
  double fit[2][kMaxInputs + 1], fx[4] = {0.0, 0.0, 0.0, 0.0};
  if (want_fit) {
    wave_affine_fit(tw + C, C, a.n, a.D, lane, fit[0], fx[0], fx[1]);  // upper
    wave_affine_fit(tw, C, a.n, a.D, lane, fit[1], fx[2], fx[3]);      // lower
  }
  if (lane == 0) {
    if (a.mode == 1) {
      write_output(a, box, j, lo, hi, epsU, epsL);
    } else {
      if (a.out_lo) a.out_lo[box * a.ld_out + a.col0 + j] = lo;
      if (a.out_hi) a.out_hi[box * a.ld_out + a.col0 + j] = hi;
      finish_neuron(a, box, j, lo, hi, epsU, epsL, l1s[0], l1s[1], fit, fx, want_fit);
    }
  }
}

// ------------------------------------------- compile-time degree variants
// For per-variable degrees 1..8 the ratio table C(k,j)/C(D,j) is a constant
// of the instruction stream and each fibre of D+1 coefficients is converted
// in registers: one LDS read and one write per coefficient and axis. The
// fastest axis is converted straight from the global load, and the extrema
// are taken from the registers of the last axis pass. Sums follow a fixed
// per-thread order, so results are reproducible run to run.
constexpr uint64_t binom_u(int n, int k) {
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}

template <int D>
struct Ratio {
  double v[D + 1][D + 1];
  constexpr Ratio() : v() {
    for (int k = 0; k <= D; ++k)
      for (int j = 0; j <= D; ++j) v[k][j] = j <= k ? (double)binom_u(k, j) / (double)binom_u(D, j) : 0.0;
  }
};

// b_k = sum_{j<=k} C(k,j)/C(D,j) a_j in place; descending k keeps a_j (j<k).
template <int D>
__device__ __forceinline__ void to_bern(double (&x)[D + 1]) {
  constexpr Ratio<D> R{};
#pragma unroll
  for (int k = D; k >= 0; --k) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j <= k; ++j) s = fma(R.v[k][j], x[j], s);
    x[k] = s;
  }
}

// Reduction of R <= kRows rows of 64 lane values in a wave's LDS scratch
// (row r at scr[kRowStride r + lane]; the stride spreads the rows over the
// banks), in a fixed order: eight partials per row (lane k 8 + q sums the
// row's elements q, q + 8, ...), then the row. Row r's result lands at
// scr[kRowResult + r].
constexpr int kRows = 8;
constexpr int kRowStride = 72;
constexpr int kRowPart = kRows * kRowStride, kRowResult = kRowPart + kRows * 8;
constexpr int kRowScratch = kRowResult + kRows;  // doubles of a wave's scratch

template <class Op>
__device__ __forceinline__ void wave_rows(double *scr, int R, int lane, Op op) {
  wave_sync();
  if (lane < R * 8) {
    const double *src = scr + (lane >> 3) * kRowStride + (lane & 7);
    double s = src[0];
#pragma unroll
    for (int i = 1; i < 8; ++i) s = op(s, src[8 * i]);
    scr[kRowPart + lane] = s;
  }
  wave_sync();
  if (lane < R) {
    const double *src = scr + kRowPart + lane * 8;
    double s = src[0];
#pragma unroll
    for (int i = 1; i < 8; ++i) s = op(s, src[i]);
    scr[kRowResult + lane] = s;
  }
  wave_sync();
}

// k/D - 1/2 for a digit k <= D: selects over the compile-time quotients,
// the same values as the division.
template <int D>
__device__ __forceinline__ double grid_c(unsigned k) {
  double v = -0.5;
#pragma unroll
  for (int q = 1; q <= D; ++q) v = k == (unsigned)q ? (double)q / D - 0.5 : v;
  return v;
}

struct WaveTeam {
  int tid;
  double *scr = nullptr;  // kRowScratch doubles of LDS for reduce(); null: shuffles
  static constexpr int nt = 64;
  __device__ void sync() const { wave_sync(); }
  __device__ double sum(double v) const { return wave_reduce(v, OpAdd()); }
  __device__ double min(double v) const { return wave_reduce(v, OpMin()); }
  __device__ double max(double v) const { return wave_reduce(v, OpMax()); }
  // K values at once, each over the wave
  template <int K, class Op>
  __device__ void reduce(double (&v)[K], Op op) const {
    static_assert(K <= kRows, "rows");
    if (!scr) {
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = wave_reduce(v[k], op);
      return;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) scr[k * kRowStride + tid] = v[k];
    wave_rows(scr, K, tid, op);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = scr[kRowResult + k];
    wave_sync();
  }
};

// Shared doubles a BlockTeam's `red` needs for reduce<K> with K <= kRows.
constexpr int kRedDoubles = 17 * kRows;

struct BlockTeam {
  int tid, nt;
  double *red;  // 16 doubles; reduce<K>() needs 17 K (kRedDoubles)
  __device__ void sync() const { __syncthreads(); }
  __device__ double sum(double v) const { return block_reduce(v, OpAdd(), red); }
  __device__ double min(double v) const { return block_reduce(v, OpMin(), red); }
  __device__ double max(double v) const { return block_reduce(v, OpMax(), red); }
  template <int K, class Op>
  __device__ void reduce(double (&v)[K], Op op) const {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_reduce(v[k], op);
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < K; ++k) red[k * 16 + wid] = v[k];
    __syncthreads();
    if (threadIdx.x < K) {
      double r = red[threadIdx.x * 16];
      for (int w = 1; w < nw; ++w) r = op(r, red[threadIdx.x * 16 + w]);
      red[16 * K + threadIdx.x] = r;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = red[16 * K + k];
    __syncthreads();
  }
};

__device__ inline double *tm_scratch(const WaveTeam &tm) { return tm.scr; }
__device__ inline double *tm_scratch(const BlockTeam &) { return nullptr; }

// One axis pass: every fibre of D+1 coefficients at stride `st` converted in
// registers. Fibre f has base (f / st) st (D+1) + f % st = f + (f / st) st D;
// the quotient is one multiply-high by magic = floor((2^32 - 1) / st) + 1,
// exact for f < 2^32 / st.
template <int D, bool kTrack, class Team>
__device__ __forceinline__ void axis_pass(double *t, int F, unsigned st, unsigned magic, const Team &tm, double &mn,
                                          double &mx) {
  constexpr int D1 = D + 1;
  for (int f = tm.tid; f < F; f += tm.nt) {
    const unsigned hi = st == 1 ? (unsigned)f : __umulhi((unsigned)f, magic);
    const int base = f + (int)(hi * st) * D;
    double x[D1];
#pragma unroll
    for (int j = 0; j < D1; ++j) x[j] = t[base + j * (int)st];
    to_bern<D>(x);
#pragma unroll
    for (int j = 0; j < D1; ++j) {
      if (kTrack) {
        mn = fmin(mn, x[j]);
        mx = fmax(mx, x[j]);
      }
      t[base + j * (int)st] = x[j];
    }
  }
}

// The same pass over the fibres whose leading exponents (axes before the
// one converted) are listed in `list` (np dense prefixes): the others are
// zero and stay zero.
template <int D, bool kTrack, class Team>
__device__ __forceinline__ void axis_pass_list(double *t, const int *list, int np, unsigned st, unsigned magic,
                                               const Team &tm, double &mn, double &mx) {
  constexpr int D1 = D + 1;
  const int W = np * (int)st;
  for (int w = tm.tid; w < W; w += tm.nt) {
    const unsigned pi = st == 1 ? (unsigned)w : __umulhi((unsigned)w, magic);
    const unsigned lo = (unsigned)w - pi * st;
    const int base = (int)((unsigned)list[pi] * (unsigned)D1 * st + lo);
    double x[D1];
#pragma unroll
    for (int j = 0; j < D1; ++j) x[j] = t[base + j * (int)st];
    to_bern<D>(x);
#pragma unroll
    for (int j = 0; j < D1; ++j) {
      if (kTrack) {
        mn = fmin(mn, x[j]);
        mx = fmax(mx, x[j]);
      }
      t[base + j * (int)st] = x[j];
    }
  }
}

// Last pass (axis 0, stride st = (D+1)^(n-1), fibre f = the digits of axes
// 1 .. n-1) with the extrema of the coefficients and of the remainders
// b_K - l(K/D) of an affine fit l (bl: beta_0, then the slope of every axis,
// each about the box centre). The results are not stored back.
template <int D, class Team>
__device__ __forceinline__ void last_pass_fit(const double *t, int st, int n, const Team &tm, const double *bl,
                                              double &mn, double &mx, double &rmn, double &rmx) {
  constexpr int D1 = D + 1;
  const double b1 = bl[1];
  for (int f = tm.tid; f < st; f += tm.nt) {
    double x[D1];
#pragma unroll
    for (int j = 0; j < D1; ++j) x[j] = t[f + j * st];
    to_bern<D>(x);
    double c = bl[0];
    unsigned q = (unsigned)f;
    for (int ax = n - 1; ax >= 1; --ax) {
      c = fma(bl[1 + ax], grid_c<D>(q % D1), c);
      q /= D1;
    }
#pragma unroll
    for (int j = 0; j < D1; ++j) {
      mn = fmin(mn, x[j]);
      mx = fmax(mx, x[j]);
      const double r = x[j] - fma(b1, (double)j / D - 0.5, c);
      rmn = fmin(rmn, r);
      rmx = fmax(rmx, r);
    }
  }
}

// Convert axes [0, na) of a tensor already in LDS whose axis na-1 has stride
// s0 (axis a has stride s0 (D+1)^(na-1-a)); `total` coefficients. Tracks the
// extrema of the last pass when `track` is set. With a prefix table `pl`
// (simplex.hpp prefix_table for (D, na), in LDS) only the fibres that can be
// nonzero are converted: valid when every nonzero coefficient of the tensor
// has exponent sum <= D. With a fit `bl` (whole tensor: s0 = 1, na = n) the
// last pass also tracks the remainder extrema into rmn / rmx and leaves axis
// 0 unconverted in LDS.
template <int D, class Team>
__device__ void team_axes(double *t, int total, int s0, int na, const Team &tm, bool track, double &mn,
                          double &mx, const int *pl = nullptr, const double *bl = nullptr,
                          double *rmn = nullptr, double *rmx = nullptr) {
  constexpr int D1 = D + 1;
  const int F = total / D1;
  unsigned stride = (unsigned)s0;
  for (int ax = na - 1; ax >= 0; --ax) {
    tm.sync();
    const unsigned magic = stride > 1 ? 0xFFFFFFFFu / stride + 1u : 0u;
    const bool last = track && ax == 0;
    if (last && bl) {
      last_pass_fit<D>(t, (int)stride, na, tm, bl, mn, mx, *rmn, *rmx);
    } else if (pl) {
      const int np = pl[ax + 1] - pl[ax];
      if (last)
        axis_pass_list<D, true>(t, pl + pl[ax], np, stride, magic, tm, mn, mx);
      else
        axis_pass_list<D, false>(t, pl + pl[ax], np, stride, magic, tm, mn, mx);
    } else {
      if (last)
        axis_pass<D, true>(t, F, stride, magic, tm, mn, mx);
      else
        axis_pass<D, false>(t, F, stride, magic, tm, mn, mx);
    }
    stride *= D1;
  }
  tm.sync();
}

// Copy the prefix table into LDS (all threads of the block, then a barrier).
__device__ inline const int *stage_prefixes(const ConvertArgs &a, int *dst) {
  if (!a.plist) return nullptr;
  for (int i = threadIdx.x; i < a.plist_len; i += blockDim.x) dst[i] = a.plist[i];
  __syncthreads();
  return dst;
}


// Least-squares affine fit l(x) = beta_0 + sum_a beta_a (x_a - 1/2) of the
// control net {(K/D, b_K)} (same quantities as lds_affine_fit), from the
// stored coefficients a_J instead of the dense net. The centred grid
// coordinates are orthogonal, so beta_0 is the mean of the b_K and beta_a
// their first moment along axis a over sum_K (k_a/D - 1/2)^2. With
// b_K = sum_J a_J prod_i C(k_i, j_i) / C(D, j_i) both sums factor over the
// axes, and the one-axis sums over k = j .. D have closed forms
// (hockey-stick identity): sum_k C(k,j)/C(D,j) = (D+1)/(j+1),
// sum_k C(k,j)/C(D,j) (k/D - 1/2) = (D+1)/(j+1) * j (D+2) / (2 D (j+2)), and
// sum_k (k/D - 1/2)^2 = (D+1)(D+2) / (12 D). What remains is
//   beta_0 = sum_J w_J,   beta_a = 6 sum_J w_J j_a / (j_a + 2),
//   w_J = a_J / prod_i (j_i + 1),
// independent of D. One wave computes it (didx gives each J's digits, axis
// n-1 fastest) into bl[0 .. n] in LDS; the caller's barrier publishes it.
// 1/(j+1) and 6 j/(j+2) for a digit j <= D (selects over constants).
template <int D>
__device__ __forceinline__ double fit_inv(unsigned j) {
  double v = 1.0;
#pragma unroll
  for (int q = 1; q <= D; ++q) v = j == (unsigned)q ? 1.0 / (q + 1) : v;
  return v;
}
template <int D>
__device__ __forceinline__ double fit_slope(unsigned j) {
  double v = 0.0;
#pragma unroll
  for (int q = 1; q <= D; ++q) v = j == (unsigned)q ? 6.0 * q / (q + 2) : v;
  return v;
}

template <int D, typename T>
__device__ void wave_fit(const T *p, const int *didx, int S, int n, int lane, double *bl, double *scr = nullptr) {
  constexpr unsigned D1 = D + 1;
  if (scr) {  // the n + 1 sums as rows of the wave's scratch, kRows at a time
    for (int r0 = 0; r0 <= n; r0 += kRows) {
      const int R = min(kRows, n + 1 - r0);
      for (int r = 0; r < R; ++r) scr[r * kRowStride + lane] = 0.0;
      for (int i = lane; i < S; i += 64) {
        unsigned d = (unsigned)didx[i];
        double w = (double)p[i];
        for (int ax = 0; ax < n; ++ax) {
          w *= fit_inv<D>(d % D1);
          d /= D1;
        }
        d = (unsigned)didx[i];
        for (int ax = n - 1; ax >= 0; --ax) {  // row 1 + ax - r0
          const unsigned k = d % D1;
          d /= D1;
          const int r = 1 + ax - r0;
          if (r >= 0 && r < R) scr[r * kRowStride + lane] += w * fit_slope<D>(k);
        }
        if (r0 == 0) scr[lane] += w;
      }
      wave_rows(scr, R, lane, OpAdd());
      if (lane < R) bl[r0 + lane] = scr[kRowResult + lane];
      wave_sync();
    }
    return;
  }
  for (int base = 0; base < S; base += 64) {
    const int i = base + lane;
    double w = 0.0;
    unsigned dig = 0u;
    if (i < S) {
      dig = (unsigned)didx[i];
      w = (double)p[i];
      unsigned d = dig;
      for (int ax = 0; ax < n; ++ax) {
        w *= fit_inv<D>(d % D1);
        d /= D1;
      }
    }
    const double b0 = wave_reduce(w, OpAdd());
    for (int ax = n - 1; ax >= 0; --ax) {
      const unsigned k = dig % D1;
      dig /= D1;
      const double ba = wave_reduce(w * fit_slope<D>(k), OpAdd());
      if (lane == 0) bl[1 + ax] = base == 0 ? ba : bl[1 + ax] + ba;
    }
    if (lane == 0) bl[0] = base == 0 ? b0 : bl[0] + b0;
  }
}

// team_convert without its reductions: the lane's own extrema (and, with a
// fit, remainder extrema) are folded into mn, mx (rmn, rmx).
template <int D, typename T, class Team>
__device__ void team_convert_lanes(double *t, const T *p, const int *didx, int C, int S, int n, const Team &tm,
                                   const int *pl, const double *bl, double &mn, double &mx, double &rmn,
                                   double &rmx) {
  for (int i = tm.tid; i < C; i += tm.nt) t[i] = 0.0;
  tm.sync();
  for (int i = tm.tid; i < S; i += tm.nt) t[didx[i]] = (double)p[i];
  team_axes<D>(t, C, 1, n, tm, true, mn, mx, pl, bl, &rmn, &rmx);
}


// Bound of one side from its Bernstein extremum (FP32 mode: widened by the
// basis-change rounding and the pre-activation radius, rounded outward).
__device__ inline double side_lo(const ConvertArgs &a, double mn, double l1, double eps) {
  if (a.fp64) return mn;
  return round_down(mn - a.gconv * l1 - eps);
}
__device__ inline double side_hi(const ConvertArgs &a, double mx, double l1, double eps) {
  if (a.fp64) return mx;
  return round_up(mx + a.gconv * l1 + eps);
}

__device__ inline bool wants_fit(const ConvertArgs &a, int64_t box, int j) {
  if (a.mode == 2) return true;
  return a.mode == 0 && a.D > 0 && (a.learned || a.fits || (a.plan && a.plan[box * a.plan_ld + a.plan_col0 + j] <= 0));
}

// Periodic linearisation (mode 2, thread 0): the affine post polynomials
// l + max remainder (upper) and l + min remainder (lower) of one neuron in
// the power basis, from the fits bU, bL (l(t) = b[0] + sum_a b[1+a] (t_a -
// 1/2)) and the remainder extrema fx = (rmaxU, rminU, rmaxL, rminL). FP32
// mode: the radius of each is the stored post's radius, the read-off's
// rounding of the Bernstein coefficients (gconv times the l1 norm) and the
// FP64 rounding of the fit's evaluation at the grid and of the conversion to
// the power basis (gamma(n + 8) times the fit's and remainder's magnitudes).
__device__ inline void write_lin(const ConvertArgs &a, int64_t box, int j, const double *bU, const double *bL,
                                 const double *fx, double epsU, double epsL, double l1U, double l1L) {
  NeuronRec &r = a.recs[box * a.h + j];
  double sU = 0.0, sL = 0.0, aU = fabs(bU[0]), aL = fabs(bL[0]);
  for (int ax = 0; ax < a.n; ++ax) {
    sU += bU[1 + ax];
    sL += bL[1 + ax];
    aU += fabs(bU[1 + ax]);
    aL += fabs(bL[1 + ax]);
  }
  r.fbU[0] = bU[0] - 0.5 * sU + fx[0];
  r.fbL[0] = bL[0] - 0.5 * sL + fx[3];
  for (int q = 1; q <= kMaxInputs; ++q) {
    r.fbU[q] = q <= a.n ? bU[q] : 0.0;
    r.fbL[q] = q <= a.n ? bL[q] : 0.0;
  }
  r.fbpadU = r.fbpadL = 0.0;
  if (!a.fp64) {
    const double ge = gamma64(a.n + 8);
    r.fbpadU = epsU + a.gconv * l1U + ge * (aU + fabs(fx[0]));
    r.fbpadL = epsL + a.gconv * l1L + ge * (aL + fabs(fx[3]));
  }
}

__device__ inline void write_neuron(const ConvertArgs &a, int64_t box, int j, double lo, double hi, double epsU,
                                    double epsL, double l1U, double l1L, const double *ext, bool fitted,
                                    bool fits_written = false) {
  if (a.mode == 1) {
    write_output(a, box, j, lo, hi, epsU, epsL);
  } else {
    if (a.out_lo) a.out_lo[box * a.ld_out + a.col0 + j] = lo;
    if (a.out_hi) a.out_hi[box * a.ld_out + a.col0 + j] = hi;
    record_neuron(a, box, j, lo, hi, epsU, epsL, l1U, l1L, ext, fitted, fits_written);
  }
}

// A neuron's fit coefficients (or zeros, fit null) written by the team's
// lanes, one coefficient each, then made visible to the team (the rule
// chosen by thread 0 may read them).
template <class Team>
__device__ inline void team_write_fit(const ConvertArgs &a, const Team &tm, double *dst, const double *fit) {
  for (int q = tm.tid; q <= kMaxInputs; q += tm.nt) dst[q] = fit && q <= a.n ? fit[q] : 0.0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  tm.sync();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Both bound tensors of neuron (box, j) by one team with `t` (C doubles) and
// `bl` (the two fits, 2 (kMaxInputs + 1) doubles) in LDS; `fitter` marks the
// team's first wave, which computes the fits.
template <int D, typename T, class Team>
__device__ void readoff_pair(const ConvertArgs &a, const Team &tm, bool fitter, int lane, double *t, double *bl,
                             const int *pl, int64_t box, int j) {
  const int C = (int)a.C, S = (int)a.S;
  const T *p = reinterpret_cast<const T *>(a.pre) + box * a.slot + (int64_t)j * 2 * a.S;
  double *scr = tm_scratch(tm);
  double *blU = bl, *blL = bl + kMaxInputs + 1;
  // l1 norms of both tensors; their loads go out before the radii's
  double l1[2] = {0.0, 0.0};
  for (int i = tm.tid; i < S; i += tm.nt) {
    l1[0] += fabs((double)p[i]);
    l1[1] += fabs((double)p[S + i]);
  }
  double epsU, epsL;
  radii_and_l1(a, box, j, tm, l1, epsU, epsL);
  const double l1U = l1[0], l1L = l1[1];
  // Affine fits (closed form from the stored coefficients) go to the
  // neurons that may take a fitted rule and turn out unstable, or to every
  // such neuron when all are fitted (a.fits): then first, with the remainder
  // ranges in the read-off's last pass; else after the extrema, with a
  // second read-off for the remainders.
  const bool want = wants_fit(a, box, j);
  const bool early = want && a.fits;
  auto fits = [&]() {
    if (fitter) {
      wave_fit<D>(p, a.didx, S, a.n, lane, blU, scr);
      wave_fit<D>(p + S, a.didx, S, a.n, lane, blL, scr);
    }
    tm.sync();
  };
  if (early) fits();
  double mnL = INFINITY, mxL = -INFINITY, rmnL = INFINITY, rmxL = -INFINITY;
  team_convert_lanes<D>(t, p + S, a.didx, C, S, a.n, tm, pl, early ? blL : nullptr, mnL, mxL, rmnL, rmxL);
  double mnU = INFINITY, mxU = -INFINITY, rmnU = INFINITY, rmxU = -INFINITY;
  team_convert_lanes<D>(t, p, a.didx, C, S, a.n, tm, pl, early ? blU : nullptr, mnU, mxU, rmnU, rmxU);
  // maxima of: max U, -min L, and the remainders' max U, -min U, max L, -min L
  double ex[6] = {mxU, -mnL, rmxU, -rmnU, rmxL, -rmnL};
  tm.reduce(ex, OpMax());
  const double lo = side_lo(a, -ex[1], l1L, epsL), hi = side_hi(a, ex[0], l1U, epsU);
  const bool fitted = want && (a.fits || (lo < 0.0 && hi > 0.0));
  if (fitted && !early) {
    fits();
    double m0 = INFINITY, m1 = -INFINITY;
    rmnL = rmnU = INFINITY;
    rmxL = rmxU = -INFINITY;
    team_convert_lanes<D>(t, p + S, a.didx, C, S, a.n, tm, pl, blL, m0, m1, rmnL, rmxL);
    team_convert_lanes<D>(t, p, a.didx, C, S, a.n, tm, pl, blU, m0, m1, rmnU, rmxU);
    double rx[4] = {rmxU, -rmnU, rmxL, -rmnL};
    tm.reduce(rx, OpMax());
    for (int q = 0; q < 4; ++q) ex[2 + q] = rx[q];
  }
  double fx[4] = {0.0, 0.0, 0.0, 0.0};  // rmaxU, rminU, rmaxL, rminL
  if (fitted) {
    fx[0] = ex[2];
    fx[1] = -ex[3];
    fx[2] = ex[4];
    fx[3] = -ex[5];
  }
  if (a.mode == 2) {
    if (tm.tid == 0) write_lin(a, box, j, blU, blL, fx, epsU, epsL, l1U, l1L);
    return;
  }
  if (a.mode == 0 && fitted) {  // the fits (an unfitted neuron's are never read)
    NeuronRec &rec = a.recs[box * a.h + j];
    team_write_fit(a, tm, rec.fitU, blU);
    team_write_fit(a, tm, rec.fitL, blL);
  }
  if (tm.tid == 0) write_neuron(a, box, j, lo, hi, epsU, epsL, l1U, l1L, fx, fitted, true);
}

// Doubles of one wave's LDS slice: reduction rows, the tensor and the two
// fits.
__host__ __device__ constexpr int wave_slice_doubles(int C) { return kRowScratch + C + 2 * (kMaxInputs + 1); }

// One wave per (box, neuron), one bound tensor at a time in the wave's LDS
// slice.
template <int D, typename T>
__global__ void __launch_bounds__(kBlock, 6) convert_wave_t(ConvertArgs a) {
  extern __shared__ double lds[];
  const WaveTeam tm{(int)(threadIdx.x & 63)};
  const int wv = threadIdx.x >> 6;
  const int C = (int)a.C;
  const int *pl = stage_prefixes(a, reinterpret_cast<int *>(lds));
  double *tw = lds + (a.plist_len + 1) / 2 + (int64_t)wv * wave_slice_doubles(C);
  const int64_t item = (int64_t)blockIdx.x * (kBlock / 64) + wv;
  if (item >= launch_boxes(a) * a.h) return;
  const int64_t box = a.bids ? a.bids[item / a.h] : item / a.h;
  const WaveTeam tmw{tm.tid, tw};
  readoff_pair<D, T>(a, tmw, true, tm.tid, tw + kRowScratch, tw + kRowScratch + C, pl, box, (int)(item % a.h));
}

// One block per (box, neuron) for tensors up to kSmallLds coefficients, one
// tensor in LDS at a time.
template <int D, typename T>
__global__ void __launch_bounds__(1024) convert_block_t(ConvertArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[kRedDoubles];
  const BlockTeam tm{(int)threadIdx.x, (int)blockDim.x, red};
  const int *pl = stage_prefixes(a, reinterpret_cast<int *>(lds));
  double *t = lds + (a.plist_len + 1) / 2;
  const int64_t item = blockIdx.x;
  if (item >= launch_boxes(a) * a.h) return;
  const int64_t box = a.bids ? a.bids[item / a.h] : item / a.h;
  readoff_pair<D, T>(a, tm, threadIdx.x < 64, (int)(threadIdx.x & 63), t, t + a.C, pl, box, (int)(item % a.h));
}

// Degree 1 (every first hidden layer, and neurons whose plan keeps degree
// 1): an affine polynomial a_0 + sum_a a_{1+a} t_a, whose per-variable
// degree-1 Bernstein coefficients are its values at the 2^n box corners. All
// the read-off needs is then in closed form over the n + 1 stored
// coefficients: the extrema a_0 + sum_a min(a_{1+a}, 0) and
// a_0 + sum_a max(a_{1+a}, 0); the least-squares fit of the corner values,
// beta_a = a_{1+a} and beta_0 = a_0 + sum_a a_{1+a} / 2 (the closed form of
// the fit below at degree 1); and its remainders, the same constant
// a_0 - beta_0 + sum_a beta_a / 2 at every corner (zero up to rounding). A
// team of lanes per neuron, several neurons per wave. For the first layer
// over every box (from_box) the kernel also forms the coefficients from the
// box, W and b (the layer-1 kernel's arithmetic) and stores them, so the
// first layer takes one launch.
// kL lanes per neuron (8 when the n + 1 coefficients fit, else 16), each
// holding coefficients l, l + kL, ...
template <int kL>
__device__ __forceinline__ double aff_sum(double v) {
#pragma unroll
  for (int m = kL / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, kL);
  return v;
}

template <typename T, int kL>
__global__ void __launch_bounds__(kBlock) convert_affine_kernel(ConvertArgs a) {
  constexpr int kAffLanes = kL;
  constexpr int kR = (kMaxInputs + 1 + kL - 1) / kL;  // coefficient slots per lane
  const int l = threadIdx.x % kAffLanes;
  const int64_t item = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kAffLanes;
  if (item >= launch_boxes(a) * a.h) return;  // whole teams leave together
  const int S = (int)a.S;
  const int64_t box = a.bids ? a.bids[item / a.h] : item / a.h;
  const int j = (int)(item % a.h);
  const T *p = reinterpret_cast<const T *>(a.pre) + box * a.slot + (int64_t)j * 2 * a.S;
  // the lane's coefficients: indices l + r kL (n + 1 <= 17)
  double u[kR], w[kR];
  if (a.from_box) {
    // the first layer's pre-activation in closed form (upper = lower): with
    // x_a = d_lo_a + (d_hi_a - d_lo_a) t_a, the constant b_j + W_j d_lo and
    // the coefficient W_ja (d_hi_a - d_lo_a) of t_a; stored, and read off
    // as stored
    const double *lo = a.box_lo + box * a.n, *hi = a.box_hi + box * a.n;
    const double *wj = a.W + (int64_t)j * a.n;
    T *pw = reinterpret_cast<T *>(const_cast<void *>(a.pre)) + box * a.slot + (int64_t)j * 2 * a.S;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      u[r] = w[r] = 0.0;
      const int i = l + r * kAffLanes;
      if (i < S) {
        double v;
        if (i == 0) {
          v = a.b[j];
          for (int k = 0; k < a.n; ++k) v = fma(wj[k], lo[k], v);
        } else {
          v = wj[i - 1] * (hi[i - 1] - lo[i - 1]);
        }
        const T sv = (T)v;
        pw[i] = sv;
        pw[S + i] = sv;
        u[r] = w[r] = (double)sv;
      }
    }
    if (a.flags && j == 0 && l == 0) {  // the box's validity, once per box
      int bad = 0;
      for (int k = 0; k < a.n; ++k)
        if (!(lo[k] <= hi[k]) || !isfinite(lo[k]) || !isfinite(hi[k])) bad = 1;
      a.flags[box] = bad;
      if (bad && a.hbad) *a.hbad = 1;
    }
  } else {
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      u[r] = w[r] = 0.0;
      const int i = l + r * kAffLanes;
      if (i < S) {
        u[r] = (double)p[i];
        w[r] = (double)p[S + i];
      }
    }
  }
  if (a.mode == 2) {
    // an affine post is its own linearisation (zero remainders): its
    // coefficients, and in FP32 mode its radius, carry over unchanged
    NeuronRec &rec = a.recs[box * a.h + j];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int q = l + r * kAffLanes;
      if (q <= kMaxInputs) {
        rec.fbU[q] = q < S ? u[r] : 0.0;
        rec.fbL[q] = q < S ? w[r] : 0.0;
      }
    }
    if (l == 0) {
      rec.fbpadU = a.fp64 ? 0.0 : rec.padU;
      rec.fbpadL = a.fp64 ? 0.0 : rec.padL;
    }
    return;
  }
  double epsU = 0.0, epsL = 0.0;
  if (!a.fp64) {
    if (a.layer == 0 && a.from_box) {
      // pre_radii's layer-0 radius on the stored values in the team's
      // registers (coefficient i on team lane i mod kL, slot i / kL), its
      // sums in the same order
      const int base = (int)(threadIdx.x & 63) & ~(kAffLanes - 1);
      auto stored = [&](int i) {
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < kR; ++r)
          if (r == i / kAffLanes) v = u[r];
        return __shfl(v, base + i % kAffLanes, 64);
      };
      const double *lo = a.box_lo + box * a.n, *hi = a.box_hi + box * a.n;
      const double *wj = a.W + (int64_t)j * a.n;
      double a0 = a.b[j], sabs = fabs(a.b[j]);
      for (int k = 0; k < a.n; ++k) {
        a0 = fma(wj[k], lo[k], a0);
        sabs += fabs(wj[k]) * (fabs(lo[k]) + fabs(hi[k] - lo[k]));
      }
      double rr = fabs(stored(0) - a0);
      for (int k = 0; k < a.n; ++k) {
        const double ak = wj[k] * (hi[k] - lo[k]);
        rr += fabs(stored(1 + k) - ak);  // coefficient of t_k
      }
      epsU = epsL = (rr + gamma64(a.n + 4) * sabs) * kPadSafety;
    } else if (a.layer == 0) {
      pre_radii(a, box, j, a.pre, 0, 1, [](double v) { return v; }, epsU, epsL);
    } else {
      double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // sU, sL, g, rU, rL
      for (int k = l; k < a.hin; k += kAffLanes) {
        const double wk = a.W[(int64_t)j * a.hin + k];
        const double4 P = *reinterpret_cast<const double4 *>(a.prad + (box * a.hin + k) * 4);
        if (wk >= 0.0) {
          v[0] += wk * P.x;
          v[1] += wk * P.y;
        } else {
          v[0] -= wk * P.y;
          v[1] -= wk * P.x;
        }
        v[2] += fabs(wk) * (P.z + P.w);
      }
      const double *rp = a.rpart + box * a.rpart_slot + (int64_t)j * 2 * a.cblocks;
      for (int64_t cb = l; cb < a.cblocks; cb += kAffLanes) {
        v[3] += rp[cb];
        v[4] += rp[a.cblocks + cb];
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) v[q] = aff_sum<kL>(v[q]);
      const double gg = a.gpre * (v[2] + fabs(a.b[j]));
      epsU = (v[0] + gg + v[3]) * kPadSafety;
      epsL = (v[1] + gg + v[4]) * kPadSafety;
    }
  }
  // l1 norms, extrema, fit constants: lane l's share of each sum
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // l1U, l1L, max U, min L, beta0 U, beta0 L
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    const int i = l + r * kAffLanes;
    s[0] += fabs(u[r]);
    s[1] += fabs(w[r]);
    const bool c0 = i == 0;
    s[2] += c0 ? u[r] : fmax(u[r], 0.0);
    s[3] += c0 ? w[r] : fmin(w[r], 0.0);
    s[4] += c0 ? u[r] : 0.5 * u[r];
    s[5] += c0 ? w[r] : 0.5 * w[r];
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) s[q] = aff_sum<kL>(s[q]);
  const double l1U = s[0], l1L = s[1];
  const double lo = side_lo(a, s[3], l1L, epsL), hi = side_hi(a, s[2], l1U, epsU);
  const bool want = wants_fit(a, box, j);
  const bool fitted = want && (a.fits || (lo < 0.0 && hi > 0.0));
  double fx[4] = {0.0, 0.0, 0.0, 0.0};  // rmaxU, rminU, rmaxL, rminL
  if (fitted) {
    // the remainder constant: a_0 - beta_0 + sum_a beta_a / 2
    double c[2] = {0.0, 0.0};
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const bool c0 = l + r * kAffLanes == 0;
      c[0] += c0 ? u[r] - s[4] : 0.5 * u[r];
      c[1] += c0 ? w[r] - s[5] : 0.5 * w[r];
    }
    c[0] = aff_sum<kL>(c[0]);
    c[1] = aff_sum<kL>(c[1]);
    fx[0] = fx[1] = c[0];
    fx[2] = fx[3] = c[1];
  }
  if (a.mode == 0 && fitted) {  // the fits: beta_0, then beta_a = a_{1+a}
    NeuronRec &rec = a.recs[box * a.h + j];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int q = l + r * kAffLanes;
      if (q <= kMaxInputs) {
        const bool on = q < S;
        rec.fitU[q] = on ? (q == 0 ? s[4] : u[r]) : 0.0;
        rec.fitL[q] = on ? (q == 0 ? s[5] : w[r]) : 0.0;
      }
    }
    // visible to lane 0, whose rule may read them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  // an unfitted neuron's fit fields are never read (fitted == 0)
  if (l == 0) write_neuron(a, box, j, lo, hi, epsU, epsL, l1U, l1L, fx, fitted, true);
}

// Executed-work counts of the read-off kernels, for the profiler (host).
// Coefficients of total degree t in nv variables: C(t + nv - 1, nv - 1).
static double count_at(int nv, int t) {
  if (nv == 0) return t == 0 ? 1.0 : 0.0;
  double c = 1.0;
  for (int i = 1; i < nv; ++i) c = c * (t + i) / i;
  return c;
}

// FP64 operations (an FMA counts 2, a min or max 1) of one tensor's tree
// read-off: the `fix` leading variables folded once per block ((D+1)^fix
// blocks, each with its own digits), the next q chain levels refolded as
// their round digits change, then per round (D+1)^q of them) e - 1
// expansions and (D+1)^e lanes, each folding its last variable (every parent
// coefficient once, ratios from LDS) and converting its (D+1)^M tile in
// registers, then a min and a max per Bernstein coefficient. A one-variable
// basis change with the compile-time ratio table costs D(D+1)/2 FMAs: its
// column j = 0 is all ones, so those products fold into the sums. The pass
// that adds the remainders of fitted neurons is not counted.
static double tree_ops(int n, int D, int M, int fix, int q, int e) {
  const double D1 = D + 1, T = 0.5 * D * (D + 1);
  // level i: folding variable i of an (n - i)-variable polynomial, summed
  // over the D + 1 digits; a child coefficient of total degree t takes
  // min(D - t, k) + 1 parents at digit k
  auto fold_all_digits = [&](int i) {
    double s = 0.0;
    for (int t = 0; t <= D; ++t) {
      double per = 0.0;
      for (int k = 0; k <= D; ++k) per += std::min(D - t, k) + 1;
      s += count_at(n - i - 1, t) * per;
    }
    return s;
  };
  double mac = 0.0;
  for (int i = 0; i < fix; ++i) mac += std::pow(D1, fix - 1) * fold_all_digits(i);
  double block = 0.0;
  for (int c = 0; c < q; ++c) block += std::pow(D1, c) * fold_all_digits(fix + c);
  double round = 0.0, V = 1.0;
  for (int st = 1; st < e; ++st) {
    const int d = n - fix - q - st + 1;
    round += V * (double)ssize(d - 1, D) * T;
    V *= D1;
  }
  const double lane = (double)ssize(M + 1, D) + M * std::pow(D1, M - 1) * T;
  round += std::pow(D1, e) * lane;
  mac += std::pow(D1, fix) * (block + std::pow(D1, q) * round);
  return 2.0 * mac + 2.0 * std::pow(D1, n);
}

// Bytes a hidden or output neuron's read-off must move: its two stored
// tensors, in FP32 mode the GEMM's rounding partials of its row, and what it
// writes (bounds and, for hidden neurons, the rule: kind, degree, interval,
// approximant, shift, radii and norms); per box the previous layer's radii.
static double readoff_neuron_bytes(const ConvertArgs &a) {
  double b = 2.0 * a.S * (a.fp64 ? 8 : 4) + 16.0;
  if (!a.fp64 && a.layer > 0) b += 2.0 * a.cblocks * 8;
  if (a.mode == 0) b += (a.L + 10) * 8.0;
  return b;
}
static double readoff_box_bytes(const ConvertArgs &a) { return (!a.fp64 && a.layer > 0) ? a.hin * 32.0 : 0.0; }

// Closed-form degree-1 read-off, per neuron: six sums over the n + 1
// coefficients of both tensors with their min / max / abs (about ten
// operations per coefficient), in FP32 mode after the first layer the
// radii's sums over the previous layer's neurons and the GEMM partials, and
// for the first layer formed from the box its coefficients.
static double affine_ops(const ConvertArgs &a) {
  double f = 10.0 * (a.n + 1);
  if (!a.fp64 && a.layer > 0) f += 5.0 * a.hin + 2.0 * a.cblocks;
  if (a.from_box) f += 4.0 * a.n;  // the coefficients formed from the box
  return f;
}

template <typename T>
static hipError_t launch_affine(const ConvertArgs &a, hipStream_t s) {
  ProfScope ps(a.mode == 2 ? kProfLin : kProfConvertSmall, s,
               a.nboxes * a.h * readoff_neuron_bytes(a) + a.nboxes * readoff_box_bytes(a),
               (double)a.nboxes * a.h * affine_ops(a));
  const int64_t teams = a.nboxes * a.h;
  if (a.S <= 8) {
    hipLaunchKernelGGL((convert_affine_kernel<T, 8>), dim3((unsigned)((teams * 8 + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL((convert_affine_kernel<T, 16>), dim3((unsigned)((teams * 16 + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

// Tensors beyond one block's LDS: the tree read-off. The basis change is a
// product over variables, so fixing the leading variable of a polynomial at
// Bernstein index k leaves the polynomial in the other variables
//   q_k(rest) = sum_j C(k, j) / C(D, j) p_j(rest)
// where p_j collects the terms with exponent j of the leading variable; its
// total degree stays <= D, so q_k is stored in the (d-1)-variable layout
// (the child table of simplex.hpp TreeTable gives the parent rank of every
// (j, rest)). Applying this to the leading n - M variables, one at a time,
// yields for every Bernstein index of those variables an M-variable
// polynomial whose own basis change gives exactly the Bernstein
// coefficients at that index; no dense tensor is formed.
//
// A block owns one tensor and the first lo leading indices (ko); it folds
// them once, then runs (D+1)^q rounds over the next q indices (a chain of
// single folds, refolded from the first changed index on), and in each round
// expands the following e-1 variables into all (D+1)^(e-1) index
// combinations in LDS; finally each lane folds the last one at its own index
// and converts its (D+1)^M tile in registers, tracking the extremum of the
// tensor's side. Every step applies one ratio per variable in a sum of at
// most D+1 terms, within the n(D+2) rounding steps of the per-axis change.
constexpr int tree_tile_axes(int D) { return D == 1 ? 5 : D == 2 ? 3 : D <= 5 ? 2 : 1; }

// Highest degree of the block-per-tensor tree read-off (the per-neuron
// kernels stop at 8; above, tensors no longer fit one block's LDS anyway).
constexpr int kTreeMaxDegree = 12;

constexpr int cpow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Calls f(std::integral_constant<int, I>) for I = B .. E-1, unrolled.
template <int B, int E>
struct Unroll {
  template <class F>
  __device__ static __forceinline__ void run(F &&f) {
    f(std::integral_constant<int, B>{});
    Unroll<B + 1, E>::run(f);
  }
};
template <int E>
struct Unroll<E, E> {
  template <class F>
  __device__ static __forceinline__ void run(F &&) {}
};

// The layout of NV variables of degree D (as simplex.hpp: graded by total
// degree, descending lexicographic within a degree) at compile time.
template <int D, int NV>
struct CSimplex {
  static constexpr int D1 = D + 1, dense = cpow(D + 1, NV), count = (int)binom_u(NV + D, D);
  int dense_of[count];  // dense index (variable 0 most significant) of each rank
  static constexpr int dsum(int v) {
    int s = 0;
    for (; v > 0; v /= D1) s += v % D1;
    return s;
  }
  constexpr CSimplex() : dense_of() {
    int r = 0;
    for (int t = 0; t <= D; ++t)
      for (int v = dense - 1; v >= 0; --v)
        if (dsum(v) == t) dense_of[r++] = v;
  }
  constexpr int rank_of(int v) const {
    for (int r = 0; r < count; ++r)
      if (dense_of[r] == v) return r;
    return -1;
  }
};

// The lane's last fold: for each coefficient c of its M-variable polynomial
// (dense tile index dl, degree budget deg = D - |c|) the parent ranks of
// (j, c), j = 0 .. deg, in the (M+1)-variable layout.
template <int D, int M>
struct LaneTab {
  static constexpr int NC = CSimplex<D, M>::count;
  int dl[NC], deg[NC], pr[NC][D + 1];
  constexpr LaneTab() : dl(), deg(), pr() {
    const CSimplex<D, M> cm{};
    const CSimplex<D, M + 1> cp{};
    for (int c = 0; c < NC; ++c) {
      dl[c] = cm.dense_of[c];
      deg[c] = D - CSimplex<D, M>::dsum(dl[c]);
      for (int j = 0; j <= D; ++j) pr[c][j] = j <= deg[c] ? cp.rank_of(j * cpow(D + 1, M) + dl[c]) : 0;
    }
  }
};
template <int D, int M>
struct LaneTabs {
  static constexpr LaneTab<D, M> t{};
};

// Basis change of an in-register block x (local index: its variables'
// digits, the first slowest) along each of its SZ variables.
template <int D, int SZ, int N>
__device__ __forceinline__ void block_to_bern(double (&x)[N]) {
  constexpr int D1 = D + 1;
  static_assert(cpow(D + 1, SZ) == N, "block size");
  Unroll<0, SZ>::run([&](auto Q) {
    constexpr int s = cpow(D + 1, SZ - 1 - Q.value);  // local stride of the variable
    Unroll<0, N / D1>::run([&](auto L) {
      constexpr int line = (L.value / s) * s * D1 + L.value % s;
      double y[D1];
#pragma unroll
      for (int j = 0; j < D1; ++j) y[j] = x[line + j * s];
      to_bern<D>(y);
#pragma unroll
      for (int j = 0; j < D1; ++j) x[line + j * s] = y[j];
    });
  });
}

// Lane stage: fold the parent's leading variable at the lane's index (ratio
// row rk), convert the M-variable tile, fold its extremum into ext.
template <int D, int M, bool kMax>
__device__ __forceinline__ void tree_lane(const double *par, const double (&rk)[D + 1], double &ext) {
  using LT = LaneTabs<D, M>;
  constexpr int N = cpow(D + 1, M);
  double x[N];
#pragma unroll
  for (int q = 0; q < N; ++q) x[q] = 0.0;
  Unroll<0, LaneTab<D, M>::NC>::run([&](auto C) {
    constexpr int c = C.value;
    double g = 0.0;
    Unroll<0, LT::t.deg[c] + 1>::run([&](auto J) { g = fma(rk[J.value], par[LT::t.pr[c][J.value]], g); });
    x[LT::t.dl[c]] = g;
  });
  block_to_bern<D, M>(x);
#pragma unroll
  for (int q = 0; q < N; ++q) ext = kMax ? fmax(ext, x[q]) : fmin(ext, x[q]);
}

// One fold of a single polynomial of d variables (in) at index k into the
// d-1 variables' layout (out, Sc coefficients); off: dimension d's offsets.
__device__ __forceinline__ void tree_fold(const double *in, double *out, const int *tb, const int *off, int Sc,
                                          const double *rk, int k, int tid, int nt) {
  for (int r = tid; r < Sc; r += nt) {
    const int b = off[r], cnt = min(off[r + 1] - b, k + 1);
    double s = 0.0;
    for (int j = 0; j < cnt; ++j) s = fma(rk[j], in[tb[b + j]], s);
    out[r] = s;
  }
}

// V polynomials of d variables (Sp coefficients each) into V (D+1) of d-1
// variables (Sc each): out variant v (D+1) + k is in variant v at index k.
// A thread takes one (v, r): the parents (j, r), j <= D - |r|, zero-padded
// to D+1 values, give all D+1 indices at once by the one-variable basis
// change.
template <int D>
__device__ __forceinline__ void tree_expand(const double *in, double *out, const int *tb, const int *off, int Sp,
                                            int Sc, int V, int tid, int nt) {
  constexpr int D1 = D + 1;
  const unsigned magic = Sc > 1 ? 0xFFFFFFFFu / (unsigned)Sc + 1u : 0u;
  const int total = V * Sc;
  for (int o = tid; o < total; o += nt) {
    const int v = Sc == 1 ? o : (int)__umulhi((unsigned)o, magic);
    const int r = o - v * Sc;
    const int b = off[r], cnt = off[r + 1] - b;
    const double *src = in + (int64_t)v * Sp;
    double x[D1];
#pragma unroll
    for (int j = 0; j < D1; ++j) x[j] = j < cnt ? src[tb[b + j]] : 0.0;
    to_bern<D>(x);
    double *dst = out + (int64_t)v * D1 * Sc + r;
#pragma unroll
    for (int k = 0; k < D1; ++k) dst[k * Sc] = x[k];
  }
}

struct TreePlan {
  int lo = -1, q = 0, e = 0;  // indices fixed per block, per round (chain), expanded per round
  int64_t nchunk = 0;         // (D+1)^lo blocks, and partials, per tensor
  int rounds = 0, lanes = 0, threads = 0;
  int S[kMaxInputs + 1] = {};  // S(d, D), d = 0 .. n
};

template <int D, int M, typename T>
__global__ void __launch_bounds__(1024) convert_tree_t(ConvertArgs a, TreePlan tp, double *partial,
                                                       double *l1part) {
  extern __shared__ double lds[];
  __shared__ double red[16];
  constexpr int D1 = D + 1;
  constexpr Ratio<D> R{};
  if ((int64_t)blockIdx.y >= launch_boxes(a) * a.h * 2) return;  // past a device count
  const int tid = threadIdx.x, nt = blockDim.x, n = a.n;
  const BlockTeam bt{tid, nt, red};
  // LDS: child tables (ints), ratio table, root, chain levels, expansions
  int *tb = reinterpret_cast<int *>(lds);
  for (int i = tid; i < a.tree_len; i += nt) tb[i] = a.tree[i];
  double *tab = lds + (a.tree_len + 1) / 2;
  double *chain = tab + D1 * D1;  // levels 1 .. lo + q
  int nchain = tp.lo + tp.q, cdim = n - nchain;
  int chain_size = 0;
  for (int i = 1; i <= nchain; ++i) chain_size += tp.S[n - i];
  // the stored coefficients: when the block fixes indices (lo >= 1) they are
  // read only by its first fold and share the expansions' area; otherwise
  // the rounds refold from them and they get their own
  double *root = chain + chain_size;
  double *expd = tp.lo >= 1 ? root : root + tp.S[n];  // expansions 1 .. e - 1
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < D1 * D1; ++i) tab[i] = R.v[i / D1][i % D1];
  }
  const int64_t tensor = blockIdx.y;
  const int side = (int)(tensor & 1);  // 1: lower bound tensor (minimum), 0: upper (maximum)
  const int64_t gb = tensor / (2 * a.h), rest = tensor % (2 * a.h);
  const int64_t box = a.bids ? a.bids[gb] : gb;
  const T *p = reinterpret_cast<const T *>(a.pre) + box * a.slot + rest * a.S;
  double l1 = 0.0;
  for (int i = tid; i < tp.S[n]; i += nt) {
    const double v = (double)p[i];
    root[i] = v;
    l1 += fabs(v);
  }
  if (blockIdx.x == 0) {
    l1 = bt.sum(l1);
    if (tid == 0) l1part[tensor] = l1;
  }
  __syncthreads();
  // level offsets of the chain: level i (1-based) at chain + cofs(i)
  auto level = [&](int i) -> double * {  // i = 0: root
    if (i == 0) return root;
    double *q = chain;
    for (int l = 1; l < i; ++l) q += tp.S[n - l];
    return q;
  };
  // the block's fixed indices
  for (int i = 0; i < tp.lo; ++i) {
    unsigned k = blockIdx.x;
    for (int s2 = tp.lo - 1; s2 > i; --s2) k /= D1;
    k %= D1;
    tree_fold(level(i), level(i + 1), tb, tb + a.tree_base[n - i], tp.S[n - i - 1], tab + k * D1, (int)k, tid, nt);
    __syncthreads();
  }
  // the lane's index and parent variant
  const int lane_k = tid % D1, pv = tid / D1;
  double rk[D1];
#pragma unroll
  for (int j = 0; j < D1; ++j) rk[j] = tab[lane_k * D1 + j];
  double ext = side ? INFINITY : -INFINITY;
  for (int rho = 0; rho < tp.rounds; ++rho) {
    // chain indices of the round (q digits, the first most significant);
    // refold from the first that changed
    int first = 0;
    if (rho > 0) {
      int a0 = rho, a1 = rho - 1;
      for (int i = tp.q - 1; i >= 0; --i) {
        if (a0 % D1 != a1 % D1) first = i;
        a0 /= D1;
        a1 /= D1;
      }
    }
    for (int i = first; i < tp.q; ++i) {
      int k = rho;
      for (int s2 = tp.q - 1; s2 > i; --s2) k /= D1;
      k %= D1;
      const int lv = tp.lo + i;
      tree_fold(level(lv), level(lv + 1), tb, tb + a.tree_base[n - lv], tp.S[n - lv - 1], tab + k * D1, k, tid,
                nt);
      __syncthreads();
    }
    // expansions into all index combinations of the next e - 1 variables
    const double *par = level(nchain);
    double *out = expd;
    int V = 1;
    for (int i = 1; i < tp.e; ++i) {
      const int d = cdim - i + 1;  // variables of the input
      tree_expand<D>(par, out, tb, tb + a.tree_base[d], tp.S[d], tp.S[d - 1], V, tid, nt);
      __syncthreads();
      par = out;
      out += (int64_t)V * D1 * tp.S[d - 1];
      V *= D1;
    }
    if (tid < tp.lanes) {
      const double *pp = par + (int64_t)pv * tp.S[M + 1];
      if (side)
        tree_lane<D, M, false>(pp, rk, ext);
      else
        tree_lane<D, M, true>(pp, rk, ext);
    }
    __syncthreads();
  }
  const double v = side ? bt.min(ext) : bt.max(ext);
  if (tid == 0) partial[tensor * tp.nchunk + blockIdx.x] = v;
}

template <typename T, int D>
static hipError_t launch_tree_t(const ConvertArgs &a, const TreePlan &tp, size_t lds, double *partial,
                                double *l1part, hipStream_t s) {
  constexpr int M = tree_tile_axes(D);
  RET_IF(hipFuncSetAttribute((const void *)convert_tree_t<D, M, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  hipLaunchKernelGGL((convert_tree_t<D, M, T>), dim3((unsigned)tp.nchunk, (unsigned)(a.nboxes * a.h * 2)),
                     dim3((unsigned)tp.threads), lds, s, a, tp, partial, l1part);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_tree(const ConvertArgs &a, const TreePlan &tp, size_t lds, double *partial, double *l1part,
                              hipStream_t s) {
  switch (a.D) {
    case 2: return launch_tree_t<T, 2>(a, tp, lds, partial, l1part, s);
    case 3: return launch_tree_t<T, 3>(a, tp, lds, partial, l1part, s);
    case 4: return launch_tree_t<T, 4>(a, tp, lds, partial, l1part, s);
    case 5: return launch_tree_t<T, 5>(a, tp, lds, partial, l1part, s);
    case 6: return launch_tree_t<T, 6>(a, tp, lds, partial, l1part, s);
    case 7: return launch_tree_t<T, 7>(a, tp, lds, partial, l1part, s);
    case 8: return launch_tree_t<T, 8>(a, tp, lds, partial, l1part, s);
    case 9: return launch_tree_t<T, 9>(a, tp, lds, partial, l1part, s);
    case 10: return launch_tree_t<T, 10>(a, tp, lds, partial, l1part, s);
    case 11: return launch_tree_t<T, 11>(a, tp, lds, partial, l1part, s);
    case 12: return launch_tree_t<T, 12>(a, tp, lds, partial, l1part, s);
    default: return hipErrorInvalidValue;
  }
}

// The tree read-off for one neuron's pair of tensors (all tensors within
// one block's reach): a block per neuron holds both trees, upper and lower,
// and lanes 0 .. lanes-1 take the upper tensor's tiles, the next lanes the
// lower's. A neuron that may take a fitted rule gets its affine fits
// (closed form, wave_fit) before the pass, which then tracks the remainders
// b_K - l(K/D) beside the extrema.
constexpr int ntree_tile_axes(int D) { return D == 1 ? 1 : D == 2 ? 3 : D <= 4 ? 2 : 1; }

struct NTreePlan {
  int e = 0, q = 0;  // variables expanded per round, folded per round (chain)
  int lanes = 0, threads = 0, rounds = 0;
  int sides = 2;     // trees per team: both bounds, or one (output layers: a block per bound)
  int area = 0;      // doubles of one tensor's tree: stored coefficients, chain, expansions
  int S[kMaxInputs + 1] = {};
};

// The lane's tile: folds the extrema of its Bernstein coefficients x into
// mn / mx and, with kFit, those of the remainders x - l into rmn / rmx, with
// l = c + sum over the tile's variables a of g[a] (digit/D - 1/2).
template <int D, int M, bool kFit>
__device__ __forceinline__ void ntree_lane(const double *par, const double (&rk)[D + 1], double c,
                                           const double (&g)[M], double &mn, double &mx, double &rmn,
                                           double &rmx) {
  using LT = LaneTabs<D, M>;
  constexpr int N = cpow(D + 1, M);
  double x[N];
#pragma unroll
  for (int q = 0; q < N; ++q) x[q] = 0.0;
  Unroll<0, LaneTab<D, M>::NC>::run([&](auto C) {
    constexpr int cc = C.value;
    double s = 0.0;
    Unroll<0, LT::t.deg[cc] + 1>::run([&](auto J) { s = fma(rk[J.value], par[LT::t.pr[cc][J.value]], s); });
    x[LT::t.dl[cc]] = s;
  });
  block_to_bern<D, M>(x);
  Unroll<0, N>::run([&](auto Q) {
    const double v = x[Q.value];
    mn = fmin(mn, v);
    mx = fmax(mx, v);
    if constexpr (kFit) {
      double l = c;
      Unroll<0, M>::run([&](auto A) {
        constexpr int t = (Q.value / cpow(D + 1, M - 1 - A.value)) % (D + 1);
        l = fma(g[A.value], (double)t / D - 0.5, l);
      });
      rmn = fmin(rmn, v - l);
      rmx = fmax(rmx, v - l);
    }
  });
}

// One pass over both trees (areas t0 and t0 + area); with kFit also the
// remainder extrema of the fits bl (upper, then lower).
template <int D, int M, bool kFit, class Team>
__device__ void ntree_pass(const ConvertArgs &a, const NTreePlan &tp, const Team &tm, const int *tb,
                           const double *tab, double *t0, const double *bl, double &mn, double &mx, double &rmn,
                           double &rmx) {
  constexpr int D1 = D + 1;
  const int tid = tm.tid, nt = tm.nt, n = a.n;
  const int side = tid / tp.lanes, tl = tid - side * tp.lanes;  // side 0: upper, 1: lower
  const bool lane = side < tp.sides;
  const int lane_k = tl % D1, pv = tl / D1;
  double rk[D1];
#pragma unroll
  for (int j = 0; j < D1; ++j) rk[j] = lane ? tab[lane_k * D1 + j] : 0.0;
  // the fit's tile part and the lane's own digits' part
  double g[M];  // the fit's slopes along the tile's variables
  double cl = 0.0;
  const double *beta = bl + (lane ? side : 0) * (kMaxInputs + 1);
  if (kFit) {
#pragma unroll
    for (int m = 0; m < M; ++m) g[m] = beta[1 + n - M + m];
    cl = beta[0];
    int rem = tl;
    for (int i = tp.e - 1; i >= 0; --i) {  // variable q + i has digit rem % D1
      cl = fma(beta[1 + tp.q + i], grid_c<D>(rem % D1), cl);
      rem /= D1;
    }
  } else {
#pragma unroll
    for (int m = 0; m < M; ++m) g[m] = 0.0;
  }
  // chain levels of a tree: level i (1 .. q) after the stored coefficients
  auto level = [&](double *root, int i) -> double * {
    double *q = root;
    for (int l = 0; l < i; ++l) q += tp.S[n - l];
    return q;
  };
  int chain_size = 0;
  for (int i = 0; i <= tp.q; ++i) chain_size += tp.S[n - i];
  for (int rho = 0; rho < tp.rounds; ++rho) {
    int first = 0;
    if (rho > 0) {
      int a0 = rho, a1 = rho - 1;
      for (int i = tp.q - 1; i >= 0; --i) {
        if (a0 % D1 != a1 % D1) first = i;
        a0 /= D1;
        a1 /= D1;
      }
    }
    double cr = cl;  // the round's chain digits' part of the fit
    if (kFit) {
      int rem = rho;
      for (int i = tp.q - 1; i >= 0; --i) {
        cr = fma(beta[1 + i], grid_c<D>(rem % D1), cr);
        rem /= D1;
      }
    }
    for (int i = first; i < tp.q; ++i) {
      int k = rho;
      for (int s2 = tp.q - 1; s2 > i; --s2) k /= D1;
      k %= D1;
      for (int sd = 0; sd < tp.sides; ++sd) {
        double *root = t0 + sd * tp.area;
        tree_fold(level(root, i), level(root, i + 1), tb, tb + a.tree_base[n - i], tp.S[n - i - 1], tab + k * D1, k,
                  tid, nt);
      }
      tm.sync();
    }
    const int cdim = n - tp.q;
    // expansions: step i reads the chain's last level (i = 1) or the
    // previous step's output
    {
      int Vx = 1;
      int64_t in_off = -1, out_off = chain_size;
      for (int i = 1; i < tp.e; ++i) {
        const int d = cdim - i + 1;
        for (int sd = 0; sd < tp.sides; ++sd) {
          double *root = t0 + sd * tp.area;
          const double *in = in_off < 0 ? level(root, tp.q) : root + in_off;
          tree_expand<D>(in, root + out_off, tb, tb + a.tree_base[d], tp.S[d], tp.S[d - 1], Vx, tid, nt);
        }
        tm.sync();
        in_off = out_off;
        out_off += (int64_t)Vx * D1 * tp.S[d - 1];
        Vx *= D1;
      }
      if (lane) {
        double *root = t0 + side * tp.area;
        const double *par = (in_off < 0 ? level(root, tp.q) : root + in_off) + (int64_t)pv * tp.S[M + 1];
        ntree_lane<D, M, kFit>(par, rk, cr, g, mn, mx, rmn, rmx);
      }
    }
    tm.sync();
  }
}

// One neuron's read-off by a team: a block (kWave false) or one wave of a
// block of four, each wave with its own neuron and LDS slice (kWave true).
// An output neuron's one bound (bside 0 upper, 1 lower) by a block with
// one tree (tp.sides == 1): its extremum, radius and output bound only.
// `pass(t0, mn, mx)` runs one pass over the tensor at t0 (the bound's
// extremum: mx for the upper tensor, mn for the lower).
template <typename T, class Team, class Pass>
__device__ void ntree_output_side(const ConvertArgs &a, const Team &tm, double *bl, int64_t item, int bside,
                                  Pass pass) {
  const int tid = tm.tid, nt = tm.nt, S = (int)a.S;
  double *t0 = bl + 2 * (kMaxInputs + 1);
  const int64_t box = a.bids ? a.bids[item / a.h] : item / a.h;
  const int j = (int)(item % a.h);
  const T *p = reinterpret_cast<const T *>(a.pre) + box * a.slot + ((int64_t)j * 2 + bside) * a.S;
  double l1[2] = {0.0, 0.0};
  for (int i = tid; i < S; i += nt) {
    const double v = (double)p[i];
    t0[i] = v;
    l1[bside] += fabs(v);
  }
  tm.sync();
  // the radii's first inputs past the barrier: they arrive while the pass runs
  RadiiIn ri;
  radii_prefetch(a, box, j, tid, ri);
  double mn = INFINITY, mx = -INFINITY;
  pass(t0, mn, mx);
  double epsU, epsL;
  radii_and_l1(a, box, j, tm, l1, epsU, epsL, &ri);
  double ex[2] = {mx, -mn};
  tm.reduce(ex, OpMax());
  if (tid != 0) return;
  const int64_t o = box * a.ld_out + a.col0 + j;
  if (bside == 0) {
    a.out_hi[o] = side_hi(a, ex[0], l1[0], epsU);
    if (a.out_eps) a.out_eps[(box * a.h + j) * 2 + 0] = epsU;
  } else {
    a.out_lo[o] = side_lo(a, -ex[1], l1[1], epsL);
    if (a.out_eps) a.out_eps[(box * a.h + j) * 2 + 1] = epsL;
  }
}

// `pass(F, t0, mn, mx, rmn, rmx)` runs one pass over both tensors (the
// upper at t0, the lower at t0 + tp.area; side = tid / tp.lanes) and, with
// F::value, tracks the remainders of the fits in bl.
template <int D, typename T, bool kWave, class Team, class Pass>
__device__ void ntree_neuron(const ConvertArgs &a, const NTreePlan &tp, const Team &tm, double *bl, int64_t item,
                             Pass pass) {
  const int tid = tm.tid, nt = tm.nt, n = a.n, S = (int)a.S;
  double *t0 = bl + 2 * (kMaxInputs + 1);
  const int64_t box = a.bids ? a.bids[item / a.h] : item / a.h;
  const int j = (int)(item % a.h);
  const T *p = reinterpret_cast<const T *>(a.pre) + box * a.slot + (int64_t)j * 2 * a.S;
  double l1[2] = {0.0, 0.0};
  for (int i = tid; i < S; i += nt) {
    const double uu = (double)p[i], ww = (double)p[S + i];
    t0[i] = uu;
    t0[tp.area + i] = ww;
    l1[0] += fabs(uu);
    l1[1] += fabs(ww);
  }
  tm.sync();
  // the radii's first inputs, loaded past the barrier (which waits for every
  // outstanding load) so that they arrive while the pass runs
  RadiiIn ri;
  radii_prefetch(a, box, j, tid, ri);
  const int side = tid / tp.lanes;
  // Affine fits (closed form from the stored coefficients) go to the
  // neurons that may take a fitted rule and turn out unstable, or to every
  // such neuron when all are fitted (a.fits): then first, with the remainder
  // ranges in the extrema's pass; else after the extrema, with a second pass
  // over the trees (their stored coefficients are kept) for the remainders.
  const bool want = wants_fit(a, box, j);
  const bool early = want && a.fits;
  auto fits = [&]() {
    if (kWave || threadIdx.x < 64) {
      double *scr = kWave ? tm_scratch(tm) : nullptr;
      wave_fit<D>(p, a.didx, S, n, (int)(threadIdx.x & 63), bl, scr);
      wave_fit<D>(p + S, a.didx, S, n, (int)(threadIdx.x & 63), bl + kMaxInputs + 1, scr);
    }
    tm.sync();
  };
  if (early) fits();
  double mn = INFINITY, mx = -INFINITY, rmn = INFINITY, rmx = -INFINITY;
  if (early)
    pass(std::true_type{}, t0, mn, mx, rmn, rmx);
  else
    pass(std::false_type{}, t0, mn, mx, rmn, rmx);
  // the radii after the pass: their loads arrive while it runs
  double epsU, epsL;
  radii_and_l1(a, box, j, tm, l1, epsU, epsL, &ri);
  const double l1U = l1[0], l1L = l1[1];
  // maxima of: max U, -min L, and the remainders' max U, -min U, max L, -min L
  double ex[6] = {side == 0 ? mx : -INFINITY, side == 1 ? -mn : -INFINITY, side == 0 ? rmx : -INFINITY,
                  side == 0 ? -rmn : -INFINITY, side == 1 ? rmx : -INFINITY, side == 1 ? -rmn : -INFINITY};
  tm.reduce(ex, OpMax());
  const double mxU = ex[0], mnL = -ex[1];
  const double lo = side_lo(a, mnL, l1L, epsL), hi = side_hi(a, mxU, l1U, epsU);
  const bool fitted = want && (a.fits || (lo < 0.0 && hi > 0.0));
  if (fitted && !early) {
    fits();
    double m0 = INFINITY, m1 = -INFINITY;
    rmn = INFINITY;
    rmx = -INFINITY;
    pass(std::true_type{}, t0, m0, m1, rmn, rmx);
    double rx[4] = {side == 0 ? rmx : -INFINITY, side == 0 ? -rmn : -INFINITY, side == 1 ? rmx : -INFINITY,
                    side == 1 ? -rmn : -INFINITY};
    tm.reduce(rx, OpMax());
    for (int q = 0; q < 4; ++q) ex[2 + q] = rx[q];
  }
  double fx[4] = {0.0, 0.0, 0.0, 0.0};  // rmaxU, rminU, rmaxL, rminL
  if (fitted) {
    fx[0] = ex[2];
    fx[1] = -ex[3];
    fx[2] = ex[4];
    fx[3] = -ex[5];
  }
  if (a.mode == 2) {
    if (tid == 0) write_lin(a, box, j, bl, bl + kMaxInputs + 1, fx, epsU, epsL, l1U, l1L);
    return;
  }
  if (a.mode == 0 && fitted) {  // the fits (an unfitted neuron's are never read)
    NeuronRec &rec = a.recs[box * a.h + j];
    team_write_fit(a, tm, rec.fitU, bl);
    team_write_fit(a, tm, rec.fitL, bl + kMaxInputs + 1);
  }
  if (tid == 0) write_neuron(a, box, j, lo, hi, epsU, epsL, l1U, l1L, fx, fitted, true);
}

// Wave teams per block of the one-wave-per-neuron form: one, so a neuron's
// wave is scheduled (and its LDS slice freed) on its own.
constexpr int kNTeams = 1;

template <int D, int M, typename T, bool kWave, bool kSide = false>
__global__ void __launch_bounds__(kWave ? 64 * kNTeams : 1024) convert_ntree_t(ConvertArgs a, NTreePlan tp) {
  extern __shared__ double lds[];
  __shared__ double red[kRedDoubles];
  constexpr int D1 = D + 1;
  constexpr Ratio<D> R{};
  {  // blocks past a device count leave before staging anything
    const int64_t items = launch_boxes(a) * a.h;
    const int64_t first = kWave ? (int64_t)blockIdx.x * (blockDim.x >> 6) : (int64_t)blockIdx.x;
    if (first >= (kSide ? 2 * items : items)) return;
  }
  int *tb = reinterpret_cast<int *>(lds);
  for (int i = threadIdx.x; i < a.tree_len; i += blockDim.x) tb[i] = a.tree[i];
  double *tab = lds + (a.tree_len + 1) / 2;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < D1 * D1; ++i) tab[i] = R.v[i / D1][i % D1];
  }
  __syncthreads();
  double *slices = tab + D1 * D1;  // per team: fits (upper, lower), then the two trees
  if (kWave) {
    const int wv = threadIdx.x >> 6;
    const int64_t item = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
    if (item >= launch_boxes(a) * a.h) return;
    double *slice = slices + (int64_t)wv * (kRowScratch + 2 * (kMaxInputs + 1) + 2 * tp.area);
    const WaveTeam tm{(int)(threadIdx.x & 63), slice};
    double *bl = slice + kRowScratch;
    ntree_neuron<D, T, true>(a, tp, tm, bl, item,
                             [&](auto F, double *t0, double &mn, double &mx, double &rmn, double &rmx) {
                               ntree_pass<D, M, decltype(F)::value>(a, tp, tm, tb, tab, t0, bl, mn, mx, rmn, rmx);
                             });
  } else {
    const BlockTeam tm{(int)threadIdx.x, (int)blockDim.x, red};
    if constexpr (kSide)
      ntree_output_side<T>(a, tm, slices, blockIdx.x >> 1, (int)(blockIdx.x & 1),
                           [&](double *t0, double &mn, double &mx) {
                             double rmn = INFINITY, rmx = -INFINITY;
                             ntree_pass<D, M, false>(a, tp, tm, tb, tab, t0, slices, mn, mx, rmn, rmx);
                           });
    else
      ntree_neuron<D, T, false>(a, tp, tm, slices, blockIdx.x,
                                [&](auto F, double *t0, double &mn, double &mx, double &rmn, double &rmx) {
                                  ntree_pass<D, M, decltype(F)::value>(a, tp, tm, tb, tab, t0, slices, mn, mx, rmn,
                                                                       rmx);
                                });
  }
}

// ------------------------------------------- quadratic tensors, one wave
// At per-variable degree 2 every stored monomial is 1, t_a, t_a^2 or
// t_a t_b, and the Bernstein coefficient at index K (Def. 2 at degree 2) is
//   b_K = sum_J a_J prod_a r(K_a, J_a),  r(k, 0) = 1, r(k, 1) = k/2,
//   r(k, 2) = [k = 2]
// (the ratios C(k,j)/C(2,j), exact in binary). A wave takes one neuron:
// lanes 0..31 the upper tensor, 32..63 the lower. Each lane fixes the
// digits of the first P variables (3^P <= 32 lanes per tensor), folds them
// out of the stored coefficients (each coefficient once, weighted by its
// prefix monomial's value at the lane's digits), then for each of the 3^R
// digit tuples of the next R variables folds those, and converts the
// remaining M-variable tile (M <= 2, which keeps the wave's registers, and
// so the waves per SIMD, in check) in registers. The stored coefficients are
// read as LDS broadcasts; the pass has no barrier. A box's neurons run on
// one XCD (xcd_item), sharing its radius inputs in one L2. Rounding: a Bernstein
// coefficient is a sum of at most S(P,2) + S(R,2) + 2M rounded terms of
// the |a_J| weighted by products of ratios in [0, 1], within the read-off's
// gamma(n (D + 2) + 4) l1 bound for every n here.
constexpr int qsize(int n) { return (n + 1) * (n + 2) / 2; }  // S(n, 2)

// Layout rank (simplex.hpp order) of the monomial t_u t_v (u <= v; -1 for
// an absent factor) among n variables: the constant, the n linear
// monomials, then t_u t_v in row order of the upper triangle.
constexpr int qrank(int n, int u, int v) {
  return u < 0 ? 0 : v < 0 ? 1 + u : 1 + n + u * n - u * (u - 1) / 2 + (v - u);
}

// The factors (u, v) of every rank of the n-variable degree-2 layout.
template <int N>
struct QuadMono {
  int u[qsize(N)], v[qsize(N)];
  constexpr QuadMono() : u(), v() {
    u[0] = v[0] = -1;
    for (int a = 0; a < N; ++a) {
      u[1 + a] = a;
      v[1 + a] = -1;
    }
    int r = 1 + N;
    for (int a = 0; a < N; ++a)
      for (int b = a; b < N; ++b) {
        u[r] = a;
        v[r] = b;
        ++r;
      }
  }
};

template <int N>
struct QuadMonos {
  static constexpr QuadMono<N> t{};
};

// Split of every rank of the N-variable layout into its monomial over the
// first P variables (rank in the P-variable layout) and over the other
// N - P (rank in that layout, variables renumbered from 0).
template <int N, int P>
struct QuadSplit {
  int pre[qsize(N)], rest[qsize(N)];
  constexpr QuadSplit() : pre(), rest() {
    const QuadMono<N> m{};
    for (int r = 0; r < qsize(N); ++r) {
      int f[2] = {m.u[r], m.v[r]}, pf[2] = {-1, -1}, rf[2] = {-1, -1}, np = 0, nr = 0;
      for (int i = 0; i < 2; ++i) {
        if (f[i] < 0) continue;
        if (f[i] < P)
          pf[np++] = f[i];
        else
          rf[nr++] = f[i] - P;
      }
      pre[r] = qrank(P, pf[0], pf[1]);
      rest[r] = qrank(N - P, rf[0], rf[1]);
    }
  }
};
template <int N, int P>
struct QuadSplits {
  static constexpr QuadSplit<N, P> t{};
};

// Dense tile position (digits, first variable slowest) of every rank of
// the M-variable layout.
template <int M>
struct QuadDense {
  int at[qsize(M)];
  constexpr QuadDense() : at() {
    const QuadMono<M> m{};
    for (int r = 0; r < qsize(M); ++r) {
      int d = 0;
      if (m.u[r] >= 0) d += cpow(3, M - 1 - m.u[r]);
      if (m.v[r] >= 0) d += cpow(3, M - 1 - m.v[r]);
      at[r] = d;
    }
  }
};
template <int M>
struct QuadDenses {
  static constexpr QuadDense<M> t{};
};

// Values of the K-variable layout's monomials at Bernstein digits k.
template <int K>
__device__ __forceinline__ void quad_weights(const int (&k)[K > 0 ? K : 1], double (&w)[qsize(K)]) {
  using QM = QuadMonos<K>;
  Unroll<0, qsize(K)>::run([&](auto R) {
    constexpr int r = R.value, u = QM::t.u[r], v = QM::t.v[r];
    if constexpr (u < 0) {
      w[r] = 1.0;
    } else if constexpr (v < 0) {
      w[r] = 0.5 * k[u];
    } else if constexpr (u == v) {
      w[r] = k[u] == 2 ? 1.0 : 0.0;
    } else {
      w[r] = (0.5 * k[u]) * (0.5 * k[v]);
    }
  });
}

template <int N>
struct QuadShape {
  static constexpr int P = N - 1 < 3 ? N - 1 : 3;          // lane variables
  static constexpr int M = N - P < 2 ? N - P : 2;          // tile variables
  static constexpr int R = N - P - M;                      // round variables
  static constexpr int lanes = cpow(3, P), rounds = cpow(3, R), tile = cpow(3, M);
};

// The degree-2 basis change of one fibre (y0, y1, y2) in place:
// b_0 = y0, b_1 = y0 + y1/2, b_2 = (y0 + y1) + y2, leaving out the entries
// that are structurally zero (kNz1, kNz2 false).
template <bool kNz1, bool kNz2>
__device__ __forceinline__ void to_bern2(double &y0, double &y1, double &y2) {
  double b1 = y0, b2 = y0;
  if constexpr (kNz1) {
    b1 = fma(0.5, y1, y0);
    b2 = y0 + y1;
  }
  if constexpr (kNz2) b2 = b2 + y2;
  y1 = b1;
  y2 = b2;
}

// Sum of the digits after axis a of dense tile position `pos` (M digits,
// the first slowest).
constexpr int tile_digits_after(int pos, int a, int M) {
  int s = 0;
  for (int b = a + 1; b < M; ++b) s += (pos / cpow(3, M - 1 - b)) % 3;
  return s;
}

// Basis change of a dense M-variable degree-2 tile whose entries of total
// degree above 2 are zero: axis by axis, an entry with digit t on the axis
// being converted can be nonzero only if t plus the digits of the axes not
// yet converted is at most 2, and such zeros are skipped.
template <int M>
__device__ __forceinline__ void tile_to_bern2(double (&x)[cpow(3, M)]) {
  Unroll<0, M>::run([&](auto A) {
    constexpr int s = cpow(3, M - 1 - A.value);
    Unroll<0, cpow(3, M) / 3>::run([&](auto L) {
      constexpr int line = (L.value / s) * s * 3 + L.value % s;
      constexpr int rest = tile_digits_after(line, A.value, M);
      to_bern2<1 + rest <= 2, 2 + rest <= 2>(x[line], x[line + s], x[line + 2 * s]);
    });
  });
}

// Value of monomial t_u t_v (layout factors; -1 absent) at Bernstein
// digits k of degree 2: 1, k_u/2, [k_u = 2] or k_u k_v / 4.
constexpr double quad_weight(int u, int v, const int *k) {
  return u < 0 ? 1.0 : v < 0 ? 0.5 * k[u] : u == v ? (k[u] == 2 ? 1.0 : 0.0) : 0.25 * k[u] * k[v];
}

// Fold of the R round variables at the digits of round `Rho` (first
// variable slowest) out of a polynomial over R + M variables: for each
// tile monomial t, the terms q (ascending) with a nonzero weight.
template <int R, int M, int Rho>
struct QuadRoundFold {
  int nt[qsize(M)], q[qsize(M)][qsize(R)];
  double w[qsize(M)][qsize(R)];
  int k[R > 0 ? R : 1];
  constexpr QuadRoundFold() : nt(), q(), w(), k() {
    int rem = Rho;
    for (int v = R - 1; v >= 0; --v) {
      k[v] = rem % 3;
      rem /= 3;
    }
    const QuadMono<R + M> m{};
    for (int r = 0; r < qsize(R + M); ++r) {
      int f[2] = {m.u[r], m.v[r]}, rf[2] = {-1, -1}, tf[2] = {-1, -1}, nr = 0, nm = 0;
      for (int i = 0; i < 2; ++i) {
        if (f[i] < 0) continue;
        if (f[i] < R)
          rf[nr++] = f[i];
        else
          tf[nm++] = f[i] - R;
      }
      const double wt = quad_weight(rf[0], rf[1], k);
      if (wt == 0.0) continue;
      const int t = qrank(M, tf[0], tf[1]);
      q[t][nt[t]] = r;
      w[t][nt[t]] = wt;
      ++nt[t];
    }
  }
};
template <int R, int M, int Rho>
struct QuadRoundFolds {
  static constexpr QuadRoundFold<R, M, Rho> t{};
};

// One pass over the lane's share of its tensor (`c`, the S(N,2) stored
// coefficients in LDS). Without kFit only the extremum the bound needs is
// kept: the maximum of the upper tensor (side 0) into mx, the minimum of
// the lower (side 1) into mn, both as a maximum over the lane's
// coefficients times +1 or -1 (the sign folded into the lane's weights,
// exact). With kFit, both extrema and those of the remainders
// b_K - l(K/2), l(x) = beta_0 + sum_a beta_a (x_a - 1/2), into rmn / rmx.
template <int N, bool kFit>
__device__ __forceinline__ void quad_pass(const double *c, const double *beta, int tl, int side, double &mn,
                                          double &mx, double &rmn, double &rmx) {
  using Q = QuadShape<N>;
  constexpr int P = Q::P, M = Q::M, R = Q::R, NT = Q::tile;
  constexpr int SRM = qsize(R + M), SM = qsize(M);
  using S1 = QuadSplits<N, P>;
  using QD = QuadDenses<M>;
  if (tl >= Q::lanes) return;
  int kp[P];
  {
    int rem = tl;
#pragma unroll
    for (int v = P - 1; v >= 0; --v) {
      kp[v] = rem % 3;
      rem /= 3;
    }
  }
  double wp[qsize(P)];
  quad_weights<P>(kp, wp);
  if constexpr (!kFit) {
    const double sgn = side ? -1.0 : 1.0;
#pragma unroll
    for (int q = 0; q < qsize(P); ++q) wp[q] *= sgn;
  }
  // fold the lane's variables: p1 over the other R + M variables
  double p1[SRM];
#pragma unroll
  for (int q = 0; q < SRM; ++q) p1[q] = 0.0;
  Unroll<0, qsize(N)>::run([&](auto Rk) {
    constexpr int r = Rk.value, q = S1::t.rest[r], w = S1::t.pre[r];
    p1[q] = fma(c[r], wp[w], p1[q]);
  });
  double cl = 0.0, g[M];
  if constexpr (kFit) {
    cl = beta[0];
#pragma unroll
    for (int v = 0; v < P; ++v) cl = fma(beta[1 + v], 0.5 * kp[v] - 0.5, cl);
#pragma unroll
    for (int m = 0; m < M; ++m) g[m] = beta[1 + P + R + m];
  }
  double best = -INFINITY;
  Unroll<0, Q::rounds>::run([&](auto Rho) {
    using F = QuadRoundFolds<R, M, Rho.value>;
    double x[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) x[i] = 0.0;
    Unroll<0, SM>::run([&](auto T) {
      constexpr int t = T.value;
      if constexpr (R == 0) {
        x[QD::t.at[t]] = p1[t];
      } else {
        constexpr int n0 = F::t.nt[t];
        static_assert(n0 >= 1, "every tile monomial keeps its round-constant term");
        constexpr double w0 = F::t.w[t][0];
        double acc = w0 == 1.0 ? p1[F::t.q[t][0]] : w0 * p1[F::t.q[t][0]];  // exact: w0 is a power of 2
        Unroll<1, n0>::run([&](auto I) {
          constexpr double wi = F::t.w[t][I.value];
          constexpr int qi = F::t.q[t][I.value];
          acc = wi == 1.0 ? acc + p1[qi] : fma(wi, p1[qi], acc);
        });
        x[QD::t.at[t]] = acc;
      }
    });
    tile_to_bern2<M>(x);
    if constexpr (!kFit) {
#pragma unroll
      for (int i = 0; i < NT; ++i) best = fmax(best, x[i]);
    } else {
      double cr = cl;
      Unroll<0, R>::run([&](auto V) {
        constexpr double gv = 0.5 * F::t.k[V.value] - 0.5;
        cr = fma(beta[1 + P + V.value], gv, cr);
      });
      Unroll<0, NT>::run([&](auto Qv) {
        const double v = x[Qv.value];
        mn = fmin(mn, v);
        mx = fmax(mx, v);
        double l = cr;
        Unroll<0, M>::run([&](auto A) {
          constexpr int t = (Qv.value / cpow(3, M - 1 - A.value)) % 3;
          l = fma(g[A.value], 0.5 * t - 0.5, l);
        });
        rmn = fmin(rmn, v - l);
        rmx = fmax(rmx, v - l);
      });
    }
  });
  if constexpr (!kFit) {
    if (side == 0)
      mx = fmax(mx, best);
    else
      mn = fmin(mn, -best);
  }
}

// LDS of the quadratic read-off: the wave's reduction scratch, the two
// fits, the two stored tensors.
constexpr size_t quad_lds(int n) { return (size_t)(kRowScratch + 2 * (kMaxInputs + 1) + 2 * qsize(n)) * sizeof(double); }

// Up to six inputs the kernel is held to six waves per SIMD (80 registers,
// a few spilled), which hides more of a neuron's load latency than five.
template <int N, typename T>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(N <= 6 ? 6 : 1)))
convert_quad_t(ConvertArgs a) {
  extern __shared__ double lds[];
  const int64_t item = xcd_item(blockIdx.x, a.h, launch_boxes(a));  // a box's neurons on one XCD
  if (item < 0) return;                                             // past the boxes (or a device count)
  const WaveTeam tm{(int)threadIdx.x, lds};
  double *bl = lds + kRowScratch;
  NTreePlan tp;  // what ntree_neuron reads of it: 32 lanes per tensor, the lower tensor's offset
  tp.lanes = 32;
  tp.area = qsize(N);
  const int tl = (int)(threadIdx.x & 31), side = (int)(threadIdx.x >> 5);
  ntree_neuron<2, T, true>(a, tp, tm, bl, item,
                           [&](auto F, double *t0, double &mn, double &mx, double &rmn, double &rmx) {
                             quad_pass<N, decltype(F)::value>(t0 + side * qsize(N), bl + side * (kMaxInputs + 1),
                                                              tl, side, mn, mx, rmn, rmx);
                           });
}

// --------------------------------- output tensors of degree 3 or 4, direct
// The same direct fold as the degree-2 read-off for an output neuron's
// bound tensor at degree D = 3 or 4 (one block per bound, as the tree's
// output form): each lane fixes the Bernstein digits of the first P
// variables ((D+1)^P <= 128 lanes), folds them out of the stored
// coefficients with the ratios C(k,j)/C(D,j) of its digits (prefix
// monomial by prefix monomial, each stored coefficient once), folds the next
// R variables per round at compile-time digits, and converts its M <= 2
// variable tile in registers, keeping only the bound's extremum.

// Exponents of the N-variable degree-D layout in rank order (simplex.hpp
// order: graded by total degree, descending lexicographic within one).
template <int D, int N>
struct DLayout {
  static constexpr int count = (int)binom_u(N + D, D);
  int e[count][N > 0 ? N : 1];
  constexpr DLayout() : e() {
    int r = 0;
    for (int t = 0; t <= D && N > 0; ++t) {
      int x[N > 0 ? N : 1] = {};
      x[0] = t;
      for (;;) {
        for (int a = 0; a < N; ++a) e[r][a] = x[a];
        ++r;
        int i = N - 2;  // the next tuple of the same degree, descending
        while (i >= 0 && x[i] == 0) --i;
        if (i < 0) break;
        int tail = 0;
        for (int b = i + 1; b < N; ++b) {
          tail += x[b];
          x[b] = 0;
        }
        --x[i];
        x[i + 1] = tail + 1;
      }
    }
  }
};
template <int D, int N>
struct DLayouts {
  static constexpr DLayout<D, N> t{};
};

// Layout rank of the exponents e[0..n) (any total degree).
constexpr int drank(int n, const int *e) {
  int d = 0;
  for (int i = 0; i < n; ++i) d += e[i];
  int r = d > 0 ? (int)binom_u(n + d - 1, n) : 0;  // every monomial of lower degree
  int rem = d;
  for (int i = 0; i + 1 < n; ++i) {
    const int m = n - 2 - i;
    for (int v = e[i] + 1; v <= rem; ++v) r += (int)binom_u(rem - v + m, m);
    rem -= e[i];
  }
  return r;
}

template <int D, int N>
struct DirectShape {
  static constexpr int D1 = D + 1;
  static constexpr int P = [] {
    int p = 1;
    while (p + 1 <= N - 1 && cpow(D + 1, p + 1) <= 128) ++p;
    return p;
  }();
  static constexpr int M = N - P < 2 ? N - P : 2;
  static constexpr int R = N - P - M;
  static constexpr int lanes = cpow(D1, P), rounds = cpow(D1, R), tile = cpow(D1, M);
  static constexpr int threads = (lanes + 63) / 64 * 64;
};

// Rank in the N-variable layout of (prefix monomial m of P variables, rest
// monomial q of N - P), -1 when the total degree exceeds D.
template <int D, int N, int P>
struct DJoin {
  static constexpr int SP = (int)binom_u(P + D, D), SQ = (int)binom_u(N - P + D, D);
  int r[SP][SQ];
  constexpr DJoin() : r() {
    const DLayout<D, P> lp{};
    const DLayout<D, N - P> lq{};
    for (int m = 0; m < SP; ++m)
      for (int q = 0; q < SQ; ++q) {
        int e[N] = {}, d = 0;
        for (int a = 0; a < P; ++a) d += e[a] = lp.e[m][a];
        for (int a = 0; a < N - P; ++a) d += e[P + a] = lq.e[q][a];
        r[m][q] = d <= D ? drank(N, e) : -1;
      }
  }
};
template <int D, int N, int P>
struct DJoins {
  static constexpr DJoin<D, N, P> t{};
};

// The round fold at compile-time digits: for each tile monomial t of M
// variables, the terms q of the (R+M)-variable polynomial with a nonzero
// weight prod_a C(k_a, e_a)/C(D, e_a) over the round variables, ascending q.
template <int D, int R, int M, int Rho>
struct DRoundFold {
  static constexpr int SRM = (int)binom_u(R + M + D, D), SM = (int)binom_u(M + D, D);
  int nt[SM], q[SM][SRM];
  double w[SM][SRM];
  int k[R > 0 ? R : 1];
  constexpr DRoundFold() : nt(), q(), w(), k() {
    const Ratio<D> rt{};
    int rem = Rho;
    for (int v = R - 1; v >= 0; --v) {
      k[v] = rem % (D + 1);
      rem /= (D + 1);
    }
    const DLayout<D, R + M> l{};
    for (int r = 0; r < SRM; ++r) {
      double wt = 1.0;
      for (int a = 0; a < R; ++a)
        if (l.e[r][a] > 0) wt = wt * rt.v[k[a]][l.e[r][a]];
      if (wt == 0.0) continue;
      int et[M > 0 ? M : 1] = {};
      for (int a = 0; a < M; ++a) et[a] = l.e[r][R + a];
      const int t = drank(M, et);
      q[t][nt[t]] = r;
      w[t][nt[t]] = wt;
      ++nt[t];
    }
  }
};
template <int D, int R, int M, int Rho>
struct DRoundFolds {
  static constexpr DRoundFold<D, R, M, Rho> t{};
};

// Dense tile position (digits, first variable slowest) of the rank-t
// monomial of the M-variable layout.
template <int D, int M>
struct DTilePos {
  static constexpr int SM = (int)binom_u(M + D, D);
  int at[SM];
  constexpr DTilePos() : at() {
    const DLayout<D, M> l{};
    for (int t = 0; t < SM; ++t) {
      int v = 0;
      for (int a = 0; a < M; ++a) v = v * (D + 1) + l.e[t][a];
      at[t] = v;
    }
  }
};
template <int D, int M>
struct DTilePoss {
  static constexpr DTilePos<D, M> t{};
};

// Sum of the digits (base b) after axis a of dense position `pos` (M digits,
// the first slowest).
constexpr int tile_digits_after_d(int pos, int a, int M, int b) {
  int s = 0;
  for (int c = a + 1; c < M; ++c) s += (pos / cpow(b, M - 1 - c)) % b;
  return s;
}

// Basis change of a dense M-variable degree-D tile whose entries of total
// degree above D are zero; along each axis the entries that can be nonzero
// (digit plus the digits of the axes not yet converted at most D) only.
template <int D, int M>
__device__ __forceinline__ void tile_to_bern(double (&x)[cpow(D + 1, M)]) {
  constexpr int D1 = D + 1;
  constexpr Ratio<D> rt{};
  Unroll<0, M>::run([&](auto A) {
    constexpr int st = cpow(D1, M - 1 - A.value);
    Unroll<0, cpow(D1, M) / D1>::run([&](auto L) {
      constexpr int line = (L.value / st) * st * D1 + L.value % st;
      constexpr int jmax = D - tile_digits_after_d(line, decltype(A)::value, M, D1);  // entries j > jmax are zero
      if constexpr (jmax >= 0) {
        double y[D1];
#pragma unroll
        for (int j = 0; j < D1; ++j) y[j] = x[line + j * st];
        Unroll<0, D1>::run([&](auto K) {
          constexpr int kk = D - K.value;  // descending k keeps y_j (j < k)
          double sacc = y[0];
          Unroll<1, (kk < jmax ? kk : jmax) + 1>::run([&](auto J) {
            constexpr double r = rt.v[kk][J.value];
            sacc = r == 1.0 ? sacc + y[J.value] : fma(r, y[J.value], sacc);
          });
          x[line + kk * st] = sacc;
        });
      }
    });
  });
}

// One bound's pass over its stored coefficients c (LDS), lanes < lanes
// active, the ratio table in LDS: the maximum of the upper tensor
// (bside 0) into mx, the minimum of the lower into mn.
template <int D, int N>
__device__ __forceinline__ void direct_side_pass(const double *c, const double *tab, int tid, int bside, double &mn,
                                                 double &mx) {
  using Q = DirectShape<D, N>;
  constexpr int D1 = D + 1, P = Q::P, M = Q::M, R = Q::R, NT = Q::tile;
  constexpr int SP = (int)binom_u(P + D, D), SRM = (int)binom_u(R + M + D, D), SM = (int)binom_u(M + D, D);
  using LP = DLayouts<D, P>;
  using J = DJoins<D, N, P>;
  using TP = DTilePoss<D, M>;
  if (tid >= Q::lanes) return;
  double rho[P][D1];  // the ratios of the lane's digits
  {
    int rem = tid;
#pragma unroll
    for (int v = P - 1; v >= 0; --v) {
      const int k = rem % D1;
      rem /= D1;
#pragma unroll
      for (int j = 0; j < D1; ++j) rho[v][j] = tab[k * D1 + j];
    }
  }
  const double sgn = bside ? -1.0 : 1.0;
  double p1[SRM];
#pragma unroll
  for (int q = 0; q < SRM; ++q) p1[q] = 0.0;
  Unroll<0, SP>::run([&](auto Mm) {
    constexpr int m = Mm.value;
    double w = sgn;
    Unroll<0, P>::run([&](auto A) {
      constexpr int e = LP::t.e[m][A.value];
      if constexpr (e > 0) w *= rho[A.value][e];
    });
    Unroll<0, SRM>::run([&](auto Qq) {
      constexpr int r = J::t.r[m][Qq.value];
      if constexpr (r >= 0) p1[Qq.value] = fma(c[r], w, p1[Qq.value]);
    });
  });
  double best = -INFINITY;
  Unroll<0, Q::rounds>::run([&](auto Rho) {
    using F = DRoundFolds<D, R, M, Rho.value>;
    double x[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) x[i] = 0.0;
    Unroll<0, SM>::run([&](auto T) {
      constexpr int t = T.value;
      if constexpr (R == 0) {
        x[TP::t.at[t]] = p1[t];
      } else {
        constexpr int n0 = F::t.nt[t];
        static_assert(n0 >= 1, "every tile monomial keeps its round-constant term");
        constexpr double w0 = F::t.w[t][0];
        double acc = w0 == 1.0 ? p1[F::t.q[t][0]] : w0 * p1[F::t.q[t][0]];
        Unroll<1, n0>::run([&](auto I) {
          constexpr double wi = F::t.w[t][I.value];
          constexpr int qi = F::t.q[t][I.value];
          acc = wi == 1.0 ? acc + p1[qi] : fma(wi, p1[qi], acc);
        });
        x[TP::t.at[t]] = acc;
      }
    });
    tile_to_bern<D, M>(x);
#pragma unroll
    for (int i = 0; i < NT; ++i) best = fmax(best, x[i]);
  });
  if (bside == 0)
    mx = fmax(mx, best);
  else
    mn = fmin(mn, -best);
}

// Rounding steps of the direct read-off beyond its terms' count: a prefix
// weight is a product of P rounded ratios (2P - 1 roundings), a round's
// weight one of R, and each tile axis adds one rounded ratio per term.
constexpr int direct_depth(int D, int N, int P, int R, int M) {
  return (int)binom_u(P + D, D) + 2 * P - 1 + (R > 0 ? (int)binom_u(R + D, D) + 2 * R - 1 : 0) + M * (D + 2);
}

template <int D, int N, typename T>
__global__ void __launch_bounds__(128) convert_direct_side_t(ConvertArgs a) {  // DirectShape::threads <= 128
  extern __shared__ double lds[];
  __shared__ double red[kRedDoubles];
  constexpr int D1 = D + 1;
  constexpr Ratio<D> Rt{};
  const int64_t item = blockIdx.x >> 1;
  if (item >= launch_boxes(a) * a.h) return;  // past a device count
  double *tab = lds;
  if (threadIdx.x < D1 * D1) tab[threadIdx.x] = Rt.v[threadIdx.x / D1][threadIdx.x % D1];
  __syncthreads();
  double *bl = tab + D1 * D1;  // the fits' space (unused here), then the tensor
  const BlockTeam tm{(int)threadIdx.x, (int)blockDim.x, red};
  const int bside = (int)(blockIdx.x & 1);
  ntree_output_side<T>(a, tm, bl, item, bside, [&](double *t0, double &mn, double &mx) {
    direct_side_pass<D, N>(t0, tab, (int)threadIdx.x, bside, mn, mx);
  });
}

static NTreePlan ntree_plan(int n, int D, int M, bool wave_team, int sides = 2);
static size_t ntree_lds(const NTreePlan &tp, int n, int D, int teams, bool wave);



template <typename T, int D, int M>
static bool launch_ntree(const ConvertArgs &a, hipStream_t s, bool wave_team, hipError_t &err) {
  const NTreePlan tp = ntree_plan(a.n, D, M, wave_team);
  if (tp.e < 1) return false;
  const int64_t items = a.nboxes * a.h;
  ProfScope ps(a.mode == 2 ? kProfLin : kProfConvertSmall, s,
               items * readoff_neuron_bytes(a) + a.nboxes * readoff_box_bytes(a),
               (double)items * 2 * tree_ops(a.n, D, M, 0, tp.q, tp.e));
  err = hipSuccess;
  if (tp.threads == 64) {  // a wave per neuron, kNTeams per block
    const size_t lds = ntree_lds(tp, a.n, D, kNTeams, true);
    if (lds <= device_lds_limit()) {
      err = hipFuncSetAttribute((const void *)convert_ntree_t<D, M, T, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (err != hipSuccess) return true;
      hipLaunchKernelGGL((convert_ntree_t<D, M, T, true>), dim3((unsigned)((items + kNTeams - 1) / kNTeams)),
                         dim3(64 * kNTeams), lds, s, a, tp);
      err = hipGetLastError();
      return true;
    }
  }
  if (a.mode == 1) {  // output neurons: a block per bound, one tree each
    const NTreePlan t1 = ntree_plan(a.n, D, M, false, 1);
    if (t1.e >= 1) {
      const size_t l1 = ntree_lds(t1, a.n, D, 1, false);
      err = hipFuncSetAttribute((const void *)convert_ntree_t<D, M, T, false, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)l1);
      if (err != hipSuccess) return true;
      hipLaunchKernelGGL((convert_ntree_t<D, M, T, false, true>), dim3((unsigned)(items * 2)), dim3((unsigned)t1.threads),
                         l1, s, a, t1);
      err = hipGetLastError();
      return true;
    }
  }
  const size_t lds = ntree_lds(tp, a.n, D, 1, false);
  err = hipFuncSetAttribute((const void *)convert_ntree_t<D, M, T, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  if (err != hipSuccess) return true;
  hipLaunchKernelGGL((convert_ntree_t<D, M, T, false>), dim3((unsigned)items), dim3((unsigned)tp.threads), lds, s, a,
                     tp);
  err = hipGetLastError();
  return true;
}

// The quadratic read-off's rank formula against the layout's own ranks,
// checked once per n (no allocation).
static bool quad_layout_ok(int n) {
  static std::atomic<int> known[kMaxInputs + 1];  // 0 unknown, 1 matches, -1 not
  if (n < 1 || n > kMaxInputs) return false;
  const int k = known[n].load(std::memory_order_relaxed);
  if (k != 0) return k > 0;
  bool good = true;
  for (int u = -1; u < n; ++u)
    for (int v = -1; v < n; ++v) {
      if ((u < 0 && v >= 0) || (v >= 0 && v < u)) continue;
      uint16_t e[kMaxInputs] = {};
      if (u >= 0) ++e[u];
      if (v >= 0) ++e[v];
      good = good && simplex_rank(n, e) == qrank(n, u, v);
    }
  known[n].store(good ? 1 : -1, std::memory_order_relaxed);
  return good;
}

// Executed FP64 operations of one neuron's quadratic read-off (both
// tensors): the lane fold (an FMA per stored coefficient), per round the
// round fold, the tile's basis change (6 FMAs per fibre and axis) and its
// extrema.
static double quad_ops(int n) {
  const int P = std::min(n - 1, 3), M = std::min(n - P, 2), R = n - P - M;
  double tile = 1, lanes = 1, rounds = 1;
  for (int i = 0; i < M; ++i) tile *= 3;
  for (int i = 0; i < P; ++i) lanes *= 3;
  for (int i = 0; i < R; ++i) rounds *= 3;
  const double round = (R > 0 ? 2.0 * qsize(R + M) : 0.0) + 12.0 * M * tile / 3 + 2.0 * tile;
  return 2.0 * lanes * (2.0 * qsize(n) + rounds * round);
}

template <typename T>
static bool launch_quad(const ConvertArgs &a, hipStream_t s, hipError_t &err) {
  if (a.n < 4 || a.n > 8 || a.S != qsize(a.n) || !quad_layout_ok(a.n)) return false;
  const int64_t items = a.nboxes * a.h;
  ProfScope ps(a.mode == 2 ? kProfLin : kProfConvertSmall, s,
               items * readoff_neuron_bytes(a) + a.nboxes * readoff_box_bytes(a), (double)items * quad_ops(a.n));
  const dim3 grid((unsigned)xcd_item_blocks(a.nboxes, a.h)), block(64);
  const size_t lds = quad_lds(a.n);
  switch (a.n) {
    case 4: hipLaunchKernelGGL((convert_quad_t<4, T>), grid, block, lds, s, a); break;
    case 5: hipLaunchKernelGGL((convert_quad_t<5, T>), grid, block, lds, s, a); break;
    case 6: hipLaunchKernelGGL((convert_quad_t<6, T>), grid, block, lds, s, a); break;
    case 7: hipLaunchKernelGGL((convert_quad_t<7, T>), grid, block, lds, s, a); break;
    default: hipLaunchKernelGGL((convert_quad_t<8, T>), grid, block, lds, s, a); break;
  }
  err = hipGetLastError();
  return true;
}

// Executed FP64 operations of one bound's direct read-off at degree D.
static double direct_side_ops(int D, int n, int P, int R, int M) {
  double lanes = 1, rounds = 1, tile = 1;
  for (int i = 0; i < P; ++i) lanes *= D + 1;
  for (int i = 0; i < R; ++i) rounds *= D + 1;
  for (int i = 0; i < M; ++i) tile *= D + 1;
  const double per_round = 2.0 * (double)ssize(R + M, D) + M * tile * (D + 2) + tile;
  return lanes * (2.0 * (double)ssize(n, D) + 2.0 * (double)ssize(P, D) + rounds * per_round);
}

template <typename T, int D, int N>
static void launch_direct_side_n(const ConvertArgs &a, hipStream_t s) {
  using Q = DirectShape<D, N>;
  const size_t lds = ((D + 1) * (D + 1) + 2 * (kMaxInputs + 1) + ssize(N, D)) * sizeof(double);
  hipLaunchKernelGGL((convert_direct_side_t<D, N, T>), dim3((unsigned)(a.nboxes * a.h * 2)), dim3(Q::threads), lds, s,
                     a);
}

// Output layers at degree 3 or 4 with 5 or 6 inputs: a block per bound.
template <typename T, int D>
static bool launch_direct_side(const ConvertArgs &a_in, hipStream_t s, hipError_t &err) {
  if (a_in.mode != 1 || a_in.n < 5 || a_in.n > 6 || a_in.S != ssize(a_in.n, D)) return false;
  ConvertArgs a = a_in;
  int P = 1;
  while (P + 1 <= a.n - 1 && ipow(D + 1, P + 1) <= 128) ++P;
  const int M = std::min(a.n - P, 2), R = a.n - P - M;
  // the read-off pad covers this kernel's rounding steps
  a.gconv = gamma64(std::max((double)a.n * (D + 2) + 4, (double)direct_depth(D, a.n, P, R, M)) + a.gextra);
  const int64_t items = a.nboxes * a.h;
  ProfScope ps(kProfConvertSmall, s, items * readoff_neuron_bytes(a) + a.nboxes * readoff_box_bytes(a),
               (double)items * direct_side_ops(D, a.n, P, R, M));
  if (a.n == 5)
    launch_direct_side_n<T, D, 5>(a, s);
  else
    launch_direct_side_n<T, D, 6>(a, s);
  err = hipGetLastError();
  return true;
}

template <typename T, int D>
static hipError_t launch_convert_t(const ConvertArgs &a, hipStream_t s) {
  // degree 1 tensors are read off in closed form, whatever n; the tree needs
  // D >= 2 to pay for its levels
  if constexpr (D == 1) {
    return launch_affine<T>(a, s);
  } else {
    if constexpr (D == 2) {  // quadratic tensors: the direct one-wave form unless tuned away
      hipError_t err = hipSuccess;
      if (a.tune.conv_wave == 0 && launch_quad<T>(a, s, err)) return err;
    }
    if constexpr (D == 3 || D == 4) {  // output bounds: the direct form unless tuned away
      hipError_t err = hipSuccess;
      if (a.tune.conv_wave == 0 && launch_direct_side<T, D>(a, s, err)) return err;
    }
    if (a.tree) {
      hipError_t err = hipSuccess;
      if (a.tune.conv_wave == 0 && launch_ntree<T, D, ntree_tile_axes(D)>(a, s, false, err)) return err;
      if (a.tune.conv_wave == 3 && launch_ntree<T, D, ntree_tile_axes(D)>(a, s, true, err)) return err;
    }
    const size_t plb = (size_t)((a.plist_len + 1) / 2) * sizeof(double);
    if (a.C <= kWaveC && a.tune.conv_wave <= 1) {
      const size_t lds = (size_t)(kBlock / 64) * wave_slice_doubles((int)a.C) * sizeof(double) + plb;
      RET_IF(hipFuncSetAttribute((const void *)convert_wave_t<D, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
      ProfScope ps(kProfConvertSmall, s, (double)a.nboxes * a.h * 2 * a.S * (a.fp64 ? 8 : 4),
                   (double)a.nboxes * a.h * 2 * a.n * a.C * (a.D + 2));
      const int64_t items = a.nboxes * a.h;
      hipLaunchKernelGGL((convert_wave_t<D, T>), dim3((unsigned)((items + kBlock / 64 - 1) / (kBlock / 64))),
                         dim3(kBlock), lds, s, a);
      return hipGetLastError();
    }
    const size_t lds = (size_t)(a.C + 2 * (kMaxInputs + 1)) * sizeof(double) + plb;
    if (lds + 256 > device_lds_limit()) return hipErrorInvalidValue;
    RET_IF(hipFuncSetAttribute((const void *)convert_block_t<D, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    // a block per neuron; when few blocks share a CU's LDS, more waves each
    static const unsigned kThreads[4] = {0, 256, 512, 1024};
    const unsigned threads = a.tune.conv_block > 0 && a.tune.conv_block < 4 ? kThreads[a.tune.conv_block]
                                                                            : (lds > 40 * 1024 ? 1024 : 256);
    ProfScope ps(kProfConvertSmall, s, (double)a.nboxes * a.h * 2 * a.S * (a.fp64 ? 8 : 4),
                 (double)a.nboxes * a.h * 2 * a.n * a.C * (a.D + 2));
    hipLaunchKernelGGL((convert_block_t<D, T>), dim3((unsigned)(a.nboxes * a.h)), dim3(threads), lds, s, a);
    return hipGetLastError();
  }
}

template <typename T>
static hipError_t launch_convert_fixed(const ConvertArgs &a, hipStream_t s) {
  switch (a.D) {
    case 1: return launch_convert_t<T, 1>(a, s);
    case 2: return launch_convert_t<T, 2>(a, s);
    case 3: return launch_convert_t<T, 3>(a, s);
    case 4: return launch_convert_t<T, 4>(a, s);
    case 5: return launch_convert_t<T, 5>(a, s);
    case 6: return launch_convert_t<T, 6>(a, s);
    case 7: return launch_convert_t<T, 7>(a, s);
    case 8: return launch_convert_t<T, 8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------- two-pass path
struct Split {
  int m;         // trailing axes converted in pass A
  int64_t Ci;    // (D+1)^m
  int64_t Co;    // (D+1)^(n-m)
  int64_t Q;     // inner columns per pass-B tile
  int64_t nchunk;
};

// FP64 elements of one staged tile: the smaller of kTileLds and what the
// device lets one block hold next to the basis-change table.
static int64_t tile_elems(int D) {
  const int64_t fit = (int64_t)(device_lds_limit() / sizeof(double)) - (int64_t)(D + 1) * (D + 1) - 64;
  return std::min<int64_t>(kTileLds, fit);
}

static Split make_split(int n, int D) {
  Split s{};
  const int64_t tile = tile_elems(D);
  s.m = 0;
  s.Ci = 1;
  while (s.m < n && s.Ci * (D + 1) <= tile) { s.Ci *= (D + 1); ++s.m; }
  s.Co = ipow(D + 1, n - s.m);
  s.Q = tile / (s.Co > 0 ? s.Co : 1);
  int64_t q = 1;
  while (q * 2 <= s.Q) q *= 2;
  s.Q = q < 1 ? 1 : q;
  if (s.Q > s.Ci) s.Q = s.Ci;
  s.nchunk = (s.Ci + s.Q - 1) / s.Q;
  return s;
}

// Pass A: one block per (tensor, outer slice): convert the m trailing axes.
template <typename T>
__global__ void __launch_bounds__(kBlock) convert_passA_kernel(ConvertArgs a, Split sp, double *l1part) {
  extern __shared__ double lds[];
  const int D1 = a.D + 1;
  double *t = lds;
  double *tab = lds + sp.Ci;
  const int64_t tensor = blockIdx.y;  // (box*h + j)*2 + s
  if (tensor >= launch_boxes(a) * a.h * 2) return;
  const int64_t o = blockIdx.x;
  fill_table(tab, a.D);
  double *red = tab + D1 * D1;
  const int64_t gb = tensor / (2 * a.h), rest = tensor % (2 * a.h);
  const int64_t box = a.bids ? a.bids[gb] : gb;
  const T *p = reinterpret_cast<const T *>(a.pre) + box * a.slot + rest * a.S;
  for (int64_t i = threadIdx.x; i < sp.Ci; i += blockDim.x) t[i] = 0.0;
  __syncthreads();
  // the stored coefficients whose leading (outer) digits are those of slice o
  double l1 = 0.0;
  for (int64_t i = threadIdx.x; i < a.S; i += blockDim.x) {
    const int64_t d = a.didx[i];
    if (d / sp.Ci == o) {
      const double v = (double)p[i];
      t[d - o * sp.Ci] = v;
      l1 += fabs(v);
    }
  }
  l1 = block_reduce(l1, OpAdd(), red);
  lds_basis_change(t, sp.Ci, sp.m, a.D, 0, sp.m, tab);
  double *q = a.scratch + tensor * a.C + o * sp.Ci;
  for (int64_t i = threadIdx.x; i < sp.Ci; i += blockDim.x) q[i] = t[i];
  if (threadIdx.x == 0) l1part[tensor * sp.Co + o] = l1;
}

// Pass B: one block per (tensor, column chunk): convert the n-m leading axes
// of a [Co][Q] tile and reduce it to one extremum (min for lower bounds,
// max for upper bounds) written to the partials area.
__global__ void __launch_bounds__(kBlock) convert_passB_kernel(ConvertArgs a, Split sp, double *partial) {
  extern __shared__ double lds[];
  const int D1 = a.D + 1;
  double *t = lds;                      // [Co][Q]
  double *tab = lds + sp.Co * sp.Q;
  double *red = tab + D1 * D1;
  const int64_t tensor = blockIdx.y;
  if (tensor >= launch_boxes(a) * a.h * 2) return;
  const int s = (int)(tensor & 1);
  const int64_t q0 = (int64_t)blockIdx.x * sp.Q;
  const int64_t qn = min(sp.Q, sp.Ci - q0);
  fill_table(tab, a.D);
  const double *src = a.scratch + tensor * a.C;
  for (int64_t i = threadIdx.x; i < sp.Co * sp.Q; i += blockDim.x) {
    const int64_t o = i / sp.Q, q = i % sp.Q;
    t[i] = (q < qn) ? src[o * sp.Ci + q0 + q] : 0.0;
  }
  __syncthreads();
  // leading axes of the [Co] part; the Q columns are the fastest index.
  const int nl = a.n - sp.m;
  int64_t stride = sp.Q;
  for (int ax = nl - 1; ax >= 0; --ax) {
    const int64_t fibres = sp.Co * sp.Q / D1;
    for (int64_t f = threadIdx.x; f < fibres; f += blockDim.x) {
      const int64_t base = (f / stride) * stride * D1 + (f % stride);
      for (int k = a.D; k >= 0; --k) {
        double acc = 0.0;
        for (int jj = 0; jj <= k; ++jj) acc = fma(tab[k * D1 + jj], t[base + (int64_t)jj * stride], acc);
        t[base + (int64_t)k * stride] = acc;
      }
    }
    __syncthreads();
    stride *= D1;
  }
  double v = s ? INFINITY : -INFINITY;
  for (int64_t i = threadIdx.x; i < sp.Co * sp.Q; i += blockDim.x) {
    if (i % sp.Q < qn) v = s ? fmin(v, t[i]) : fmax(v, t[i]);
  }
  v = s ? block_reduce(v, OpMin(), red) : block_reduce(v, OpMax(), red);
  if (threadIdx.x == 0) partial[tensor * sp.nchunk + blockIdx.x] = v;
}

// Fold the per-chunk extrema of both bounds of one neuron: one wave each.
__global__ void __launch_bounds__(kBlock) convert_final_kernel(ConvertArgs a, Split sp, const double *partial,
                                                               const double *l1part) {
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (item >= launch_boxes(a) * a.h) return;
  const int64_t box = a.bids ? a.bids[item / a.h] : item / a.h;
  const int j = (int)(item % a.h);
  double mn = INFINITY, mx = -INFINITY, l1U = 0.0, l1L = 0.0;
  for (int64_t c = lane; c < sp.nchunk; c += 64) {
    mn = fmin(mn, partial[(item * 2 + 1) * sp.nchunk + c]);
    mx = fmax(mx, partial[(item * 2 + 0) * sp.nchunk + c]);
  }
  for (int64_t o = lane; o < sp.Co; o += 64) {
    l1U += l1part[(item * 2 + 0) * sp.Co + o];
    l1L += l1part[(item * 2 + 1) * sp.Co + o];
  }
  mn = wave_reduce(mn, OpMin());
  mx = wave_reduce(mx, OpMax());
  l1U = wave_reduce(l1U, OpAdd());
  l1L = wave_reduce(l1L, OpAdd());
  double lo, hi, epsU, epsL;
  padded_bounds(a, box, j, mn, mx, l1L, l1U, lane, 64, [](double v) { return wave_reduce(v, OpAdd()); }, lo, hi,
                epsU, epsL);
  if (lane != 0) return;
  if (a.mode == 1) {
    write_output(a, box, j, lo, hi, epsU, epsL);
  } else {
    if (a.out_lo) a.out_lo[box * a.ld_out + a.col0 + j] = lo;
    if (a.out_hi) a.out_hi[box * a.ld_out + a.col0 + j] = hi;
    finish_neuron(a, box, j, lo, hi, epsU, epsL, l1U, l1L, nullptr, nullptr, false);
  }
}

static bool use_small(int64_t C) {
  const int64_t fit = (int64_t)(device_lds_limit() / sizeof(double)) - 17 * 17 - 64;
  return C <= kSmallLds && C <= fit;
}


// Ints of the tree table of n variables and degree D.
static int64_t tree_ints(int n, int D) {
  int64_t t = 0;
  for (int d = 2; d <= n; ++d) t += ssize(d - 1, D) + 1 + ssize(d, D);
  return t;
}

// LDS of a plan: tables, ratio table, chain levels, the stored coefficients
// and the expansions (sharing one area when lo >= 1).
static size_t tree_lds(const TreePlan &tp, int n, int D) {
  const int D1 = D + 1;
  int64_t dbl = (tree_ints(n, D) + 1) / 2 + D1 * D1, ex = 0;
  for (int i = 1; i <= tp.lo + tp.q; ++i) dbl += tp.S[n - i];
  int64_t V = 1;
  for (int i = 1; i < tp.e; ++i) {
    V *= D1;
    ex += V * tp.S[n - tp.lo - tp.q - i];
  }
  return (size_t)(dbl + (tp.lo >= 1 ? std::max<int64_t>(ex, tp.S[n]) : ex + tp.S[n])) * sizeof(double);
}

// Blocks the tree read-off aims for (some 32 per CU); the partials stay
// within tensors + kTreeBlocks (D+1).
constexpr int64_t kTreeBlocks = 8192;

// Plan of the tree read-off: lanes per round (D+1)^e, the count that fills
// whole waves best (the smaller of equals), then the fewest block-fixed
// indices giving kTreeBlocks blocks, the rest folded per round. e shrinks
// until the levels fit LDS. lo < 0 when the path does not apply.
static TreePlan tree_plan(int n, int D, int64_t tensors) {
  TreePlan none;
  if (D < 1 || D > kTreeMaxDegree || n < 2 || n > kMaxInputs) return none;
  const int M = tree_tile_axes(D), D1 = D + 1, lead = n - M;
  if (lead < 1 || ssize(n, D, (int64_t)1 << 24) < 0) return none;
  TreePlan tp;
  for (int d = 0; d <= n; ++d) tp.S[d] = (int)ssize(d, D);
  // e: the most busy lanes per CU (blocks resident by LDS, at most 32
  // waves), counting blocks beyond four waves at half (their barriers wait
  // on more waves), the smaller e of equals
  TreePlan best;
  double best_score = 0.0;
  for (int e = 1; e <= lead; ++e) {
    const int64_t lanes = ipow(D1, e);
    if (lanes > 1024) break;
    TreePlan c = tp;
    c.e = e;
    c.lanes = (int)lanes;
    c.threads = (int)std::max<int64_t>(64, (lanes + 63) / 64 * 64);
    c.lo = 0;
    while (c.lo < lead - e && tensors * ipow(D1, c.lo) < kTreeBlocks) ++c.lo;
    c.q = lead - e - c.lo;
    c.rounds = (int)ipow(D1, c.q);
    c.nchunk = ipow(D1, c.lo);
    const size_t lds = tree_lds(c, n, D);
    if (lds > device_lds_limit()) continue;
    const int64_t wpb = c.threads / 64;
    const int64_t blocks = std::min<int64_t>(device_lds_limit() / lds, 32 / wpb);
    const double score = (double)(blocks * lanes) * (wpb > 4 ? 0.5 : 1.0);
    if (blocks >= 1 && score > best_score * 1.05) {
      best_score = score;
      best = c;
    }
  }
  return best;
}

// Plan of the neuron tree: e the most variables with 2 (D+1)^e lanes in one
// block (one wave with wave_team), the rest folded per round; e shrinks
// until both trees fit LDS.
static NTreePlan ntree_plan(int n, int D, int M, bool wave_team, int sides) {
  NTreePlan none;
  if (D < 1 || D > 8 || n > kMaxInputs) return none;
  const int D1 = D + 1, lead = n - M;
  if (lead < 1) return none;
  NTreePlan tp;
  tp.sides = sides;
  for (int d = 0; d <= n; ++d) tp.S[d] = (int)ssize(d, D);
  // one tree per block: the same expansion as with two, half the block
  const int64_t max_lanes = wave_team ? 64 : (sides == 1 ? 512 : 1024);
  int e = 0;
  while (e < lead && sides * ipow(D1, e + 1) <= max_lanes) ++e;
  for (; e >= 1; --e) {
    tp.e = e;
    tp.q = lead - e;
    tp.lanes = (int)ipow(D1, e);
    tp.threads = std::max(64, (sides * tp.lanes + 63) / 64 * 64);
    tp.rounds = (int)ipow(D1, tp.q);
    int64_t area = 0;
    for (int i = 0; i <= tp.q; ++i) area += tp.S[n - i];
    int64_t V = 1;
    for (int i = 1; i < e; ++i) {
      V *= D1;
      area += V * tp.S[n - tp.q - i];
    }
    tp.area = (int)area;
    const size_t lds =
        (size_t)((tree_ints(n, D) + 1) / 2 + D1 * D1 + 2 * (kMaxInputs + 1) + sides * area) * sizeof(double);
    if (lds <= device_lds_limit()) return tp;
  }
  return none;
}

static size_t ntree_lds(const NTreePlan &tp, int n, int D, int teams, bool wave) {
  // wave teams also hold their reduction scratch
  return (size_t)((tree_ints(n, D) + 1) / 2 + (D + 1) * (D + 1) +
                  (int64_t)teams * ((wave ? kRowScratch : 0) + 2 * (kMaxInputs + 1) + (int64_t)tp.sides * tp.area)) *
         sizeof(double);
}

bool convert_tree(int n, int D) {
  if (D == 1) return false;  // read off at the corners
  const int64_t C = tsize(n, D);
  if (C < 0 || use_small(C)) return false;
  return tree_plan(n, D, 1).lo >= 0;
}

size_t convert_scratch_bytes(int n, int D, int h, int64_t nboxes) {
  const int64_t C = ipow(D + 1, n);
  if (D == 1 || use_small(C)) return 0;
  if (tree_plan(n, D, nboxes * h * 2).lo >= 0)
    return align256(((size_t)nboxes * h * 2 + kTreeBlocks * (D + 1)) * sizeof(double)) +
           align256((size_t)nboxes * h * 2 * sizeof(double));
  const Split sp = make_split(n, D);
  return align256((size_t)nboxes * h * 2 * C * sizeof(double)) +
         align256((size_t)nboxes * h * 2 * sp.nchunk * sizeof(double)) +
         align256((size_t)nboxes * h * 2 * sp.Co * sizeof(double));
}

// One block per (box, output neuron, bound): zero the dense tensor, then
// place the stored coefficients at their dense positions (rank 0, the
// constant, widened by the tensor's radius in FP32 mode and rounded
// outward, so the polynomial stays a bound).
template <typename T>
__global__ void __launch_bounds__(kBlock) out_polys_kernel(OutPolyArgs a) {
  const int64_t item = blockIdx.x;
  const int side = (int)(item & 1);
  const int64_t gj = item >> 1, g = gj / a.h;
  const int j = (int)(gj - g * a.h);
  const int64_t box = a.bids ? a.bids[g] : g;
  double *dst = (side == 0 ? a.U : a.L) + (box * a.h + j) * a.C;
  for (int64_t i = threadIdx.x; i < a.C; i += blockDim.x) dst[i] = 0.0;
  __syncthreads();
  const T *src = reinterpret_cast<const T *>(a.pre) + box * a.slot + ((int64_t)j * 2 + side) * a.S;
  for (int64_t r = threadIdx.x; r < a.S; r += blockDim.x) {
    double v = (double)src[r];
    if (r == 0 && a.eps) {
      const double e = a.eps[(box * a.h + j) * 2 + side];
      v = side == 0 ? round_up(v + e) : round_down(v - e);
    }
    dst[a.didx[r]] = v;
  }
}

hipError_t launch_out_polys(const OutPolyArgs &a, hipStream_t s) {
  if (a.nboxes < 1) return hipSuccess;
  if (a.S > a.C || !a.didx || !a.U || !a.L) return hipErrorInvalidValue;
  const int64_t blocks = a.nboxes * a.h * 2;
  if (a.fp64)
    hipLaunchKernelGGL(out_polys_kernel<double>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(out_polys_kernel<float>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

bool convert_one_block(int n, int D) {
  if (D == 1) return true;
  const int64_t C = tsize(n, D);
  return D >= 2 && D <= 8 && C >= 0 && (C <= kWaveC || use_small(C));
}

hipError_t launch_convert(const ConvertArgs &a_in, hipStream_t s) {
  // the rounding factors the kernels apply, once per launch
  ConvertArgs a = a_in;
  a.gconv = gamma64((double)a.n * (a.D + 2) + 4 + a.gextra);
  a.gpre = gamma64(2.0 * a.hin + 6);
  const int D1 = a.D + 1;
  if (a.mode == 2) {  // linearisation: the kernels that fit every neuron
    if (!convert_one_block(a.n, a.D) || (a.D >= 2 && !a.didx)) return hipErrorInvalidValue;
    a.fits = 1;
    a.used = nullptr;
    a.out_lo = a.out_hi = nullptr;
    if (a.tune.conv_wave == 1 || a.tune.conv_wave == 2) {
      // the dense variants need the wave kernel's reach or a block's LDS
      if (a.tune.conv_wave == 1 && a.C > kWaveC) a.tune.conv_wave = 2;
    } else if (!a.tree && a.D >= 2) {
      a.tune.conv_wave = a.C <= kWaveC ? 1 : 2;
    }
    return a.fp64 ? launch_convert_fixed<double>(a, s) : launch_convert_fixed<float>(a, s);
  }
  if (a.D == 1 || (a.D >= 2 && a.D <= 8 && ((a.C <= kWaveC && a.tune.conv_wave == 0) || use_small(a.C))))
    return a.fp64 ? launch_convert_fixed<double>(a, s) : launch_convert_fixed<float>(a, s);
  if (a.C <= kWaveC) {
    const size_t lds = (D1 * D1 + (kBlock / 64) * 2 * a.C) * sizeof(double);
    auto k = a.fp64 ? convert_wave_kernel<double> : convert_wave_kernel<float>;
    RET_IF(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ProfScope ps(kProfConvertSmall, s, (double)a.nboxes * a.h * 2 * a.S * (a.fp64 ? 8 : 4),
                 (double)a.nboxes * a.h * 2 * a.n * a.C * (a.D + 2));
    const int64_t items = a.nboxes * a.h;
    hipLaunchKernelGGL(k, dim3((unsigned)((items + kBlock / 64 - 1) / (kBlock / 64))), dim3(kBlock), lds, s, a);
    return hipGetLastError();
  }
  if (use_small(a.C)) {
    const size_t lds = (a.C + D1 * D1 + 16) * sizeof(double);
    auto k = a.fp64 ? convert_small_kernel<double> : convert_small_kernel<float>;
    RET_IF(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ProfScope ps(kProfConvertSmall, s, (double)a.nboxes * a.h * 2 * a.S * (a.fp64 ? 8 : 4),
                 (double)a.nboxes * a.h * 2 * a.n * a.C * (a.D + 2));
    hipLaunchKernelGGL(k, dim3((unsigned)(a.nboxes * a.h)), dim3(kBlock), lds, s, a);
    return hipGetLastError();
  }
  const int64_t tensors = a.nboxes * a.h * 2;
  const TreePlan tp = tree_plan(a.n, a.D, tensors);
  if (tp.lo >= 0) {  // the workspace holds no staging for this shape
    if (!a.tree || a.tree_len != (int)tree_ints(a.n, a.D) || tensors * tp.nchunk > tensors + kTreeBlocks * (a.D + 1))
      return hipErrorInvalidValue;
    const size_t lds = tree_lds(tp, a.n, a.D);
    ConvertArgs b = a;
    b.gextra = 0;  // one ratio per variable and step: within the per-axis count
    b.gconv = gamma64((double)b.n * (b.D + 2) + 4);
    double *partial = a.scratch;
    double *l1part = reinterpret_cast<double *>(
        reinterpret_cast<char *>(partial) +
        align256(((size_t)a.nboxes * a.h * 2 + kTreeBlocks * (a.D + 1)) * sizeof(double)));
    {
      ProfScope ps(kProfConvertChunk, s,
                   (double)(a.nboxes * a.h) * readoff_neuron_bytes(a) + a.nboxes * readoff_box_bytes(a),
                   (double)tensors * tree_ops(a.n, a.D, tree_tile_axes(a.D), tp.lo, tp.q, tp.e));
      RET_IF(a.fp64 ? launch_tree<double>(b, tp, lds, partial, l1part, s)
                    : launch_tree<float>(b, tp, lds, partial, l1part, s));
    }
    Split fsp{};
    fsp.nchunk = tp.nchunk;
    fsp.Co = 1;
    ProfScope ps(kProfConvertFinal, s, (double)tensors * tp.nchunk * 8);
    hipLaunchKernelGGL(convert_final_kernel, dim3((unsigned)((a.nboxes * a.h + 3) / 4)), dim3(kBlock), 0, s, b, fsp,
                       (const double *)partial, (const double *)l1part);
    return hipGetLastError();
  }
  const Split sp = make_split(a.n, a.D);
  if (sp.Co > tile_elems(a.D)) return hipErrorInvalidValue;
  double *partial = reinterpret_cast<double *>(reinterpret_cast<char *>(a.scratch) +
                                               align256((size_t)a.nboxes * a.h * 2 * a.C * sizeof(double)));
  double *l1part = reinterpret_cast<double *>(reinterpret_cast<char *>(partial) +
                                              align256((size_t)a.nboxes * a.h * 2 * sp.nchunk * sizeof(double)));
  {
    const size_t lds = (sp.Ci + D1 * D1 + 16) * sizeof(double);
    auto k = a.fp64 ? convert_passA_kernel<double> : convert_passA_kernel<float>;
    RET_IF(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ProfScope ps(kProfConvertPassA, s, (double)tensors * (a.S * (a.fp64 ? 8 : 4) + a.C * 8));
    hipLaunchKernelGGL(k, dim3((unsigned)sp.Co, (unsigned)tensors), dim3(kBlock), lds, s, a, sp, l1part);
  }
  {
    const size_t lds = (sp.Co * sp.Q + D1 * D1 + 16) * sizeof(double);
    RET_IF(hipFuncSetAttribute((const void *)convert_passB_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ProfScope ps(kProfConvertPassB, s, (double)tensors * a.C * 8);
    hipLaunchKernelGGL(convert_passB_kernel, dim3((unsigned)sp.nchunk, (unsigned)tensors), dim3(kBlock), lds, s, a,
                       sp, partial);
  }
  {
    ProfScope ps(kProfConvertFinal, s, (double)tensors * sp.nchunk * 8);
    hipLaunchKernelGGL(convert_final_kernel, dim3((unsigned)((a.nboxes * a.h + 3) / 4)), dim3(kBlock), 0, s, a, sp,
                       (const double *)partial, (const double *)l1part);
  }
  return hipGetLastError();
}

// ------------------------------------------------- step-level primitives

// Basis change of `count` independent tensors: Bernstein coefficients (if
// requested), min, max and sum of |power coefficients|; one block per tensor.
template <typename T>
__global__ void __launch_bounds__(kBlock) basis_minmax_kernel(int n, int D, int64_t C, const T *coef, double *bern,
                                                              double *mn, double *mx, double *l1) {
  extern __shared__ double lds[];
  const int D1 = D + 1;
  double *t = lds;
  double *tab = lds + C;
  double *red = tab + D1 * D1;
  const int64_t item = blockIdx.x;
  fill_table(tab, D);
  double s1 = 0.0;
  for (int64_t i = threadIdx.x; i < C; i += blockDim.x) {
    t[i] = (double)coef[item * C + i];
    s1 += fabs(t[i]);
  }
  __syncthreads();
  lds_basis_change(t, C, n, D, 0, n, tab);
  double vmin = INFINITY, vmax = -INFINITY;
  for (int64_t i = threadIdx.x; i < C; i += blockDim.x) {
    vmin = fmin(vmin, t[i]);
    vmax = fmax(vmax, t[i]);
    if (bern) bern[item * C + i] = t[i];
  }
  vmin = block_reduce(vmin, OpMin(), red);
  vmax = block_reduce(vmax, OpMax(), red);
  s1 = block_reduce(s1, OpAdd(), red);
  if (threadIdx.x == 0) {
    mn[item] = vmin;
    mx[item] = vmax;
    if (l1) l1[item] = s1;
  }
}

size_t basis_minmax_scratch(int, int, int64_t) { return 0; }

hipError_t launch_basis_minmax(int n, int D, int64_t count, const void *coef, int fp64, double *bern, double *mn,
                               double *mx, double *l1, double *, hipStream_t s) {
  const int64_t C = ipow(D + 1, n);
  if (!use_small(C)) return hipErrorInvalidValue;
  const int D1 = D + 1;
  const size_t lds = (C + D1 * D1 + 16) * sizeof(double);
  if (fp64) {
    RET_IF(hipFuncSetAttribute((const void *)basis_minmax_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds));
    hipLaunchKernelGGL(basis_minmax_kernel<double>, dim3((unsigned)count), dim3(kBlock), lds, s, n, D, C,
                       (const double *)coef, bern, mn, mx, l1);
  } else {
    RET_IF(hipFuncSetAttribute((const void *)basis_minmax_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds));
    hipLaunchKernelGGL(basis_minmax_kernel<float>, dim3((unsigned)count), dim3(kBlock), lds, s, n, D, C,
                       (const float *)coef, bern, mn, mx, l1);
  }
  return hipGetLastError();
}

__global__ void relu_poly_kernel(int64_t count, int L, const double *lo, const double *hi, double *c, double *e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double cc[kMaxOrder + 1], ee;
  relu_poly_dev(lo[i], hi[i], L, cc, &ee);
  for (int k = 0; k <= L; ++k) c[i * (L + 1) + k] = cc[k];
  e[i] = ee;
}

hipError_t launch_relu_poly(int64_t count, int L, const double *lo, const double *hi, double *c, double *e,
                            hipStream_t s) {
  hipLaunchKernelGGL(relu_poly_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, L, lo, hi, c,
                     e);
  return hipGetLastError();
}

}  // namespace bern
