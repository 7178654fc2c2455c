// Per-neuron rule of Step 2 (device-side, shared by the read-off kernels and
// the predictor's kernels): the ReLU over-approximant's power series and the
// choice of rule for stable / unstable neurons.
#pragma once

#include "common.hpp"

namespace bern {

__device__ inline double binom_d(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  if (k > n - k) k = n - k;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
  return rint(r);
}

// ReLU over-approximant on [lo, hi] (lo < 0 < hi) of order L: power
// coefficients c[0..L] in u and e = value at y = 0.
__device__ inline void relu_poly_dev(double lo, double hi, int L, double *c, double *e) {
  double d[kMaxOrder + 1];
#pragma unroll
  for (int k = 0; k <= kMaxOrder; ++k) {
    const double y = lo + (hi - lo) * (double)k / (double)L;
    d[k] = (k <= L) ? fmax(y, 0.0) : 0.0;
  }
#pragma unroll
  for (int j = 1; j <= kMaxOrder; ++j) {
#pragma unroll
    for (int k = kMaxOrder; k >= j; --k)
      if (j <= L && k <= L) d[k] -= d[k - 1];
  }
#pragma unroll
  for (int j = 0; j <= kMaxOrder; ++j) c[j] = (j <= L) ? binom_d(L, j) * d[j] : 0.0;
  const double u0 = -lo / (hi - lo);
  double v = 0.0;
#pragma unroll
  for (int j = kMaxOrder; j >= 0; --j)
    if (j <= L) v = fma(v, u0, c[j]);
  *e = v;
}

// Rule of one hidden neuron (thread-level). The fallback needs the affine fits
// of the record; without them (tensors converted in two passes) code 0 is
// taken as order 1, the same relaxation before its linearisation.
__device__ inline void decide_neuron(NeuronRec &r, int code, bool uniform, int L, int n, int D, int cap, int fp64) {
  const double lo = r.lo, hi = r.hi;
  if (!uniform) {
    // keep every tensor within the plain form's size: code * D <= cap
    if (code > kMaxOrder) code = kMaxOrder;
    while (code > 1 && code * D > cap) --code;
    if (code < 1 && !r.fitted) code = 1;
  } else {
    code = L;
  }
  int kind, deg;
  if (!(hi > 0.0)) { kind = kInactive; deg = 0; }     // hi <= 0 (also NaN) -> zero polynomial
  else if (lo >= 0.0) { kind = kActive; deg = D; }
  else if (code >= 1) { kind = code; deg = code * D; }
  else { kind = kFallback; deg = 1; }
  if (uniform) deg = L * D;  // plain rule: uniform degree per layer
  r.kind = kind;
  r.deg = deg;
  r.padU = r.padL = r.pl1U = r.pl1L = 0.0;
  r.fbpadU = r.fbpadL = 0.0;
  r.dB = 0.0;
#pragma unroll
  for (int k = 0; k <= kMaxOrder; ++k) r.c[k] = 0.0;
  r.e = 0.0;
  const double mag = fabs(lo) + fabs(hi);
  if (kind >= 1) {
    relu_poly_dev(lo, hi, kind, r.c, &r.e);
    if (!fp64) {
      double sc = 0.0;
      for (int k = 0; k <= kind; ++k) sc += fabs(r.c[k]);
      double p3 = 1.0;
      for (int k = 0; k < kind; ++k) p3 *= 3.0;
      r.dB = mag * (gamma64(4) + gamma64(kind + 2) * p3);
      r.e = round_up(r.e + r.dB + gamma64(2.0 * kind + 2) * sc + (hi - lo) * gamma64(3));
    }
  }
  if (kind == kFallback) {
    // degree-1 approximant: upper lambda (U^ - lo), lower lambda L^ (with the
    // radii folded in), each replaced by its least-squares affine fit plus
    // the extreme remainder (largest for the upper, smallest for the lower).
    const double lam = hi / (hi - lo);
    const double *fitU = r.fitU, *fitL = r.fitL;
    const double extU = r.rmaxU, extL = r.rminL;
    double sU = 0.0, sL = 0.0, aU = fabs(fitU[0]), aL = fabs(fitL[0]);
    for (int ax = 0; ax < n; ++ax) {
      sU += fitU[1 + ax];
      sL += fitL[1 + ax];
      aU += fabs(fitU[1 + ax]);
      aL += fabs(fitL[1 + ax]);
    }
    r.fbU[0] = lam * (fitU[0] - lo - 0.5 * sU + extU + r.epsU);
    r.fbL[0] = lam * (fitL[0] - 0.5 * sL + extL - r.epsL);
    for (int ax = 0; ax < n; ++ax) {
      r.fbU[1 + ax] = lam * fitU[1 + ax];
      r.fbL[1 + ax] = lam * fitL[1 + ax];
    }
    if (!fp64) {
      const double g = gamma64((double)n * (D + 2) + 4);
      const double ge = gamma64(n + 8);
      r.fbpadU = lam * (g * r.l1U + ge * (aU + fabs(extU) + fabs(lo) + r.epsU)) + gamma64(4) * lam * (mag + hi - lo);
      r.fbpadL = lam * (g * r.l1L + ge * (aL + fabs(extL) + r.epsL)) + gamma64(4) * lam * (mag + hi - lo);
    }
  }
}

}  // namespace bern
