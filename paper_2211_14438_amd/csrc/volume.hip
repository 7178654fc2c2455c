// Relative volume of the output set (Section 6): the integral over the input
// box of the upper minus the lower output polynomial, divided by the box's
// volume. With the polynomials in t in [0,1]^n (x = lo + t (hi - lo)), that
// is their mean over the unit cube, and the mean of t^k is
// prod_a 1 / (k_a + 1): a weighted sum of the stored power coefficients.
#include "volume.hpp"

namespace bern {

constexpr int kVolWaves = 4;  // waves per block, one (box, output) each

template <typename T>
__global__ void __launch_bounds__(64 * kVolWaves) rel_volume_kernel(OutPolyArgs a, int n, int D, double *vol) {
  const int lane = (int)(threadIdx.x & 63);
  const int64_t item = (int64_t)blockIdx.x * kVolWaves + (threadIdx.x >> 6);
  if (item >= a.nboxes * a.h) return;  // uniform over the wave
  const int64_t g = item / a.h;
  const int j = (int)(item - g * a.h);
  const int64_t box = a.bids ? a.bids[g] : g;
  const T *up = reinterpret_cast<const T *>(a.pre) + box * a.slot + (int64_t)j * 2 * a.S;
  const T *lw = up + a.S;
  const int D1 = D + 1;
  double s = 0.0;
  for (int64_t r = lane; r < a.S; r += 64) {
    int v = a.didx[r];
    double den = 1.0;  // prod (k_a + 1) <= (D+1)^n: an exact integer
    for (int q = 0; q < n; ++q) {
      den *= (double)(v % D1 + 1);
      v /= D1;
    }
    s += ((double)up[r] - (double)lw[r]) / den;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) {
    const int64_t o = box * a.h + j;
    if (a.eps) s += a.eps[o * 2] + a.eps[o * 2 + 1];
    vol[o] = s;
  }
}

hipError_t launch_rel_volume(const OutPolyArgs &a, int n, int D, double *vol, hipStream_t s) {
  if (a.nboxes < 1) return hipSuccess;
  if (!a.didx || !vol || n < 1 || D < 0 || a.S < 1) return hipErrorInvalidValue;
  const int64_t items = a.nboxes * a.h;
  const unsigned blocks = (unsigned)((items + kVolWaves - 1) / kVolWaves);
  if (a.fp64)
    hipLaunchKernelGGL(rel_volume_kernel<double>, dim3(blocks), dim3(64 * kVolWaves), 0, s, a, n, D, vol);
  else
    hipLaunchKernelGGL(rel_volume_kernel<float>, dim3(blocks), dim3(64 * kVolWaves), 0, s, a, n, D, vol);
  return hipGetLastError();
}

}  // namespace bern
