// Affine steps of the hot path on gfx950.
//
//  * layer-1 pre-activation in closed form (Section 5.3 input initialisation
//    followed by eqs. upper/lower_bounds_layer): with x_a = d_lo_a + w_a t_a the
//    pre-activation W x + b is affine in t: the constant b + W d_lo and the
//    coefficient W_ja w_a of t_a, ranks 0 and 1 + a of the total-degree
//    layout (simplex.hpp) at degree 1; upper = lower.
//  * interval affine map of a hidden/output layer (eqs. upper_bounds_layer,
//    lower_bounds_layer): U^ = W+ U + W- L + b, L^ = W+ L + W- U + b, computed
//    in midpoint-radius form U^, L^ = W M +- |W| R + b with M = (U+L)/2 and
//    R = (U-L)/2 (equal in exact arithmetic, half the multiply-adds). In the
//    power basis the bias only touches the constant coefficient.
//
// Layout: tensors [box][neuron][bound 0=upper,1=lower][coefficient], the
// coefficients in the total-degree layout of simplex.hpp.
#include "common.hpp"

namespace bern {

template <typename T>
__global__ void __launch_bounds__(kBlock) layer1_kernel(Layer1Args a) {
  const int64_t C = a.n + 1;  // total-degree layout at degree 1: constant, then t_1 .. t_n
  const int64_t total = a.nboxes * a.h * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = i % C;
    const int64_t bj = i / C;  // launch box * h + j
    const int j = (int)(bj % a.h);
    const int64_t box = a.bids ? a.bids[bj / a.h] : bj / a.h;
    const double *lo = a.box_lo + box * a.n;
    const double *hi = a.box_hi + box * a.n;
    const double *w = a.W + (int64_t)j * a.n;
    double v;
    if (c == 0) {
      v = a.b[j];
      for (int k = 0; k < a.n; ++k) v = fma(w[k], lo[k], v);
    } else {
      const int axis = (int)c - 1;
      v = w[axis] * (hi[axis] - lo[axis]);
    }
    T *out = reinterpret_cast<T *>(a.pre) + box * a.slot + (int64_t)j * 2 * C;
    out[c] = (T)v;
    out[C + c] = (T)v;
  }
}

hipError_t launch_layer1(const Layer1Args &a, hipStream_t s) {
  const int64_t total = a.nboxes * a.h * (int64_t)(a.n + 1);
  const int64_t blocks = (total + kBlock - 1) / kBlock;
  const unsigned grid = (unsigned)std::min<int64_t>(blocks, 65536);
  ProfScope ps(kProfLayer1, s, (double)total * 2 * (a.fp64 ? 8 : 4));
  if (a.fp64)
    hipLaunchKernelGGL(layer1_kernel<double>, dim3(grid), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(layer1_kernel<float>, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// Multiply-adds of the inputs in `list` (count entries) into the MB
// accumulator pairs: X points at the thread's coefficient of input 0's upper
// tensor, input k's tensors sit at k*st (upper) and k*st + C (lower). `on`
// false makes every value an exact zero (loads stay in bounds). KU inputs
// per step, the next step's loads issued before this step's multiply-adds.
template <typename T, int MB, int KU>
__device__ __forceinline__ void gemm_rows(const T *X, int64_t st, int64_t C, const int *list, int count, bool on,
                                          const double *wt, int hp, double (&accM)[MB], double (&accR)[MB]) {
  int k = 0;
  T u[KU], l[KU];
  if (KU <= count) {
#pragma unroll
    for (int q = 0; q < KU; ++q) {
      const int64_t r = (int64_t)list[q] * st;
      u[q] = X[r];
      l[q] = X[r + C];
    }
  }
  for (; k + KU <= count; k += KU) {
    T un[KU], ln[KU];
    const bool more = k + 2 * KU <= count;
    if (more) {
#pragma unroll
      for (int q = 0; q < KU; ++q) {
        const int64_t r = (int64_t)list[k + KU + q] * st;
        un[q] = X[r];
        ln[q] = X[r + C];
      }
    }
#pragma unroll
    for (int q = 0; q < KU; ++q) {
      const double uu = on ? (double)u[q] : 0.0, ll = on ? (double)l[q] : 0.0;
      const double M = (uu + ll) * 0.5;
      const double R = (uu - ll) * 0.5;
      const double *w = wt + (int64_t)list[k + q] * hp;
#pragma unroll
      for (int mm = 0; mm < MB; ++mm) {
        accM[mm] = fma(w[mm], M, accM[mm]);
        accR[mm] = fma(fabs(w[mm]), R, accR[mm]);
      }
    }
    if (more) {
#pragma unroll
      for (int q = 0; q < KU; ++q) {
        u[q] = un[q];
        l[q] = ln[q];
      }
    }
  }
  for (; k < count; ++k) {
    const int64_t r = (int64_t)list[k] * st;
    const double uu = on ? (double)X[r] : 0.0, ll = on ? (double)X[r + C] : 0.0;
    const double M = (uu + ll) * 0.5;
    const double R = (uu - ll) * 0.5;
    const double *w = wt + (int64_t)list[k] * hp;
#pragma unroll
    for (int mm = 0; mm < MB; ++mm) {
      accM[mm] = fma(w[mm], M, accM[mm]);
      accR[mm] = fma(fabs(w[mm]), R, accR[mm]);
    }
  }
}

// One thread per output coefficient c (degree Dout); MB output neurons per
// block row. Block x index runs over output-neuron chunks first so that the
// blocks reading the same coefficient range of the previous layer run
// together and share L2. Only the box's live inputs are read: composed
// neurons' full tensors, the tensors of order-1 and fallback neurons, which
// hold only the coefficients of their own degree (a prefix in the
// total-degree layout), and active neurons' pre-activation tensors in place.
// The weights come from the transposed, zero-padded copy W^T[k][hp]: for one
// input k the block's MB weights are contiguous and uniform, so they load as
// a few wide scalar loads and no row guard sits in the inner loop; |w| is the
// FMA's source modifier. Arithmetic is FP64 whatever the storage type; in
// FP32 mode each block also reports, per output neuron and bound, the sum of
// |fl32(y) - y| over its coefficients (the exact rounding of the stored
// tensor), reduced in a fixed order.
template <typename T, int MB, int KU>
__global__ void __launch_bounds__(kBlock) gemm_kernel(GemmArgs a) {
  __shared__ double red[kBlock / 64][MB][2];
  const int m0 = blockIdx.x * MB;
  const int64_t c = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  const int64_t box = a.bids ? a.bids[blockIdx.z] : blockIdx.z;
  const bool valid = c < a.C;
  const T *X = reinterpret_cast<const T *>(a.post) + box * a.slot_in;
  double accM[MB], accR[MB];
#pragma unroll
  for (int mm = 0; mm < MB; ++mm) accM[mm] = accR[mm] = 0.0;
  const int mcount = min(MB, a.h - m0);
  const int *lv = a.live + box * a.live_ld;
  const int64_t st = 2 * a.C;
  const double *wt = a.WT + m0;
  // lanes past the tensor read its last coefficient; their sums are dropped
  const int64_t cc = valid ? c : a.C - 1;
  gemm_rows<T, MB, KU>(X + cc, st, a.C, lv + 3, lv[0], true, wt, a.hp, accM, accR);
  if (lv[1] > 0) {
    // degree-preserving inputs hold the first Cs coefficients (graded order:
    // the monomials of their degree); beyond, their lifted tensor is zero
    const bool inside = cc < a.Cs;
    gemm_rows<T, MB, KU>(X + (inside ? cc : 0), st, a.C, lv + 3 + a.hin, lv[1], inside, wt, a.hp, accM, accR);
  }
  if (lv[2] > 0) {
    // active neurons: post = pre, read from the previous pre-activation arena
    const bool inside = cc < a.Cact;
    const T *Xa = reinterpret_cast<const T *>(a.act) + box * a.act_slot;
    gemm_rows<T, MB, KU>(Xa + (inside ? cc : 0), 2 * a.Cact, a.Cact, lv + 3 + 2 * a.hin, lv[2], inside, wt, a.hp, accM,
                         accR);
  }
  T *Y = reinterpret_cast<T *>(a.pre) + box * a.slot_out;
  const bool track = a.rpart != nullptr;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int mm = 0; mm < MB; ++mm) {
    double ru = 0.0, rl = 0.0;
    if (mm < mcount && valid) {
      const int m = m0 + mm;
      const double bias = (c == 0) ? a.b[m] : 0.0;
      const double yu = accM[mm] + accR[mm] + bias;
      const double yl = accM[mm] - accR[mm] + bias;
      const T su = (T)yu, sl = (T)yl;
      Y[(int64_t)m * 2 * a.C + c] = su;
      Y[(int64_t)m * 2 * a.C + a.C + c] = sl;
      ru = fabs((double)su - yu);
      rl = fabs((double)sl - yl);
    }
    if (track && mm < mcount) {
      for (int off = 32; off > 0; off >>= 1) {
        ru += __shfl_xor(ru, off, 64);
        rl += __shfl_xor(rl, off, 64);
      }
      if (lane == 0) {
        red[wid][mm][0] = ru;
        red[wid][mm][1] = rl;
      }
    }
  }
  if (!track) return;
  __syncthreads();
  if (threadIdx.x < 2 * mcount) {
    const int mm = threadIdx.x >> 1, s = threadIdx.x & 1;
    double v = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w][mm][s];
    a.rpart[box * a.rpart_slot + ((int64_t)(m0 + mm) * 2 + s) * a.cblocks + blockIdx.y] = v;
  }
}

int64_t gemm_cblocks(int64_t C) { return (C + kBlock - 1) / kBlock; }

template <int MB, int KU>
static hipError_t launch_gemm_mb(const GemmArgs &a, hipStream_t s) {
  dim3 grid((a.h + MB - 1) / MB, (unsigned)a.cblocks, (unsigned)a.nboxes);
  if (a.fp64)
    hipLaunchKernelGGL((gemm_kernel<double, MB, KU>), grid, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((gemm_kernel<float, MB, KU>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// Narrow output layers are bound by reading the input tensors: fewer rows
// per block and more loads in flight; wide layers by the FP64 multiply-adds.
hipError_t launch_gemm(const GemmArgs &a0, hipStream_t s) {
  GemmArgs a = a0;
  a.cblocks = gemm_cblocks(a.C);
  if (a.hp % 16 != 0 || a.hp < a.h || !a.live || a.Cs > a.C || !a.act) return hipErrorInvalidValue;
  ProfScope ps(kProfGemm, s, (double)a.nboxes * (2.0 * a.hin + 2.0 * a.h) * a.C * (a.fp64 ? 8 : 4),
               4.0 * a.nboxes * a.h * a.hin * a.C);
  if (a.h <= 4) {
    switch (a.tune.gemm_narrow) {
      case 1: return launch_gemm_mb<4, 4>(a, s);
      case 2: return launch_gemm_mb<4, 16>(a, s);
      default: return launch_gemm_mb<4, 8>(a, s);
    }
  }
  if (a.h <= 8) return launch_gemm_mb<8, 4>(a, s);
  switch (a.tune.gemm_wide) {
    case 1: return launch_gemm_mb<16, 4>(a, s);
    case 2: return launch_gemm_mb<8, 2>(a, s);
    case 3: return launch_gemm_mb<8, 4>(a, s);
    default: return launch_gemm_mb<16, 2>(a, s);
  }
}

}  // namespace bern
