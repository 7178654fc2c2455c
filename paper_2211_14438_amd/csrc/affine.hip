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
    if (a.flags && c == 0 && j == 0) {  // the box's validity, once per box
      int bad = 0;
      for (int k = 0; k < a.n; ++k)
        if (!(lo[k] <= hi[k]) || !isfinite(lo[k]) || !isfinite(hi[k])) bad = 1;
      a.flags[box] = bad;
    }
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
  if ((int64_t)blockIdx.z >= launch_boxes(a)) return;  // past a device count
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
  int64_t Cs = a.Cs, Cact = a.Cact;
  if (a.box_din) {  // the box's own pre degree
    const int din = box_degree(a.box_din, box);
    Cact = a.counts.at(a.n, din);
    Cs = a.counts.at(a.n, min(din, a.Dout));
  }
  // lanes past the tensor read its last coefficient; their sums are dropped
  const int64_t cc = valid ? c : a.C - 1;
  gemm_rows<T, MB, KU>(X + cc, st, a.C, lv + 3, lv[0], true, wt, a.hp, accM, accR);
  if (lv[1] > 0) {
    // degree-preserving inputs hold the first Cs coefficients (graded order:
    // the monomials of their degree); beyond, their lifted tensor is zero
    const bool inside = cc < Cs;
    gemm_rows<T, MB, KU>(X + (inside ? cc : 0), st, a.C, lv + 3 + a.hin, lv[1], inside, wt, a.hp, accM, accR);
  }
  if (lv[2] > 0) {
    // active neurons: post = pre, read from the previous pre-activation arena
    const bool inside = cc < Cact;
    const T *Xa = reinterpret_cast<const T *>(a.act) + box * a.act_slot;
    gemm_rows<T, MB, KU>(Xa + (inside ? cc : 0), 2 * Cact, Cact, lv + 3 + 2 * a.hin, lv[2], inside, wt, a.hp, accM,
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

// Tensors of at most 64 coefficients: one output coefficient per lane as
// above, but G = 64 / C boxes share a wave (lanes g C .. g C + C - 1 hold box
// g of the block's G), and the block's four waves take one quarter of the
// inputs each, their sums added in wave order at the end. The inputs run
// densely over k with a kind per (box, input) staged in LDS from the kind
// bytes of the live lists (0 none, 1 full, 2 degree-preserving prefix, 3
// active in place), so
// k and the weights stay uniform across the wave; an input a lane's box does
// not use reads an in-bounds element and contributes an exact zero. The
// per-lane order of the sums depends neither on MB nor on the box's place in
// the block; the FP32 rounding sums are added over the box's coefficients in
// index order.
constexpr int kPackMaxC = 64;
constexpr int kPackWaves = 4;
constexpr int kPackKU = 4;

__host__ __device__ inline int pack_groups(int64_t C) { return (int)(64 / C); }

// Dynamic LDS: the block's weights W^T[k][m0 .. m0 + MB) (hin MB doubles),
// one slot of wave partials (2 MB x 64 doubles, reused for the rounding
// sums), then the kind table (G hin bytes).
inline size_t pack_lds(int G, int hin, int MB) {
  return ((size_t)hin * MB + (size_t)2 * MB * 64) * sizeof(double) + (size_t)G * hin;
}

template <typename T, int MB>
__global__ void __launch_bounds__(kPackWaves * 64) gemm_pack_kernel(GemmArgs a) {
  extern __shared__ double pk_lds[];
  const int C = (int)a.C, G = pack_groups(a.C), hin = a.hin;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane / C, c = lane - g * C;
  // logical block: row chunk fastest, the row chunks of one box group on one XCD
  const int nx = (a.h + MB - 1) / MB;
  const int64_t lb = xcd_block(blockIdx.x, (int64_t)gridDim.x);
  const int m0 = (int)(lb % nx) * MB;
  const int64_t slot0 = lb / nx * G;
  const int64_t bslot = slot0 + g;
  const int64_t nb = launch_boxes(a);
  if (slot0 >= nb) return;  // past a device count
  const bool valid = g < G && bslot < nb;
  double *wl = pk_lds;
  double *part = wl + (size_t)hin * MB;
  unsigned char *kind = reinterpret_cast<unsigned char *>(part + (size_t)2 * MB * 64);
  // weights through LDS: one uniform read per row instead of scalar loads
  // whose latency each step would wait for; the block's boxes' input kinds
  // from the kind bytes of their lists, both behind one barrier
  for (int i = threadIdx.x; i < hin * MB; i += blockDim.x) wl[i] = a.WT[(int64_t)(i / MB) * a.hp + m0 + i % MB];
  for (int t = threadIdx.x; t < G * hin; t += blockDim.x) {
    const int gg = t / hin;
    unsigned char kk = 0;
    if (slot0 + gg < nb) {
      const int64_t bx = a.bids ? a.bids[slot0 + gg] : slot0 + gg;
      kk = live_kinds(a.live + bx * a.live_ld, hin)[t - gg * hin];
    }
    kind[t] = kk;
  }
  __syncthreads();
  const int64_t box = a.bids ? a.bids[valid ? bslot : slot0] : (valid ? bslot : slot0);
  const T *X = reinterpret_cast<const T *>(a.post) + box * a.slot_in;
  const T *Xa = reinterpret_cast<const T *>(a.act) + box * a.act_slot;
  const unsigned char *kd = kind + (valid ? g : 0) * hin;
  int Cs = (int)a.Cs, Ca = (int)a.Cact;
  if (a.box_din) {  // the lane's box's own pre degree
    const int din = box_degree(a.box_din, box);
    Ca = (int)a.counts.at(a.n, din);
    Cs = (int)a.counts.at(a.n, min(din, a.Dout));
  }
  const int kq = (hin + kPackWaves - 1) / kPackWaves;
  const int k0 = min(hin, w * kq), k1 = min(hin, k0 + kq);
  double accM[MB], accR[MB];
#pragma unroll
  for (int mm = 0; mm < MB; ++mm) accM[mm] = accR[mm] = 0.0;
  // loads of kPackKU inputs from kb on; inputs the lane's box does not use,
  // and those past k1, read an in-bounds element marked out
  auto load = [&](int kb, T (&u)[kPackKU], T (&l)[kPackKU], bool (&in)[kPackKU]) {
#pragma unroll
    for (int q = 0; q < kPackKU; ++q) {
      const int k = kb + q;
      const bool live = k < k1;
      const int kk = live && valid ? kd[k] : 0;
      const int lim = kk == 1 ? C : kk == 2 ? Cs : kk == 3 ? Ca : 0;
      in[q] = c < lim;
      const bool ac = kk == 3;
      const int kc = live ? k : k0;
      const T *base = ac ? Xa + (int64_t)kc * 2 * Ca : X + (int64_t)kc * 2 * C;
      const int off = in[q] ? c : 0;
      u[q] = base[off];
      l[q] = base[off + (ac ? Ca : C)];
    }
  };
  T u[kPackKU], l[kPackKU];
  bool in[kPackKU];
  if (k0 < k1) load(k0, u, l, in);
  for (int kb = k0; kb < k1; kb += kPackKU) {
    T un[kPackKU], ln[kPackKU];
    bool inn[kPackKU];
    const bool more = kb + kPackKU < k1;
    if (more) load(kb + kPackKU, un, ln, inn);
#pragma unroll
    for (int q = 0; q < kPackKU; ++q) {
      if (kb + q < k1) {
        const double uu = in[q] ? (double)u[q] : 0.0, ll = in[q] ? (double)l[q] : 0.0;
        const double M = (uu + ll) * 0.5;
        const double R = (uu - ll) * 0.5;
        const double *wk = wl + (kb + q) * MB;
#pragma unroll
        for (int mm = 0; mm < MB; ++mm) {
          accM[mm] = fma(wk[mm], M, accM[mm]);
          accR[mm] = fma(fabs(wk[mm]), R, accR[mm]);
        }
      }
    }
    if (more) {
#pragma unroll
      for (int q = 0; q < kPackKU; ++q) {
        u[q] = un[q];
        l[q] = ln[q];
        in[q] = inn[q];
      }
    }
  }
  // the quarters' sums, added in wave order by wave 0 through one LDS slot
  // that waves 1, 2, ... fill in turn (a smaller block footprint, so more
  // blocks share a CU)
  for (int v = 1; v < kPackWaves; ++v) {
    if (w == v) {
#pragma unroll
      for (int mm = 0; mm < MB; ++mm) {
        part[(2 * mm) * 64 + lane] = accM[mm];
        part[(2 * mm + 1) * 64 + lane] = accR[mm];
      }
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int mm = 0; mm < MB; ++mm) {
        accM[mm] += part[(2 * mm) * 64 + lane];
        accR[mm] += part[(2 * mm + 1) * 64 + lane];
      }
    }
    __syncthreads();
  }
  const bool track = a.rpart != nullptr;
  if (w == 0) {
    T *Y = reinterpret_cast<T *>(a.pre) + box * a.slot_out;
#pragma unroll
    for (int mm = 0; mm < MB; ++mm) {
      const int m = m0 + mm;
      double ru = 0.0, rl = 0.0;
      if (valid && m < a.h) {
        const double bias = c == 0 ? a.b[m] : 0.0;
        const double yu = accM[mm] + accR[mm] + bias;
        const double yl = accM[mm] - accR[mm] + bias;
        const T su = (T)yu, sl = (T)yl;
        Y[(int64_t)m * 2 * C + c] = su;
        Y[(int64_t)m * 2 * C + C + c] = sl;
        ru = fabs((double)su - yu);
        rl = fabs((double)sl - yl);
      }
      if (track) {
        part[(2 * mm) * 64 + lane] = ru;
        part[(2 * mm + 1) * 64 + lane] = rl;
      }
    }
  }
  if (!track) return;
  __syncthreads();
  // per (box, row, bound): its coefficients' rounding in index order
  for (int t = threadIdx.x; t < G * MB * 2; t += blockDim.x) {
    const int gg = t / (2 * MB), r = t - gg * 2 * MB, mm = r >> 1, sd = r & 1;
    if (slot0 + gg >= nb || m0 + mm >= a.h) continue;
    double v = 0.0;
    for (int q = 0; q < C; ++q) v += part[r * 64 + gg * C + q];
    const int64_t bx = a.bids ? a.bids[slot0 + gg] : slot0 + gg;
    a.rpart[bx * a.rpart_slot + ((int64_t)(m0 + mm) * 2 + sd) * a.cblocks] = v;
  }
}

int64_t gemm_cblocks(int64_t C) { return (C + kBlock - 1) / kBlock; }

template <int MB>
static hipError_t launch_gemm_pack(const GemmArgs &a, hipStream_t s) {
  const int G = pack_groups(a.C);
  const size_t lds = pack_lds(G, a.hin, MB);
  const int64_t blocks = (int64_t)((a.h + MB - 1) / MB) * ((a.nboxes + G - 1) / G);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)blocks);
  if (a.fp64) {
    RET_IF(hipFuncSetAttribute((const void *)gemm_pack_kernel<double, MB>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((gemm_pack_kernel<double, MB>), grid, dim3(kPackWaves * 64), lds, s, a);
  } else {
    RET_IF(hipFuncSetAttribute((const void *)gemm_pack_kernel<float, MB>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((gemm_pack_kernel<float, MB>), grid, dim3(kPackWaves * 64), lds, s, a);
  }
  return hipGetLastError();
}

template <int MB, int KU>
static hipError_t launch_gemm_mb(const GemmArgs &a, hipStream_t s) {
  dim3 grid((a.h + MB - 1) / MB, (unsigned)a.cblocks, (unsigned)a.nboxes);
  // one coefficient block: only the waves that hold coefficients
  const unsigned threads = a.C < kBlock ? (unsigned)((a.C + 63) / 64 * 64) : kBlock;
  if (a.fp64)
    hipLaunchKernelGGL((gemm_kernel<double, MB, KU>), grid, dim3(threads), 0, s, a);
  else
    hipLaunchKernelGGL((gemm_kernel<float, MB, KU>), grid, dim3(threads), 0, s, a);
  return hipGetLastError();
}

// Narrow output layers are bound by reading the input tensors: fewer rows
// per block and more loads in flight; wide layers by the FP64 multiply-adds.
hipError_t launch_gemm(const GemmArgs &a0, hipStream_t s) {
  GemmArgs a = a0;
  a.cblocks = gemm_cblocks(a.C);
  if (a.hp % 16 != 0 || a.hp < a.h || !a.live || a.Cs > a.C || !a.act) return hipErrorInvalidValue;
  if (a.box_din && (a.n < 1 || stored_count(a.n, a.Dout) != a.C)) return hipErrorInvalidValue;
  if (a.box_din) a.counts.fill(a.n);
  ProfScope ps(kProfGemm, s, (double)a.nboxes * (2.0 * a.hin + 2.0 * a.h) * a.C * (a.fp64 ? 8 : 4),
               4.0 * a.nboxes * a.h * a.hin * a.C);
  if (a.C <= kPackMaxC && pack_lds(pack_groups(a.C), a.hin, 16) <= device_lds_limit()) {
    if (a.h <= 4) return launch_gemm_pack<4>(a, s);
    if (a.h <= 8 || a.tune.gemm_wide != 1) return launch_gemm_pack<8>(a, s);
    return launch_gemm_pack<16>(a, s);
  }
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
