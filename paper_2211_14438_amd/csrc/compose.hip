// Composition of the ReLU approximant with a neuron's input polynomials
// (Step 3 of Section 5.1, eqs. post_bounds_1/2) on gfx950.
//
// For an unstable neuron with pre-activation interval [lo, hi] and ReLU order
// L, with nu(P) = (P - lo)/(hi - lo) and the power series c_0..c_L of Step 2:
//     U = sum_j c_j nu(U^)^j,        L = sum_j c_j nu(L^)^j - e.
// Powers of a polynomial are products "Prod" (Section 4.2): n-d convolutions
// of coefficient tensors. In the power basis, lifting a tensor to a higher
// degree (Prop. 4 elevation) is a zero pad, and adding a constant only
// touches the constant coefficient.
//
// The network's tensors are stored in the total-degree layout (simplex.hpp),
// so a product runs over the index pairs (I, J) of stored coefficients with
// I + J = K, listed per output coefficient K in a table built once per
// degree pair:
//  * order 2 (the common case): U = c_2 nu^2 + c_1 nu + c_0 over the square
//    table (pairs I < J once, doubled, plus the diagonal);
//  * order >= 3: Horner steps Q <- nu * Q + c_j, one launch per step;
//  * order 1, active (identity) and the linear fallback are element-wise
//    writes at the input degree; inactive neurons (zero) store nothing and
//    are left out of the next affine map's input lists.
// Composed results are written whole at the layer's post degree Dout.
// The dense per-variable-degree square kernel below serves the step-level
// product entry point, whose tensors are dense.
//
// Arithmetic is FP64 for both storage types: with packed FP32 math off, FP32
// and FP64 FMAs issue at the same rate on gfx950, and FP64 keeps the rounding
// radius of FP32 mode down to the final FP32 stores. In FP32 mode the input
// radius is folded into nu (U^ + epsU, L^ - epsL keep nu in [0,1] exactly),
// and every block reports the exact sum of |fl32(q) - q| over the
// coefficients it stored, plus their l1 norm, for the radius of the result.
#include "common.hpp"

namespace bern {

__host__ __device__ constexpr int cpow(int b, int e) { return e == 0 ? 1 : b * cpow(b, e - 1); }

__device__ inline int64_t wave_box(const ComposeArgs &a, int64_t g) { return a.bids ? a.bids[g] : g; }

// item index of (launch box g, neuron j, bound s) among the wave's boxes
__device__ inline int64_t item_of(const ComposeArgs &a, int64_t g, int j, int s) {
  return (wave_box(a, g) * a.h + j) * a.nbounds + s;
}

// partial slots per item: every class of a layer uses the layer's stride
__device__ inline int64_t pslots(const ComposeArgs &a) { return a.pstride > 0 ? a.pstride : a.nbx; }

template <typename T>
__device__ inline const T *in_tensor(const ComposeArgs &a, int64_t box, int j, int s, int64_t Cin) {
  return reinterpret_cast<const T *>(a.pre) + box * a.slot_in + ((int64_t)j * a.nbounds + s) * Cin;
}
template <typename T>
__device__ inline T *out_tensor(const ComposeArgs &a, int64_t box, int j, int s, int64_t Cout) {
  return reinterpret_cast<T *>(a.post) + box * a.slot_out + ((int64_t)j * a.nbounds + s) * Cout;
}
template <typename T>
__device__ inline const T *in_tensor(const ComposeArgs &a, int64_t box, int j, int s) {
  return in_tensor<T>(a, box, j, s, a.Cin);
}
template <typename T>
__device__ inline T *out_tensor(const ComposeArgs &a, int64_t box, int j, int s) {
  return out_tensor<T>(a, box, j, s, a.Cout);
}

// A box's degrees and stored-coefficient counts in a launch: the launch's
// own, or the box's from the per-box degree arrays.
struct BoxDeg {
  int Din, Dout;
  int64_t Cin, Cout, Cs;
};
__device__ inline BoxDeg box_deg(const ComposeArgs &a, int64_t box) {
  BoxDeg d{a.Din, a.Dout, a.Cin, a.Cout, a.Cs};
  if (a.box_din) {
    d.Din = box_degree(a.box_din, box);
    d.Cin = a.counts.at(a.n, d.Din);
  }
  if (a.box_dout) {
    d.Dout = box_degree(a.box_dout, box);
    d.Cout = a.counts.at(a.n, d.Dout);
  }
  if (a.box_din || a.box_dout) d.Cs = a.counts.at(a.n, min(d.Din, d.Dout));
  return d;
}

// Block-wide sums of (rounding, l1) in a fixed order; thread 0 writes them
// to partial slot `slot` of item `it`.
__device__ void block_partials_slot(const ComposeArgs &a, int64_t it, int64_t slot, double r, double l1) {
  __shared__ double red[kBlock / 64][2];
  for (int off = 32; off > 0; off >>= 1) {
    r += __shfl_xor(r, off, 64);
    l1 += __shfl_xor(l1, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[wid][0] = r;
    red[wid][1] = l1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sr = 0.0, sl = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      sr += red[w][0];
      sl += red[w][1];
    }
    a.part[(it * pslots(a) + slot) * 2 + 0] = sr;
    a.part[(it * pslots(a) + slot) * 2 + 1] = sl;
    if (slot == 0)  // the slots past this class's blocks
      for (int64_t b = a.nbx; b < pslots(a); ++b) a.part[(it * pslots(a) + b) * 2 + 0] =
                                                     a.part[(it * pslots(a) + b) * 2 + 1] = 0.0;
  }
}

__device__ inline void block_partials(const ComposeArgs &a, int64_t it, double r, double l1) {
  block_partials_slot(a, it, blockIdx.x, r, l1);
}

// One wave's item: its (rounding, l1) sums in slot 0, zeros in the others.
__device__ void wave_partials(const ComposeArgs &a, int64_t it, double r, double l1) {
  for (int off = 32; off > 0; off >>= 1) {
    r += __shfl_xor(r, off, 64);
    l1 += __shfl_xor(l1, off, 64);
  }
  const int lane = threadIdx.x & 63;
  for (int64_t b = lane; b < pslots(a); b += 64) {
    a.part[(it * pslots(a) + b) * 2 + 0] = b == 0 ? r : 0.0;
    a.part[(it * pslots(a) + b) * 2 + 1] = b == 0 ? l1 : 0.0;
  }
}

// Items of a launch are (launch box, neuron, bound) in that order; the boxes
// are a.nboxes, or the count a.dcount reads from device memory.
__device__ inline int64_t launch_items(const ComposeArgs &a) {
  return launch_boxes(a) * (int64_t)a.h * a.nbounds;
}

// Every item of the launch with work to do: a wave takes `chunks`
// consecutive wave slots per item (chunk index c), one item after another
// over a grid that may hold fewer waves than items, and runs f(g, j, s, c)
// for each item that passes need(kind, s). With grouping (a.group > 1, at
// most 64) a wave slot covers a.group consecutive items, whose kinds it reads
// at once, and runs those that pass in order. Either way an item's work is
// the same.
template <class Need, class F>
__device__ inline void for_wave_items(const ComposeArgs &a, int chunks, Need need, F f) {
  const int64_t per = (int64_t)a.h * a.nbounds, total = launch_items(a);
  const int grp = a.group > 1 ? a.group : 1;
  const int64_t slots = (total + grp - 1) / grp * chunks;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int lane = threadIdx.x & 63;
  for (int64_t w0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w0 < slots; w0 += stride) {
    const int c = (int)(w0 % chunks);
    const int64_t w = w0 / chunks;
    if (grp == 1) {
      const int64_t g = w / per;
      const int rest = (int)(w - g * per);
      const int j = rest / a.nbounds, s = rest - j * a.nbounds;
      if (need(a.recs[wave_box(a, g) * a.h + j].kind, s)) f(g, j, s, c);
      continue;
    }
    const int64_t i0 = w * grp;
    bool mine = false;
    if (lane < grp && i0 + lane < total) {
      const int64_t it = i0 + lane, g = it / per;
      const int rest = (int)(it - g * per);
      mine = need(a.recs[wave_box(a, g) * a.h + rest / a.nbounds].kind, rest % a.nbounds);
    }
    unsigned long long todo = __ballot(mine);
    while (todo) {
      const int b = __ffsll((long long)todo) - 1;
      todo &= todo - 1;
      const int64_t it = i0 + b, g = it / per;
      const int rest = (int)(it - g * per);
      f(g, rest / a.nbounds, rest % a.nbounds, c);
    }
  }
}

// Store one coefficient; track its rounding and magnitude.
template <typename T>
__device__ __forceinline__ void store(T *dst, double q, double &r, double &l1) {
  const T v = (T)q;
  *dst = v;
  r += fabs((double)v - q);
  l1 += fabs((double)v);
}

struct NuSource {
  double lo, w, shift;  // nu = (p + shift*[K=0] - lo) / w
};

__device__ inline NuSource nu_of(const ComposeArgs &a, const NeuronRec *r, int s) {
  if (!r) return {0.0, 1.0, 0.0};  // plain product mode: nu = p
  NuSource v;
  v.lo = r->lo;
  v.w = r->hi - r->lo;
  v.shift = a.fp64 ? 0.0 : (s == 0 ? r->epsU : -r->epsL);
  return v;
}

// ------------------------------------------------------------ row conv
template <int D, int NI>
__device__ __forceinline__ void row_conv(const double *ra, const double *rb, double *acc) {
  constexpr int D1 = D + 1, E1 = 2 * D + 1;
  if constexpr (NI == 1) {
#pragma unroll
    for (int i = 0; i < D1; ++i)
#pragma unroll
      for (int j = 0; j < D1; ++j) acc[i + j] = fma(ra[i], rb[j], acc[i + j]);
  } else {
#pragma unroll
    for (int i0 = 0; i0 < D1; ++i0)
#pragma unroll
      for (int i1 = 0; i1 < D1; ++i1)
#pragma unroll
        for (int j0 = 0; j0 < D1; ++j0)
#pragma unroll
          for (int j1 = 0; j1 < D1; ++j1)
            acc[(i0 + j0) * E1 + i1 + j1] = fma(ra[i0 * D1 + i1], rb[j0 * D1 + j1], acc[(i0 + j0) * E1 + i1 + j1]);
  }
}

template <int D, int NI>
struct SqGeom {
  static constexpr int D1 = D + 1, E1 = 2 * D + 1;
  static constexpr int R = cpow(D1, NI), RO = cpow(E1, NI);
  static constexpr int RP = (R + 1) & ~1;  // row pitch in doubles (16-byte aligned rows)
};

// Square path: nu in LDS (FP64) as rows of R = (D+1)^NI coefficients;
// thread = one output row of the layer's post tensor. Rows of nu that are
// exactly zero are flagged while nu is staged (their products add exact
// zeros, so skipping them leaves every result bit unchanged); output rows whose
// outer digit sum exceeds twice the largest digit sum of a nonzero row only
// receive such products and are written as zeros without the loop.
template <typename T, int D, int NI>
__global__ void __launch_bounds__(kBlock) compose_sq_kernel(ComposeArgs a) {
  using G = SqGeom<D, NI>;
  constexpr int D1 = G::D1, E1 = G::E1, R = G::R, RO = G::RO, RP = G::RP;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *rows = reinterpret_cast<double *>(smem_raw);
  __shared__ int tmax;

  const int j = blockIdx.y / a.nbounds, s = blockIdx.y % a.nbounds;
  const int64_t g = blockIdx.z, box = wave_box(a, g);
  const NeuronRec *rec = a.recs ? &a.recs[box * a.h + j] : nullptr;
  if (rec && rec->kind != 2) return;
  const NuSource ns = nu_of(a, rec, s);

  const int no = a.n - NI;
  const int64_t nrows = a.Cin / R;
  unsigned char *nz = smem_raw + nrows * RP * sizeof(double);  // one flag per row
  const int64_t it = item_of(a, g, j, s);
  const T *p = in_tensor<T>(a, box, j, s);
  if (threadIdx.x == 0) tmax = -1;
  for (int64_t i = threadIdx.x; i < a.Cin; i += blockDim.x) {
    double v = (double)p[i];
    if (i == 0) v += ns.shift - ns.lo;
    rows[(i / R) * RP + (i % R)] = v / ns.w;
  }
  __syncthreads();
  for (int64_t r = threadIdx.x; r < nrows; r += blockDim.x) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < R; ++q) any |= rows[r * RP + q] != 0.0;
    nz[r] = any ? 1 : 0;
    if (any) {
      int ds = 0;
      int64_t rem = r;
      for (int q = 0; q < no; ++q) {
        ds += (int)(rem % D1);
        rem /= D1;
      }
      atomicMax(&tmax, ds);
    }
  }
  __syncthreads();
  const int dsmax = 2 * tmax;  // -2 when nu is the zero polynomial

  const int Do1 = a.Dout + 1;
  int64_t Mo = 1;
  for (int q = 0; q < no; ++q) Mo *= Do1;
  const int64_t ko = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int Rout = (NI == 1) ? Do1 : Do1 * Do1;
  T *out = out_tensor<T>(a, box, j, s) + (ko < Mo ? ko : 0) * Rout;
  double rsum = 0.0, l1sum = 0.0;

  // outer digits of ko (base Dout+1): per-axis pair ranges packed 4 bits/axis
  uint64_t lop = 0, hip = 0;
  int64_t rK = 0, cnt = 1;
  bool work = ko < Mo, lin_ok = true, origin = true;
  if (work) {
    int64_t rem = ko, pw = 1;
    int dsum = 0;
    for (int q = no - 1; q >= 0; --q) {
      const int k = (int)(rem % Do1);
      rem /= Do1;
      dsum += k;
      if (k > 2 * D) work = false;
      const int l = max(0, k - D), hh = min(k, D);
      const int sh = 4 * (no - 1 - q);
      lop |= (uint64_t)(l & 15) << sh;
      hip |= (uint64_t)(hh & 15) << sh;
      cnt *= (hh - l + 1);
      rK += (int64_t)k * pw;
      pw *= D1;
      if (k > D) lin_ok = false;
      if (k != 0) origin = false;
    }
    if (dsum > dsmax && !origin) work = false;
  }
  {
    // Rows that only receive exact-zero products (or lie past degree 2D) are
    // zero: written by the whole block with coalesced stores over its
    // contiguous range of rows.
    __shared__ unsigned char busy[kBlock];
    busy[threadIdx.x] = (work || ko >= Mo) ? 1 : 0;
    __syncthreads();
    const int64_t ko0 = (int64_t)blockIdx.x * blockDim.x;
    const int nr = (int)min((int64_t)blockDim.x, Mo - ko0);
    const unsigned magic = 0xFFFFFFFFu / (unsigned)Rout + 1u;  // e / Rout = umulhi(e, magic) for e < 2^32 / Rout
    T *base = out_tensor<T>(a, box, j, s) + ko0 * Rout;
    for (unsigned e = threadIdx.x; e < (unsigned)(nr * Rout); e += blockDim.x)
      if (!busy[Rout == 1 ? e : __umulhi(e, magic)]) base[e] = (T)0;
  }
  if (work) {
    double acc[RO];
#pragma unroll
    for (int q = 0; q < RO; ++q) acc[q] = 0.0;
    int64_t rI = 0;
    {
      int64_t pw = 1;
      for (int q = no - 1; q >= 0; --q) {
        rI += (int64_t)((lop >> (4 * (no - 1 - q))) & 15) * pw;
        pw *= D1;
      }
    }
    uint64_t iv = lop;
    const int64_t half = cnt >> 1;
    for (int64_t t = 0; t < half; ++t) {
      if (nz[rI] & nz[rK - rI]) {
        double ra[R], rb[R];
        const double *pa = rows + rI * RP;
        const double *pb = rows + (rK - rI) * RP;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          ra[q] = pa[q];
          rb[q] = pb[q];
        }
        row_conv<D, NI>(ra, rb, acc);
      }
      int64_t pw = 1;
      for (int q = no - 1; q >= 0; --q) {
        const int sh = 4 * (no - 1 - q);
        const int d = (int)((iv >> sh) & 15), hh = (int)((hip >> sh) & 15);
        if (d < hh) {
          iv += (uint64_t)1 << sh;
          rI += pw;
          break;
        }
        const int l = (int)((lop >> sh) & 15);
        iv = (iv & ~((uint64_t)15 << sh)) | ((uint64_t)l << sh);
        rI -= (int64_t)(d - l) * pw;
        pw *= D1;
      }
    }
#pragma unroll
    for (int q = 0; q < RO; ++q) acc[q] = acc[q] + acc[q];
    if ((cnt & 1) && nz[rI]) {  // middle pair I = K - I
      double ra[R];
      const double *pa = rows + rI * RP;
#pragma unroll
      for (int q = 0; q < R; ++q) ra[q] = pa[q];
      row_conv<D, NI>(ra, ra, acc);
    }

    // epilogue: c2 nu^2 + c1 nu + (c0 - e for the lower bound)
    const double c2 = rec ? rec->c[2] : 1.0;
    const double c1 = rec ? rec->c[1] : 0.0;
    const double cst = rec ? rec->c[0] - (s == 1 ? rec->e : 0.0) : 0.0;
    double lin[R];
#pragma unroll
    for (int q = 0; q < R; ++q) lin[q] = 0.0;
    if (lin_ok) {
      const double *pl = rows + rK * RP;
#pragma unroll
      for (int q = 0; q < R; ++q) lin[q] = pl[q];
    }
    if constexpr (NI == 1) {
#pragma unroll
      for (int q0 = 0; q0 < E1; ++q0) {
        double v = c2 * acc[q0];
        if (q0 <= D) v = fma(c1, lin[q0], v);
        if (origin && q0 == 0) v += cst;
        store(out + q0, v, rsum, l1sum);
      }
      for (int q0 = E1; q0 < Do1; ++q0) out[q0] = (T)0;  // layer degree above 2D
    } else {
      if (Do1 > E1) {
        for (int q0 = 0; q0 < Do1; ++q0)
          for (int q1 = 0; q1 < Do1; ++q1)
            if (q0 >= E1 || q1 >= E1) out[q0 * Do1 + q1] = (T)0;
      }
#pragma unroll
      for (int q0 = 0; q0 < E1; ++q0)
#pragma unroll
        for (int q1 = 0; q1 < E1; ++q1) {
          double v = c2 * acc[q0 * E1 + q1];
          if (q0 <= D && q1 <= D) v = fma(c1, lin[q0 * D1 + q1], v);
          if (origin && q0 == 0 && q1 == 0) v += cst;
          store(out + q0 * Do1 + q1, v, rsum, l1sum);
        }
    }
  }
  if (a.part) block_partials(a, it, rsum, l1sum);
}

// ------------------------------------------------- element-wise rules
// Input lists of the next affine map, one wave per box: composed neurons
// (order >= 2, full tensors at the layer's post degree), order-1 and
// fallback neurons (post tensors stored at degree Din), and active neurons
// (post = pre, read in place from the pre-activation arena). Inactive
// neurons are left out.
__global__ void __launch_bounds__(kBlock) live_kernel(ComposeArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (g >= a.nboxes) return;
  const int64_t box = wave_box(a, g);
  int *lv = a.live + box * a.live_ld;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int nf = 0, ns = 0, na = 0;
  for (int j0 = 0; j0 < a.h; j0 += 64) {
    const int j = j0 + lane;
    const int kind = j < a.h ? a.recs[box * a.h + j].kind : (int)kInactive;
    // after a linearisation every neuron that is not inactive holds a full
    // degree-1 post tensor
    const bool full = a.lin ? (j < a.h && kind != kInactive) : kind >= 2;
    const bool small = !a.lin && (kind == 1 || kind == kFallback);
    const bool act = !a.lin && kind == kActive;
    const unsigned long long bf = __ballot(full), bs = __ballot(small), ba = __ballot(act);
    if (full) lv[3 + nf + __popcll(bf & below)] = j;
    if (small) lv[3 + a.h + ns + __popcll(bs & below)] = j;
    if (act) lv[3 + 2 * a.h + na + __popcll(ba & below)] = j;
    if (j < a.h) live_kinds(lv, a.h)[j] = (unsigned char)(full ? 1 : small ? 2 : act ? 3 : 0);
    nf += __popcll(bf);
    ns += __popcll(bs);
    na += __popcll(ba);
  }
  if (lane == 0) {
    lv[0] = nf;
    lv[1] = ns;
    lv[2] = na;
  }
}

// One item (box, neuron, bound) of order 1 (c1 nu + c0, minus e for the
// lower bound) or the linear fallback (n+1 affine coefficients), each stored
// at degree Ds = min(Din, Dout) at the start of its post tensor. Active
// neurons (post = pre, read in place by the next affine map) and inactive
// ones store nothing. Writes the wave's rounding and l1 sums to partial
// slot 0 and zeros to the item's other slots.
template <typename T>
struct ScatterJob {
  const T *p;        // pre tensor (order 1)
  T *out;            // post tensor
  const double *fb;  // fallback coefficients
  double a0, w, c1, b0;  // order 1: q_I = c1 (p_I + a0 [I=0]) / w + b0 [I=0]
  int64_t it;        // item index, for the partials
  int mode;          // 1 order 1, 2 fallback, 0 nothing
  int n;             // coefficients stored
  int lim;           // fallback: last nonzero coefficient
};

template <typename T>
__device__ inline ScatterJob<T> scatter_job(const ComposeArgs &a, int64_t g, int j, int s) {
  ScatterJob<T> J{};
  const int64_t box = wave_box(a, g);
  const NeuronRec &r = a.recs[box * a.h + j];
  const int kind = r.kind;
  const BoxDeg bd = box_deg(a, box);
  // storage degree: Din, or the layer's post degree when that is lower (only
  // fallback and inactive neurons then); a prefix of the total-degree layout
  const int Ds = min(bd.Din, bd.Dout);
  J.it = (box * a.h + j) * a.nbounds + s;
  J.p = in_tensor<T>(a, box, j, s, bd.Cin);
  J.out = out_tensor<T>(a, box, j, s, bd.Cout);
  if (kind == 1) {  // these neurons take degree Din <= Dout
    const NuSource ns = nu_of(a, &r, s);
    J.mode = 1;
    J.n = Ds == bd.Din ? (int)bd.Cin : 0;
    J.a0 = ns.shift - ns.lo;
    J.w = ns.w;
    J.c1 = r.c[1];
    J.b0 = r.c[0] - (s == 1 ? r.e : 0.0);
  } else if (kind == kFallback) {
    // rank 0: constant; rank 1 + axis: t_axis; the rest zero
    J.mode = 2;
    J.n = (int)bd.Cs;
    J.lim = Ds >= 1 ? a.n : 0;
    J.fb = (s == 0) ? r.fbU : r.fbL;
  }
  return J;
}

__device__ inline int lane_int(int v, int b) { return __builtin_amdgcn_readlane(v, b); }
__device__ inline int64_t lane_i64(int64_t v, int b) {
  const uint32_t lo = (uint32_t)lane_int((int)(uint32_t)v, b);
  const uint32_t hi = (uint32_t)lane_int((int)(uint32_t)((uint64_t)v >> 32), b);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline double lane_f64(double v, int b) { return __longlong_as_double(lane_i64(__double_as_longlong(v), b)); }
template <class P>
__device__ inline P *lane_ptr(P *v, int b) { return reinterpret_cast<P *>(lane_i64(reinterpret_cast<int64_t>(v), b)); }

// Lane b's job, read by the whole wave.
template <typename T>
__device__ inline ScatterJob<T> job_of_lane(const ScatterJob<T> &J, int b) {
  ScatterJob<T> K;
  K.p = lane_ptr(J.p, b);
  K.out = lane_ptr(J.out, b);
  K.fb = lane_ptr(J.fb, b);
  K.a0 = lane_f64(J.a0, b);
  K.w = lane_f64(J.w, b);
  K.c1 = lane_f64(J.c1, b);
  K.b0 = lane_f64(J.b0, b);
  K.it = lane_i64(J.it, b);
  K.mode = lane_int(J.mode, b);
  K.n = lane_int(J.n, b);
  K.lim = lane_int(J.lim, b);
  return K;
}

// The first two pre coefficients of each lane (order 1 with at most 128
// coefficients), loaded ahead of the job's stores.
template <typename T>
__device__ inline void scatter_prefetch(const ScatterJob<T> &J, T &x0, T &x1) {
  const int lane = threadIdx.x & 63;
  x0 = x1 = (T)0;
  if (J.mode != 1 || J.n > 128) return;
  if (lane < J.n) x0 = J.p[lane];
  if (lane + 64 < J.n) x1 = J.p[lane + 64];
}

template <typename T>
__device__ inline void scatter_run(const ComposeArgs &a, const ScatterJob<T> &J, T x0, T x1) {
  const int lane = threadIdx.x & 63;
  double rsum = 0.0, l1sum = 0.0;
  auto one = [&](int64_t I, T x) {
    double v = (double)x;
    if (I == 0) v += J.a0;
    v = J.c1 * (v / J.w);
    if (I == 0) v += J.b0;
    store(J.out + I, v, rsum, l1sum);
  };
  if (J.mode == 1 && J.n <= 128) {
    if (lane < J.n) one(lane, x0);
    if (lane + 64 < J.n) one(lane + 64, x1);
  } else if (J.mode == 1) {
    for (int64_t I = lane; I < J.n; I += 64) one(I, J.p[I]);
  } else if (J.mode == 2) {
    for (int64_t I = lane; I < J.n; I += 64) {
      if (I <= J.lim)
        store(J.out + I, J.fb[I], rsum, l1sum);
      else
        J.out[I] = (T)0;
    }
  }
  if (a.part) wave_partials(a, J.it, rsum, l1sum);
}

template <typename T>
__device__ void scatter_item(const ComposeArgs &a, int64_t g, int j, int s) {
  const ScatterJob<T> J = scatter_job<T>(a, g, j, s);
  T x0, x1;
  scatter_prefetch(J, x0, x1);
  scatter_run(a, J, x0, x1);
}

// Grouped items (a.group > 1, at most 64): lane b builds the job of the
// slot's item b, all at once; the wave then runs the jobs in item order,
// loading each job's coefficients before the previous job's stores. The
// work and sums of every item are those of scatter_item.
template <typename T>
__device__ void scatter_grouped(const ComposeArgs &a) {
  const int64_t per = (int64_t)a.h * a.nbounds, total = launch_items(a);
  const int grp = a.group;
  const int64_t slots = (total + grp - 1) / grp;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int lane = threadIdx.x & 63;
  for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < slots; w += stride) {
    const int64_t i0 = w * grp;
    ScatterJob<T> mine{};
    if (lane < grp && i0 + lane < total) {
      const int64_t it = i0 + lane, g = it / per;
      const int rest = (int)(it - g * per);
      mine = scatter_job<T>(a, g, rest / a.nbounds, rest % a.nbounds);
    }
    unsigned long long todo = __ballot(mine.mode != 0);
    if (!todo) continue;
    int b = __ffsll((long long)todo) - 1;
    todo &= todo - 1;
    ScatterJob<T> J = job_of_lane(mine, b);
    T x0, x1;
    scatter_prefetch(J, x0, x1);
    while (true) {
      const bool more = todo != 0;
      ScatterJob<T> K{};
      T y0 = (T)0, y1 = (T)0;
      if (more) {
        b = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        K = job_of_lane(mine, b);
        scatter_prefetch(K, y0, y1);
      }
      scatter_run(a, J, x0, x1);
      if (!more) break;
      J = K;
      x0 = y0;
      x1 = y1;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) compose_scatter_kernel(ComposeArgs a) {
  // order-1 and fallback neurons (the partials of the others are not read)
  if (a.group > 1) {
    scatter_grouped<T>(a);
    return;
  }
  for_wave_items(a, 1, [](int kind, int) { return kind == 1 || kind == kFallback; },
                 [&](int64_t g, int j, int s, int) { scatter_item<T>(a, g, j, s); });
}

// ---------------------------------------------- total-degree products
// Load nu = (p + shift [K = 0] - lo) / (hi - lo) of the item into LDS (FP64).
template <typename T>
__device__ inline void load_nu(const ComposeArgs &a, const T *p, const NuSource &ns, double *nu) {
  for (int64_t i = threadIdx.x; i < a.Cin; i += blockDim.x) {
    double v = (double)p[i];
    if (i == 0) v += ns.shift - ns.lo;
    nu[i] = v / ns.w;
  }
  __syncthreads();
}

// Order 2 (the common case): U = c2 nu^2 + c1 nu + c0, minus e for the
// lower bound. One thread per output coefficient K at the layer's degree;
// the pairs (I, J) with I + J = K come from the square table: pairs with
// I < J listed once and doubled, plus the diagonal term. Coefficients past
// degree 2 Din (a layer stored at a higher degree) are zero.
template <typename T>
__device__ void sq2_item(const ComposeArgs &a, int64_t g, int j, int s, int bx, double *nu) {
  // chunk bx: outputs [bx kBlock, (bx + 1) kBlock)
  const int lane = threadIdx.x & 63;
  const int64_t box = wave_box(a, g);
  const NeuronRec &r = a.recs[box * a.h + j];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // the previous item's reads of nu are done
  __builtin_amdgcn_wave_barrier();
  {
    const T *p = in_tensor<T>(a, box, j, s);
    const NuSource ns = nu_of(a, &r, s);
    for (int64_t i = lane; i < a.Cin; i += 64) {
      double v = (double)p[i];
      if (i == 0) v += ns.shift - ns.lo;
      nu[i] = v / ns.w;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  T *out = out_tensor<T>(a, box, j, s);
  double rsum = 0.0, l1sum = 0.0;
  const int64_t K1 = min((int64_t)(bx + 1) * kBlock, a.Cout);
  for (int64_t K = (int64_t)bx * kBlock + lane; K < K1; K += 64) {
    double v = 0.0;
    if (K < a.Sm[2]) {
      double acc = 0.0;
      const int e = a.sq_off[K + 1];
      for (int q = a.sq_off[K]; q < e; ++q) {
        const int2 pr = a.sq_pairs[q];
        acc = fma(nu[pr.x], nu[pr.y], acc);
      }
      acc = acc + acc;
      const int d = a.sq_diag[K];
      if (d >= 0) acc = fma(nu[d], nu[d], acc);
      v = r.c[2] * acc;
      if (K < a.Cin) v = fma(r.c[1], nu[K], v);
      if (K == 0) v += r.c[0] - (s == 1 ? r.e : 0.0);
    }
    store(out + K, v, rsum, l1sum);
  }
  if (a.part) {  // the chunk's own slot
    for (int off = 32; off > 0; off >>= 1) {
      rsum += __shfl_xor(rsum, off, 64);
      l1sum += __shfl_xor(l1sum, off, 64);
    }
    const int64_t it = item_of(a, g, j, s);
    if (lane == 0) {
      a.part[(it * pslots(a) + bx) * 2 + 0] = rsum;
      a.part[(it * pslots(a) + bx) * 2 + 1] = l1sum;
    }
    if (bx == 0)  // the slots past this class's chunks
      for (int64_t b = a.nbx + lane; b < pslots(a); b += 64)
        a.part[(it * pslots(a) + b) * 2 + 0] = a.part[(it * pslots(a) + b) * 2 + 1] = 0.0;
  }
}

// Both bounds of a neuron in one wave (nu of each in the wave's LDS): every
// pair of the table is read once for the two sums; each bound's sums are
// those of sq2_item, in the same order.
template <typename T>
__device__ void sq2_pair(const ComposeArgs &a, int64_t g, int j, int bx, double *nu) {
  const int lane = threadIdx.x & 63;
  const int64_t box = wave_box(a, g);
  const NeuronRec &r = a.recs[box * a.h + j];
  double *nu0 = nu, *nu1 = nu + a.Cin;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // the previous item's reads of nu are done
  __builtin_amdgcn_wave_barrier();
  for (int s = 0; s < 2; ++s) {
    const T *p = in_tensor<T>(a, box, j, s);
    const NuSource ns = nu_of(a, &r, s);
    double *q = s == 0 ? nu0 : nu1;
    for (int64_t i = lane; i < a.Cin; i += 64) {
      double v = (double)p[i];
      if (i == 0) v += ns.shift - ns.lo;
      q[i] = v / ns.w;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  T *out0 = out_tensor<T>(a, box, j, 0), *out1 = out_tensor<T>(a, box, j, 1);
  double rsum0 = 0.0, l1sum0 = 0.0, rsum1 = 0.0, l1sum1 = 0.0;
  const int64_t K1 = min((int64_t)(bx + 1) * kBlock, a.Cout);
  for (int64_t K = (int64_t)bx * kBlock + lane; K < K1; K += 64) {
    double v0 = 0.0, v1 = 0.0;
    if (K < a.Sm[2]) {
      double acc0 = 0.0, acc1 = 0.0;
      const int e = a.sq_off[K + 1];
      for (int q = a.sq_off[K]; q < e; ++q) {
        const int2 pr = a.sq_pairs[q];
        acc0 = fma(nu0[pr.x], nu0[pr.y], acc0);
        acc1 = fma(nu1[pr.x], nu1[pr.y], acc1);
      }
      acc0 = acc0 + acc0;
      acc1 = acc1 + acc1;
      const int d = a.sq_diag[K];
      if (d >= 0) {
        acc0 = fma(nu0[d], nu0[d], acc0);
        acc1 = fma(nu1[d], nu1[d], acc1);
      }
      v0 = r.c[2] * acc0;
      v1 = r.c[2] * acc1;
      if (K < a.Cin) {
        v0 = fma(r.c[1], nu0[K], v0);
        v1 = fma(r.c[1], nu1[K], v1);
      }
      if (K == 0) {
        v0 += r.c[0] - 0.0;
        v1 += r.c[0] - r.e;
      }
    }
    store(out0 + K, v0, rsum0, l1sum0);
    store(out1 + K, v1, rsum1, l1sum1);
  }
  if (a.part) {  // each bound's own slot for the chunk
    for (int off = 32; off > 0; off >>= 1) {
      rsum0 += __shfl_xor(rsum0, off, 64);
      l1sum0 += __shfl_xor(l1sum0, off, 64);
      rsum1 += __shfl_xor(rsum1, off, 64);
      l1sum1 += __shfl_xor(l1sum1, off, 64);
    }
    for (int s = 0; s < 2; ++s) {
      const int64_t it = item_of(a, g, j, s);
      if (lane == 0) {
        a.part[(it * pslots(a) + bx) * 2 + 0] = s == 0 ? rsum0 : rsum1;
        a.part[(it * pslots(a) + bx) * 2 + 1] = s == 0 ? l1sum0 : l1sum1;
      }
      if (bx == 0)  // the slots past this class's chunks
        for (int64_t b = a.nbx + lane; b < pslots(a); b += 64)
          a.part[(it * pslots(a) + b) * 2 + 0] = a.part[(it * pslots(a) + b) * 2 + 1] = 0.0;
    }
  }
}

// Grouped order-2 neurons, both bounds per wave (a.group > 1, at most 64):
// lane b finds whether the slot's item b is one (all at once), and the
// lanes read the square table's ranges of their outputs in the slot's chunk
// once; the wave then runs the neurons in item order, loading each one's
// coefficients (at most 128 per bound) and record fields ahead of the
// previous neuron's products and stores. Every sum is that of sq2_pair, in
// the same order.
template <typename T>
struct Sq2Job {
  const T *p0, *p1;  // pre tensors of the two bounds
  T *out0, *out1;    // post tensors
  int64_t it;        // item of the upper bound (the lower bound's is it + 1)
  double f;          // lane f < 8: field f of the record (c0, c1, c2, e, lo, hi, epsU, epsL)
  T x[4];            // the lane's first two coefficients of each bound (Cin <= 128)
};

template <typename T>
__device__ inline Sq2Job<T> sq2_job(const ComposeArgs &a, int64_t box, int j) {
  const int lane = threadIdx.x & 63;
  Sq2Job<T> J;
  J.p0 = in_tensor<T>(a, box, j, 0);
  J.p1 = in_tensor<T>(a, box, j, 1);
  J.out0 = out_tensor<T>(a, box, j, 0);
  J.out1 = out_tensor<T>(a, box, j, 1);
  J.it = (box * a.h + j) * a.nbounds;
  const NeuronRec &r = a.recs[box * a.h + j];
  const int fl = lane & 7;
  const double *fp = fl < 3 ? &r.c[fl] : fl == 3 ? &r.e : fl == 4 ? &r.lo : fl == 5 ? &r.hi : fl == 6 ? &r.epsU : &r.epsL;
  J.f = *fp;
  J.x[0] = J.x[1] = J.x[2] = J.x[3] = (T)0;
  if (a.Cin <= 128) {
    if (lane < a.Cin) {
      J.x[0] = J.p0[lane];
      J.x[2] = J.p1[lane];
    }
    if (lane + 64 < a.Cin) {
      J.x[1] = J.p0[lane + 64];
      J.x[3] = J.p1[lane + 64];
    }
  }
  return J;
}

// The square table's range and diagonal of the lane's outputs in a chunk.
struct Sq2Tab {
  int off[kBlock / 64], end[kBlock / 64], diag[kBlock / 64];
};

template <typename T>
__device__ void sq2_pair_run(const ComposeArgs &a, const Sq2Job<T> &J, int bx, double *nu, const Sq2Tab &tb) {
  const int lane = threadIdx.x & 63;
  const double c0 = lane_f64(J.f, 0), c1 = lane_f64(J.f, 1), c2 = lane_f64(J.f, 2), e = lane_f64(J.f, 3);
  const double lo = lane_f64(J.f, 4), hi = lane_f64(J.f, 5);
  const double shift0 = a.fp64 ? 0.0 : lane_f64(J.f, 6), shift1 = a.fp64 ? 0.0 : -lane_f64(J.f, 7);
  const double w = hi - lo;  // nu_s = (p_s + shift_s [I = 0] - lo) / w
  double *nu0 = nu, *nu1 = nu + a.Cin;
  wave_sync();  // the previous neuron's reads of nu are done
  for (int s = 0; s < 2; ++s) {
    const T *p = s == 0 ? J.p0 : J.p1;
    const double a0 = (s == 0 ? shift0 : shift1) - lo;
    double *q = s == 0 ? nu0 : nu1;
    if (a.Cin <= 128) {
      for (int u = 0; u < 2; ++u) {
        const int i = lane + 64 * u;
        if (i < a.Cin) {
          double v = (double)J.x[2 * s + u];
          if (i == 0) v += a0;
          q[i] = v / w;
        }
      }
    } else {
      for (int64_t i = lane; i < a.Cin; i += 64) {
        double v = (double)p[i];
        if (i == 0) v += a0;
        q[i] = v / w;
      }
    }
  }
  wave_sync();
  double rsum0 = 0.0, l1sum0 = 0.0, rsum1 = 0.0, l1sum1 = 0.0;
  const int64_t K1 = min((int64_t)(bx + 1) * kBlock, a.Cout);
#pragma unroll
  for (int t = 0; t < kBlock / 64; ++t) {
    const int64_t K = (int64_t)bx * kBlock + lane + 64 * t;
    if (K >= K1) continue;
    double v0 = 0.0, v1 = 0.0;
    if (K < a.Sm[2]) {
      double acc0 = 0.0, acc1 = 0.0;
      int q = tb.off[t];
      const int qe = tb.end[t];
      for (; q < qe; ++q) {
        const int2 pr = a.sq_pairs[q];
        acc0 = fma(nu0[pr.x], nu0[pr.y], acc0);
        acc1 = fma(nu1[pr.x], nu1[pr.y], acc1);
      }
      acc0 = acc0 + acc0;
      acc1 = acc1 + acc1;
      const int d = tb.diag[t];
      if (d >= 0) {
        acc0 = fma(nu0[d], nu0[d], acc0);
        acc1 = fma(nu1[d], nu1[d], acc1);
      }
      v0 = c2 * acc0;
      v1 = c2 * acc1;
      if (K < a.Cin) {
        v0 = fma(c1, nu0[K], v0);
        v1 = fma(c1, nu1[K], v1);
      }
      if (K == 0) {
        v0 += c0 - 0.0;
        v1 += c0 - e;
      }
    }
    store(J.out0 + K, v0, rsum0, l1sum0);
    store(J.out1 + K, v1, rsum1, l1sum1);
  }
  if (a.part) {  // each bound's own slot for the chunk
    for (int off = 32; off > 0; off >>= 1) {
      rsum0 += __shfl_xor(rsum0, off, 64);
      l1sum0 += __shfl_xor(l1sum0, off, 64);
      rsum1 += __shfl_xor(rsum1, off, 64);
      l1sum1 += __shfl_xor(l1sum1, off, 64);
    }
    for (int s = 0; s < 2; ++s) {
      const int64_t it = J.it + s;
      if (lane == 0) {
        a.part[(it * pslots(a) + bx) * 2 + 0] = s == 0 ? rsum0 : rsum1;
        a.part[(it * pslots(a) + bx) * 2 + 1] = s == 0 ? l1sum0 : l1sum1;
      }
      if (bx == 0)  // the slots past this class's chunks
        for (int64_t b = a.nbx + lane; b < pslots(a); b += 64)
          a.part[(it * pslots(a) + b) * 2 + 0] = a.part[(it * pslots(a) + b) * 2 + 1] = 0.0;
    }
  }
}

template <typename T>
__device__ void sq2_pair_grouped(const ComposeArgs &a, double *nu) {
  const int64_t per = (int64_t)a.h * a.nbounds, total = launch_items(a);
  const int grp = a.group, chunks = (int)a.nbx;
  const int64_t slots = (total + grp - 1) / grp * chunks;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int lane = threadIdx.x & 63;
  for (int64_t w0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w0 < slots; w0 += stride) {
    const int bx = (int)(w0 % chunks);
    const int64_t i0 = w0 / chunks * grp;
    int64_t mbox = 0;
    int mj = 0;
    bool mine = false;
    if (lane < grp && i0 + lane < total) {
      const int64_t it = i0 + lane, g = it / per;
      const int rest = (int)(it - g * per);
      mj = rest / a.nbounds;
      mbox = wave_box(a, g);
      mine = rest % a.nbounds == 0 && a.recs[mbox * a.h + mj].kind == 2;
    }
    unsigned long long todo = __ballot(mine);
    if (!todo) continue;
    Sq2Tab tb;
    const int64_t K1 = min((int64_t)(bx + 1) * kBlock, a.Cout);
#pragma unroll
    for (int t = 0; t < kBlock / 64; ++t) {
      const int64_t K = (int64_t)bx * kBlock + lane + 64 * t;
      tb.off[t] = tb.end[t] = 0;
      tb.diag[t] = -1;
      if (K < K1 && K < a.Sm[2]) {
        tb.off[t] = a.sq_off[K];
        tb.end[t] = a.sq_off[K + 1];
        tb.diag[t] = a.sq_diag[K];
      }
    }
    int b = __ffsll((long long)todo) - 1;
    todo &= todo - 1;
    Sq2Job<T> J = sq2_job<T>(a, lane_i64(mbox, b), lane_int(mj, b));
    while (true) {
      const bool more = todo != 0;
      Sq2Job<T> K;
      if (more) {
        b = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        K = sq2_job<T>(a, lane_i64(mbox, b), lane_int(mj, b));
      }
      sq2_pair_run(a, J, bx, nu, tb);
      if (!more) break;
      J = K;
    }
  }
}

// kPair: both bounds per wave (the items of bound 1 are then skipped).
template <typename T, bool kPair>
__global__ void __launch_bounds__(kBlock) compose_sq2_kernel(ComposeArgs a) {
  extern __shared__ double lds_nu[];
  double *nu = lds_nu + (threadIdx.x >> 6) * (kPair ? 2 : 1) * a.Cin;  // the wave's nu
  if constexpr (kPair) {
    if (a.group > 1) {
      sq2_pair_grouped<T>(a, nu);
      return;
    }
    for_wave_items(a, (int)a.nbx, [](int kind, int s) { return kind == 2 && s == 0; },
                   [&](int64_t g, int j, int, int bx) { sq2_pair<T>(a, g, j, bx, nu); });
  } else {
    for_wave_items(a, (int)a.nbx, [](int kind, int) { return kind == 2; },
                   [&](int64_t g, int j, int s, int bx) { sq2_item<T>(a, g, j, s, bx, nu); });
  }

}

// Orders L >= 3: Horner steps Q^(m) = nu Q^(m-1) + c_{L-1-m}, m = 1 .. L-1,
// with Q^(0) = c_L nu + c_{L-1}; Q^(m) has degree (m+1) Din and step m reads
// the product table (Din, m Din). Intermediates stay in FP64 scratch; the
// last step subtracts e for the lower bound and stores the post tensor.
template <typename T>
__global__ void __launch_bounds__(kBlock) compose_hz_kernel(ComposeArgs a, int m) {
  extern __shared__ double nu[];
  const int j = blockIdx.y / a.nbounds, s = blockIdx.y % a.nbounds;
  const int64_t nb = launch_boxes(a);
  for (int64_t g = blockIdx.z; g < nb; g += gridDim.z) {
  const int64_t box = wave_box(a, g);
  const NeuronRec &r = a.recs[box * a.h + j];
  const int L = r.kind;
  if (L < 3 || m > L - 1) continue;  // uniform over the block
  __syncthreads();                    // the previous item's reads of nu are done
  load_nu(a, in_tensor<T>(a, box, j, s), nu_of(a, &r, s), nu);
  const bool last = (m == L - 1);
  const int64_t it = item_of(a, g, j, s);
  double *scr = reinterpret_cast<double *>(a.scratch);
  const double *qprev = scr + (it * 2 + ((m - 1) & 1)) * a.Cq;
  double *qcur = scr + (it * 2 + (m & 1)) * a.Cq;
  const double cL = r.c[L], cL1 = r.c[L - 1], cadd = r.c[L - 1 - m];
  const int64_t Sq = a.Sm[m + 1];  // coefficients of Q^(m)
  const int64_t Ct = last ? a.Cout : Sq;
  const int *off = a.hz_off[m];
  const int2 *pairs = a.hz_pairs[m];
  const int64_t K0 = (int64_t)blockIdx.x * kBlock, K1 = min(K0 + kBlock, Ct);
  double rsum = 0.0, l1sum = 0.0;
  for (int64_t K = K0 + threadIdx.x; K < K1; K += blockDim.x) {
    double v = 0.0;
    if (K < Sq) {
      const int e = off[K + 1];
      for (int q = off[K]; q < e; ++q) {
        const int2 pr = pairs[q];
        const double qv = (m == 1) ? fma(cL, nu[pr.y], pr.y == 0 ? cL1 : 0.0) : qprev[pr.y];
        v = fma(nu[pr.x], qv, v);
      }
      if (K == 0) v += cadd - ((last && s == 1) ? r.e : 0.0);
    }
    if (last)
      store(out_tensor<T>(a, box, j, s) + K, v, rsum, l1sum);
    else
      qcur[K] = v;
  }
  if (last && a.part) block_partials(a, it, rsum, l1sum);
  }
}

// ---------------------------------------------- post radii (FP32 mode)
// One thread per (box, neuron, bound): fold the blocks' partial sums and add the
// analytic part of the radius of each post polynomial:
//  * the perturbation of nu by FP64 rounding: |nu~ - nu| <= dnu in sup norm,
//    and since nu and nu~ stay in [0, 1 + dnu] on the box,
//    |Q(nu~) - Q(nu)| <= sum_j |c_j| j dnu (1 + dnu)^(j-1);
//  * the rounding of the approximant's coefficients (dB);
//  * FP64 accumulation of the products: gamma(L (C + 4)) sum_j |c_j| N^j with
//    N >= ||nu~||_1 + 1.
__global__ void post_radii_kernel(ComposeArgs a, NeuronRec *recs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.nboxes * a.h * 2) return;
  const int64_t item = t >> 1;
  const int s = (int)(t & 1);
  const int64_t box = wave_box(a, item / a.h);
  const int j = (int)(item % a.h);
  NeuronRec &r = recs[box * a.h + j];
  const int kind = r.kind;
  // coefficients of the stored pre-activation tensors (degree r.dpre)
  double cin = 1.0;
  for (int q = 1; q <= a.n; ++q) cin = cin * (r.dpre + q) / q;
  {
    const int64_t it = (box * a.h + j) * 2 + s;
    double rs = 0.0, l1 = 0.0;
    if (kind != kActive && kind != kInactive) {  // stored by one of the kernels above
      for (int64_t b = 0; b < pslots(a); ++b) {
        rs += a.part[(it * pslots(a) + b) * 2 + 0];
        l1 += a.part[(it * pslots(a) + b) * 2 + 1];
      }
    }
    const double eps_pre = s == 0 ? r.epsU : r.epsL;
    const double l1_pre = s == 0 ? r.l1U : r.l1L;
    double pad = 0.0;
    if (kind == kInactive) {
      l1 = 0.0;
    } else if (kind == kActive) {
      pad = eps_pre;
      l1 = l1_pre;
    } else if (kind == kFallback) {
      pad = rs + (s == 0 ? r.fbpadU : r.fbpadL);
    } else {
      const double w = r.hi - r.lo;
      const double src = l1_pre + eps_pre + fabs(r.lo);
      const double dnu = gamma64(6) * src / w;
      const double N = src / w * (1.0 + gamma64(6)) + 1.0;
      // (1 + dnu)^(j-1) by repeated products: exact for j <= 2, within an
      // ulp per further factor after (covered by kPadSafety)
      double t1 = 0.0, t3 = 0.0, pw = 1.0, gr = 1.0;
      for (int jj = 1; jj <= kind; ++jj) {
        t1 += fabs(r.c[jj]) * jj * dnu * gr;
        gr *= 1.0 + dnu;
      }
      for (int jj = 0; jj <= kind; ++jj) {
        t3 += fabs(r.c[jj]) * pw;
        pw *= N;
      }
      pad = rs + t1 + r.dB + gamma64((double)kind * (cin + 4.0)) * t3;
    }
    pad *= kPadSafety;
    if (s == 0) {
      r.padU = pad;
      r.pl1U = l1;
    } else {
      r.padL = pad;
      r.pl1L = l1;
    }
    if (a.rad) {  // padU, padL, pl1U, pl1L: this bound's two
      double *q = a.rad + (box * a.h + j) * 4;
      q[s] = pad;
      q[2 + s] = l1;
    }
  }
}

// ------------------------------------- periodic linearisation (Lin)
// One wave per (box, neuron, bound): the neuron's post polynomial as a full
// tensor of Cout coefficients (degree Dout) in the post arena, for the
// mode-2 read-off. Composed neurons (order >= 2) already hold it; order-1
// and fallback ones hold their first Cs coefficients; active ones take their
// pre-activation (Cin coefficients, Din <= Dout); the rest is zero, which in
// the total-degree layout is the elevation to Dout (Prop. 4).
template <typename T>
__global__ void __launch_bounds__(64) lin_stage_kernel(ComposeArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t items = launch_items(a);
  for (int64_t w = blockIdx.x; w < items; w += gridDim.x) {
  const int64_t g = w / ((int64_t)a.h * a.nbounds);
  const int rest = (int)(w - g * a.h * a.nbounds);
  const int j = rest / a.nbounds, s = rest - j * a.nbounds;
  const int64_t box = wave_box(a, g);
  const int kind = a.recs[box * a.h + j].kind;
  if (kind >= 2) continue;
  const BoxDeg bd = box_deg(a, box);
  T *out = out_tensor<T>(a, box, j, s, bd.Cout);
  int64_t from = 0;
  if (kind == kActive) {  // degree Din <= Dout (the box's post degree is the largest)
    const T *p = in_tensor<T>(a, box, j, s, bd.Cin);
    const int64_t cc = min(bd.Cin, bd.Cout);
    for (int64_t I = lane; I < cc; I += 64) out[I] = p[I];
    from = cc;
  } else if (kind == 1 || kind == kFallback) {
    from = bd.Cs;
  }
  for (int64_t I = from + lane; I < bd.Cout; I += 64) out[I] = (T)0;
  }
}

// One thread per (box, neuron): the linearised posts (fbU, fbL) stored at
// degree 1, n + 1 coefficients per tensor, and the record updated: degree 1,
// FP32 radii = the linearisation's radius plus the exact rounding of the
// stores, l1 norms of the stored coefficients. Inactive neurons store
// nothing (they stay out of the next affine map's lists).
template <typename T>
__global__ void __launch_bounds__(kBlock) lin_scatter_kernel(ComposeArgs a, NeuronRec *recs) {
  const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= a.nboxes * a.h) return;
  const int64_t box = wave_box(a, item / a.h);
  const int j = (int)(item % a.h);
  NeuronRec &r = recs[box * a.h + j];
  const int64_t C1 = a.n + 1;
  double pad[2] = {0.0, 0.0}, l1[2] = {0.0, 0.0};
  if (r.kind != kInactive) {
    for (int s = 0; s < 2; ++s) {
      const double *fb = s == 0 ? r.fbU : r.fbL;
      T *out = reinterpret_cast<T *>(a.post) + box * a.slot_out + ((int64_t)j * 2 + s) * C1;
      double rs = 0.0;
      for (int q = 0; q <= a.n; ++q) store(out + q, fb[q], rs, l1[s]);
      if (!a.fp64) pad[s] = ((s == 0 ? r.fbpadU : r.fbpadL) + rs) * kPadSafety;
    }
  }
  r.deg = r.kind == kInactive ? 0 : 1;
  r.padU = pad[0];
  r.padL = pad[1];
  r.pl1U = l1[0];
  r.pl1L = l1[1];
  if (a.rad) {
    double *q = a.rad + (box * a.h + j) * 4;
    q[0] = pad[0];
    q[1] = pad[1];
    q[2] = l1[0];
    q[3] = l1[1];
  }
}

hipError_t launch_lin_stage(const ComposeArgs &a_in, hipStream_t s) {
  if (a_in.nboxes < 1) return hipSuccess;
  // a class below its pre degree (Dout < Din) holds fallback and inactive
  // neurons only (with per-box degrees this holds by construction: a box's
  // post degree is the largest of its neurons')
  const bool per_box = a_in.box_din || a_in.box_dout;
  if ((!per_box && a_in.Cs > a_in.Cout) || a_in.nbounds != 2) return hipErrorInvalidValue;
  ComposeArgs a = a_in;
  a.group = 1;
  if (per_box) a.counts.fill(a.n);
  const int64_t items = a.nboxes * a.h * a.nbounds;
  ProfScope ps(kProfLin, s, 0.0);
  if (a.fp64)
    hipLaunchKernelGGL(lin_stage_kernel<double>, dim3((unsigned)dev_grid(items, a.dcount)), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(lin_stage_kernel<float>, dim3((unsigned)dev_grid(items, a.dcount)), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lin_scatter(const ComposeArgs &a, hipStream_t s) {
  if (a.nboxes < 1) return hipSuccess;
  if (!a.recs || !a.post || a.dcount) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((a.nboxes * a.h + kBlock - 1) / kBlock);
  ProfScope ps(kProfLin, s, 0.0);
  if (a.fp64)
    hipLaunchKernelGGL(lin_scatter_kernel<double>, dim3(blocks), dim3(kBlock), 0, s, a,
                       const_cast<NeuronRec *>(a.recs));
  else
    hipLaunchKernelGGL(lin_scatter_kernel<float>, dim3(blocks), dim3(kBlock), 0, s, a,
                       const_cast<NeuronRec *>(a.recs));
  return hipGetLastError();
}

// ------------------------------------------------ plain product kernel
template <typename T>
__global__ void __launch_bounds__(kBlock) polymul_kernel(int n, int da, int db, int64_t count, const T *A, const T *B,
                                                         T *out) {
  const int dc = da + db;
  const int64_t Ca = ipow(da + 1, n), Cb = ipow(db + 1, n), Cc = ipow(dc + 1, n);
  const int64_t it = blockIdx.y;
  for (int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; K < Cc; K += (int64_t)gridDim.x * blockDim.x) {
    int k[kMaxInputs], lo_[kMaxInputs], hi_[kMaxInputs], i[kMaxInputs];
    int64_t rem = K;
    for (int q = n - 1; q >= 0; --q) {
      k[q] = (int)(rem % (dc + 1));
      rem /= (dc + 1);
    }
    for (int q = 0; q < n; ++q) {
      lo_[q] = max(0, k[q] - db);
      hi_[q] = min(k[q], da);
      i[q] = lo_[q];
    }
    double v = 0.0;
    bool more = true;
    while (more) {
      int64_t iI = 0, iJ = 0;
      for (int q = 0; q < n; ++q) {
        iI = iI * (da + 1) + i[q];
        iJ = iJ * (db + 1) + (k[q] - i[q]);
      }
      v = fma((double)A[it * Ca + iI], (double)B[it * Cb + iJ], v);
      int q = n - 1;
      for (; q >= 0; --q) {
        if (i[q] < hi_[q]) {
          ++i[q];
          break;
        }
        i[q] = lo_[q];
      }
      if (q < 0) more = false;
    }
    out[it * Cc + K] = (T)v;
  }
}

// ------------------------------------------------------------ dispatch
static int sq_ni(int n, int D) { return (D <= 4 && n >= 2) ? 2 : 1; }

// LDS bytes of the square kernel for (n, D), or 0 if there is none.
static size_t sq_lds(int n, int D) {
  if (D < 1 || D > 8) return 0;
  const int NI = sq_ni(n, D);
  const int64_t R = ipow(D + 1, NI), RP = (R + 1) & ~1;
  const int64_t nrows = ipow(D + 1, n) / R;
  return (size_t)nrows * RP * sizeof(double) + (size_t)((nrows + 15) & ~15);
}

static bool sq_handles(int n, int Din, int Dout) {
  const size_t l = sq_lds(n, Din);
  return l > 0 && l <= device_lds_limit() && Dout >= 2 * Din;
}

int64_t compose_nbx(int64_t Cout) { return std::max<int64_t>(1, (Cout + kBlock - 1) / kBlock); }

// Threads of the per-item composition blocks: one wave (most items return
// at once by kind; the few that work loop over their kBlock outputs).
constexpr unsigned kComposeThreads = 64;

template <typename T, int D, int NI>
static hipError_t launch_sq(const ComposeArgs &a, hipStream_t s) {
  const size_t lds = sq_lds(a.n, D);
  RET_IF(hipFuncSetAttribute((const void *)compose_sq_kernel<T, D, NI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  const int64_t Mo = ipow(a.Dout + 1, a.n - NI);
  dim3 grid((unsigned)((Mo + kBlock - 1) / kBlock), (unsigned)(a.h * a.nbounds), (unsigned)a.nboxes);
  ProfScope ps(a.recs ? kProfComposeSquare : kProfPolyMul, s, 0.0);
  hipLaunchKernelGGL((compose_sq_kernel<T, D, NI>), grid, dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

// Launch the square kernel if one handles this degree; returns that degree
// (or -1 when the Horner path must take the order-2 neurons).
template <typename T>
static int sq_dispatch(const ComposeArgs &a, hipStream_t s, hipError_t &err) {
  const int D = a.Din;
  err = hipSuccess;
  if (!sq_handles(a.n, D, a.Dout)) return -1;
  const bool ni2 = sq_ni(a.n, D) == 2;
  switch (D) {
    case 1: err = ni2 ? launch_sq<T, 1, 2>(a, s) : launch_sq<T, 1, 1>(a, s); break;
    case 2: err = ni2 ? launch_sq<T, 2, 2>(a, s) : launch_sq<T, 2, 1>(a, s); break;
    case 3: err = ni2 ? launch_sq<T, 3, 2>(a, s) : launch_sq<T, 3, 1>(a, s); break;
    case 4: err = ni2 ? launch_sq<T, 4, 2>(a, s) : launch_sq<T, 4, 1>(a, s); break;
    case 5: err = launch_sq<T, 5, 1>(a, s); break;
    case 6: err = launch_sq<T, 6, 1>(a, s); break;
    case 7: err = launch_sq<T, 7, 1>(a, s); break;
    case 8: err = launch_sq<T, 8, 1>(a, s); break;
    default: return -1;
  }
  return err == hipSuccess ? D : -1;
}

// Waves per block of the one-wave-per-item kernels (scatter, square).
constexpr int kComposeWaves = 1;

template <typename T>
static hipError_t compose_all(const ComposeArgs &a_in, hipStream_t s) {
  ComposeArgs a = a_in;
  // with a device count the lists and radii are the caller's, over all boxes
  if ((a.dcount || a.stage != 0) && (!a.lists_ready || !a.radii_later)) return hipErrorInvalidValue;
  const unsigned gx = (unsigned)a.nbx;
  // many items: a wave takes a group of items and reads their kinds at
  // once; 16 for the scatter (its items are few and light), 8 for the
  // square (heavier items, which the group's wave takes one after another)
  const int64_t items_all = a.nboxes * a.h * a.nbounds;
  const bool group = items_all >= 65536;
  if (a.live && !a.lists_ready) {
    ProfScope ps(kProfMisc, s, 0.0);
    hipLaunchKernelGGL(live_kernel, dim3((unsigned)((a.nboxes + kBlock / 64 - 1) / (kBlock / 64))), dim3(kBlock), 0,
                       s, a);
    RET_IF(hipGetLastError());
  }
  if (a.stage != 2) {
    ProfScope ps(kProfComposeSimple, s, 0.0);
    ComposeArgs ag = a;
    ag.group = group ? 16 : 1;
    const int64_t waves = (items_all + ag.group - 1) / ag.group;
    hipLaunchKernelGGL(compose_scatter_kernel<T>,
                       dim3((unsigned)dev_grid((waves + kComposeWaves - 1) / kComposeWaves, a.dcount)),
                       dim3(64 * kComposeWaves), 0, s, ag);
    RET_IF(hipGetLastError());
  }
  const size_t lds = (size_t)a.Cin * sizeof(double);
  if (a.stage == 1) return hipSuccess;  // the products run per class
  if (a.box_din || a.box_dout) return hipErrorInvalidValue;  // products take one (Din, Dout) class
  if (a.Lmax >= 2) {
    if (!a.sq_off || kComposeWaves * lds > device_lds_limit() || (int64_t)gx * kBlock < a.Cout)
      return hipErrorInvalidValue;
    // both bounds of a neuron per wave when their two nu fit
    const bool pair = a.nbounds == 2 && 2 * kComposeWaves * lds <= device_lds_limit();
    const void *k = pair ? (const void *)compose_sq2_kernel<T, true> : (const void *)compose_sq2_kernel<T, false>;
    const size_t klds = (pair ? 2 : 1) * kComposeWaves * lds;
    RET_IF(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)klds));
    ComposeArgs ag = a;
    ag.group = group ? 8 : 1;
    const int64_t waves = (items_all + ag.group - 1) / ag.group * a.nbx;
    ProfScope ps(kProfComposeSquare, s, 0.0);
    const dim3 grid((unsigned)dev_grid((waves + kComposeWaves - 1) / kComposeWaves, a.dcount));
    if (pair)
      hipLaunchKernelGGL((compose_sq2_kernel<T, true>), grid, dim3(64 * kComposeWaves), klds, s, ag);
    else
      hipLaunchKernelGGL((compose_sq2_kernel<T, false>), grid, dim3(64 * kComposeWaves), klds, s, ag);
    RET_IF(hipGetLastError());
  }
  if (a.Lmax >= 3) {
    RET_IF(hipFuncSetAttribute((const void *)compose_hz_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    for (int m = 1; m <= a.Lmax - 1; ++m) {
      if (!a.hz_off[m]) return hipErrorInvalidValue;
      dim3 grid(gx, (unsigned)(a.h * a.nbounds), (unsigned)dev_grid(a.nboxes, a.dcount, (int64_t)gx * a.h * a.nbounds));
      ProfScope ps(kProfComposeHorner, s, 0.0);
      hipLaunchKernelGGL(compose_hz_kernel<T>, grid, dim3(kComposeThreads), lds, s, a, m);
      RET_IF(hipGetLastError());
    }
  }
  if (a.part && !a.radii_later) RET_IF(launch_post_radii(a, s));
  return hipSuccess;
}

hipError_t launch_post_radii(const ComposeArgs &a, hipStream_t s) {
  if (!a.part || !a.recs || a.dcount) return hipErrorInvalidValue;
  ProfScope ps(kProfMisc, s, 0.0);
  hipLaunchKernelGGL(post_radii_kernel, dim3((unsigned)((a.nboxes * a.h * 2 + 63) / 64)), dim3(64), 0, s, a,
                     const_cast<NeuronRec *>(a.recs));
  return hipGetLastError();
}

hipError_t launch_live(const ComposeArgs &a, hipStream_t s) {
  if (!a.live || a.nboxes < 1 || a.dcount) return hipErrorInvalidValue;
  ProfScope ps(kProfMisc, s, 0.0);
  hipLaunchKernelGGL(live_kernel, dim3((unsigned)((a.nboxes + kBlock / 64 - 1) / (kBlock / 64))), dim3(kBlock), 0, s,
                     a);
  return hipGetLastError();
}

hipError_t launch_compose(const ComposeArgs &a_in, hipStream_t s) {
  ComposeArgs a = a_in;
  if (a.box_din || a.box_dout) a.counts.fill(a.n);
  return a.fp64 ? compose_all<double>(a, s) : compose_all<float>(a, s);
}

size_t compose_scratch_bytes(int64_t Cq, int Lmax, int h, int64_t nboxes) {
  if (Lmax < 3) return 0;
  return align256((size_t)nboxes * h * 2 * 2 * Cq * sizeof(double));
}

hipError_t launch_poly_mul(int n, int da, int db, int64_t count, const void *A, const void *B, void *out, int fp64,
                           hipStream_t s) {
  const int64_t Cc = ipow(da + db + 1, n);
  if (A == B && da == db && sq_handles(n, da, 2 * da)) {
    ComposeArgs a{};
    a.n = n;
    a.Din = da;
    a.Dout = 2 * da;
    a.h = 1;
    a.nbounds = 1;
    a.Lmax = 2;
    a.Cin = ipow(da + 1, n);
    a.Cout = Cc;
    a.slot_in = a.Cin;
    a.slot_out = Cc;
    a.bids = nullptr;
    a.nboxes = count;
    a.pre = A;
    a.post = out;
    a.recs = nullptr;
    a.part = nullptr;
    a.fp64 = fp64;
    hipError_t err = hipSuccess;
    const int d = fp64 ? sq_dispatch<double>(a, s, err) : sq_dispatch<float>(a, s, err);
    RET_IF(err);
    if (d == da) return hipSuccess;
  }
  const int64_t blocks = std::min<int64_t>((Cc + kBlock - 1) / kBlock, 4096);
  dim3 grid((unsigned)blocks, (unsigned)count);
  ProfScope ps(kProfPolyMul, s, 0.0);
  if (fp64)
    hipLaunchKernelGGL(polymul_kernel<double>, grid, dim3(kBlock), 0, s, n, da, db, count, (const double *)A,
                       (const double *)B, (double *)out);
  else
    hipLaunchKernelGGL(polymul_kernel<float>, grid, dim3(kBlock), 0, s, n, da, db, count, (const float *)A,
                       (const float *)B, (float *)out);
  return hipGetLastError();
}

}  // namespace bern
