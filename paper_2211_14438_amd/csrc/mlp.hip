// Degree predictor: a small MLP 8 -> 64 -> 64 -> 4 (ReLU hidden layers) that
// proposes, for each unstable neuron, the order of its Bernstein ReLU
// approximant (classes 1, 2, 3) or the linear fallback (class 0). Any class
// yields sound bounds (Props. 1-2 hold for every order; the fallback is
// sound by Def. 2), so the predictor only trades tightness for work.
//
// Parameter vector (FP32), in this order:
//   mean[8], std[8]            feature normalisation (not trained)
//   W1[64][8], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]
//
// Training kernels are FP32 and deterministic (fixed summation order): the
// forward pass stores both hidden activations, the backward pass forms the
// per-record deltas and then sums the weight gradients over the batch with one
// thread per parameter. Inference inside the bounds pipeline runs in BF16
// (weights and activations rounded to BF16, FP32 accumulation).
#include "common.hpp"
#include "rules.hpp"

namespace bern {

constexpr int kF = 8, kH = 64, kC = 4;
constexpr int kOffMean = 0, kOffStd = 8, kOffW1 = 16, kOffB1 = kOffW1 + kH * kF, kOffW2 = kOffB1 + kH,
              kOffB2 = kOffW2 + kH * kH, kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kC * kH, kParams = kOffB3 + kC;
static_assert(kParams == 5012, "parameter layout");

__device__ inline float bf16_round(float x) {
  // round to nearest even on the upper 16 bits (finite inputs)
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// Forward pass, one thread per record. hid (optional): [N][128] = h1 | h2.
__global__ void __launch_bounds__(256) mlp_forward_kernel(const float *P, int64_t N, const float *X, float *logits,
                                                          float *hid, int bf16) {
  __shared__ float w[kParams];
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) w[i] = bf16 && i >= kOffW1 ? bf16_round(P[i]) : P[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  float x[kF], h1[kH];
  for (int f = 0; f < kF; ++f) {
    float v = (X[r * kF + f] - w[kOffMean + f]) / w[kOffStd + f];
    x[f] = bf16 ? bf16_round(v) : v;
  }
  for (int o = 0; o < kH; ++o) {
    float s = w[kOffB1 + o];
    for (int f = 0; f < kF; ++f) s = fmaf(w[kOffW1 + o * kF + f], x[f], s);
    s = fmaxf(s, 0.f);
    h1[o] = bf16 ? bf16_round(s) : s;
    if (hid) hid[r * 2 * kH + o] = h1[o];
  }
  float z[kC];
  for (int c = 0; c < kC; ++c) z[c] = w[kOffB3 + c];
  for (int o = 0; o < kH; ++o) {
    float s = w[kOffB2 + o];
    for (int i = 0; i < kH; ++i) s = fmaf(w[kOffW2 + o * kH + i], h1[i], s);
    s = fmaxf(s, 0.f);
    if (bf16) s = bf16_round(s);
    if (hid) hid[r * 2 * kH + kH + o] = s;
    for (int c = 0; c < kC; ++c) z[c] = fmaf(w[kOffW3 + c * kH + o], s, z[c]);
  }
  for (int c = 0; c < kC; ++c) logits[r * kC + c] = z[c];
}

// Per-record deltas of the mean softmax cross-entropy:
// dZ = (softmax(z) - onehot(y)) / N, dH2 = (W3^T dZ) * [h2 > 0],
// dH1 = (W2^T dH2) * [h1 > 0]. Also the per-record loss terms.
__global__ void __launch_bounds__(256) mlp_delta_kernel(const float *P, int64_t N, const float *logits,
                                                        const int8_t *y, const float *hid, float *dz, float *dh,
                                                        float *lossr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  float z[kC], m = -INFINITY;
  for (int c = 0; c < kC; ++c) {
    z[c] = logits[r * kC + c];
    m = fmaxf(m, z[c]);
  }
  float se = 0.f;
  for (int c = 0; c < kC; ++c) se += expf(z[c] - m);
  const int lab = y[r];
  lossr[r] = (logf(se) + m - z[lab]) / (float)N;
  float d[kC];
  for (int c = 0; c < kC; ++c) {
    d[c] = (expf(z[c] - m) / se - (c == lab ? 1.f : 0.f)) / (float)N;
    dz[r * kC + c] = d[c];
  }
  const float *h1 = hid + r * 2 * kH, *h2 = h1 + kH;
  float d2[kH];
  for (int o = 0; o < kH; ++o) {
    float s = 0.f;
    for (int c = 0; c < kC; ++c) s = fmaf(P[kOffW3 + c * kH + o], d[c], s);
    d2[o] = h2[o] > 0.f ? s : 0.f;
    dh[r * 2 * kH + kH + o] = d2[o];
  }
  for (int i = 0; i < kH; ++i) {
    float s = 0.f;
    for (int o = 0; o < kH; ++o) s = fmaf(P[kOffW2 + o * kH + i], d2[o], s);
    dh[r * 2 * kH + i] = h1[i] > 0.f ? s : 0.f;
  }
}

// Weight gradients: one thread per trainable parameter, sum over the batch
// in record order. Also the total loss (thread of parameter 0).
__global__ void __launch_bounds__(256) mlp_grad_kernel(const float *P, int64_t N, const float *X, const float *hid,
                                                       const float *dz, const float *dh, const float *lossr,
                                                       float *G, float *loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  double s = 0.0;
  if (p < kOffW1) {
    s = 0.0;  // normalisation is fixed
  } else if (p < kOffB1) {
    const int o = (p - kOffW1) / kF, f = (p - kOffW1) % kF;
    const float mu = P[kOffMean + f], sd = P[kOffStd + f];
    for (int64_t r = 0; r < N; ++r) s += (double)dh[r * 2 * kH + o] * (double)((X[r * kF + f] - mu) / sd);
  } else if (p < kOffW2) {
    const int o = p - kOffB1;
    for (int64_t r = 0; r < N; ++r) s += dh[r * 2 * kH + o];
  } else if (p < kOffB2) {
    const int o = (p - kOffW2) / kH, i = (p - kOffW2) % kH;
    for (int64_t r = 0; r < N; ++r) s += (double)dh[r * 2 * kH + kH + o] * hid[r * 2 * kH + i];
  } else if (p < kOffW3) {
    const int o = p - kOffB2;
    for (int64_t r = 0; r < N; ++r) s += dh[r * 2 * kH + kH + o];
  } else if (p < kOffB3) {
    const int c = (p - kOffW3) / kH, o = (p - kOffW3) % kH;
    for (int64_t r = 0; r < N; ++r) s += (double)dz[r * kC + c] * hid[r * 2 * kH + kH + o];
  } else {
    const int c = p - kOffB3;
    for (int64_t r = 0; r < N; ++r) s += dz[r * kC + c];
  }
  G[p] = (float)s;
  if (p == 0 && loss) {
    double l = 0.0;
    for (int64_t r = 0; r < N; ++r) l += lossr[r];
    *loss = (float)l;
  }
}

// Adam step on the trainable parameters (normalisation entries untouched).
__global__ void mlp_adam_kernel(float *P, const float *G, float *m, float *v, int64_t step, float lr, float b1,
                                float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kOffW1 || p >= kParams) return;
  const float g = G[p];
  m[p] = b1 * m[p] + (1.f - b1) * g;
  v[p] = b2 * v[p] + (1.f - b2) * g * g;
  const float mh = m[p] / (1.f - powf(b1, (float)step));
  const float vh = v[p] / (1.f - powf(b2, (float)step));
  P[p] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void argmax_kernel(int64_t N, const float *logits, int8_t *cls) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  int best = 0;
  for (int c = 1; c < kC; ++c)
    if (logits[r * kC + c] > logits[r * kC + best]) best = c;
  cls[r] = (int8_t)best;
}

// ------------------------------------------------ predictor in the pipeline
// Eight features of one hidden neuron from its record (interval, affine fits
// of the Bernstein control nets) and its downstream sensitivity s_j:
//   f0 = -lo/w (where zero sits in [lo, hi]), f1 = log w, f2 = layer/(H-1),
//   f3 = log(D+1), f4 = mean gap of the Bernstein coefficients of U^ and L^
//   over w, f5 = log(s_j w), f6 = spread of the fit remainders over w,
//   f7 = slope mass of the upper fit over w;  w = hi - lo.
__device__ void neuron_features(const LearnArgs &a, const NeuronRec &r, int j, float *f) {
  double w = r.hi - r.lo;
  if (!(w > 1e-300)) w = 1e-300;
  const double iw = 1.0 / w;
  double slope = 0.0;
  for (int ax = 0; ax < a.n; ++ax) slope += fabs(r.fitU[1 + ax]);
  f[0] = (float)(-r.lo * iw);
  f[1] = (float)log(w);
  f[2] = a.H > 1 ? (float)a.layer / (float)(a.H - 1) : 0.f;
  f[3] = logf((float)r.dpre + 1.f);
  f[4] = r.fitted ? (float)((r.fitU[0] - r.fitL[0]) * iw) : 0.f;
  f[5] = (float)log(fmax(a.sens[j] * w, 1e-30));
  f[6] = r.fitted ? (float)(((r.rmaxU - r.rminU) + (r.rmaxL - r.rminL)) * iw) : 0.f;
  f[7] = r.fitted ? (float)(slope * iw) : 0.f;
  for (int q = 0; q < kF; ++q)
    if (!isfinite(f[q])) f[q] = 0.f;
}

__global__ void __launch_bounds__(256) features_kernel(LearnArgs a) {
  const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= a.nboxes * a.h) return;
  const int64_t box = a.bids ? a.bids[it / a.h] : it / a.h;
  const int j = (int)(it % a.h);
  float f[kF];
  neuron_features(a, a.recs[box * a.h + j], j, f);
  for (int q = 0; q < kF; ++q) a.feat[(box * a.nh + a.noff + j) * kF + q] = f[q];
}

// Per box and layer: the layer is stored at the largest degree any of its
// neurons takes, so classes below that degree cost tightness while saving
// only composition and affine-map work. With a.raise they are raised: if
// some unstable neuron takes order >= 2, the others take at least order 2;
// otherwise, if some takes order 1, the fallback neurons take order 1. Then
// apply the rules: one wave per box (list position g), its lanes over the
// neurons.
__device__ void box_rules(const LearnArgs &a, int64_t g, int lane) {
  const int64_t box = a.bids ? a.bids[g] : g;
  int8_t *cl = a.codes + box * a.nh + a.noff;
  int top = -1;  // class as the degree it gives: fallback (0) lowest
  for (int j = lane; j < a.h; j += 64) top = max(top, (int)cl[j]);
  for (int off = 32; off > 0; off >>= 1) top = max(top, __shfl_xor(top, off, 64));
  int deg = 0;
  for (int j = lane; j < a.h; j += 64) {
    NeuronRec &r = a.recs[box * a.h + j];
    int c = cl[j];
    if (c >= 0 && a.raise) {
      if (top >= 2 && c < 2) c = 2;
      else if (top == 1 && c == 0) c = 1;
      cl[j] = (int8_t)c;
    }
    decide_neuron(r, c < 0 ? 1 : c, false, a.L, a.n, r.dpre, a.cap, a.fp64);
    if (a.used) a.used[box * a.nh + a.noff + j] = (int8_t)r.kind;
    deg = max(deg, r.deg);
  }
  if (a.degs) {  // the box's largest post degree, for the next layer's classes
    for (int off = 32; off > 0; off >>= 1) deg = max(deg, __shfl_xor(deg, off, 64));
    if (lane == 0) {
      a.degs[box] = deg;
      if (a.hdegs) a.hdegs[box] = deg;  // the host's copy (mapped host memory)
    }
  }
  if (a.live) {  // the next affine map's input lists (as live_kernel, from the kinds just decided)
    int *lv = a.live + box * a.live_ld;
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int nf = 0, ns = 0, na = 0;
    for (int j0 = 0; j0 < a.h; j0 += 64) {
      const int j = j0 + lane;
      const int kind = j < a.h ? a.recs[box * a.h + j].kind : (int)kInactive;
      const bool full = kind >= 2, small = kind == 1 || kind == kFallback, act = kind == kActive;
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
}

__global__ void __launch_bounds__(256) learned_rules_kernel(LearnArgs a) {
  const int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (g < a.nboxes) box_rules(a, g, (int)(threadIdx.x & 63));
}

// Features -> BF16 MLP -> class. A block takes kClassItems (box, neuron)
// items: one thread each reads the features, and the unstable items (the
// only ones whose rule depends on the predictor; the others get class -1)
// are listed. The block's waves then take the listed items in turn: lane o
// holds hidden unit o's weights of both hidden layers in registers (loaded
// once per wave), computes unit o of each layer, and passes the layer to
// the other lanes through the wave's LDS row. The output layer is summed
// as four quarters of 16 hidden units each, each quarter in ascending unit
// order (lanes 4c .. 4c + 3 for class c), added as (q0 + q1) + (q2 + q3):
// every sum in the same order as a neuron taken by four threads, so the
// class does not depend on the form or on where the item sits in the list.
constexpr int kClassItems = 256;  // items per block of learned_classes_kernel
constexpr int kClassWaves = 16;   // waves per block
static_assert(kClassItems < 64 * kClassWaves, "threads past the items stage the weights");

__device__ inline float mlp_param(const float *P, int i) { return i >= kOffW1 ? bf16_round(P[i]) : P[i]; }

// The MLP of the listed unstable items u = wv, wv + kClassWaves, ... by one
// wave (see learned_classes_kernel).
__device__ void classes_of_wave(const LearnArgs &a, int wv, int nu, int lane, const float *fs, const int *ulist,
                                float *hr, const float *w3s, const float *w1s, const float *w2s) {
  const float *P = a.params;
  // lane o: unit o's weights (from the block's padded rows in LDS); lanes
  // 4c + k (16 lanes): class c over the quarter k of the second hidden layer
  float w1[kF], w2[kH];
  const int o = lane;
  for (int q = 0; q < kF; ++q) w1[q] = w1s[o * (kF + 1) + q];
  for (int i = 0; i < kH; ++i) w2[i] = w2s[o * (kH + 1) + i];
  const float b1 = mlp_param(P, kOffB1 + o), b2 = mlp_param(P, kOffB2 + o);
  const int oc = (lane >> 2) & (kC - 1), ok = lane & 3;
  const float *w3 = w3s + oc * kH + ok * (kH / 4);
  const float b3 = mlp_param(P, kOffB3 + oc);
  for (int u = wv; u < nu; u += kClassWaves) {
    const int slot = ulist[u];
    float s1 = b1;
    for (int q = 0; q < kF; ++q) s1 = fmaf(w1[q], fs[slot * kF + q], s1);
    const float h1 = bf16_round(fmaxf(s1, 0.f));
    wave_sync();  // the row's previous readers are done
    hr[o] = h1;
    wave_sync();
    float s2 = b2;
    for (int i = 0; i < kH; ++i) s2 = fmaf(w2[i], hr[i], s2);
    const float h2 = bf16_round(fmaxf(s2, 0.f));
    wave_sync();
    hr[o] = h2;
    wave_sync();
    float z = ok == 0 ? b3 : 0.f;
    for (int v = 0; v < kH / 4; ++v) z = fmaf(w3[v], hr[ok * (kH / 4) + v], z);
    z += __shfl_xor(z, 1, 64);  // (q0 + q1) + (q2 + q3) over lanes 4c .. 4c + 3
    z += __shfl_xor(z, 2, 64);
    float zc[kC];
    for (int c = 0; c < kC; ++c) zc[c] = __shfl(z, 4 * c, 64);
    if (lane == 0) {
      int best = 0;
      for (int c = 1; c < kC; ++c)
        if (zc[c] > zc[best]) best = c;
      const int64_t it = (int64_t)blockIdx.x * kClassItems + slot;
      const int64_t box = a.bids ? a.bids[it / a.h] : it / a.h;
      a.codes[box * a.nh + a.noff + (int)(it % a.h)] = (int8_t)best;
    }
  }
}

// kRules: the block's items are whole boxes (h divides kClassItems), and
// once every class is written the block applies their rules (box_rules),
// one wave per box, in place of learned_rules_kernel.
template <bool kRules>
__global__ void __launch_bounds__(64 * kClassWaves) learned_classes_kernel(LearnArgs a) {
  __shared__ float fs[kClassItems][kF];
  __shared__ int ulist[kClassItems];  // the block's unstable items (slots), in no fixed order
  __shared__ int ucount;
  __shared__ float hrow[kClassWaves][kH];  // per wave: the hidden layer passed between lanes
  __shared__ float w3s[kC * kH];           // the output layer's weights
  __shared__ float w1s[kH * (kF + 1)];     // the hidden layers' weights, rows padded by one
  __shared__ float w2s[kH * (kH + 1)];     //   (a lane reading its row hits its own bank)
  if (threadIdx.x == 0) ucount = 0;
  __syncthreads();
  // the items' features (the first kClassItems threads) and the weights (the
  // other threads) load at once, behind one barrier
  if (threadIdx.x >= kClassItems) {
    const int t0 = threadIdx.x - kClassItems, nt = blockDim.x - kClassItems;
    for (int i = t0; i < kC * kH; i += nt) w3s[i] = mlp_param(a.params, kOffW3 + i);
    for (int i = t0; i < kH * kF; i += nt) w1s[(i / kF) * (kF + 1) + i % kF] = mlp_param(a.params, kOffW1 + i);
    for (int i = t0; i < kH * kH; i += nt) w2s[(i / kH) * (kH + 1) + i % kH] = mlp_param(a.params, kOffW2 + i);
  }
  // features of the block's items, one thread each; only unstable neurons
  // (lo < 0 < hi) go through the network
  if (threadIdx.x < kClassItems) {
    const int slot = threadIdx.x;
    const int64_t it = (int64_t)blockIdx.x * kClassItems + slot;
    if (it < a.nboxes * a.h) {
      const int64_t box = a.bids ? a.bids[it / a.h] : it / a.h;
      const int j = (int)(it % a.h);
      const NeuronRec &r = a.recs[box * a.h + j];
      // a stable neuron's record is read no further than its interval (the
      // first cache line) unless the features are exported
      const bool unstable = r.lo < 0.0 && r.hi > 0.0;
      if (unstable || a.feat) {
        float f[kF];
        neuron_features(a, r, j, f);
        // the network's input: the features normalised and rounded to BF16
        for (int q = 0; q < kF; ++q) fs[slot][q] = bf16_round((f[q] - a.params[kOffMean + q]) / a.params[kOffStd + q]);
        if (a.feat)
          for (int q = 0; q < kF; ++q) a.feat[(box * a.nh + a.noff + j) * kF + q] = f[q];
      }
      if (unstable)
        ulist[atomicAdd(&ucount, 1)] = slot;
      else
        a.codes[box * a.nh + a.noff + j] = -1;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nu = ucount;
  if (wv < nu) classes_of_wave(a, wv, nu, lane, &fs[0][0], ulist, hrow[wv], w3s, w1s, w2s);
  if constexpr (kRules) {
    __syncthreads();  // every class of the block's boxes written
    const int per = kClassItems / a.h;
    const int64_t g = (int64_t)blockIdx.x * per + wv;
    if (wv < per && g < a.nboxes) box_rules(a, g, lane);
  }
}

hipError_t launch_learned_rules(const LearnArgs &a, hipStream_t s) {
  {
    ProfScope ps(kProfPredictor, s, 0.0);
    const dim3 grid((unsigned)((a.nboxes * a.h + kClassItems - 1) / kClassItems)), block(64 * kClassWaves);
    if (kClassItems % a.h == 0 && kClassItems / a.h <= kClassWaves) {  // whole boxes per block: rules fused
      hipLaunchKernelGGL(learned_classes_kernel<true>, grid, block, 0, s, a);
      return hipGetLastError();
    }
    hipLaunchKernelGGL(learned_classes_kernel<false>, grid, block, 0, s, a);
    RET_IF(hipGetLastError());
  }
  ProfScope ps(kProfPredictor, s, 0.0);
  hipLaunchKernelGGL(learned_rules_kernel, dim3((unsigned)((a.nboxes + 3) / 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_features(const LearnArgs &a, hipStream_t s) {
  ProfScope ps(kProfMisc, s, 0.0);
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((a.nboxes * a.h + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

int mlp_params() { return kParams; }

hipError_t launch_mlp_forward(const float *P, int64_t N, const float *X, float *logits, float *hid, int bf16,
                              hipStream_t s) {
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, P, N, X, logits, hid,
                     bf16);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *P, int64_t N, const float *X, const int8_t *y, float *G, float *loss,
                               float *scratch, hipStream_t s) {
  float *logits = scratch;                 // [N][4]
  float *hid = logits + N * kC;            // [N][128]
  float *dz = hid + N * 2 * kH;            // [N][4]
  float *dh = dz + N * kC;                 // [N][128]
  float *lossr = dh + N * 2 * kH;          // [N]
  RET_IF(launch_mlp_forward(P, N, X, logits, hid, 0, s));
  hipLaunchKernelGGL(mlp_delta_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, P, N, logits, y, hid, dz,
                     dh, lossr);
  RET_IF(hipGetLastError());
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, P, N, X, hid, dz, dh, lossr, G,
                     loss);
  return hipGetLastError();
}

size_t mlp_backward_scratch(int64_t N) { return (size_t)N * (2 * kC + 4 * kH + 1) * sizeof(float); }

hipError_t launch_mlp_adam(float *P, const float *G, float *m, float *v, int64_t step, float lr, float b1, float b2,
                           float eps, hipStream_t s) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, P, G, m, v, step, lr, b1, b2,
                     eps);
  return hipGetLastError();
}

hipError_t launch_mlp_classify(const float *P, int64_t N, const float *X, float *logits, int8_t *cls, int bf16,
                               hipStream_t s) {
  RET_IF(launch_mlp_forward(P, N, X, logits, nullptr, bf16, s));
  hipLaunchKernelGGL(argmax_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, logits, cls);
  return hipGetLastError();
}

}  // namespace bern
