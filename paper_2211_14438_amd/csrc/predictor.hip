// Degree predictor files and training (host side of the learned plan).
//
// bern_pred_train fits the MLP of mlp.hip to (features, class) records with
// the library's own FP32 kernels: mean softmax cross-entropy, minibatch Adam
// with a cosine learning-rate schedule. The host only shuffles the records
// and moves them; every forward, backward and update step runs on the GPU.
// The trained parameters go to a file that bern_pred_load reads:
//   bytes 0..7   "BERNPRED"
//   uint32       format version (1)
//   uint32       number of parameters (bern_pred_params())
//   float32[]    the parameters, in bern_pred_params() order
//   uint32       length of a free-form metadata text, then its bytes
// all little-endian.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"

namespace bern {

static const char kMagic[8] = {'B', 'E', 'R', 'N', 'P', 'R', 'E', 'D'};
constexpr uint32_t kFormat = 1;

// SplitMix64 (Steele, Lea and Flood, 2014): the k-th output of a stream.
static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
static double unit_open(uint64_t bits) { return ((bits >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
// Standard normal from two uniforms (Box-Muller).
static double normal_at(uint64_t seed, uint64_t k) {
  const double u1 = unit_open(splitmix64(seed ^ (2 * k))), u2 = unit_open(splitmix64(seed ^ (2 * k + 1)));
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

static bern_status write_file(const char *path, const std::vector<float> &P, const char *meta) {
  FILE *f = std::fopen(path, "wb");
  if (!f) {
    set_error("cannot open %s for writing", path);
    return BERN_E_ARG;
  }
  const uint32_t ver = kFormat, np = (uint32_t)P.size();
  const uint32_t ml = meta ? (uint32_t)std::strlen(meta) : 0;
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&ver, 4, 1, f) == 1 && std::fwrite(&np, 4, 1, f) == 1 &&
            std::fwrite(P.data(), 4, P.size(), f) == P.size() && std::fwrite(&ml, 4, 1, f) == 1 &&
            (ml == 0 || std::fwrite(meta, 1, ml, f) == ml);
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) {
    set_error("writing %s failed", path);
    return BERN_E_ARG;
  }
  return BERN_OK;
}

}  // namespace bern

using namespace bern;

extern "C" bern_status bern_pred_load(const char *path, bern_pred **out) {
  if (!path || !out) {
    set_error("null path or output");
    return BERN_E_ARG;
  }
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) {
    set_error("cannot open %s", path);
    return BERN_E_ARG;
  }
  char magic[8];
  uint32_t ver = 0, np = 0;
  const bool head = std::fread(magic, 1, 8, f) == 8 && std::fread(&ver, 4, 1, f) == 1 && std::fread(&np, 4, 1, f) == 1;
  if (!head || std::memcmp(magic, kMagic, 8) != 0 || ver != kFormat || (int64_t)np != mlp_params()) {
    std::fclose(f);
    set_error("%s is not a predictor file of format %u with %d parameters", path, kFormat, mlp_params());
    return BERN_E_ARG;
  }
  std::vector<float> P(np);
  const bool body = std::fread(P.data(), 4, np, f) == np;
  std::fclose(f);
  if (!body) {
    set_error("%s is truncated", path);
    return BERN_E_ARG;
  }
  return bern_pred_create(P.data(), (int64_t)np, out);
}

extern "C" void bern_train_opts_default(bern_train_opts *t) {
  if (!t) return;
  std::memset(t, 0, sizeof(*t));
  t->epochs = 40;
  t->batch = 8192;
  t->lr = 3e-3f;
  t->beta1 = 0.9f;
  t->beta2 = 0.999f;
  t->eps = 1e-8f;
  t->seed = 0;
}

extern "C" bern_status bern_pred_train(const float *X, const int8_t *y, int64_t N, const bern_train_opts *t,
                                       const char *path, const char *meta, bern_pred **out) {
  if (out) *out = nullptr;
  if (!X || !y || N < 1 || !t || t->epochs < 1 || t->batch < 1 || !(t->lr > 0.f)) {
    set_error("bad training arguments (N = %lld)", (long long)N);
    return BERN_E_ARG;
  }
  const int F = 8, H = 64, C = 4;
  const int np = mlp_params();
  for (int64_t r = 0; r < N; ++r) {
    if (y[r] < 0 || y[r] >= C) {
      set_error("label %d of record %lld outside 0..3", y[r], (long long)r);
      return BERN_E_ARG;
    }
    for (int q = 0; q < F; ++q)
      if (!std::isfinite(X[r * F + q])) {
        set_error("non-finite feature %d of record %lld", q, (long long)r);
        return BERN_E_NUMERIC;
      }
  }
  const int64_t batch = std::min<int64_t>(t->batch, N);
  // feature normalisation (mean, standard deviation + 1e-3), not trained
  std::vector<float> P(np, 0.f);
  for (int q = 0; q < F; ++q) {
    double s = 0.0, s2 = 0.0;
    for (int64_t r = 0; r < N; ++r) s += X[r * F + q];
    const double mu = s / (double)N;
    for (int64_t r = 0; r < N; ++r) s2 += (X[r * F + q] - mu) * (X[r * F + q] - mu);
    P[q] = (float)mu;
    P[F + q] = (float)(std::sqrt(s2 / (double)N) + 1e-3);
  }
  // He initialisation of W1, W2 (variance 2 / fan-in), W3 with 1 / fan-in; zero biases
  {
    int o = 2 * F;
    uint64_t k = 0;
    for (int i = 0; i < H * F; ++i) P[o + i] = (float)(normal_at(t->seed, k++) * std::sqrt(2.0 / F));
    o += H * F + H;
    for (int i = 0; i < H * H; ++i) P[o + i] = (float)(normal_at(t->seed, k++) * std::sqrt(2.0 / H));
    o += H * H + H;
    for (int i = 0; i < C * H; ++i) P[o + i] = (float)(normal_at(t->seed, k++) * std::sqrt(1.0 / H));
  }
  // device buffers, released on every return
  struct Bufs {
    std::vector<void *> p;
    ~Bufs() {
      for (void *q : p) (void)hipFree(q);
    }
    hipError_t get(void **q, size_t b) {
      *q = nullptr;
      hipError_t e = hipMalloc(q, b);
      if (e == hipSuccess) p.push_back(*q);
      return e;
    }
  } d;
  void *dX, *dy, *dP, *dG, *dm, *dv, *dloss, *dscr;
  const int64_t steps_per_epoch = N / batch;
  BERN_HIP_TRY(d.get(&dX, (size_t)N * F * sizeof(float)));
  BERN_HIP_TRY(d.get(&dy, (size_t)N));
  BERN_HIP_TRY(d.get(&dP, (size_t)np * sizeof(float)));
  BERN_HIP_TRY(d.get(&dG, (size_t)np * sizeof(float)));
  BERN_HIP_TRY(d.get(&dm, (size_t)np * sizeof(float)));
  BERN_HIP_TRY(d.get(&dv, (size_t)np * sizeof(float)));
  BERN_HIP_TRY(d.get(&dloss, (size_t)std::max<int64_t>(steps_per_epoch, 1) * sizeof(float)));
  BERN_HIP_TRY(d.get(&dscr, mlp_backward_scratch(batch)));
  BERN_HIP_TRY(hipMemcpy(dP, P.data(), (size_t)np * sizeof(float), hipMemcpyHostToDevice));
  std::vector<float> zeros(np, 0.f);
  BERN_HIP_TRY(hipMemcpy(dm, zeros.data(), (size_t)np * sizeof(float), hipMemcpyHostToDevice));
  BERN_HIP_TRY(hipMemcpy(dv, zeros.data(), (size_t)np * sizeof(float), hipMemcpyHostToDevice));
  std::vector<int64_t> perm(N);
  for (int64_t r = 0; r < N; ++r) perm[r] = r;
  std::vector<float> Xp((size_t)N * F);
  std::vector<int8_t> yp(N);
  std::vector<float> losses((size_t)std::max<int64_t>(steps_per_epoch, 1));
  hipStream_t s = nullptr;
  int64_t step = 0;
  uint64_t draw = 0;
  for (int ep = 0; ep < t->epochs; ++ep) {
    // Fisher-Yates shuffle with the seeded stream, then the epoch's records in order
    for (int64_t r = N - 1; r > 0; --r) {
      const int64_t q = (int64_t)(splitmix64(t->seed + 0x5851F42D4C957F2Dull * (++draw)) % (uint64_t)(r + 1));
      std::swap(perm[r], perm[q]);
    }
    for (int64_t r = 0; r < N; ++r) {
      std::memcpy(&Xp[(size_t)r * F], &X[perm[r] * F], F * sizeof(float));
      yp[r] = y[perm[r]];
    }
    BERN_HIP_TRY(hipMemcpy(dX, Xp.data(), Xp.size() * sizeof(float), hipMemcpyHostToDevice));
    BERN_HIP_TRY(hipMemcpy(dy, yp.data(), (size_t)N, hipMemcpyHostToDevice));
    const float lr = (float)(t->lr * 0.5 * (1.0 + std::cos(3.141592653589793 * ep / t->epochs)));
    for (int64_t b = 0; b < steps_per_epoch; ++b) {
      const float *xb = reinterpret_cast<const float *>(dX) + b * batch * F;
      const int8_t *yb = reinterpret_cast<const int8_t *>(dy) + b * batch;
      BERN_HIP_TRY(launch_mlp_backward(reinterpret_cast<const float *>(dP), batch, xb, yb,
                                       reinterpret_cast<float *>(dG), reinterpret_cast<float *>(dloss) + b,
                                       reinterpret_cast<float *>(dscr), s));
      ++step;
      BERN_HIP_TRY(launch_mlp_adam(reinterpret_cast<float *>(dP), reinterpret_cast<const float *>(dG),
                                   reinterpret_cast<float *>(dm), reinterpret_cast<float *>(dv), step, lr, t->beta1,
                                   t->beta2, t->eps, s));
    }
    if (t->loss_out) {  // the epoch's mean minibatch loss
      BERN_HIP_TRY(hipMemcpy(losses.data(), dloss, (size_t)steps_per_epoch * sizeof(float), hipMemcpyDeviceToHost));
      double sum = 0.0;
      for (int64_t b = 0; b < steps_per_epoch; ++b) sum += losses[b];
      t->loss_out[ep] = (float)(sum / (double)std::max<int64_t>(steps_per_epoch, 1));
    }
  }
  BERN_HIP_TRY(hipMemcpy(P.data(), dP, (size_t)np * sizeof(float), hipMemcpyDeviceToHost));
  if (path) {
    const bern_status st = write_file(path, P, meta);
    if (st != BERN_OK) return st;
  }
  if (out) return bern_pred_create(P.data(), np, out);
  return BERN_OK;
}
