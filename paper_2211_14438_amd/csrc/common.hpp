// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "bernnn.h"

namespace bern {

constexpr int kMaxInputs = 16;   // n
constexpr int kMaxOrder = 8;     // ReLU approximation order L
constexpr int kBlock = 256;      // threads per block of the streaming kernels

void set_error(const char *fmt, ...);

#define BERN_HIP_TRY(expr)                                                        \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess) {                                                       \
      ::bern::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e),   \
                        __FILE__, __LINE__);                                      \
      return BERN_E_DEVICE;                                                       \
    }                                                                             \
  } while (0)

#define RET_IF(expr)                   \
  do {                                 \
    hipError_t _r = (expr);            \
    if (_r != hipSuccess) return _r;   \
  } while (0)

// (d+1)^n, or -1 when it exceeds `cap`.
inline int64_t tsize(int n, int d, int64_t cap = (int64_t)1 << 40) {
  int64_t s = 1;
  for (int a = 0; a < n; ++a) {
    if (s > cap / (d + 1)) return -1;
    s *= (d + 1);
  }
  return s;
}

__host__ __device__ inline int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// What the library knows about one hidden neuron of one box after its
// pre-activation bounds were read (Step 1) and its rule chosen (Step 2).
struct NeuronRec {
  double lo, hi;          // pre-activation interval [lo, hi]
  double c[kMaxOrder + 1];// over-approximant, power series in u = (y-lo)/(hi-lo)
  double e;               // its value at y = 0 (Prop. 2 shift)
  double padU, padL;      // FP32 mode: rounding radius of the post polynomials
  int32_t kind;           // 0 inactive, -1 active, -2 linear fallback, k >= 1 order k
  int32_t deg;            // per-variable degree of the post polynomials
  // Linear fallback: affine post polynomials a0 + sum_a a_{1+a} t_a (power basis).
  double fbU[kMaxInputs + 1];
  double fbL[kMaxInputs + 1];
};

// Per-neuron kind codes.
enum : int32_t { kInactive = 0, kActive = -1, kFallback = -2 };

// ----------------------------------------------------------- kernel launchers
// Defined in the .hip files; every launcher enqueues on `stream` and returns a
// HIP error code (no host synchronisation).

struct Layer1Args {
  int n, h;
  int64_t nboxes;
  const double *box_lo, *box_hi;  // [B][n]
  const double *W, *b;            // W^(1) [h][n], b^(1) [h], FP64
  void *pre;                      // [B][h][2][2^n]
  int fp64;
};
hipError_t launch_layer1(const Layer1Args &a, hipStream_t s);

struct GemmArgs {
  int hin, h;
  int64_t C, nboxes;
  const void *post;               // [B][hin][2][C]
  void *pre;                      // [B][h][2][C]
  const void *W;                  // [h][hin] in the tensor precision
  const double *b;                // [h]
  int fp64;
};
hipError_t launch_gemm(const GemmArgs &a, hipStream_t s);

struct ConvertArgs {
  int n, D, h, L;                 // L: ReLU order of the plain rule
  int64_t C, nboxes;
  const void *pre;                // [B][h][2][C] power coefficients
  int fp64;
  NeuronRec *recs;                // [B][h] (hidden layers)
  double *out_lo, *out_hi;        // [B][ld_out] bounds written at column col0 + j
  int64_t ld_out, col0;
  int8_t *used;                   // [B][ld_out] or null (hidden layers)
  const int8_t *plan;             // [B][plan_ld] degree codes or null (plain rule)
  int64_t plan_ld, plan_col0;
  int mode;                       // 0 hidden layer, 1 output layer
  double *scratch;                // FP64 staging for tensors too large for LDS
  size_t scratch_bytes;
};
hipError_t launch_convert(const ConvertArgs &a, hipStream_t s);
size_t convert_scratch_bytes(int n, int D, int h, int64_t nboxes);

struct ComposeArgs {
  int n, Din, Dout, h;
  int nbounds;                    // 2 (upper, lower) for the network, 1 for plain products
  int Lmax;                       // largest ReLU order any neuron of the launch may use
  int64_t Cin, Cout, nboxes;
  int64_t Cq;                     // coefficients per Horner intermediate buffer
  const void *pre;                // [B][h][2][Cin]
  void *post;                     // [B][h][2][Cout]
  const NeuronRec *recs;          // [B][h]
  int fp64;
  void *scratch;                  // Horner intermediates for orders >= 3
  size_t scratch_bytes;
};
hipError_t launch_compose(const ComposeArgs &a, hipStream_t s);
size_t compose_scratch_bytes(int n, int Din, int Lmax, int h, int64_t nboxes, int fp64);

// Largest dynamic LDS allocation one block may use on the current device.
size_t device_lds_limit();

// Step-level primitives behind the public entry points of the same names.
hipError_t launch_basis_minmax(int n, int D, int64_t count, const void *coef, int fp64, double *bern,
                               double *mn, double *mx, double *l1, double *scratch, hipStream_t s);
size_t basis_minmax_scratch(int n, int D, int64_t count);
hipError_t launch_poly_mul(int n, int da, int db, int64_t count, const void *A, const void *B, void *out,
                           int fp64, hipStream_t s);
hipError_t launch_relu_poly(int64_t count, int L, const double *lo, const double *hi, double *c, double *e,
                            hipStream_t s);

}  // namespace bern
