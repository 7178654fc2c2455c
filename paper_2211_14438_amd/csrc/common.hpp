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

// Blocks go to the chip's 8 XCDs round-robin (hardware block b to XCD b % 8),
// each XCD with its own L2. xcd_block maps a hardware block index to a
// logical one under which consecutive logical blocks (those sharing inputs)
// run on one XCD: the first 8 floor(n / 8) of n blocks are regrouped, the
// tail keeps its index (a bijection of [0, n)).
__device__ inline int64_t xcd_block(int64_t b, int64_t n) {
  const int64_t full = n / 8 * 8;
  if (b >= full) return b;
  return (b % 8) * (full / 8) + b / 8;
}

// Orders a wave's LDS accesses (and the compiler's) around a point where the
// wave's lanes read what other lanes wrote.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Box-major order with the boxes dealt to the XCDs in turn: hardware block b
// takes item (box, j) of an h-item-per-box launch with box = 8 (b / 8 / h) +
// b % 8 and j = (b / 8) % h, so one box's items share an XCD and its L2, and
// the live boxes under a device count stay spread over all XCDs. The grid
// holds 8 ceil(nboxes / 8) h blocks; blocks past nboxes get -1.
__device__ inline int64_t xcd_item(int64_t b, int h, int64_t nboxes) {
  const int64_t idx = b >> 3, box = (idx / h) * 8 + (b & 7);
  return box < nboxes ? box * h + idx % h : -1;
}
__host__ __device__ inline int64_t xcd_item_blocks(int64_t nboxes, int h) { return (nboxes + 7) / 8 * 8 * h; }

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

// C(n + d, n): the stored coefficients of a degree-d tensor in n variables
// (total-degree layout), on either side; every partial product is exact.
__host__ __device__ inline int64_t stored_count(int n, int d) {
  int64_t r = 1;
  for (int i = 1; i <= n; ++i) r = r * (d + i) / i;
  return r;
}
// A box's degree from a per-box degree array (negative values count as 0).
__device__ inline int box_degree(const int *deg, int64_t box) { return max(deg[box], 0); }

// A box's input lists of an affine map (lv: counts of full, prefix and
// active inputs, then the three lists of h entries each) end with one kind
// byte per input neuron: 0 none, 1 full tensor, 2 degree-Din prefix, 3
// active (read in place).
__host__ __device__ inline unsigned char *live_kinds(int *lv, int h) {
  return reinterpret_cast<unsigned char *>(lv + 3 + 3 * h);
}
__host__ __device__ inline const unsigned char *live_kinds(const int *lv, int h) {
  return reinterpret_cast<const unsigned char *>(lv + 3 + 3 * h);
}

// C(n + d, n) for d < kCountTable, carried by launches with per-box degrees
// (a table lookup instead of the divisions of stored_count on the device).
constexpr int kCountTable = 65;
struct CountTable {
  int64_t c[kCountTable];
  __host__ void fill(int n) {
    for (int d = 0; d < kCountTable; ++d) c[d] = stored_count(n, d);
  }
  __device__ int64_t at(int n, int d) const { return d < kCountTable ? c[d] : stored_count(n, d); }
};

// Launches whose box count lives on the device (a device-side
// classification wrote it to `dcount`): the host only knows the upper bound
// `nboxes`. The read-off and affine-map kernels take the grid of `nboxes`
// boxes and their blocks past the count leave at once (a loop over items
// would keep more values live and cost them occupancy); the composition
// kernels take a grid of at most kDevGrid blocks over which they loop.
// Without a device count the grid covers the items and each block takes one.
constexpr int64_t kDevGrid = 4096;
template <class A>
__device__ __forceinline__ int64_t launch_boxes(const A &a) {
  return a.dcount ? min((int64_t)*a.dcount, a.nboxes) : a.nboxes;
}
inline int64_t dev_grid(int64_t blocks, const int *dcount, int64_t per = 1) {
  const int64_t cap = std::max<int64_t>(1, kDevGrid / std::max<int64_t>(1, per));
  return dcount && blocks > cap ? cap : blocks;
}

// What the library knows about one hidden neuron of one box after its
// pre-activation bounds were read (Step 1) and its rule chosen (Step 2).
// FP32 mode: every stored polynomial p~ carries a radius eps such that the
// exact neuron value stays within [L~(t) - epsL, U~(t) + epsU] on the box.
struct alignas(64) NeuronRec {
  // read by the next layer for every box neuron: kept in the first 64 bytes
  double padU, padL;       // radii of the stored post polynomials
  double pl1U, pl1L;       // sum of |coefficients| of the stored post polynomials
  double lo, hi;           // pre-activation interval [lo, hi] (padded in FP32 mode)
  int32_t kind;            // 0 inactive, -1 active, -2 linear fallback, k >= 1 order k
  int32_t deg;             // per-variable degree of the post polynomials
  double c[kMaxOrder + 1]; // over-approximant, power series in u = (y-lo)/(hi-lo)
  double e;                // its value at y = 0 (Prop. 2 shift), rounded up in FP32 mode
  double dB;               // FP32 mode: bound on the rounding of c (sup over u in [0,1])
  double epsU, epsL;       // radii of the stored pre-activation polynomials
  double l1U, l1L;         // sum of |coefficients| of the stored pre-activation polynomials
  // Linear fallback: affine post polynomials a0 + sum_a a_{1+a} t_a (power basis).
  double fbU[kMaxInputs + 1];
  double fbL[kMaxInputs + 1];
  double fbpadU, fbpadL;   // radii of the fallback's own FP64 arithmetic
  // Least-squares affine fit l(t) = f[0] + sum_a f[1+a] (t_a - 1/2) of the
  // Bernstein control net of U^ and L^, and the range [rmin, rmax] of the
  // remainders b_K - l(K/D) (valid when fitted != 0).
  double fitU[kMaxInputs + 1], fitL[kMaxInputs + 1];
  double rmaxU, rminU, rmaxL, rminL;
  int32_t fitted;
  int32_t dpre;            // per-variable degree of the stored pre-activation polynomials
};

// Rounding-error helpers (FP32 mode). gamma(m) = m u / (1 - m u) for FP64.
__host__ __device__ inline double gamma64(double m) {
  const double u = 1.1102230246251565e-16;  // 2^-53
  return m * u / (1.0 - m * u);
}
// Push an FP64 value outward by more than its own rounding.
__host__ __device__ inline double round_down(double x) { return x - fabs(x) * 8.9e-16 - 1e-300; }
__host__ __device__ inline double round_up(double x) { return x + fabs(x) * 8.9e-16 + 1e-300; }
constexpr double kPadSafety = 1.0 + 1.0 / (1 << 20);  // covers the FP64 sums that build the radii

// Per-neuron kind codes.
enum : int32_t { kInactive = 0, kActive = -1, kFallback = -2 };

// --------------------------------------------------------------- profiling
// When enabled (bern_prof_enable), every kernel launch is bracketed by two
// HIP events recorded on its own stream; bern_prof_read sums the elapsed times
// per kernel class. `bytes` is the launch's algorithmic HBM traffic when the
// shape alone fixes it (0 otherwise).
enum ProfClass : int {
  kProfLayer1 = 0,
  kProfGemm,
  kProfConvertSmall,
  kProfConvertPassA,
  kProfConvertPassB,
  kProfConvertFinal,
  kProfConvertChunk,
  kProfComposeSimple,
  kProfComposeFill,
  kProfComposeSquare,
  kProfComposeHorner,
  kProfPolyMul,
  kProfPredictor,
  kProfMisc,
  kProfLin,
  kProfCount
};
struct ProfScope {
  ProfScope(int cls, hipStream_t s, double bytes, double flops = 0.0);
  ~ProfScope();
  int cls;
  hipStream_t s;
  double bytes, flops;
  void *ev0;
};

// Kernel variants an autotuner may pick; 0 everywhere is the built-in choice.
struct Tune {
  int gemm_wide = 0;    // layers wider than 8: 0 16 rows x 2 inputs/step, 1 16x4, 2 8x2, 3 8x4
                        // (tensors of <= 64 coefficients, packed: 1 16 rows, else 8)
  int gemm_narrow = 0;  // layers of <= 4 neurons: 0 4 rows x 8 inputs/step, 1 4x4, 2 4x16
  int conv_block = 0;   // threads of the block-per-neuron conversion: 0 by LDS use, 1 256, 2 512, 3 1024
  int conv_wave = 0;    // per-neuron read-off: 0 tree, 1 dense (one wave per neuron up to 1024
                        // coefficients, else one block), 2 dense, one block per neuron,
                        // 3 tree with one wave per neuron (more variables folded per round)
};
constexpr int kTuneParams = 4;
constexpr int kTuneVariants[kTuneParams] = {4, 3, 4, 4};

// ----------------------------------------------------------- kernel launchers
// Defined in the .hip files; every launcher enqueues on `stream` and returns a
// HIP error code (no host synchronisation).

// Box addressing shared by the launchers: a launch covers `nboxes` boxes of
// one degree class; box g of the launch is wave box bids[g] (identity when
// bids is null); each wave box owns a fixed slot of `slot_*` elements in the
// tensor arenas, filled densely at the box's own degree.
struct Layer1Args {
  int n, h;
  int64_t nboxes;
  const int *bids;
  int64_t slot;
  const double *box_lo, *box_hi;  // [B][n]
  const double *W, *b;            // W^(1) [h][n], b^(1) [h], FP64
  void *pre;                      // [B][h][2][n+1] (total-degree layout at degree 1)
  int fp64;
  int *flags = nullptr;           // [B] when set: 1 for a box with lo > hi or a non-finite end, else 0
};
hipError_t launch_layer1(const Layer1Args &a, hipStream_t s);

struct GemmArgs {
  int hin, h;
  int64_t C, nboxes;
  const int *bids;
  int64_t slot_in, slot_out;
  const void *post;               // [B][hin][2][C]
  void *pre;                      // [B][h][2][C]
  // Per box input lists: live[0] full post tensors (composed neurons) of C
  // coefficients, indices at live[3..]; live[1] post tensors of order-1 and
  // fallback neurons stored with their first Cs coefficients only, indices
  // at live[3 + hin..]; live[2] active neurons, read in place from their
  // pre-activation tensors (first Cact coefficients, arena `act`), indices at
  // live[3 + 2 hin..]. Inactive neurons contribute nothing.
  const int *live;
  int64_t live_ld;
  int64_t Cs;
  const void *act;                // [B][hin][2][Cact] pre-activations of the previous layer
  int64_t act_slot, Cact;
  const double *WT;               // [hin][hp]: W transposed, rows h..hp-1 zero
  int hp;                         // h rounded up to a multiple of 16
  const double *b;                // [h]
  int fp64;
  double *rpart;                  // FP32 mode: per wave box (stride rpart_slot): [h][2][cblocks]
  int64_t rpart_slot;             //   sums of |fl32(y) - y| per coefficient block
  int64_t cblocks;                // coefficient blocks of the launch (set by the launcher)
  Tune tune;
  const int *dcount = nullptr;    // device count of the launch's boxes (nboxes: its upper bound)
  // Boxes of one post degree but different pre degrees (per-neuron plans):
  // each box's pre degree Din from box_din, its Cact = C(n + Din, n) and
  // Cs = C(n + min(Din, Dout), n); null: Cact and Cs above for every box.
  const int *box_din = nullptr;
  int n = 0, Dout = 0;
  CountTable counts;              // filled by the launcher when box_din is set
};
int64_t gemm_cblocks(int64_t C);
hipError_t launch_gemm(const GemmArgs &a, hipStream_t s);

struct ConvertArgs {
  int n, D, h, L;                 // L: ReLU order of the plain rule
  int64_t C, nboxes;              // C: (D+1)^n, the dense tensor the basis change runs on
  int64_t S;                      // stored coefficients per tensor (total-degree layout)
  const int *didx;                // [S] position of each stored coefficient in the dense tensor
  const int *bids;
  int64_t slot;
  int cap;                        // largest post degree a neuron may take (plan codes are clamped)
  const void *pre;                // [B][h][2][S] power coefficients
  int fp64;
  NeuronRec *recs;                // [B][h] (hidden layers)
  // FP32 mode: inputs of the pre-activation radii
  int layer;                      // 0 = first layer (closed form), else GEMM output
  int hin;
  const NeuronRec *prev;          // [B][hin] records of the previous layer (layer > 0)
  const double *prad;             // [B][hin][4] their padU, padL, pl1U, pl1L (FP32 mode, layer > 0)
  const double *W, *b;            // this layer's W [h][hin] and b [h] (FP64)
  const double *box_lo, *box_hi;  // [B][n] (layer 0)
  int from_box;                   // layer 0 at degree 1, every box (bids null): the read-off forms
                                  // the pre tensors from the box, W and b itself and stores them
  int *flags;                     // with from_box, optional: [B] 1 for an invalid box, else 0
  int *hbad;                      // with from_box, optional: set to 1 (mapped host memory) when a box
                                  // is invalid
  const double *rpart;            // GEMM rounding partials, per wave box (stride rpart_slot):
  int64_t rpart_slot;             //   [h][2][cblocks] (layer > 0)
  int64_t cblocks;
  double *out_lo, *out_hi;        // [B][ld_out] bounds written at column col0 + j
  double *out_eps;                // mode 1, optional: [B][h][2] radii (epsU, epsL) of the output tensors
  int64_t ld_out, col0;
  int8_t *used;                   // [B][ld_out] or null (hidden layers)
  const int8_t *plan;             // [B][plan_ld] degree codes or null (plain rule)
  int64_t plan_ld, plan_col0;
  int learned;                    // rules are chosen later by the predictor (fits always needed)
  int fits;                       // compute the affine fits of every hidden neuron (features)
  int mode;                       // 0 hidden layer, 1 output layer, 2 periodic linearisation
                                  // (Lin): `pre` holds the hidden layer's post tensors at degree
                                  // D, every neuron is fitted, and the affine post (fit plus the
                                  // extreme remainder) goes to the record's fbU / fbL with its
                                  // radius in fbpadU / fbpadL (the stored posts' radii padU /
                                  // padL take the place of the pre-activation radii)
  double *scratch;                // staging and partial extrema for tensors too large for LDS
  size_t scratch_bytes;
  Tune tune;
  // tensors beyond LDS: the child tables of the tree read-off (simplex.hpp
  // TreeTable for degree D), or null
  const int *tree;
  int tree_len;
  int tree_base[17];
  int gextra;                     // rounding steps beyond the per-axis basis change (set by the launcher)
  double gconv;                   // gamma(n (D+2) + 4 + gextra): read-off rounding factor (set by the launcher)
  double gpre;                    // gamma(2 hin + 6): affine-map rounding factor of the radii (set by the launcher)
  // simplex.hpp prefix_table for (D, n), or (D, m) of the split
  // convert_nest(n, D) for tensors beyond LDS; null for degrees without a
  // compile-time kernel
  const int *plist;
  int plist_len;
  const int *dcount = nullptr;    // device count of the launch's boxes (nboxes: its upper bound)
};
hipError_t launch_convert(const ConvertArgs &a, hipStream_t s);

// The output layer's stored tensors of one class as dense power tensors at a
// caller's degree: [box][j][C] in U (upper) and L (lower), zero beyond the
// stored degree, the radii (FP32 mode) folded into the constant term.
struct OutPolyArgs {
  const void *pre;    // the output layer's pre-activation arena, [B][h][2][S] per box slot
  int64_t slot, S, C;
  const int *didx;    // rank -> dense index at the caller's degree
  const int *bids;
  int64_t nboxes;
  int h;
  const double *eps;  // [B][h][2] or null (FP64)
  int fp64;
  double *U, *L;      // [B][h][C], wave boxes
};
hipError_t launch_out_polys(const OutPolyArgs &a, hipStream_t s);
size_t convert_scratch_bytes(int n, int D, int h, int64_t nboxes);
// Whether tensors of n variables and degree D are read off by one block each
// (no staging): the read-offs that can fit every neuron (mode 2 needs it).
bool convert_one_block(int n, int D);
// Whether tensors of n variables and degree D take the tree read-off (they
// then need the TreeTable of degree D).
bool convert_tree(int n, int D);

struct ComposeArgs {
  int n, Din, Dout, h;
  const int *bids;
  int64_t slot_in, slot_out;
  double *part;                   // FP32 mode: [B*h*nbounds][nbx][2] (rounding sum, l1 sum) per block
  int64_t nbx;                    // blocks per item of every compose launch of the layer
  int nbounds;                    // 2 (upper, lower) for the network, 1 for plain products
  int group;                      // set by the launcher: items per wave (for_wave_items)
  int lists_ready;                // the live lists were built for every box (launch_live)
  int64_t pstride;                // partial slots per item (>= nbx; 0: nbx); the slots past nbx hold zeros
  int radii_later;                // launch_post_radii runs once for all the layer's classes
  int Lmax;                       // largest ReLU order any neuron of the launch may use
  int64_t Cin, Cout, nboxes;      // stored coefficients at degrees Din and Dout
  int64_t Cs;                     // stored coefficients of degree-preserving posts (degree min(Din, Dout))
  int64_t Cq;                     // coefficients per Horner intermediate buffer
  int64_t Sm[kMaxOrder + 1];      // Sm[m]: coefficients at degree m * Din
  const int *sq_off;              // square table (Din, Din) (simplex.hpp)
  const int2 *sq_pairs;
  const int *sq_diag;
  const int *hz_off[kMaxOrder];   // product tables (Din, m Din), m = 1 .. Lmax - 1
  const int2 *hz_pairs[kMaxOrder];
  const void *pre;                // [B][h][2][Cin]
  void *post;                     // [B][h][2][Cout]
  const NeuronRec *recs;          // [B][h]
  int fp64;
  void *scratch;                  // Horner intermediates for orders >= 3
  size_t scratch_bytes;
  int *live;                      // per box input lists for the next affine map (GemmArgs::live)
  double *rad;                    // FP32 mode: [B][h][4] copies of the records' padU, padL, pl1U,
                                  // pl1L, read densely by the next layer's radii
  int64_t live_ld;
  int lin;                        // the layer was linearised: every neuron that is not inactive
                                  // holds a full degree-1 post tensor (live lists, Lin launchers)
  const int *dcount = nullptr;    // device count of the launch's boxes (nboxes: its upper bound)
  // Per-box degrees (per-neuron plans, launches over boxes of several
  // classes: the scatter of order-1 and fallback posts, the Lin staging):
  // Din from box_din (null: Din above), Dout from box_dout (null: Dout), and
  // Cin, Cout, Cs from them.
  const int *box_din = nullptr, *box_dout = nullptr;
  int stage = 0;                  // launch_compose: 0 everything, 1 the scatter only, 2 the products only
  CountTable counts;              // filled by the launchers when per-box degrees are set
};
hipError_t launch_compose(const ComposeArgs &a, hipStream_t s);
// The input lists (ComposeArgs::live) of a.nboxes boxes (bids, h, recs,
// live, live_ld used) in one launch; launch_compose then skips them when
// a.lists_ready is set.
hipError_t launch_live(const ComposeArgs &a, hipStream_t s);
// The post radii (FP32 mode) of a.nboxes boxes in one launch (n, h, bids,
// recs, part, pstride or nbx, rad used), after every class's composition.
hipError_t launch_post_radii(const ComposeArgs &a, hipStream_t s);
// Periodic linearisation (Lin) of a hidden layer, around a mode-2 read-off:
// launch_lin_stage writes every neuron's post polynomials of a.nboxes boxes
// (bids) as full tensors of a.Cout coefficients (degree Dout) in the post
// arena: composed ones are already there, order-1 and fallback ones are
// zero-padded past their a.Cs stored coefficients, active ones copied from
// their pre-activations (a.Cin coefficients) and zero-padded, inactive ones
// zeroed. launch_lin_scatter then stores the records' affine posts (fbU /
// fbL) of a.nboxes boxes at degree 1 (n + 1 coefficients per tensor, the
// post arena's layout for Dout = 1), sets each record's degree to 1, and in
// FP32 mode its radii (fbpad plus the stores' rounding) and l1 norms, also
// into a.rad.
hipError_t launch_lin_stage(const ComposeArgs &a, hipStream_t s);
hipError_t launch_lin_scatter(const ComposeArgs &a, hipStream_t s);
// Blocks per item the compose launches of a layer use (partials stride).
int64_t compose_nbx(int64_t Cout);
size_t compose_scratch_bytes(int64_t Cq, int Lmax, int h, int64_t nboxes);

// bern_bounds of the plain rule on a caller-independent scratch buffer,
// allocating nothing (api.hip; used by bern_bounds_noalloc).
bern_status bounds_on_scratch(const bern_net *net, const bern_opts *opts, int64_t n_boxes, const double *box_lo,
                              const double *box_hi, double *neuron_lo, double *neuron_hi, double *out_lo,
                              double *out_hi, int8_t *used_plan, void *scratch, size_t scratch_bytes, void *stream,
                              bern_stats *stats);

// Largest dynamic LDS allocation one block may use on the current device.
size_t device_lds_limit();

struct LearnArgs {
  int n, h, H, layer;
  int64_t nboxes;
  const int *bids;
  NeuronRec *recs;                // [B][h]
  const double *sens;             // downstream sensitivity of this layer's neurons [h]
  float *feat;                    // [B][nh][8] (column block noff); optional copy of the features
  int64_t nh, noff;
  const float *params;            // predictor parameters (FP32 master copy)
  int8_t *codes;                  // [B][nh] predicted codes (column block noff)
  int8_t *used;                   // [B][nh] or null
  int *degs;                      // [B] or null: each box's largest post degree (the rules kernel)
  int *hdegs = nullptr;           // [B] or null: the same, into mapped host memory
  int cap, fp64, L;
  int raise;                      // raise classes below the layer's top class (bern_opts.no_raise == 0)
  int *live = nullptr;            // or null: the next affine map's input lists, written with the rules
  int64_t live_ld = 0;            //   (live_kernel's layout, per box stride live_ld)
};
// features -> (optional) BF16 MLP -> codes -> rules, for one class of boxes.
hipError_t launch_learned_rules(const LearnArgs &a, hipStream_t s);
// features only (any plan), for collecting training records.
hipError_t launch_features(const LearnArgs &a, hipStream_t s);

int mlp_params();
hipError_t launch_mlp_forward(const float *P, int64_t N, const float *X, float *logits, float *hid, int bf16,
                              hipStream_t s);
hipError_t launch_mlp_backward(const float *P, int64_t N, const float *X, const int8_t *y, float *G, float *loss,
                               float *scratch, hipStream_t s);
size_t mlp_backward_scratch(int64_t N);
hipError_t launch_mlp_adam(float *P, const float *G, float *m, float *v, int64_t step, float lr, float b1, float b2,
                           float eps, hipStream_t s);
hipError_t launch_mlp_classify(const float *P, int64_t N, const float *X, float *logits, int8_t *cls, int bf16,
                               hipStream_t s);

// Step-level primitives behind the public entry points of the same names.
hipError_t launch_basis_minmax(int n, int D, int64_t count, const void *coef, int fp64, double *bern,
                               double *mn, double *mx, double *l1, double *scratch, hipStream_t s);
size_t basis_minmax_scratch(int n, int D, int64_t count);
hipError_t launch_poly_mul(int n, int da, int db, int64_t count, const void *A, const void *B, void *out,
                           int fp64, hipStream_t s);
hipError_t launch_relu_poly(int64_t count, int L, const double *lo, const double *hi, double *c, double *e,
                            hipStream_t s);

}  // namespace bern
