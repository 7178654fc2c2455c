// C ABI of the bound-propagation library: validation, planning of degrees and
// workspace, waves of boxes, and the per-layer launch sequence (the top-level loop of
// Section 5.3: input initialisation, then for each layer the affine map of
// Section 5.2, the bounds of Step 1, the approximant of Step 2 and the
// composition of Step 3, and finally the output bounds).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "simplex.hpp"
#include "volume.hpp"

namespace bern {

static thread_local char g_err[1024] = "";
static thread_local bool g_no_alloc = false;

bool no_alloc_active() { return g_no_alloc; }

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

// ---------------------------------------------------------------- profiler
static std::mutex g_prof_mu;
static bool g_prof_on = false;
struct ProfRec {
  int cls;
  hipEvent_t a, b;
  double bytes, flops;
};
static std::vector<ProfRec> g_prof;
static std::vector<hipEvent_t> g_pool;  // idle events, created ahead of the timed work

static hipEvent_t pool_get() {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (g_no_alloc) return nullptr;  // no new events: the launch goes untimed
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static void pool_fill(size_t n) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  while (g_pool.size() < n) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) break;
    g_pool.push_back(e);
  }
}

ProfScope::ProfScope(int c, hipStream_t st, double by, double fl)
    : cls(c), s(st), bytes(by), flops(fl), ev0(nullptr) {
  if (!g_prof_on) return;
  hipEvent_t e = pool_get();
  if (!e) return;
  if (hipEventRecord(e, s) != hipSuccess) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_pool.push_back(e);
    return;
  }
  ev0 = e;
}

ProfScope::~ProfScope() {
  if (!ev0) return;
  hipEvent_t e = pool_get();
  if (!e || hipEventRecord(e, s) != hipSuccess) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_pool.push_back((hipEvent_t)ev0);
    if (e) g_pool.push_back(e);
    return;
  }
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof.push_back({cls, (hipEvent_t)ev0, e, bytes, flops});
}

static const char *kProfNames[kProfCount] = {
    "layer1",          "gemm",         "convert_small",  "convert_passA",  "convert_passB", "convert_final",
    "convert_chunk",   "compose_scatter", "compose_fill", "compose_square", "compose_horner", "poly_mul",
    "predictor",       "misc",         "lin"};

size_t device_lds_limit() {
  static std::mutex mu;
  static int cached[64];
  static bool init[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
  std::lock_guard<std::mutex> g(mu);
  if (!init[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 64 * 1024;
    cached[dev] = v;
    init[dev] = true;
  }
  return (size_t)cached[dev];
}

// Device-side classes of per-neuron plans (no host round trip, so the wave
// can be captured as one graph): every pre degree a box can hold at each
// layer and every (pre, post) pair the rules can give at each hidden layer.
// A neuron of a box at pre degree Din takes degree 0 (inactive), Din
// (active, order 1), k Din (order k <= the plan's largest: 3 for the
// predictor's classes, kMaxOrder for given codes; k Din within the layer's
// cap) or 1 (the linear fallback); the box's post degree is the largest, so
// the pairs are (0, {0, 1}) and (Din, {0, 1} + {k Din}). Every pair is
// launched with its device count, an empty one costing its launches, so
// the device path is taken only while the pairs stay few.
constexpr int kMaxDevLists = 64;  // lists per hidden layer: pairs + the next layer's pre degrees
constexpr int kMaxDevPairs = 48;  // pairs over all hidden layers

struct DevClasses {
  std::vector<std::vector<int>> din;                    // [layer] pre degrees, ascending
  std::vector<std::vector<std::pair<int, int>>> pairs;  // [hidden layer] (Din, Dout)
  std::vector<std::vector<int>> dout;                   // [hidden layer] post degrees, ascending
  int slots = 0;                                        // lists per layer: pairs, then post degrees
};

// Host-side plan of one network under one set of options: degree of every
// layer's pre-activation and post tensors and the per-box workspace layout.
struct Plan {
  int H, n, L, Lmax, mode;
  int lin;                          // periodic linearisation: every lin-th hidden layer (0 off)
  int lin_layers;                   // hidden layers linearised
  bool fp64;
  std::vector<int> Dpre, Dpost;     // per layer i = 1..H (index i-1); Dpost for hidden layers
  std::vector<int64_t> Cpre, Cpost;
  size_t elem;
  std::vector<int64_t> nbx;         // compose blocks per item, hidden layers
  // per-box bytes of each region
  size_t recs, rad, arenaA, arenaB, conv, horner, flags, gpart, cpart, live, oeps;
  size_t per_box() const {
    return 2 * recs + 2 * rad + 2 * arenaA + arenaB + conv + horner + flags + gpart + cpart + live + oeps;
  }
  size_t list_ints = 0;             // ints per box of the class id lists
  bool dev_ok = false;              // per-neuron plan whose classes the device can list
  DevClasses dc;
};

static bool dev_classes(const Plan &p, DevClasses &dc) {
  const int top = p.mode == BERN_PLAN_LEARNED ? 3 : kMaxOrder;
  std::vector<int> cur{1};
  int total = 0;
  dc = DevClasses{};
  for (int i = 0; i < p.H; ++i) {
    dc.din.push_back(cur);
    if (i == p.H - 1) break;
    const int cap = p.Dpost[i];
    std::vector<std::pair<int, int>> pr;
    std::vector<int> nxt;
    for (int d : cur) {
      std::vector<int> outs{0, 1};
      for (int k = 1; d >= 1 && k <= top && k * d <= cap; ++k) outs.push_back(k * d);
      std::sort(outs.begin(), outs.end());
      outs.erase(std::unique(outs.begin(), outs.end()), outs.end());
      for (int o : outs) {
        pr.emplace_back(d, o);
        nxt.push_back(o);
      }
    }
    std::sort(nxt.begin(), nxt.end());
    nxt.erase(std::unique(nxt.begin(), nxt.end()), nxt.end());
    const bool lin = p.lin > 0 && (i + 1) % p.lin == 0;
    total += (int)pr.size();
    dc.slots = std::max(dc.slots, (int)(pr.size() + nxt.size()));
    dc.pairs.push_back(pr);
    dc.dout.push_back(nxt);
    cur = lin ? std::vector<int>{1} : nxt;  // after a linearisation every box restarts at degree 1
  }
  return dc.slots <= kMaxDevLists && total <= kMaxDevPairs;
}


}  // namespace bern

struct bern_net {
  int H = 0, n = 0, nh = 0, o = 0, hmax = 0;
  std::vector<int> widths;
  std::vector<int64_t> woff, boff, noff;  // per layer offsets into W, b and hidden neurons
  double *W64 = nullptr, *b64 = nullptr;
  double *WT = nullptr;                   // per layer W^T [w_{i-1}][hp_i], zero-padded to hp_i columns
  std::vector<int64_t> wtoff;
  std::vector<int> hpad;
  double *sens = nullptr;  // [nh] downstream sensitivity of every hidden neuron
  int device = 0;
  bern::Tune tune;         // kernel variants (autotuner)
  // captured launch sequences of sync-free runs, keyed by every argument
  struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t capture = nullptr;  // stream the sequences are captured on
  bern::SimplexTables *tab = nullptr;  // index tables of the total-degree layout (built on demand)
  // pinned host staging of the per-layer box classes (box degrees in, box id
  // lists out), so those copies run asynchronously
  mutable int *host_ids = nullptr;
  mutable int *host_dev = nullptr;  // host_ids as kernels address it (mapped, coherent)
  mutable size_t host_n = 0;
};

struct bern_pred {
  float *params = nullptr;  // device, bern_pred_params() floats
};

using namespace bern;

static bern_status plan_net(const bern_net *net, const bern_opts *o, Plan &p) {
  p.H = net->H;
  p.n = net->n;
  p.fp64 = o->precision == BERN_FP64;
  p.elem = p.fp64 ? 8 : 4;
  p.L = o->L;
  p.mode = o->plan;
  p.lin = o->lin;
  p.lin_layers = 0;
  if (o->L < 1 || o->L > kMaxOrder) {
    set_error("L = %d outside 1..%d", o->L, kMaxOrder);
    return BERN_E_DEGREE;
  }
  if (o->plan == BERN_PLAN_LEARNED && !o->pred) {
    set_error("BERN_PLAN_LEARNED needs a predictor");
    return BERN_E_ARG;
  }
  // Every box's tensors stay within the plain rule's sizes at order L (plan
  // codes are clamped to that), so one fixed slot per box suffices.
  p.Lmax = o->L;
  p.Dpre.assign(p.H, 0);
  p.Dpost.assign(p.H, 0);
  p.Cpre.assign(p.H, 0);
  p.Cpost.assign(p.H, 0);
  p.nbx.assign(p.H, 0);
  int D = 1;
  const int64_t cap = (int64_t)1 << 36;
  p.recs = p.arenaA = p.arenaB = p.conv = p.horner = p.gpart = p.cpart = 0;
  for (int i = 0; i < p.H; ++i) {
    const int h = net->widths[i + 1];
    p.Dpre[i] = D;
    // stored coefficients (total-degree layout); the read-off still expands
    // them to the dense (D+1)^n tensor
    p.Cpre[i] = ssize(p.n, D, cap);
    if (p.Cpre[i] < 0 || tsize(p.n, D, cap) < 0) {
      set_error("layer %d: (%d+1)^%d coefficients overflow", i + 1, D, p.n);
      return BERN_E_TOO_LARGE;
    }
    p.arenaA = std::max(p.arenaA, align256((size_t)h * 2 * p.Cpre[i] * p.elem));
    p.conv = std::max(p.conv, convert_scratch_bytes(p.n, D, h, 1));
    // per-neuron plans leave boxes at any degree up to the plain one, and a
    // lower degree may take a read-off with more staging
    if (p.mode != BERN_PLAN_PLAIN)
      for (int d = 2; d < D; ++d) p.conv = std::max(p.conv, convert_scratch_bytes(p.n, d, h, 1));
    if (!p.fp64 && i > 0) p.gpart = std::max(p.gpart, align256((size_t)h * 2 * gemm_cblocks(p.Cpre[i]) * 8));
    if (i < p.H - 1) {
      const int Dn = p.Lmax * D;
      p.Dpost[i] = Dn;
      p.Cpost[i] = ssize(p.n, Dn, cap);
      if (p.Cpost[i] < 0) {
        set_error("layer %d post: degree %d in %d variables overflows", i + 1, Dn, p.n);
        return BERN_E_TOO_LARGE;
      }
      p.arenaB = std::max(p.arenaB, align256((size_t)h * 2 * p.Cpost[i] * p.elem));
      p.recs = std::max(p.recs, align256((size_t)h * sizeof(NeuronRec)));
      // blocks per item: every class of the layer stores at most Cpost coefficients
      const int64_t nb = compose_nbx(p.Cpost[i]);
      p.nbx[i] = nb;
      if (!p.fp64) p.cpart = std::max(p.cpart, align256((size_t)h * 2 * nb * 2 * 8));
      if (p.Lmax >= 3) {
        const int64_t Cq = ssize(p.n, (p.Lmax - 1) * D, cap);
        if (Cq < 0) {
          set_error("layer %d: Horner intermediates of degree %d overflow", i + 1, (p.Lmax - 1) * D);
          return BERN_E_TOO_LARGE;
        }
        p.horner = std::max(p.horner, compose_scratch_bytes(Cq, p.Lmax, h, 1));
      }
      if (p.mode != BERN_PLAN_PLAIN && Dn >= 3) {
        // a box at a lower degree may take orders up to Dn / Din (at most
        // 3 for learned classes, 8 for given codes): Horner intermediates
        // of degree up to Dn - 1
        const int64_t Cq = ssize(p.n, Dn - 1, cap);
        if (Cq < 0) {
          set_error("layer %d: Horner intermediates of degree %d overflow", i + 1, Dn - 1);
          return BERN_E_TOO_LARGE;
        }
        p.horner = std::max(p.horner, compose_scratch_bytes(Cq, 3, h, 1));
      }
      D = Dn;
      if (p.lin > 0 && (i + 1) % p.lin == 0) {
        // the post tensors are read off whole (fits and remainders) by one
        // block each, then the next layer starts at degree 1
        if (!convert_one_block(p.n, Dn)) {
          set_error("Lin at hidden layer %d: post degree %d in %d variables exceeds one block's read-off", i + 1,
                    Dn, p.n);
          return BERN_E_TOO_LARGE;
        }
        ++p.lin_layers;
        D = 1;
      }
    }
  }
  // per box: validity flag, post degree (two layers), the class id lists
  // (host classes: one per layer and phase; device classes: one per list
  // slot and layer parity, then their counts), and the predicted code of
  // every hidden neuron
  p.list_ints = 2 * (size_t)p.H;
  p.dev_ok = p.mode != BERN_PLAN_PLAIN && dev_classes(p, p.dc);
  if (p.dev_ok) p.list_ints = std::max(p.list_ints, 4 * (size_t)p.dc.slots);
  p.flags = align256(sizeof(int) * (3 + p.list_ints) + (size_t)net->nh);
  p.live = align256(sizeof(int) * (3 + 3 * (size_t)net->hmax) + (size_t)net->hmax);  // lists, then kind bytes
  p.rad = align256(sizeof(double) * 4 * (size_t)net->hmax);
  p.oeps = align256(sizeof(double) * 2 * (size_t)net->o);
  if (o->mem_budget_bytes > 0 && p.per_box() > o->mem_budget_bytes) {
    set_error("one box needs %zu bytes of workspace, over the budget of %llu", p.per_box(),
              (unsigned long long)o->mem_budget_bytes);
    return BERN_E_TOO_LARGE;
  }
  return BERN_OK;
}

extern "C" {

void bern_opts_default(bern_opts *opts) {
  if (!opts) return;
  memset(opts, 0, sizeof(*opts));
  opts->L = 2;
  opts->precision = BERN_FP64;
  opts->plan = BERN_PLAN_PLAIN;
  opts->sched = BERN_SCHED_PER_BOX;
}

const char *bern_status_str(int32_t s) {
  switch (s) {
    case BERN_OK: return "BERN_OK";
    case BERN_E_ARG: return "BERN_E_ARG";
    case BERN_E_SHAPE: return "BERN_E_SHAPE";
    case BERN_E_BOX: return "BERN_E_BOX";
    case BERN_E_DEGREE: return "BERN_E_DEGREE";
    case BERN_E_TOO_LARGE: return "BERN_E_TOO_LARGE";
    case BERN_E_OOM: return "BERN_E_OOM";
    case BERN_E_WORKSPACE: return "BERN_E_WORKSPACE";
    case BERN_E_DEVICE: return "BERN_E_DEVICE";
    case BERN_E_NUMERIC: return "BERN_E_NUMERIC";
    default: return "BERN_UNKNOWN";
  }
}

const char *bern_last_error(void) { return g_err; }

bern_status bern_net_create(int32_t H, const int32_t *widths, const double *W, const double *b, bern_net **out) {
  if (!out) { set_error("out is null"); return BERN_E_ARG; }
  *out = nullptr;
  if (H < 1 || H > 64 || !widths || !W || !b) {
    set_error("bad network description (H = %d)", H);
    return BERN_E_ARG;
  }
  if (widths[0] < 1 || widths[0] > kMaxInputs) {
    set_error("input dimension %d outside 1..%d", widths[0], kMaxInputs);
    return BERN_E_ARG;
  }
  int64_t nw = 0, nb = 0;
  for (int i = 1; i <= H; ++i) {
    if (widths[i] < 1 || widths[i] > 65535) {
      set_error("width h_%d = %d outside 1..65535", i, widths[i]);
      return BERN_E_ARG;
    }
    nw += (int64_t)widths[i] * widths[i - 1];
    nb += widths[i];
  }
  for (int64_t i = 0; i < nw; ++i)
    if (!std::isfinite(W[i])) { set_error("non-finite weight at %lld", (long long)i); return BERN_E_NUMERIC; }
  for (int64_t i = 0; i < nb; ++i)
    if (!std::isfinite(b[i])) { set_error("non-finite bias at %lld", (long long)i); return BERN_E_NUMERIC; }
  bern_net *net = new (std::nothrow) bern_net();
  if (!net) { set_error("out of host memory"); return BERN_E_OOM; }
  net->H = H;
  net->n = widths[0];
  net->widths.assign(widths, widths + H + 1);
  net->o = widths[H];
  int64_t wo = 0, bo = 0, no = 0;
  for (int i = 1; i <= H; ++i) {
    net->woff.push_back(wo);
    net->boff.push_back(bo);
    net->noff.push_back(no);
    wo += (int64_t)widths[i] * widths[i - 1];
    bo += widths[i];
    if (i < H) no += widths[i];
    net->hmax = std::max(net->hmax, widths[i]);
  }
  net->nh = (int)no;
  // downstream sensitivity of hidden layer i: 1^T |W^(H)| ... |W^(i+1)|
  std::vector<double> sens(std::max(1, net->nh), 0.0);
  {
    std::vector<double> v(widths[H], 1.0);
    for (int i = H; i >= 2; --i) {  // v over layer i -> over layer i-1
      const int hi_ = widths[i], hp = widths[i - 1];
      std::vector<double> u(hp, 0.0);
      const double *Wi = W + net->woff[i - 1];
      for (int r = 0; r < hi_; ++r)
        for (int c = 0; c < hp; ++c) u[c] += v[r] * std::fabs(Wi[(int64_t)r * hp + c]);
      v.swap(u);
      for (int c = 0; c < hp; ++c) sens[net->noff[i - 2] + c] = v[c];
    }
  }
  // transposed, zero-padded weights for the interval GEMM
  std::vector<double> wt;
  for (int i = 1; i <= H; ++i) {
    const int h = widths[i], hin = widths[i - 1], hp = (h + 15) / 16 * 16;
    net->wtoff.push_back((int64_t)wt.size());
    net->hpad.push_back(hp);
    const size_t base = wt.size();
    wt.resize(base + (size_t)hin * hp, 0.0);
    const double *Wi = W + net->woff[i - 1];
    for (int r = 0; r < h; ++r)
      for (int c = 0; c < hin; ++c) wt[base + (size_t)c * hp + r] = Wi[(int64_t)r * hin + c];
  }
  (void)hipGetDevice(&net->device);
  net->tab = new (std::nothrow) bern::SimplexTables();
  if (!net->tab) {
    delete net;
    set_error("out of host memory");
    return BERN_E_OOM;
  }
  net->tab->n = net->n;
  auto fail = [&](hipError_t e) {
    set_error("device allocation/copy failed: %s", hipGetErrorString(e));
    (void)hipFree(net->W64); (void)hipFree(net->b64); (void)hipFree(net->sens); (void)hipFree(net->WT);
    delete net->tab;
    delete net;
    return BERN_E_DEVICE;
  };
  hipError_t e;
  if ((e = hipMalloc(&net->W64, nw * 8)) != hipSuccess) return fail(e);
  if ((e = hipMalloc(&net->WT, wt.size() * 8)) != hipSuccess) return fail(e);
  if ((e = hipMemcpy(net->WT, wt.data(), wt.size() * 8, hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
  if ((e = hipMalloc(&net->b64, nb * 8)) != hipSuccess) return fail(e);
  if ((e = hipMalloc(&net->sens, sens.size() * 8)) != hipSuccess) return fail(e);
  if ((e = hipMemcpy(net->W64, W, nw * 8, hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
  if ((e = hipMemcpy(net->b64, b, nb * 8, hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
  if ((e = hipMemcpy(net->sens, sens.data(), sens.size() * 8, hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
  *out = net;
  return BERN_OK;
}

void bern_net_destroy(bern_net *net) {
  if (!net) return;
  (void)hipFree(net->W64);
  (void)hipFree(net->b64);
  (void)hipFree(net->sens);
  (void)hipFree(net->WT);
  for (auto &g : net->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  if (net->capture) (void)hipStreamDestroy(net->capture);
  if (net->host_ids) (void)hipHostFree(net->host_ids);
  delete net->tab;
  delete net;
}

int32_t bern_net_inputs(const bern_net *net) { return net ? net->n : 0; }
int32_t bern_net_hidden(const bern_net *net) { return net ? net->nh : 0; }
int32_t bern_net_outputs(const bern_net *net) { return net ? net->o : 0; }

static bern_status check_opts(const bern_net *net, const bern_opts *o) {
  if (!net || !o) { set_error("null net or options"); return BERN_E_ARG; }
  if (o->precision != BERN_FP64 && o->precision != BERN_FP32_PADDED) {
    set_error("unknown precision %d", o->precision);
    return BERN_E_ARG;
  }
  if (o->sched != BERN_SCHED_PER_BOX && o->sched != BERN_SCHED_BATCHED) {
    set_error("unknown schedule %d", o->sched);
    return BERN_E_ARG;
  }
  if (o->plan < BERN_PLAN_PLAIN || o->plan > BERN_PLAN_LEARNED) {
    set_error("unknown plan %d", o->plan);
    return BERN_E_ARG;
  }
  if (o->lin < 0 || o->lin > 64) {
    set_error("lin = %d outside 0..64", o->lin);
    return BERN_E_ARG;
  }
  return BERN_OK;
}

bern_status bern_workspace_size(const bern_net *net, const bern_opts *opts, int64_t n_boxes, size_t *bytes,
                                size_t *one_box) {
  bern_status st = check_opts(net, opts);
  if (st != BERN_OK) return st;
  if (!bytes || n_boxes < 1) { set_error("bad arguments"); return BERN_E_ARG; }
  Plan p;
  if ((st = plan_net(net, opts, p)) != BERN_OK) return st;
  const int64_t wave = opts->sched == BERN_SCHED_PER_BOX ? 1 : n_boxes;
  *bytes = p.per_box() * (size_t)wave;
  if (one_box) *one_box = p.per_box();
  return BERN_OK;
}

}  // extern "C"

// Boxes of a wave flagged invalid (flag[b] = 1: d_lo > d_hi or a non-finite
// coordinate, set where the first layer's coefficients are formed) get NaN
// bounds.
__global__ void poison_kernel(int64_t nb, const int *flag, int nh, int o, double *nlo, double *nhi, double *olo,
                              double *ohi) {
  const int64_t b = blockIdx.x;
  if (b >= nb || !flag[b]) return;
  const double nan = __builtin_nan("");
  for (int j = threadIdx.x; j < nh; j += blockDim.x) {
    if (nlo) nlo[b * nh + j] = nan;
    if (nhi) nhi[b * nh + j] = nan;
  }
  for (int j = threadIdx.x; j < o; j += blockDim.x) {
    olo[b * o + j] = nan;
    ohi[b * o + j] = nan;
  }
}

// Largest per-neuron post degree of every box of the wave: one wave per box,
// its lanes over the neurons.
__global__ void box_degree_kernel(int64_t nb, int h, const NeuronRec *recs, int *deg, int *hdeg) {
  const int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (b >= nb) return;
  const int lane = threadIdx.x & 63;
  int d = 0;
  for (int j = lane; j < h; j += 64) d = max(d, recs[b * h + j].deg);
  for (int off = 32; off > 0; off >>= 1) d = max(d, __shfl_xor(d, off, 64));
  if (lane == 0) {
    deg[b] = d;
    if (hdeg) hdeg[b] = d;  // the host's copy (mapped host memory)
  }
}

// Counters (bern_opts.counters): cleared by one block, then per hidden layer
// one wave per box counts its neurons' rules, and after the output layer one
// thread per box folds the output radii into the largest pad.
__global__ void counters_clear_kernel(long long *cnt) {
  if (threadIdx.x < BERN_NCOUNTERS) cnt[threadIdx.x] = 0;
}

__global__ void counters_rules_kernel(int64_t nb, int h, const NeuronRec *recs, long long *cnt) {
  const int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (b >= nb) return;
  const int lane = threadIdx.x & 63;
  long long c[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int j = lane; j < h; j += 64) {
    const int k = recs[b * h + j].kind;
    c[0] += 1;
    c[1] += k == kInactive;
    c[2] += k == kActive;
    c[3] += k == kFallback;
    c[4] += k == 1;
    c[5] += k == 2;
    c[6] += k >= 3;
  }
  for (int q = 0; q < 7; ++q) {
    long long v = c[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0 && v) atomicAdd(reinterpret_cast<unsigned long long *>(cnt + q), (unsigned long long)v);
  }
}

__global__ void counters_pad_kernel(int64_t nb, int o, const double *eps, long long *cnt) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double m = 0.0;
  for (int q = 0; q < 2 * o; ++q) m = fmax(m, eps[b * 2 * o + q]);
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long *>(cnt + BERN_CNT_MAXPAD), (unsigned long long)__double_as_longlong(m));
}

// Index tables of one layer's degree class: the dense positions for the
// read-off at Din and, for compositions, the square table (Din, Din) and the
// Horner tables (Din, m Din), m = 1 .. Lmax - 1. Built once per network.
struct LayerTables {
  const int *didx = nullptr;
  const TreeTable *tree = nullptr;
  const int *plist = nullptr;
  int plist_len = 0;
  const ProdTable *sq = nullptr;
  const ProdTable *hz[kMaxOrder] = {};
};

static bern_status layer_tables(const bern_net *net, int Din, int Lmax, bool compose, LayerTables &t) {
  hipError_t e = dense_index_table(*net->tab, Din, &t.didx);
  const bool tree = convert_tree(net->n, Din);
  // degree 1 is read off at the box corners and needs neither
  if (e == hipSuccess && Din >= 2 && Din <= 12 && net->n >= 2) e = tree_table(*net->tab, Din, &t.tree);
  if (e == hipSuccess && !tree && Din >= 2 && Din <= 8) e = prefix_table(*net->tab, Din, net->n, &t.plist, &t.plist_len);
  if (e == hipSuccess && compose && Lmax >= 2) e = product_table(*net->tab, Din, Din, true, &t.sq);
  for (int m = 1; e == hipSuccess && compose && m <= Lmax - 1 && Lmax >= 3; ++m)
    e = product_table(*net->tab, Din, m * Din, false, &t.hz[m]);
  if (e == hipErrorInvalidValue) {
    set_error("index tables for degree %d in %d variables exceed their limits", Din, net->n);
    return BERN_E_TOO_LARGE;
  }
  if (e != hipSuccess) {
    set_error("index tables: %s", hipGetErrorString(e));
    return BERN_E_DEVICE;
  }
  return BERN_OK;
}

// Boxes of one degree class within a wave (host-side classification).
struct BoxClass {
  int Din, Dout;
  std::vector<int> ids;
};

// The boxes one launch takes: `nboxes` boxes listed in `bids` (null: the
// wave's boxes in order) or, with `dcount`, the first *dcount of them, a
// count the device wrote (nboxes then bounds it).
struct LaunchClass {
  int Din = 1, Dout = 0;
  const int *bids = nullptr;
  int64_t nboxes = 0;
  const int *dcount = nullptr;
};

struct ClassTab {
  int npairs, nvals;
  int din[kMaxDevLists], dout[kMaxDevLists], vals[kMaxDevLists];
};

// One block per list, boxes in order: list k < npairs holds the boxes whose
// (pre degree, post degree) is pair k, list npairs + m those whose post
// degree is vals[m] (the next layer's read-off classes), and counts[k] their
// lengths. The last block flags every box no pair covers (none, as the
// pairs are every combination the rules give; a flagged box ends with NaN
// bounds rather than stale ones). Degrees below 0 count as 0; a null dpre
// puts every box at pre degree 1.
__global__ void __launch_bounds__(1024) classify_kernel(int64_t B, const int *dpre, const int *dpost, ClassTab t,
                                                        int *ids, int *counts, int *flags) {
  __shared__ int wsum[16];
  __shared__ int base;
  const int k = blockIdx.x;
  const int lists = t.npairs + t.nvals;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < B; b0 += blockDim.x) {
    const int64_t b = b0 + threadIdx.x;
    bool m = false;
    if (b < B) {
      const int di = dpre ? max(dpre[b], 0) : 1, dq = max(dpost[b], 0);
      if (k < t.npairs) {
        m = di == t.din[k] && dq == t.dout[k];
      } else if (k < lists) {
        m = dq == t.vals[k - t.npairs];
      } else {
        bool any = false;
        for (int q = 0; q < t.npairs; ++q) any |= di == t.din[q] && dq == t.dout[q];
        m = !any;
      }
    }
    const unsigned long long bal = __ballot(m);
    if (lane == 0) wsum[wid] = __popcll(bal);
    __syncthreads();
    if (m) {
      if (k < lists) {
        int pos = base;
        for (int w = 0; w < wid; ++w) pos += wsum[w];
        ids[(int64_t)k * B + pos + __popcll(bal & ((1ull << lane) - 1ull))] = (int)b;
      } else {
        flags[b] = 1;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < nw; ++w) tot += wsum[w];
      base += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && k < lists) counts[k] = base;
}

// Output polynomials requested by bern_output_polys: dense power tensors at
// per-variable degree D (C = (D+1)^n coefficients each), [n_boxes][o][C];
// or, by bern_rel_volume, only their relative volumes vol [n_boxes][o].
struct OutPolys {
  double *U, *L;
  int D;
  int64_t C;
  const int *didx;  // rank -> dense index at degree D
  double *vol = nullptr;
};

// Largest ReLU order a neuron of a box class (Din, Dout) may hold: the plain
// rule's L; under per-neuron plans an order-k neuron has degree k Din <=
// Dout, so at most Dout / Din (and at most 3 for the predictor's classes,
// kMaxOrder for given codes).
static int class_order(const Plan &p, int Din, int Dout) {
  if (p.mode == BERN_PLAN_PLAIN) return p.L;
  if (Din < 1) return 1;
  const int top = p.mode == BERN_PLAN_LEARNED ? 3 : kMaxOrder;
  return std::max(1, std::min(top, Dout / Din));
}

// Compose arguments of hidden layer i for the boxes of class cl (bids).
static bern_status compose_args(const bern_net *net, const Plan &p, int i, const LaunchClass &cl, void *pre,
                                void *post, int64_t slotA, int64_t slotB, NeuronRec *recs, double *rad,
                                double *cpart, void *horner, size_t horner_bytes, int *live, int64_t live_ld,
                                ComposeArgs &m) {
  const int n = net->n;
  m = ComposeArgs{};
  m.n = n;
  m.Din = cl.Din;
  m.Dout = cl.Dout;
  m.h = net->widths[i + 1];
  m.bids = cl.bids;
  m.dcount = cl.dcount;
  m.slot_in = slotA;
  m.slot_out = slotB;
  m.nbounds = 2;
  m.Lmax = class_order(p, cl.Din, cl.Dout);
  LayerTables lt;
  bern_status st = layer_tables(net, cl.Din, m.Lmax, true, lt);
  if (st != BERN_OK) return st;
  m.Cin = ssize(n, cl.Din);
  m.Cout = ssize(n, cl.Dout);
  m.Cs = ssize(n, std::min(cl.Din, cl.Dout));
  for (int q = 0; q <= kMaxOrder; ++q) m.Sm[q] = q <= m.Lmax ? ssize(n, q * cl.Din) : 0;
  m.Cq = m.Lmax >= 3 ? ssize(n, (m.Lmax - 1) * cl.Din) : 0;
  if (lt.sq) {
    m.sq_off = lt.sq->off;
    m.sq_pairs = lt.sq->pairs;
    m.sq_diag = lt.sq->diag;
  }
  for (int q = 1; q < kMaxOrder; ++q)
    if (lt.hz[q]) {
      m.hz_off[q] = lt.hz[q]->off;
      m.hz_pairs[q] = lt.hz[q]->pairs;
    }
  m.nboxes = cl.nboxes;
  m.pre = pre;
  m.post = post;
  m.recs = recs;
  m.rad = p.fp64 ? nullptr : rad;
  m.fp64 = p.fp64 ? 1 : 0;
  m.scratch = horner;
  m.scratch_bytes = horner_bytes;
  m.nbx = compose_nbx(m.Cout);
  m.pstride = p.nbx[i];
  m.part = p.fp64 ? nullptr : cpart;
  m.live = live;
  m.live_ld = live_ld;
  return BERN_OK;
}

// The compositions of hidden layer i (Section 5.1 Step 3): the order-1
// and fallback posts of every box in one launch (each box at its own
// degrees din / dout, or at the uniform uDin / uDout where those are null),
// the products of every (Din, Dout) class that can hold an order >= 2 (its
// own square and Horner tables), then the post radii of every box (FP32).
// The composition's first stage over every box (order-1 and fallback
// neurons, each box at its own degrees din / dout): it needs no host
// classes, so a host-class run enqueues it before waiting for them.
static bern_status compose_scatter_stage(const bern_net *net, const Plan &p, int i, int uDin, int uDout,
                                         const int *din, const int *dout, int64_t B, void *pre, void *post,
                                         int64_t slotA, int64_t slotB, NeuronRec *recs, double *rad, double *cpart,
                                         int *live, int64_t live_ld, hipStream_t s) {
  const int n = net->n, h = net->widths[i + 1];
  ComposeArgs m{};
  m.n = n;
  m.Din = uDin;
  m.Dout = uDout;
  m.h = h;
  m.bids = nullptr;
  m.nboxes = B;
  m.slot_in = slotA;
  m.slot_out = slotB;
  m.nbounds = 2;
  m.Lmax = 1;
  m.Cin = ssize(n, uDin);
  m.Cout = ssize(n, uDout);
  m.Cs = ssize(n, std::min(uDin, uDout));
  m.pre = pre;
  m.post = post;
  m.recs = recs;
  m.rad = p.fp64 ? nullptr : rad;
  m.fp64 = p.fp64 ? 1 : 0;
  m.nbx = p.nbx[i];
  m.pstride = p.nbx[i];
  m.part = p.fp64 ? nullptr : cpart;
  m.live = live;
  m.live_ld = live_ld;
  m.box_din = din;
  m.box_dout = dout;
  m.stage = 1;
  m.lists_ready = 1;
  m.radii_later = 1;
  BERN_HIP_TRY(launch_compose(m, s));
  return BERN_OK;
}

// A hidden layer's composition: the first stage (unless already enqueued),
// the products per (Din, Dout) class, then the post radii.
static bern_status compose_layer(const bern_net *net, const Plan &p, int i, const std::vector<LaunchClass> &pairs,
                                 int uDin, int uDout, const int *din, const int *dout, int64_t B, void *pre,
                                 void *post, int64_t slotA, int64_t slotB, NeuronRec *recs, double *rad,
                                 double *cpart, void *horner, int *live, int64_t live_ld, bool stage1,
                                 hipStream_t s) {
  const int n = net->n, h = net->widths[i + 1];
  if (stage1) {
    const bern_status st = compose_scatter_stage(net, p, i, uDin, uDout, din, dout, B, pre, post, slotA, slotB,
                                                 recs, rad, cpart, live, live_ld, s);
    if (st != BERN_OK) return st;
  }
  for (const LaunchClass &cl : pairs) {
    if (class_order(p, cl.Din, cl.Dout) < 2) continue;  // no neuron of the class has a product
    ComposeArgs mp;
    const bern_status st = compose_args(net, p, i, cl, pre, post, slotA, slotB, recs, rad, cpart, horner,
                                        p.horner * B, live, live_ld, mp);
    if (st != BERN_OK) return st;
    mp.stage = 2;
    mp.lists_ready = 1;
    mp.radii_later = 1;
    BERN_HIP_TRY(launch_compose(mp, s));
  }
  if (!p.fp64) {
    ComposeArgs mr{};
    mr.n = n;
    mr.h = h;
    mr.nboxes = B;
    mr.nbounds = 2;
    mr.recs = recs;
    mr.part = cpart;
    mr.nbx = p.nbx[i];
    mr.pstride = p.nbx[i];
    mr.rad = rad;
    mr.fp64 = 0;
    BERN_HIP_TRY(launch_post_radii(mr, s));
  }
  return BERN_OK;
}

// The affine map after hidden layer i (Section 5.2), one launch per post
// degree class: every box of the class holds its posts at that degree and
// reads its active neurons' pre-activations at its own pre degree (din, or
// the uniform uDin where din is null).
static bern_status gemm_layer(const bern_net *net, const Plan &p, int i, const std::vector<LaunchClass> &gc, int uDin,
                              const int *din, void *const *Aa, void *Bp, int64_t slotA, int64_t slotB, int *live,
                              int64_t live_ld, double *gpart, hipStream_t s) {
  const int n = net->n;
  for (const LaunchClass &cl : gc) {
    GemmArgs a{};
    a.hin = net->widths[i + 1];
    a.h = net->widths[i + 2];
    a.C = ssize(n, cl.Dout);
    a.nboxes = cl.nboxes;
    a.bids = cl.bids;
    a.dcount = cl.dcount;
    a.slot_in = slotB;
    a.slot_out = slotA;
    a.post = Bp;
    a.pre = Aa[(i + 1) & 1];
    a.act = Aa[i & 1];
    a.act_slot = slotA;
    if (din) {
      a.box_din = din;
      a.n = n;
      a.Dout = cl.Dout;
      a.Cs = a.C;
      a.Cact = a.C;
    } else {
      a.Cact = ssize(n, uDin);
      a.Cs = ssize(n, std::min(uDin, cl.Dout));
    }
    a.live = live;
    a.live_ld = live_ld;
    a.tune = net->tune;
    a.WT = net->WT + net->wtoff[i + 1];
    a.hp = net->hpad[i + 1];
    a.b = net->b64 + net->boff[i + 1];
    a.fp64 = p.fp64 ? 1 : 0;
    a.rpart = p.fp64 ? nullptr : gpart;
    a.rpart_slot = (int64_t)(p.gpart / sizeof(double));
    BERN_HIP_TRY(launch_gemm(a, s));
  }
  return BERN_OK;
}

// Hidden layer i under periodic linearisation (opts.lin), after its
// compositions: every neuron's post polynomials staged whole at its box's
// post degree, read off per post degree class with fits and remainders
// (mode 2), the affine posts stored at degree 1 for all boxes, and the next
// layer's affine map over every box at degree 1 (Section 5.4, the Lin
// parameter).
static bern_status lin_layer_run(const bern_net *net, const Plan &p, int i, const std::vector<LaunchClass> &gc,
                                 int uDin, int uDout, const int *din, const int *dout, int64_t B, void *const *Aa,
                                 void *Bp, int64_t slotA, int64_t slotB, NeuronRec *recs, double *rad, int *live,
                                 int64_t live_ld, double *gpart, double *conv, hipStream_t s) {
  const int n = net->n, h = net->widths[i + 1];
  {
    ComposeArgs m{};
    m.n = n;
    m.Din = uDin;
    m.Dout = uDout;
    m.h = h;
    m.nboxes = B;
    m.nbounds = 2;
    m.slot_in = slotA;
    m.slot_out = slotB;
    m.Cin = ssize(n, uDin);
    m.Cout = ssize(n, uDout);
    m.Cs = ssize(n, std::min(uDin, uDout));
    m.pre = Aa[i & 1];
    m.post = Bp;
    m.recs = recs;
    m.fp64 = p.fp64 ? 1 : 0;
    m.box_din = din;
    m.box_dout = dout;
    BERN_HIP_TRY(launch_lin_stage(m, s));
  }
  for (const LaunchClass &cl : gc) {
    if (cl.Dout < 1) continue;  // every neuron inactive: nothing to linearise
    LayerTables lt;
    bern_status st = layer_tables(net, cl.Dout, p.Lmax, false, lt);
    if (st != BERN_OK) return st;
    ConvertArgs c{};
    c.n = n;
    c.D = cl.Dout;
    c.h = h;
    c.L = p.L;
    c.C = ipow(cl.Dout + 1, n);
    c.S = ssize(n, cl.Dout);
    c.didx = lt.didx;
    c.plist = lt.plist;
    c.plist_len = lt.plist_len;
    if (lt.tree) {
      c.tree = lt.tree->buf;
      c.tree_len = lt.tree->len;
      for (int d = 0; d <= n && d < 17; ++d) c.tree_base[d] = lt.tree->base[d];
    }
    c.nboxes = cl.nboxes;
    c.bids = cl.bids;
    c.dcount = cl.dcount;
    c.slot = slotB;
    c.cap = cl.Dout;
    c.pre = Bp;
    c.fp64 = p.fp64 ? 1 : 0;
    c.recs = recs;
    c.scratch = conv;
    c.scratch_bytes = p.conv * B;
    c.layer = i;
    c.hin = net->widths[i];
    c.W = net->W64 + net->woff[i];
    c.b = net->b64 + net->boff[i];
    c.mode = 2;
    c.tune = net->tune;
    const hipError_t e = launch_convert(c, s);
    if (e == hipErrorInvalidValue) {
      set_error("Lin read-off at degree %d in %d variables is not available", cl.Dout, n);
      return BERN_E_TOO_LARGE;
    }
    BERN_HIP_TRY(e);
  }
  // the affine posts of every box at degree 1, then their input lists
  ComposeArgs ml{};
  ml.n = n;
  ml.h = h;
  ml.nboxes = B;
  ml.nbounds = 2;
  ml.recs = recs;
  ml.post = Bp;
  ml.slot_out = slotB;
  ml.rad = p.fp64 ? nullptr : rad;
  ml.fp64 = p.fp64 ? 1 : 0;
  ml.live = live;
  ml.live_ld = live_ld;
  ml.lin = 1;
  BERN_HIP_TRY(launch_lin_scatter(ml, s));
  BERN_HIP_TRY(launch_live(ml, s));
  const std::vector<LaunchClass> all{LaunchClass{1, 1, nullptr, B, nullptr}};
  return gemm_layer(net, p, i, all, 1, nullptr, Aa, Bp, slotA, slotB, live, live_ld, gpart, s);
}

// A wait for the work enqueued on a stream up to a mark, by polling an event
// of the calling thread's on the current device (spin_mark records it; work
// enqueued after the mark is not waited for; spin_poll waits for it) instead
// of a blocking stream synchronisation: the host resumes within microseconds
// of the kernel it waits for, which the per-layer degree read-back of host
// classes pays once per hidden layer.
static hipEvent_t *spin_event() {
  static thread_local hipEvent_t ev[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  if (!ev[dev] && hipEventCreateWithFlags(&ev[dev], hipEventDisableTiming) != hipSuccess) return nullptr;
  return &ev[dev];
}
static hipError_t spin_mark(hipStream_t s) {
  hipEvent_t *ev = spin_event();
  return ev ? hipEventRecord(*ev, s) : hipErrorInvalidResourceHandle;
}
static hipError_t spin_poll() {
  hipEvent_t *ev = spin_event();
  if (!ev) return hipErrorInvalidResourceHandle;
  hipError_t e;
  while ((e = hipEventQuery(*ev)) == hipErrorNotReady) {
  }
  return e;
}

// Enqueue the launch sequence of one wave of `B` boxes. The plain rule keeps
// every box at the same degrees: one class, no host round trip. Plans with
// per-neuron degrees launch each degree class of boxes on its own (a box's
// tensors stay dense at the box's own degree inside its fixed slot): with
// `dc`, every class the rules can give, its box list and count written by a
// classification kernel (no host round trip); without, the classes that
// occur, read back once per hidden layer (the box degrees to the host, the
// id lists to the device).
static bern_status run_wave(const bern_net *net, const Plan &p, const bern_opts *o, int64_t b0, int64_t B,
                            const double *box_lo, const double *box_hi, const int8_t *plan, double *nlo, double *nhi,
                            double *olo, double *ohi, int8_t *used, char *ws, hipStream_t s,
                            const OutPolys *op = nullptr, const DevClasses *dc = nullptr) {
  char *cur = ws;
  NeuronRec *recbuf[2];
  recbuf[0] = reinterpret_cast<NeuronRec *>(cur); cur += p.recs * B;
  recbuf[1] = reinterpret_cast<NeuronRec *>(cur); cur += p.recs * B;
  // dense copies of the records' post radii, alternating like the records
  double *radbuf[2];
  radbuf[0] = reinterpret_cast<double *>(cur); cur += p.rad * B;
  radbuf[1] = reinterpret_cast<double *>(cur); cur += p.rad * B;
  double *gpart = reinterpret_cast<double *>(cur); cur += p.gpart * B;
  double *cpart = reinterpret_cast<double *>(cur); cur += p.cpart * B;
  // pre-activation arenas alternate between layers: the affine map of layer
  // i+1 reads active neurons' pre-activations of layer i in place
  void *Aa[2];
  Aa[0] = cur; cur += p.arenaA * B;
  Aa[1] = cur; cur += p.arenaA * B;
  void *Bp = cur; cur += p.arenaB * B;
  double *conv = reinterpret_cast<double *>(cur); cur += p.conv * B;
  void *horner = cur; cur += p.horner * B;
  int *live = reinterpret_cast<int *>(cur); cur += p.live * B;
  double *oeps = reinterpret_cast<double *>(cur); cur += p.oeps * B;
  const int64_t live_ld = (int64_t)(p.live / sizeof(int));
  int *flags = reinterpret_cast<int *>(cur);
  int *degs = flags + B;          // [2][B] box post degrees, alternating by layer
  int *idlists = flags + 3 * B;   // host classes: [H][2][B]; device classes: [2][slots][B], then [2][slots] counts
  int8_t *codes = reinterpret_cast<int8_t *>(idlists + (int64_t)p.list_ints * B);  // [B][nh]
  const bool learned = p.mode == BERN_PLAN_LEARNED;
  const int n = net->n;
  const int64_t slotA = (int64_t)(p.arenaA / p.elem), slotB = (int64_t)(p.arenaB / p.elem);
  const bool plain = p.mode == BERN_PLAN_PLAIN;
  const bool dev = !plain && dc != nullptr;
  const int64_t slots = dev ? dc->slots : 0;
  auto dev_ids = [&](int layer, int64_t k) -> const int * { return idlists + ((layer & 1) * slots + k) * B; };
  auto dev_cnt = [&](int layer, int64_t k) -> int * { return idlists + 2 * slots * B + (layer & 1) * slots + k; };

  // host-side degree classes of the current layer's pre-activations
  std::vector<const int *> carried;  // device id lists the next layer's read-off can reuse
  std::vector<BoxClass> classes(1);
  classes[0].Din = 1;
  classes[0].Dout = 0;
  std::vector<int> dcur(B, 1);
  // pinned staging: B box degrees, then one id list per (layer, phase); a
  // list is written once per wave, and every wave's first copy follows a
  // stream synchronisation, so no staged list is rewritten in flight
  // (and last, one int the first layer's read-off sets when a box is invalid)
  const size_t need = (size_t)B * (1 + 2 * (size_t)p.H) + 1;
  if (!plain && !dev && net->host_n < need) {
    BERN_HIP_TRY(hipStreamSynchronize(s));
    if (net->host_ids) (void)hipHostFree(net->host_ids);
    net->host_ids = net->host_dev = nullptr;
    net->host_n = 0;
    // mapped and coherent: the kernels that find the box degrees store them
    // here as well, so the host reads them with no copy
    BERN_HIP_TRY(hipHostMalloc((void **)&net->host_ids, need * sizeof(int),
                               hipHostMallocMapped | hipHostMallocCoherent));
    net->host_n = need;
    BERN_HIP_TRY(hipHostGetDevicePointer((void **)&net->host_dev, net->host_ids, 0));
  }
  // Host classes: the first layer's read-off reports an invalid box through
  // the staging's last int, so that a run with none skips the NaN step.
  volatile int *bad_h = (!plain && !dev) ? net->host_ids + need - 1 : nullptr;
  int *bad_d = (!plain && !dev) ? net->host_dev + need - 1 : nullptr;
  if (bad_h) *bad_h = 0;
  bool bad_known = false, any_bad = true, from_box_0 = false;
  // a phase's lists into the pinned staging, their device addresses into
  // devl; the ints to copy (0: one class of every box, the identity)
  auto stage = [&](std::vector<BoxClass> &cl, int layer, int phase, std::vector<const int *> &devl) -> size_t {
    devl.assign(cl.size(), nullptr);
    if (cl.size() == 1 && (int64_t)cl[0].ids.size() == B) return 0;  // identity
    int *all = net->host_ids + B + ((int64_t)layer * 2 + phase) * B;
    size_t cnt = 0;
    for (auto &c : cl) {
      std::copy(c.ids.begin(), c.ids.end(), all + cnt);
      cnt += c.ids.size();
    }
    int *dst = idlists + ((int64_t)layer * 2 + phase) * B;
    int64_t off = 0;
    for (size_t k = 0; k < cl.size(); ++k) {
      devl[k] = dst + off;
      off += cl[k].ids.size();
    }
    return cnt;
  };
  // both phases of a layer (adjacent slots of B ints) in one copy
  auto upload2 = [&](size_t c0, size_t c1, int layer) -> bern_status {
    const int64_t base = ((int64_t)layer * 2) * B;
    if (c0 == 0 && c1 == 0) return BERN_OK;
    const int64_t from = c0 > 0 ? base : base + B, count = c1 > 0 ? base + B + (int64_t)c1 - from : (int64_t)c0;
    BERN_HIP_TRY(hipMemcpyAsync(idlists + from, net->host_ids + B + from, (size_t)count * sizeof(int),
                                hipMemcpyHostToDevice, s));
    return BERN_OK;
  };
  for (auto &c : classes) {
    c.ids.resize(B);
    for (int64_t b = 0; b < B; ++b) c.ids[b] = (int)b;
  }
  bool restart = true;  // every box at pre degree 1 (the first layer, or after a linearisation)

  for (int i = 0; i < p.H; ++i) {
    const int hin = net->widths[i], h = net->widths[i + 1];
    const bool last = (i == p.H - 1);
    NeuronRec *recs = recbuf[i & 1];
    const NeuronRec *prev = recbuf[(i + 1) & 1];
    // plan codes are clamped to the plain rule's post degree of the layer
    const int cap = last ? 1 : p.Dpost[i];
    const bool lin_layer = !last && p.lin > 0 && (i + 1) % p.lin == 0;
    int *ldeg = degs + (i & 1) * B;  // this layer's box post degrees
    // the read-off classes of the layer
    std::vector<LaunchClass> rc;
    bern_status st = BERN_OK;
    if (dev) {
      if (restart) {
        rc.push_back(LaunchClass{1, 0, nullptr, B, nullptr});
      } else {
        const int64_t np = (int64_t)dc->pairs[i - 1].size();
        for (size_t m = 0; m < dc->din[i].size(); ++m)
          rc.push_back(LaunchClass{dc->din[i][m], 0, dev_ids(i - 1, np + m), B, dev_cnt(i - 1, np + m)});
      }
    } else {
      std::vector<const int *> cid;
      if (carried.size() == classes.size()) {
        cid = carried;  // the previous layer's composition lists, same classes in the same order
      } else {
        st = upload2(stage(classes, i, 0, cid), 0, i);
        if (st != BERN_OK) return st;
      }
      for (size_t k = 0; k < classes.size(); ++k)
        rc.push_back(LaunchClass{classes[k].Din, 0, cid[k], (int64_t)classes[k].ids.size(), nullptr});
    }
    carried.clear();
    // The first layer's pre tensors: formed by its read-off when that is one
    // degree-1 class of every box, else by the layer-1 kernel first; either
    // sets every box's validity flag (read by the last step).
    const bool from_box = i == 0 && rc.size() == 1 && rc[0].Din == 1 && !rc[0].bids && !rc[0].dcount &&
                          rc[0].nboxes == B;
    if (i == 0) from_box_0 = from_box;
    if (i == 0 && !from_box) {
      Layer1Args a{n, net->widths[1], B, nullptr, slotA, box_lo, box_hi, net->W64 + net->woff[0],
                   net->b64 + net->boff[0], Aa[0], p.fp64 ? 1 : 0, flags};
      BERN_HIP_TRY(launch_layer1(a, s));
    }
    // bounds read-off (+ rules and approximants for hidden layers), per class
    for (const LaunchClass &cl : rc) {
      ConvertArgs c{};
      c.n = n;
      c.D = cl.Din;
      c.h = h;
      c.L = p.L;
      LayerTables lt;
      st = layer_tables(net, cl.Din, p.Lmax, false, lt);
      if (st != BERN_OK) return st;
      c.C = ipow(cl.Din + 1, n);
      c.S = ssize(n, cl.Din);
      c.didx = lt.didx;
      c.plist = lt.plist;
      c.plist_len = lt.plist_len;
      if (lt.tree) {
        c.tree = lt.tree->buf;
        c.tree_len = lt.tree->len;
        for (int d = 0; d <= n && d < 17; ++d) c.tree_base[d] = lt.tree->base[d];
      }
      c.nboxes = cl.nboxes;
      c.bids = cl.bids;
      c.dcount = cl.dcount;
      c.slot = slotA;
      c.cap = cap;
      c.pre = Aa[i & 1];
      c.fp64 = p.fp64 ? 1 : 0;
      c.recs = recs;
      c.scratch = conv;
      c.scratch_bytes = p.conv * B;
      c.plan = (plain || learned) ? nullptr : plan;
      c.learned = learned && !last;
      c.fits = o->features && !last;  // export: every neuron fitted
      c.layer = i;
      c.hin = hin;
      c.prev = prev;
      c.prad = radbuf[(i + 1) & 1];
      c.W = net->W64 + net->woff[i];
      c.b = net->b64 + net->boff[i];
      c.box_lo = box_lo;
      c.box_hi = box_hi;
      c.from_box = from_box ? 1 : 0;
      c.flags = from_box ? flags : nullptr;
      c.hbad = from_box ? bad_d : nullptr;
      c.rpart = gpart;
      c.rpart_slot = (int64_t)(p.gpart / sizeof(double));
      c.cblocks = gemm_cblocks(c.S);
      c.tune = net->tune;
      c.plan_ld = net->nh;
      c.plan_col0 = last ? 0 : net->noff[i];
      if (last) {
        c.mode = 1;
        c.out_lo = olo;
        c.out_hi = ohi;
        c.ld_out = net->o;
        c.col0 = 0;
        c.used = nullptr;
        c.out_eps = ((op || o->counters) && !p.fp64) ? oeps : nullptr;
      } else {
        c.mode = 0;
        c.out_lo = nlo;
        c.out_hi = nhi;
        c.ld_out = net->nh;
        c.col0 = net->noff[i];
        c.used = used;
      }
      BERN_HIP_TRY(launch_convert(c, s));
    }
    // predictor and rules (learned plans), or the exported features: one
    // launch over the wave's boxes, every record holding its own degree
    if (!last && (learned || o->features)) {
      LearnArgs la{};
      la.n = n;
      la.h = h;
      la.H = p.H;
      la.layer = i;
      la.nboxes = B;
      la.bids = nullptr;
      la.recs = recs;
      la.sens = net->sens + net->noff[i];
      la.feat = o->features ? o->features + (size_t)b0 * net->nh * 8 : nullptr;
      la.nh = net->nh;
      la.noff = net->noff[i];
      la.params = learned ? o->pred->params : nullptr;
      la.codes = codes;
      la.used = used;
      la.degs = learned ? ldeg : nullptr;  // the rules kernel also gives each box's post degree
      la.hdegs = learned && !plain && !dev ? net->host_dev : nullptr;  // and the host's copy
      la.cap = cap;
      la.fp64 = p.fp64 ? 1 : 0;
      la.L = p.L;
      la.raise = o->no_raise ? 0 : 1;
      if (learned && !lin_layer) {  // the rules also write the next affine map's input lists
        la.live = live;
        la.live_ld = live_ld;
      }
      if (learned)
        BERN_HIP_TRY(launch_learned_rules(la, s));
      else
        BERN_HIP_TRY(launch_features(la, s));
    }
    if (!last && o->counters) {
      ProfScope ps(kProfMisc, s, 0.0);
      hipLaunchKernelGGL(counters_rules_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, B, h,
                         (const NeuronRec *)recs, (long long *)o->counters);
      BERN_HIP_TRY(hipGetLastError());
    }
    if (last && o->counters && !p.fp64) {
      ProfScope ps(kProfMisc, s, 0.0);
      hipLaunchKernelGGL(counters_pad_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, B, net->o,
                         (const double *)oeps, (long long *)o->counters);
      BERN_HIP_TRY(hipGetLastError());
    }
    if (last) {
      if (op) {  // the output layer's stored tensors, per class, into the caller's dense tensors
        for (const LaunchClass &cl : rc) {
          if (cl.dcount) {
            set_error("output tensors are taken with host-side classes only");
            return BERN_E_ARG;
          }
          if (op->vol) {  // relative volume at the class's own degree
            OutPolyArgs a{};
            a.pre = Aa[i & 1];
            a.slot = slotA;
            a.S = ssize(n, cl.Din);
            BERN_HIP_TRY(dense_index_table(*net->tab, cl.Din, &a.didx));  // built for this layer's read-off
            a.bids = cl.bids;
            a.nboxes = cl.nboxes;
            a.h = h;
            a.eps = p.fp64 ? nullptr : oeps;
            a.fp64 = p.fp64 ? 1 : 0;
            BERN_HIP_TRY(launch_rel_volume(a, n, cl.Din, op->vol + (size_t)b0 * h, s));
            continue;
          }
          if (cl.Din > op->D) {
            set_error("output degree %d of some box exceeds the requested %d", cl.Din, op->D);
            return BERN_E_DEGREE;
          }
          OutPolyArgs a{};
          a.pre = Aa[i & 1];
          a.slot = slotA;
          a.S = ssize(n, cl.Din);
          a.C = op->C;
          a.didx = op->didx;
          a.bids = cl.bids;
          a.nboxes = cl.nboxes;
          a.h = h;
          a.eps = p.fp64 ? nullptr : oeps;
          a.fp64 = p.fp64 ? 1 : 0;
          a.U = op->U + (size_t)b0 * h * op->C;
          a.L = op->L + (size_t)b0 * h * op->C;
          BERN_HIP_TRY(launch_out_polys(a, s));
        }
      }
      break;
    }

    // this layer's box degrees: pre (null: every box at the uniform uDin)
    // and post (null: uniform, the plain rule)
    const int uDin = plain ? rc[0].Din : 1;
    const int uDout = plain ? p.L * uDin : 0;
    const int *din = (plain || restart) ? nullptr : degs + ((i + 1) & 1) * B;
    const int *dout = plain ? nullptr : ldeg;
    // a learned plan's host classes: the composition's first stage goes
    // ahead of the wait for them (its inputs are on the device: the degrees
    // and, from the rules kernel, the lists)
    const bool early_scatter = learned && !plain && !dev;
    // (Din, Dout) classes for the products; post degree classes for the
    // affine map and the next layer's read-off
    std::vector<BoxClass> next, nc;  // host classes
    std::vector<LaunchClass> pc, gc;
    std::vector<const int *> gid;
    if (plain) {
      pc.push_back(LaunchClass{uDin, uDout, rc[0].bids, rc[0].nboxes, nullptr});
      gc = pc;
      nc = classes;
      nc[0].Din = uDout;
      gid.assign(1, rc[0].bids);
    } else {
      if (!learned) {  // (the learned rules kernel wrote them)
        ProfScope ps(kProfMisc, s, 0.0);
        hipLaunchKernelGGL(box_degree_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, B, h,
                           (const NeuronRec *)recs, ldeg, dev ? nullptr : net->host_dev);
      }
      BERN_HIP_TRY(hipGetLastError());
      if (dev) {
        const auto &pr = dc->pairs[i];
        const auto &dv = dc->dout[i];
        ClassTab t{};
        t.npairs = (int)pr.size();
        t.nvals = (int)dv.size();
        for (int k = 0; k < t.npairs; ++k) {
          t.din[k] = pr[k].first;
          t.dout[k] = pr[k].second;
        }
        for (int m = 0; m < t.nvals; ++m) t.vals[m] = dv[m];
        {
          ProfScope ps(kProfMisc, s, 0.0);
          hipLaunchKernelGGL(classify_kernel, dim3((unsigned)(t.npairs + t.nvals + 1)), dim3(1024), 0, s, B,
                             restart ? (const int *)nullptr : (const int *)(degs + ((i + 1) & 1) * B),
                             (const int *)ldeg, t, idlists + (i & 1) * slots * B, dev_cnt(i, 0), flags);
        }
        BERN_HIP_TRY(hipGetLastError());
        for (int k = 0; k < t.npairs; ++k)
          pc.push_back(LaunchClass{pr[k].first, pr[k].second, dev_ids(i, k), B, dev_cnt(i, k)});
        for (int m = 0; m < t.nvals; ++m)
          gc.push_back(LaunchClass{0, dv[m], dev_ids(i, t.npairs + m), B, dev_cnt(i, t.npairs + m)});
      } else {
        // the degrees' host copy, stored by the kernel that found them; the
        // composition's first stage runs while the host waits for them
        const int *hd = net->host_ids;
        BERN_HIP_TRY(spin_mark(s));
        if (early_scatter) {
          st = compose_scatter_stage(net, p, i, uDin, uDout, din, dout, B, Aa[i & 1], Bp, slotA, slotB, recs,
                                     radbuf[i & 1], cpart, live, live_ld, s);
          if (st != BERN_OK) return st;
        }
        BERN_HIP_TRY(spin_poll());
        if (i == 0 && from_box_0) {  // the first layer's read-off is done
          any_bad = *bad_h != 0;
          bad_known = true;
        }
        for (int64_t b = 0; b < B; ++b) {
          const int din_b = dcur[b], dout_b = std::max(hd[b], 0);
          size_t k = 0;
          for (; k < next.size(); ++k)
            if (next[k].Din == din_b && next[k].Dout == dout_b) break;
          if (k == next.size()) next.push_back(BoxClass{din_b, dout_b, {}});
          next[k].ids.push_back((int)b);
        }
        for (auto &cl : next) {
          size_t k = 0;
          for (; k < nc.size(); ++k)
            if (nc[k].Din == cl.Dout) break;
          if (k == nc.size()) nc.push_back(BoxClass{cl.Dout, 0, {}});
          nc[k].ids.insert(nc[k].ids.end(), cl.ids.begin(), cl.ids.end());
        }
        for (auto &cl : nc) std::sort(cl.ids.begin(), cl.ids.end());
        std::vector<const int *> pid;
        const size_t c0 = stage(next, i, 0, pid), c1 = stage(nc, i, 1, gid);
        st = upload2(c0, c1, i);
        if (st != BERN_OK) return st;
        for (size_t k = 0; k < next.size(); ++k)
          pc.push_back(LaunchClass{next[k].Din, next[k].Dout, pid[k], (int64_t)next[k].ids.size(), nullptr});
        for (size_t k = 0; k < nc.size(); ++k)
          gc.push_back(LaunchClass{0, nc[k].Din, gid[k], (int64_t)nc[k].ids.size(), nullptr});
      }
    }
    // the next affine map's input lists of every box (a linearised layer
    // builds its own after the linearisation; a learned plan's rules kernel
    // has written them)
    if (!lin_layer && !learned) {
      ComposeArgs ml{};
      ml.h = h;
      ml.nboxes = B;
      ml.recs = recs;
      ml.live = live;
      ml.live_ld = live_ld;
      BERN_HIP_TRY(launch_live(ml, s));
    }
    st = compose_layer(net, p, i, pc, uDin, uDout, din, dout, B, Aa[i & 1], Bp, slotA, slotB, recs, radbuf[i & 1],
                       cpart, horner, live, live_ld, !early_scatter, s);
    if (st != BERN_OK) return st;
    if (lin_layer) {
      st = lin_layer_run(net, p, i, gc, uDin, uDout, din, dout, B, Aa, Bp, slotA, slotB, recs, radbuf[i & 1], live,
                         live_ld, gpart, conv, s);
      if (st != BERN_OK) return st;
      classes.assign(1, BoxClass{1, 0, {}});
      classes[0].ids.resize(B);
      for (int64_t b = 0; b < B; ++b) {
        classes[0].ids[b] = (int)b;
        dcur[b] = 1;
      }
      carried.clear();
      restart = true;
      continue;
    }
    restart = false;
    st = gemm_layer(net, p, i, gc, uDin, din, Aa, Bp, slotA, slotB, live, live_ld, gpart, s);
    if (st != BERN_OK) return st;
    if (dev) continue;  // the classification kernel listed the next read-off's classes
    // next layer's classes: by the new pre degree, the lists just uploaded
    for (auto &cl : nc)
      for (int b : cl.ids) dcur[b] = cl.Din;
    carried = gid;
    classes.swap(nc);
  }
  if (!bad_known || any_bad) {
    ProfScope ps(kProfMisc, s, 0.0);
    hipLaunchKernelGGL(poison_kernel, dim3((unsigned)B), dim3(64), 0, s, B, (const int *)flags, net->nh, net->o,
                       nlo, nhi, olo, ohi);
    BERN_HIP_TRY(hipGetLastError());
  }
  return BERN_OK;
}

// Capture the launch sequence `run` once per distinct argument set on the
// network's own capture stream, then replay it on `s` as one graph launch.
template <typename Run>
static bern_status run_graph(bern_net *net, const bern_opts *o, int64_t n_boxes, std::vector<uint64_t> key,
                             Run &run, hipStream_t s) {
  key.push_back((uint64_t)n_boxes);
  key.push_back((uint64_t)o->L);
  key.push_back((uint64_t)o->precision);
  key.push_back((uint64_t)o->sched);
  key.push_back((uint64_t)o->max_wave);
  key.push_back((uint64_t)(uintptr_t)o->features);
  key.push_back((uint64_t)o->lin);
  key.push_back((uint64_t)o->no_raise);
  key.push_back((uint64_t)(uintptr_t)o->counters);
  key.push_back((uint64_t)net->tune.gemm_wide | (uint64_t)net->tune.gemm_narrow << 8 |
                (uint64_t)net->tune.conv_block << 16 | (uint64_t)net->tune.conv_wave << 24);
  int dev = 0;
  BERN_HIP_TRY(hipGetDevice(&dev));
  key.push_back((uint64_t)dev);
  for (auto &g : net->graphs) {
    if (g.key == key) {
      BERN_HIP_TRY(hipGraphLaunch(g.exec, s));
      return BERN_OK;
    }
  }
  if (!net->capture) BERN_HIP_TRY(hipStreamCreateWithFlags(&net->capture, hipStreamNonBlocking));
  const bool prof = g_prof_on;
  g_prof_on = false;  // no timing events inside a captured sequence
  BERN_HIP_TRY(hipStreamBeginCapture(net->capture, hipStreamCaptureModeRelaxed));
  bern_status st = run(net->capture);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(net->capture, &graph);
  g_prof_on = prof;
  if (st != BERN_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  BERN_HIP_TRY(ce);
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    set_error("graph instantiation failed");
    return BERN_E_DEVICE;
  }
  if (net->graphs.size() >= 8) {  // keep the most recent few
    (void)hipGraphExecDestroy(net->graphs.front().exec);
    (void)hipGraphDestroy(net->graphs.front().graph);
    net->graphs.erase(net->graphs.begin());
  }
  net->graphs.push_back({key, graph, exec});
  BERN_HIP_TRY(hipGraphLaunch(exec, s));
  return BERN_OK;
}

// Every index table the device classes of plan p can use (built here, once
// per network, before any capture; without allocations only looked up):
// the read-off at every pre degree, the products of every class that can
// hold an order >= 2, and the Lin read-off at every post degree. False when
// one of them exceeds its limits or, without allocations, is missing.
static bool dev_class_tables(const bern_net *net, const Plan &p) {
  const DevClasses &dc = p.dc;
  for (int i = 0; i < p.H; ++i) {
    LayerTables lt;
    for (int d : dc.din[i])
      if (layer_tables(net, d, p.Lmax, false, lt) != BERN_OK) return false;
    if (i == p.H - 1) continue;
    for (const auto &pr : dc.pairs[i]) {
      const int order = class_order(p, pr.first, pr.second);
      if (order >= 2 && layer_tables(net, pr.first, order, true, lt) != BERN_OK) return false;
    }
    const bool lin = p.lin > 0 && (i + 1) % p.lin == 0;
    for (int d : dc.dout[i])
      if (lin && d >= 1 && layer_tables(net, d, p.Lmax, false, lt) != BERN_OK) return false;
  }
  return true;
}

static bern_status bounds_impl(const bern_net *net, const bern_opts *opts, int64_t n_boxes, const double *box_lo,
                               const double *box_hi, const int8_t *plan, double *neuron_lo, double *neuron_hi,
                               double *out_lo, double *out_hi, int8_t *used_plan, void *workspace, size_t ws_bytes,
                               void *stream, bern_stats *stats, const OutPolys *op) {
  const auto t_enter = std::chrono::steady_clock::now();
  bern_status st = check_opts(net, opts);
  if (st != BERN_OK) return st;
  if (n_boxes < 1 || !box_lo || !box_hi || !out_lo || !out_hi) {
    set_error("bad arguments (n_boxes = %lld)", (long long)n_boxes);
    return BERN_E_ARG;
  }
  if (!workspace || ((uintptr_t)workspace & 255)) {
    set_error("workspace must be a non-null 256-byte aligned device pointer");
    return BERN_E_WORKSPACE;
  }
  if (opts->plan == BERN_PLAN_GIVEN && !plan) {
    set_error("BERN_PLAN_GIVEN needs a plan array");
    return BERN_E_ARG;
  }

  Plan p;
  if ((st = plan_net(net, opts, p)) != BERN_OK) return st;
  const size_t per_box = p.per_box();
  if (ws_bytes < per_box) {
    set_error("workspace of %zu bytes is smaller than one box needs (%zu)", ws_bytes, per_box);
    return BERN_E_WORKSPACE;
  }
  int64_t wave = (int64_t)(ws_bytes / per_box);
  if (opts->sched == BERN_SCHED_PER_BOX) wave = 1;
  if (opts->max_wave > 0) wave = std::min<int64_t>(wave, opts->max_wave);
  wave = std::min<int64_t>(wave, std::min<int64_t>(n_boxes, 65535));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int nwaves = (int)((n_boxes + wave - 1) / wave);
  // Per-neuron plans in a graph: the device lists every class the rules can
  // give (when they are few), so the wave needs no host round trip.
  bool graph = opts->graph && !op && (p.mode == BERN_PLAN_PLAIN || p.dev_ok);
  // device classes: under a graph, and always without allocations (the
  // host classes stage box degrees in pinned host memory)
  const bool plain_rule = p.mode == BERN_PLAN_PLAIN;
  const DevClasses *dc = !plain_rule && !op && p.dev_ok && (graph || g_no_alloc) ? &p.dc : nullptr;
  if (dc && !dev_class_tables(net, p)) {
    // a class whose tables exceed their limits leaves the run to the host
    // classes, which build only those of the classes that occur
    if (g_no_alloc) {
      set_error("the network's index tables for these options are not built yet");
      return BERN_E_ARG;
    }
    dc = nullptr;
    graph = false;
  }
  if (!plain_rule && !dc && g_no_alloc) {
    set_error("the degree classes of this plan exceed what the device lists");
    return BERN_E_ARG;
  }
  if (!plain_rule && !dc) {
    // host classes synchronise the stream once per hidden layer, which a
    // stream under capture does not allow
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    BERN_HIP_TRY(hipStreamIsCapturing(reinterpret_cast<hipStream_t>(stream), &cs));
    if (cs != hipStreamCaptureStatusNone) {
      set_error("a per-neuron plan run with host-side degree classes synchronises its stream, which is being "
                "captured (set opts.graph to list the classes on the device)");
      return BERN_E_ARG;
    }
  }
  auto run_all = [&](hipStream_t rs) -> bern_status {
    if (opts->counters) {
      ProfScope ps(kProfMisc, rs, 0.0);
      hipLaunchKernelGGL(counters_clear_kernel, dim3(1), dim3(64), 0, rs, (long long *)opts->counters);
      BERN_HIP_TRY(hipGetLastError());
    }
    for (int64_t b0 = 0; b0 < n_boxes; b0 += wave) {
      const int64_t B = std::min<int64_t>(wave, n_boxes - b0);
      bern_status r = run_wave(net, p, opts, b0, B, box_lo + b0 * net->n, box_hi + b0 * net->n,
                               plan ? plan + b0 * net->nh : nullptr, neuron_lo ? neuron_lo + b0 * net->nh : nullptr,
                               neuron_hi ? neuron_hi + b0 * net->nh : nullptr, out_lo + b0 * net->o,
                               out_hi + b0 * net->o, used_plan ? used_plan + b0 * net->nh : nullptr,
                               reinterpret_cast<char *>(workspace), rs, op, dc);
      if (r != BERN_OK) return r;
    }
    return BERN_OK;
  };
  // Runs with no host round trip (the plain rule, or per-neuron plans with
  // device classes) are captured once per argument set and replayed as one
  // graph launch; per-neuron plans otherwise read every box's degree back
  // once per hidden layer and run eagerly.
  if (graph) {
    // index tables are built (device allocations) before any capture
    for (int i = 0; i < p.H && !dc; ++i) {
      LayerTables lt;
      st = layer_tables(net, p.Dpre[i], p.Lmax, i < p.H - 1, lt);
      if (st != BERN_OK) return st;
      if (i < p.H - 1 && p.lin > 0 && (i + 1) % p.lin == 0) {  // the Lin read-off at the post degree
        st = layer_tables(net, p.Dpost[i], p.Lmax, false, lt);
        if (st != BERN_OK) return st;
      }
    }
    st = run_graph(const_cast<bern_net *>(net), opts, n_boxes,
                   {(uint64_t)(uintptr_t)box_lo, (uint64_t)(uintptr_t)box_hi, (uint64_t)(uintptr_t)neuron_lo,
                    (uint64_t)(uintptr_t)neuron_hi, (uint64_t)(uintptr_t)out_lo, (uint64_t)(uintptr_t)out_hi,
                    (uint64_t)(uintptr_t)used_plan, (uint64_t)(uintptr_t)workspace, (uint64_t)ws_bytes,
                    (uint64_t)wave, (uint64_t)opts->plan, (uint64_t)(uintptr_t)plan,
                    (uint64_t)(uintptr_t)(opts->pred ? opts->pred->params : nullptr)},
                   run_all, s);
  } else {
    st = run_all(s);
  }
  if (st != BERN_OK) return st;
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->n_waves = nwaves;
    stats->boxes_per_wave = (int32_t)wave;
    stats->out_degree = p.Dpre[p.H - 1];
    stats->lin_layers = p.lin_layers;
    stats->workspace_used = per_box * (size_t)wave;
    stats->graph = graph ? 1 : 0;
    stats->device_classes = dc ? 1 : 0;
    stats->enqueue_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_enter).count();
  }
  return BERN_OK;
}

extern "C" bern_status bern_bounds(const bern_net *net, const bern_opts *opts, int64_t n_boxes, const double *box_lo,
                                   const double *box_hi, const int8_t *plan, double *neuron_lo, double *neuron_hi,
                                   double *out_lo, double *out_hi, int8_t *used_plan, void *workspace,
                                   size_t ws_bytes, void *stream, bern_stats *stats) {
  return bounds_impl(net, opts, n_boxes, box_lo, box_hi, plan, neuron_lo, neuron_hi, out_lo, out_hi, used_plan,
                     workspace, ws_bytes, stream, stats, nullptr);
}

namespace bern {
// bern_bounds on a library-owned scratch buffer (bern_bounds_noalloc): the
// plain rule, or the learned plan with its degree classes listed on the
// device (no host staging of per-box degrees), run eagerly (no graph
// objects), and only once every index table the options need exists
// (checked before anything is enqueued); while it runs, table builders and
// the profiler's event pool allocate nothing.
bern_status bounds_on_scratch(const bern_net *net, const bern_opts *opts, int64_t n_boxes, const double *box_lo,
                              const double *box_hi, double *neuron_lo, double *neuron_hi, double *out_lo,
                              double *out_hi, int8_t *used_plan, void *scratch, size_t scratch_bytes, void *stream,
                              bern_stats *stats) {
  bern_status st = check_opts(net, opts);
  if (st != BERN_OK) return st;
  if (opts->plan == BERN_PLAN_GIVEN) {
    set_error("bern_bounds_noalloc takes the plain rule or the learned plan (it has no codes argument)");
    return BERN_E_ARG;
  }
  Plan p;
  if ((st = plan_net(net, opts, p)) != BERN_OK) return st;
  if (p.mode == BERN_PLAN_LEARNED && !p.dev_ok) {
    set_error("the learned plan's degree classes exceed what the device lists (over %d (pre, post) pairs or %d "
              "lists in a layer), which bern_bounds_noalloc needs", kMaxDevPairs, kMaxDevLists);
    return BERN_E_ARG;
  }
  if (p.per_box() > scratch_bytes) {
    set_error("one box needs %zu bytes of scratch, over the %zu bytes bern_bounds_noalloc holds", p.per_box(),
              scratch_bytes);
    return BERN_E_TOO_LARGE;
  }
  struct Guard {
    Guard() { g_no_alloc = true; }
    ~Guard() { g_no_alloc = false; }
  } guard;
  bool ok = true;
  if (p.mode == BERN_PLAN_PLAIN) {
    for (int i = 0; i < p.H && ok; ++i) {
      LayerTables lt;
      ok = layer_tables(net, p.Dpre[i], p.Lmax, i < p.H - 1, lt) == BERN_OK;
      if (ok && i < p.H - 1 && p.lin > 0 && (i + 1) % p.lin == 0)
        ok = layer_tables(net, p.Dpost[i], p.Lmax, false, lt) == BERN_OK;
    }
  } else {
    ok = dev_class_tables(net, p);
  }
  if (!ok) {
    set_error("the network's index tables for these options are not built yet (a bern_bounds call with the "
              "same options builds them; for the learned plan, with opts.graph set)");
    return BERN_E_ARG;
  }
  bern_opts o = *opts;
  o.graph = 0;
  return bounds_impl(net, &o, n_boxes, box_lo, box_hi, nullptr, neuron_lo, neuron_hi, out_lo, out_hi, used_plan,
                     scratch, scratch_bytes, stream, stats, nullptr);
}
}  // namespace bern

extern "C" bern_status bern_output_polys(const bern_net *net, const bern_opts *opts, int64_t n_boxes,
                                         const double *box_lo, const double *box_hi, const int8_t *plan,
                                         int32_t degree, double *poly_U, double *poly_L, double *out_lo,
                                         double *out_hi, void *workspace, size_t ws_bytes, void *stream) {
  bern_status st = check_opts(net, opts);
  if (st != BERN_OK) return st;
  if (!poly_U || !poly_L || degree < 1) {
    set_error("bern_output_polys needs both polynomial arrays and a degree >= 1 (got %d)", degree);
    return BERN_E_ARG;
  }
  const int64_t C = tsize(net->n, degree);
  if (C < 0 || C > ((int64_t)1 << 31)) {
    set_error("(%d+1)^%d dense coefficients overflow", degree, net->n);
    return BERN_E_TOO_LARGE;
  }
  OutPolys op{poly_U, poly_L, degree, C, nullptr};
  hipError_t e = dense_index_table(*net->tab, degree, &op.didx);
  if (e == hipErrorInvalidValue) {
    set_error("index table for degree %d in %d variables exceeds its limits", degree, net->n);
    return BERN_E_TOO_LARGE;
  }
  BERN_HIP_TRY(e);
  return bounds_impl(net, opts, n_boxes, box_lo, box_hi, plan, nullptr, nullptr, out_lo, out_hi, nullptr, workspace,
                     ws_bytes, stream, nullptr, &op);
}

extern "C" bern_status bern_rel_volume(const bern_net *net, const bern_opts *opts, int64_t n_boxes,
                                       const double *box_lo, const double *box_hi, const int8_t *plan,
                                       double *rel_vol, double *out_lo, double *out_hi, void *workspace,
                                       size_t ws_bytes, void *stream) {
  bern_status st = check_opts(net, opts);
  if (st != BERN_OK) return st;
  if (!rel_vol) {
    set_error("bern_rel_volume needs an output array");
    return BERN_E_ARG;
  }
  OutPolys op{nullptr, nullptr, 0, 0, nullptr, rel_vol};
  return bounds_impl(net, opts, n_boxes, box_lo, box_hi, plan, nullptr, nullptr, out_lo, out_hi, nullptr, workspace,
                     ws_bytes, stream, nullptr, &op);
}

// ------------------------------------------------- host-memory convenience
namespace {
// Device buffers of one bern_bounds_host call, released on every return.
struct DeviceBufs {
  std::vector<void *> ptrs;
  ~DeviceBufs() {
    for (void *q : ptrs) (void)hipFree(q);
  }
  hipError_t alloc(void **out, size_t bytes) {
    *out = nullptr;
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMalloc(out, bytes);
    if (e == hipSuccess) ptrs.push_back(*out);
    return e;
  }
};
}  // namespace

extern "C" bern_status bern_bounds_host(const bern_net *net, const bern_opts *opts, int64_t n_boxes,
                                        const double *box_lo, const double *box_hi, const int8_t *plan,
                                        double *neuron_lo, double *neuron_hi, double *out_lo, double *out_hi,
                                        int8_t *used_plan, bern_stats *stats) {
  bern_status st = check_opts(net, opts);
  if (st != BERN_OK) return st;
  if (n_boxes < 1 || !box_lo || !box_hi || !out_lo || !out_hi) {
    set_error("bad arguments (n_boxes = %lld)", (long long)n_boxes);
    return BERN_E_ARG;
  }
  size_t ws_all = 0, ws_one = 0;
  if ((st = bern_workspace_size(net, opts, n_boxes, &ws_all, &ws_one)) != BERN_OK) return st;
  const size_t nb = (size_t)n_boxes, nbox = nb * (size_t)net->n * sizeof(double);
  const size_t nhid = nb * (size_t)net->nh, nout = nb * (size_t)net->o * sizeof(double);
  DeviceBufs d;
  void *dlo, *dhi, *dplan = nullptr, *dnlo = nullptr, *dnhi = nullptr, *dolo, *dohi, *dused = nullptr, *ws = nullptr;
  BERN_HIP_TRY(d.alloc(&dlo, nbox));
  BERN_HIP_TRY(d.alloc(&dhi, nbox));
  if (plan) BERN_HIP_TRY(d.alloc(&dplan, nhid));
  if (neuron_lo) BERN_HIP_TRY(d.alloc(&dnlo, nhid * sizeof(double)));
  if (neuron_hi) BERN_HIP_TRY(d.alloc(&dnhi, nhid * sizeof(double)));
  BERN_HIP_TRY(d.alloc(&dolo, nout));
  BERN_HIP_TRY(d.alloc(&dohi, nout));
  if (used_plan) BERN_HIP_TRY(d.alloc(&dused, nhid));
  // the whole batch in one wave if it fits, else the smallest usable workspace
  if (d.alloc(&ws, ws_all) != hipSuccess) {
    (void)hipGetLastError();
    BERN_HIP_TRY(d.alloc(&ws, ws_one));
    ws_all = ws_one;
  }
  BERN_HIP_TRY(hipMemcpy(dlo, box_lo, nbox, hipMemcpyHostToDevice));
  BERN_HIP_TRY(hipMemcpy(dhi, box_hi, nbox, hipMemcpyHostToDevice));
  if (plan) BERN_HIP_TRY(hipMemcpy(dplan, plan, nhid, hipMemcpyHostToDevice));
  st = bern_bounds(net, opts, n_boxes, (const double *)dlo, (const double *)dhi, (const int8_t *)dplan,
                   (double *)dnlo, (double *)dnhi, (double *)dolo, (double *)dohi, (int8_t *)dused, ws, ws_all,
                   nullptr, stats);
  if (st != BERN_OK) return st;
  BERN_HIP_TRY(hipStreamSynchronize(nullptr));
  BERN_HIP_TRY(hipMemcpy(out_lo, dolo, nout, hipMemcpyDeviceToHost));
  BERN_HIP_TRY(hipMemcpy(out_hi, dohi, nout, hipMemcpyDeviceToHost));
  if (neuron_lo) BERN_HIP_TRY(hipMemcpy(neuron_lo, dnlo, nhid * sizeof(double), hipMemcpyDeviceToHost));
  if (neuron_hi) BERN_HIP_TRY(hipMemcpy(neuron_hi, dnhi, nhid * sizeof(double), hipMemcpyDeviceToHost));
  if (used_plan) BERN_HIP_TRY(hipMemcpy(used_plan, dused, nhid, hipMemcpyDeviceToHost));
  return BERN_OK;
}

// ------------------------------------------------------- branch and bound
// One branch-and-bound round (bern_verify) in one block: every pending box is
// decided from the bounds of output k -- verified (+1) when out_hi <= thr,
// violated (-1) when out_lo > thr, open (0) otherwise -- and, when the round
// may split and the halves of the open boxes fit max_boxes, each open box is
// bisected along its widest input dimension into the next buffer (box
// order: open box number q gives boxes 2q and 2q + 1). The volume fractions
// (box volume over `total`) are summed in a fixed order: each thread over a
// contiguous run of boxes, then thread 0 over the threads. out: [0] open
// boxes, [1] split (1/0), [2] verified, [3] violated, [4] open-and-unsplit
// volume fractions.
static __global__ void __launch_bounds__(1024) bb_round_kernel(int n, int o, int64_t nb, const double *lo, const double *hi,
                                                        const double *olo, const double *ohi, int k, double thr,
                                                        double total, int64_t max_boxes, int may_split, double *nlo,
                                                        double *nhi, int8_t *status, int64_t *pos, double *out) {
  __shared__ int wsum[16];
  __shared__ int64_t base;
  __shared__ int split;
  __shared__ double part[3][1024];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  if (tid == 0) base = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += blockDim.x) {  // decisions, and the open boxes' numbers
    const int64_t b = b0 + tid;
    bool open = false;
    if (b < nb) {
      const double bl = olo[b * o + k], bh = ohi[b * o + k];
      const int8_t st = bh <= thr ? 1 : (bl > thr ? -1 : 0);
      status[b] = st;
      open = st == 0;
    }
    const unsigned long long bal = __ballot(open);
    if (lane == 0) wsum[wid] = __popcll(bal);
    __syncthreads();
    if (open) {
      int64_t q = base;
      for (int w = 0; w < wid; ++w) q += wsum[w];
      pos[b] = q + __popcll(bal & ((1ull << lane) - 1ull));
    }
    __syncthreads();
    if (tid == 0) {
      int tot = 0;
      for (int w = 0; w < nw; ++w) tot += wsum[w];
      base += tot;
    }
    __syncthreads();
  }
  if (tid == 0) split = may_split && base * 2 <= max_boxes;
  __syncthreads();
  double v[3] = {0.0, 0.0, 0.0};
  const int64_t run = (nb + blockDim.x - 1) / blockDim.x;
  for (int64_t b = tid * run; b < nb && b < (tid + 1) * run; ++b) {
    const double *l = lo + b * n, *h = hi + b * n;
    double vol = 1.0;
    int wide = 0;
    for (int a = 0; a < n; ++a) {
      vol *= h[a] - l[a];
      if (a > 0 && h[a] - l[a] > h[wide] - l[wide]) wide = a;
    }
    vol /= total;
    const int st = status[b];
    if (st == 1) {
      v[0] += vol;
    } else if (st == -1) {
      v[1] += vol;
    } else if (!split) {
      v[2] += vol;
    } else {
      const double mid = 0.5 * (l[wide] + h[wide]);
      for (int half = 0; half < 2; ++half) {
        double *cl = nlo + (2 * pos[b] + half) * n, *ch = nhi + (2 * pos[b] + half) * n;
        for (int a = 0; a < n; ++a) {
          cl[a] = a == wide && half == 1 ? mid : l[a];
          ch[a] = a == wide && half == 0 ? mid : h[a];
        }
      }
    }
  }
  for (int q = 0; q < 3; ++q) part[q][tid] = v[q];
  __syncthreads();
  if (tid == 0) {
    double t[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < (int)blockDim.x; ++i)
      for (int q = 0; q < 3; ++q) t[q] += part[q][i];
    out[0] = (double)base;
    out[1] = split ? 1.0 : 0.0;
    out[2] = t[0];
    out[3] = t[1];
    out[4] = t[2];
  }
}

extern "C" bern_status bern_verify(const bern_net *net, const bern_opts *opts, int64_t n_boxes,
                                   const double *box_lo, const double *box_hi, int32_t out_index, double threshold,
                                   int32_t max_rounds, int64_t max_boxes, bern_verify_result *res) {
  bern_status st = check_opts(net, opts);
  if (st != BERN_OK) return st;
  if (n_boxes < 1 || !box_lo || !box_hi || !res || out_index < 0 || out_index >= net->o || max_rounds < 1 ||
      max_boxes < n_boxes) {
    set_error("bad arguments (n_boxes %lld, out_index %d, max_rounds %d, max_boxes %lld)", (long long)n_boxes,
              out_index, max_rounds, (long long)max_boxes);
    return BERN_E_ARG;
  }
  const int n = net->n, o = net->o;
  std::vector<double> lo(box_lo, box_lo + n_boxes * n), hi(box_hi, box_hi + n_boxes * n);
  double total = 0.0;
  auto volume = [&](const double *l, const double *h) {
    double v = 1.0;
    for (int a = 0; a < n; ++a) v *= h[a] - l[a];
    return v;
  };
  for (int64_t b = 0; b < n_boxes; ++b) {
    for (int a = 0; a < n; ++a)
      if (!(lo[b * n + a] < hi[b * n + a])) {
        set_error("box %lld: d_lo >= d_hi in dimension %d", (long long)b, a);
        return BERN_E_BOX;
      }
    total += volume(&lo[b * n], &hi[b * n]);
  }
  // keep the caller's decision log settings, clear the rest
  const int64_t log_cap = res->log_cap;
  double *log_lo = res->log_lo, *log_hi = res->log_hi, *log_olo = res->log_out_lo, *log_ohi = res->log_out_hi;
  int8_t *log_st = res->log_status;
  const bool logging = log_cap > 0 && log_lo && log_hi && log_olo && log_ohi && log_st;
  memset(res, 0, sizeof(*res));
  res->log_cap = log_cap;
  res->log_lo = log_lo;
  res->log_hi = log_hi;
  res->log_out_lo = log_olo;
  res->log_out_hi = log_ohi;
  res->log_status = log_st;
  auto log_box = [&](const double *l, const double *h, double olo_, double ohi_, int8_t status) {
    if (!logging || res->log_count >= log_cap) return;
    const int64_t k = res->log_count++;
    std::copy(l, l + n, log_lo + k * n);
    std::copy(h, h + n, log_hi + k * n);
    log_olo[k] = olo_;
    log_ohi[k] = ohi_;
    log_st[k] = status;
  };
  // the rounds on the device: the pending boxes (two buffers, alternating),
  // their output bounds, decisions and halves stay in device memory; each
  // round reads back its open count and volume sums (and, when the caller
  // logs decisions, the round's boxes and bounds)
  size_t ws_bytes = 0, ws_one = 0;
  if ((st = bern_workspace_size(net, opts, max_boxes, &ws_bytes, &ws_one)) != BERN_OK) return st;
  DeviceBufs d;
  void *blo[2], *bhi[2], *dolo, *dohi, *dstat, *dpos, *dout, *ws;
  const size_t boxb = (size_t)max_boxes * n * sizeof(double), outb = (size_t)max_boxes * o * sizeof(double);
  for (int q = 0; q < 2; ++q) {
    BERN_HIP_TRY(d.alloc(&blo[q], boxb));
    BERN_HIP_TRY(d.alloc(&bhi[q], boxb));
  }
  BERN_HIP_TRY(d.alloc(&dolo, outb));
  BERN_HIP_TRY(d.alloc(&dohi, outb));
  BERN_HIP_TRY(d.alloc(&dstat, (size_t)max_boxes));
  BERN_HIP_TRY(d.alloc(&dpos, (size_t)max_boxes * sizeof(int64_t)));
  BERN_HIP_TRY(d.alloc(&dout, 8 * sizeof(double)));
  // a round in one wave if the largest one fits, else the smallest usable workspace
  if (d.alloc(&ws, ws_bytes) != hipSuccess) {
    (void)hipGetLastError();
    BERN_HIP_TRY(d.alloc(&ws, ws_one));
    ws_bytes = ws_one;
  }
  BERN_HIP_TRY(hipMemcpy(blo[0], lo.data(), (size_t)n_boxes * n * sizeof(double), hipMemcpyHostToDevice));
  BERN_HIP_TRY(hipMemcpy(bhi[0], hi.data(), (size_t)n_boxes * n * sizeof(double), hipMemcpyHostToDevice));
  std::vector<double> hlo, hhi, holo, hohi;
  std::vector<int8_t> hst;
  int cur = 0;
  int64_t nb = n_boxes;
  for (int round = 0; round < max_rounds && nb > 0; ++round) {
    if ((st = bern_bounds(net, opts, nb, (const double *)blo[cur], (const double *)bhi[cur], nullptr, nullptr,
                          nullptr, (double *)dolo, (double *)dohi, nullptr, ws, ws_bytes, nullptr, nullptr)) != BERN_OK)
      return st;
    res->rounds = round + 1;
    res->boxes_bounded += nb;
    {
      ProfScope ps(kProfMisc, nullptr, 0.0);
      hipLaunchKernelGGL(bb_round_kernel, dim3(1), dim3(1024), 0, nullptr, n, o, nb, (const double *)blo[cur],
                         (const double *)bhi[cur], (const double *)dolo, (const double *)dohi, out_index, threshold,
                         total, max_boxes, round + 1 < max_rounds ? 1 : 0, (double *)blo[cur ^ 1],
                         (double *)bhi[cur ^ 1], (int8_t *)dstat, (int64_t *)dpos, (double *)dout);
    }
    BERN_HIP_TRY(hipGetLastError());
    double hout[8];
    BERN_HIP_TRY(hipMemcpy(hout, dout, sizeof(hout), hipMemcpyDeviceToHost));  // waits for the round
    const int64_t open = (int64_t)hout[0];
    const bool split = hout[1] != 0.0;
    res->verified += hout[2];
    res->violated += hout[3];
    if (!split) {
      res->undecided += hout[4];
      res->undecided_boxes += open;
    }
    if (logging && res->log_count < log_cap) {
      hlo.resize((size_t)nb * n);
      hhi.resize((size_t)nb * n);
      holo.resize((size_t)nb * o);
      hohi.resize((size_t)nb * o);
      hst.resize((size_t)nb);
      BERN_HIP_TRY(hipMemcpy(hlo.data(), blo[cur], (size_t)nb * n * sizeof(double), hipMemcpyDeviceToHost));
      BERN_HIP_TRY(hipMemcpy(hhi.data(), bhi[cur], (size_t)nb * n * sizeof(double), hipMemcpyDeviceToHost));
      BERN_HIP_TRY(hipMemcpy(holo.data(), dolo, (size_t)nb * o * sizeof(double), hipMemcpyDeviceToHost));
      BERN_HIP_TRY(hipMemcpy(hohi.data(), dohi, (size_t)nb * o * sizeof(double), hipMemcpyDeviceToHost));
      BERN_HIP_TRY(hipMemcpy(hst.data(), dstat, (size_t)nb, hipMemcpyDeviceToHost));
      for (int pass = 0; pass < 2; ++pass)  // the decided boxes, then the open ones left unsplit
        for (int64_t b = 0; b < nb; ++b) {
          const bool take = pass == 0 ? hst[b] != 0 : (hst[b] == 0 && !split);
          if (take)
            log_box(&hlo[b * n], &hhi[b * n], holo[b * o + out_index], hohi[b * o + out_index], hst[b]);
        }
    }
    nb = split ? 2 * open : 0;
    cur ^= 1;
  }
  return BERN_OK;
}

// --------------------------------------------------------------- autotuner
static void tune_to(const Tune &t, int32_t *v) {
  v[0] = t.gemm_wide;
  v[1] = t.gemm_narrow;
  v[2] = t.conv_block;
  v[3] = t.conv_wave;
}
static void tune_from(const int32_t *v, Tune &t) {
  t.gemm_wide = v[0];
  t.gemm_narrow = v[1];
  t.conv_block = v[2];
  t.conv_wave = v[3];
}

extern "C" int32_t bern_tune_params(void) { return kTuneParams; }

extern "C" int32_t bern_tune_variants(int32_t param) {
  return (param >= 0 && param < kTuneParams) ? kTuneVariants[param] : 0;
}

extern "C" bern_status bern_tune_get(const bern_net *net, int32_t *choice) {
  if (!net || !choice) { set_error("null argument"); return BERN_E_ARG; }
  tune_to(net->tune, choice);
  return BERN_OK;
}

extern "C" bern_status bern_tune_set(bern_net *net, const int32_t *choice) {
  if (!net || !choice) { set_error("null argument"); return BERN_E_ARG; }
  for (int q = 0; q < kTuneParams; ++q)
    if (choice[q] < 0 || choice[q] >= kTuneVariants[q]) {
      set_error("tuning parameter %d: variant %d outside 0..%d", q, choice[q], kTuneVariants[q] - 1);
      return BERN_E_ARG;
    }
  tune_from(choice, net->tune);
  return BERN_OK;
}

// Coordinate search over the kernel variants: for each parameter in turn,
// time `reps` full runs of bern_bounds under every variant (the others at
// their current choice) with events on `stream`, keep the fastest. The
// arguments are those of bern_bounds; the outputs hold the last run's
// results. Synchronises `stream`.
extern "C" bern_status bern_autotune(bern_net *net, const bern_opts *opts, int64_t n_boxes, const double *box_lo,
                                     const double *box_hi, const int8_t *plan, double *neuron_lo, double *neuron_hi,
                                     double *out_lo, double *out_hi, int8_t *used_plan, void *workspace,
                                     size_t ws_bytes, void *stream, int32_t reps, int32_t *choice, float *best_ms) {
  if (!net || !opts || reps < 1) { set_error("bad arguments"); return BERN_E_ARG; }
  bern_opts o = *opts;
  o.graph = 0;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  BERN_HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("event creation failed");
    return BERN_E_DEVICE;
  }
  auto timed = [&](float &ms) -> bern_status {
    bern_status st = bern_bounds(net, &o, n_boxes, box_lo, box_hi, plan, neuron_lo, neuron_hi, out_lo, out_hi,
                                 used_plan, workspace, ws_bytes, stream, nullptr);  // warm-up
    if (st != BERN_OK) return st;
    BERN_HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) {
      st = bern_bounds(net, &o, n_boxes, box_lo, box_hi, plan, neuron_lo, neuron_hi, out_lo, out_hi, used_plan,
                       workspace, ws_bytes, stream, nullptr);
      if (st != BERN_OK) return st;
    }
    BERN_HIP_TRY(hipEventRecord(e1, s));
    BERN_HIP_TRY(hipEventSynchronize(e1));
    BERN_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    ms /= (float)reps;
    return BERN_OK;
  };
  int32_t cur[kTuneParams];
  tune_to(net->tune, cur);
  float best = 0.0f;
  bern_status st = timed(best);
  for (int q = 0; q < kTuneParams && st == BERN_OK; ++q) {
    const int keep = cur[q];
    int pick = keep;
    for (int v = 0; v < kTuneVariants[q] && st == BERN_OK; ++v) {
      if (v == keep) continue;
      cur[q] = v;
      tune_from(cur, net->tune);
      float ms = 0.0f;
      st = timed(ms);
      if (st == BERN_OK && ms < best) {
        best = ms;
        pick = v;
      }
    }
    cur[q] = pick;
    tune_from(cur, net->tune);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != BERN_OK) return st;
  if (choice) tune_to(net->tune, choice);
  if (best_ms) *best_ms = best;
  return BERN_OK;
}

// ---------------------------------------------------------------- profiler
extern "C" bern_status bern_prof_enable(int32_t on) {
  if (on) pool_fill(8192);
  g_prof_on = on != 0;
  return BERN_OK;
}

extern "C" bern_status bern_prof_reset(void) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (auto &r : g_prof) {
    (void)hipEventSynchronize(r.b);
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_prof.clear();
  return BERN_OK;
}

extern "C" int32_t bern_prof_classes(void) { return kProfCount; }

extern "C" const char *bern_prof_name(int32_t cls) {
  return (cls >= 0 && cls < kProfCount) ? kProfNames[cls] : "";
}

extern "C" bern_status bern_prof_read(int32_t cls, int64_t *launches, double *ms, double *bytes, double *flops) {
  if (cls < 0 || cls >= kProfCount || !launches || !ms || !bytes) {
    set_error("bad arguments");
    return BERN_E_ARG;
  }
  std::lock_guard<std::mutex> g(g_prof_mu);
  int64_t n = 0;
  double t = 0.0, by = 0.0, fl = 0.0;
  for (auto &r : g_prof) {
    if (r.cls != cls) continue;
    BERN_HIP_TRY(hipEventSynchronize(r.b));
    float e = 0.f;
    BERN_HIP_TRY(hipEventElapsedTime(&e, r.a, r.b));
    ++n;
    t += e;
    by += r.bytes;
    fl += r.flops;
  }
  *launches = n;
  *ms = t;
  *bytes = by;
  if (flops) *flops = fl;
  return BERN_OK;
}

// ---------------------------------------------------- step-level entry points
extern "C" size_t bern_basis_minmax_scratch(int32_t n, int32_t D, int64_t count) {
  return basis_minmax_scratch(n, D, count);
}

extern "C" bern_status bern_basis_minmax(int32_t n, int32_t D, int64_t count, const void *coef, int32_t fp64,
                                         double *bern_out, double *mn, double *mx, double *l1, void *scratch,
                                         size_t scratch_bytes, void *stream) {
  if (n < 1 || n > kMaxInputs || D < 0 || D > 64 || count < 1 || count > 65535 || !coef || !mn || !mx) {
    set_error("bad arguments");
    return BERN_E_ARG;
  }
  (void)scratch_bytes;
  hipError_t e = launch_basis_minmax(n, D, count, coef, fp64, bern_out, mn, mx, l1, (double *)scratch,
                                     reinterpret_cast<hipStream_t>(stream));
  if (e == hipErrorInvalidValue) {
    set_error("tensor of (%d+1)^%d coefficients exceeds the one-block limit", D, n);
    return BERN_E_TOO_LARGE;
  }
  BERN_HIP_TRY(e);
  return BERN_OK;
}

extern "C" bern_status bern_poly_mul(int32_t n, int32_t da, int32_t db, int64_t count, const void *A,
                                     const void *B, void *out, int32_t fp64, void *stream) {
  if (n < 1 || n > kMaxInputs || da < 0 || db < 0 || da > 64 || db > 64 || count < 1 || count > 65535 || !A || !B ||
      !out) {
    set_error("bad arguments");
    return BERN_E_ARG;
  }
  BERN_HIP_TRY(launch_poly_mul(n, da, db, count, A, B, out, fp64, reinterpret_cast<hipStream_t>(stream)));
  return BERN_OK;
}

extern "C" bern_status bern_relu_poly(int64_t count, int32_t L, const double *lo, const double *hi, double *c,
                                      double *e, void *stream) {
  if (count < 1 || L < 1 || L > kMaxOrder || !lo || !hi || !c || !e) {
    set_error("bad arguments");
    return BERN_E_ARG;
  }
  BERN_HIP_TRY(launch_relu_poly(count, L, lo, hi, c, e, reinterpret_cast<hipStream_t>(stream)));
  return BERN_OK;
}

// ------------------------------------------------------ degree predictor
extern "C" int32_t bern_pred_params(void) { return mlp_params(); }

extern "C" bern_status bern_pred_create(const float *params, int64_t n_params, bern_pred **out) {
  if (!out || !params || n_params != mlp_params()) {
    set_error("bern_pred_create needs %d parameters", mlp_params());
    return BERN_E_ARG;
  }
  *out = nullptr;
  for (int64_t i = 0; i < n_params; ++i)
    if (!std::isfinite(params[i])) {
      set_error("non-finite predictor parameter at %lld", (long long)i);
      return BERN_E_NUMERIC;
    }
  for (int f = 0; f < 8; ++f)
    if (!(params[8 + f] > 0.f)) {
      set_error("feature scale %d must be positive", f);
      return BERN_E_NUMERIC;
    }
  bern_pred *p = new (std::nothrow) bern_pred();
  if (!p) { set_error("out of host memory"); return BERN_E_OOM; }
  hipError_t e = hipMalloc(&p->params, n_params * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(p->params, params, n_params * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    set_error("predictor upload failed: %s", hipGetErrorString(e));
    (void)hipFree(p->params);
    delete p;
    return BERN_E_DEVICE;
  }
  *out = p;
  return BERN_OK;
}

extern "C" void bern_pred_destroy(bern_pred *p) {
  if (!p) return;
  (void)hipFree(p->params);
  delete p;
}

extern "C" size_t bern_mlp_backward_scratch(int64_t N) { return mlp_backward_scratch(N); }

extern "C" bern_status bern_mlp_forward(const float *P, int64_t N, const float *X, float *logits, int32_t bf16,
                                        void *stream) {
  if (!P || N < 1 || !X || !logits) { set_error("bad arguments"); return BERN_E_ARG; }
  BERN_HIP_TRY(launch_mlp_forward(P, N, X, logits, nullptr, bf16, reinterpret_cast<hipStream_t>(stream)));
  return BERN_OK;
}

extern "C" bern_status bern_mlp_backward(const float *P, int64_t N, const float *X, const int8_t *y, float *G,
                                         float *loss, void *scratch, void *stream) {
  if (!P || N < 1 || !X || !y || !G || !scratch) { set_error("bad arguments"); return BERN_E_ARG; }
  BERN_HIP_TRY(launch_mlp_backward(P, N, X, y, G, loss, (float *)scratch, reinterpret_cast<hipStream_t>(stream)));
  return BERN_OK;
}

extern "C" bern_status bern_mlp_adam(float *P, const float *G, float *m, float *v, int64_t step, float lr,
                                     float beta1, float beta2, float eps, void *stream) {
  if (!P || !G || !m || !v || step < 1) { set_error("bad arguments"); return BERN_E_ARG; }
  BERN_HIP_TRY(launch_mlp_adam(P, G, m, v, step, lr, beta1, beta2, eps, reinterpret_cast<hipStream_t>(stream)));
  return BERN_OK;
}

extern "C" bern_status bern_mlp_classify(const float *P, int64_t N, const float *X, float *logits, int8_t *cls,
                                         int32_t bf16, void *stream) {
  if (!P || N < 1 || !X || !logits || !cls) { set_error("bad arguments"); return BERN_E_ARG; }
  BERN_HIP_TRY(launch_mlp_classify(P, N, X, logits, cls, bf16, reinterpret_cast<hipStream_t>(stream)));
  return BERN_OK;
}
