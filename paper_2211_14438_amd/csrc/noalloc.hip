// bern_bounds_noalloc: bern_bounds for callers that cannot allocate device
// memory. Its scratch is a file-scope device array of kNoAllocScratch bytes,
// one copy per GPU the library runs on (held until the process ends). Host
// code never passes the array's name to a kernel: its device address is
// looked up once per device with hipGetSymbolAddress and kept here.
#include <mutex>

#include "common.hpp"

namespace bern {

constexpr size_t kNoAllocScratch = BERN_NOALLOC_SCRATCH_BYTES;  // per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// The current device's copy of the scratch array (looked up on the first
// call on that device, with it current).
static bern_status scratch_for_current_device(void **out) {
  int dev = 0;
  BERN_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d outside the 0..%d the library tracks", dev, kMaxDevices - 1);
    return BERN_E_DEVICE;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error("hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
      return BERN_E_DEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BERN_OK;
}

}  // namespace bern

extern "C" bern_status bern_bounds_noalloc(const bern_net *net, const bern_opts *opts, int64_t n_boxes,
                                           const double *box_lo, const double *box_hi, double *neuron_lo,
                                           double *neuron_hi, double *out_lo, double *out_hi, int8_t *used_plan,
                                           void *stream, bern_stats *stats) {
  if (!net || !opts) {
    bern::set_error("null net or options");
    return BERN_E_ARG;
  }
  void *ptr = nullptr;
  const bern_status st = bern::scratch_for_current_device(&ptr);
  if (st != BERN_OK) return st;
  return bern::bounds_on_scratch(net, opts, n_boxes, box_lo, box_hi, neuron_lo, neuron_hi, out_lo, out_hi, used_plan,
                                 ptr, bern::kNoAllocScratch, stream, stats);
}
