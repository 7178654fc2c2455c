// Relative volume of the output set (Section 6, evaluation metrics).
#pragma once
#include "common.hpp"

namespace bern {

// vol[box][j] = mean over the input box of the upper minus the lower output
// polynomial of output j: the stored total-degree power coefficients of the
// output layer (a.pre, a.slot, a.S, a.bids, a.nboxes, a.h, a.fp64), each
// weighted by the mean of its monomial over [0,1]^n; a.didx maps a rank to
// its dense index at the stored per-variable degree D. In FP32 mode a.eps
// (the tensors' radii) is added, so the volume is that of the padded pair.
hipError_t launch_rel_volume(const OutPolyArgs &a, int n, int D, double *vol, hipStream_t s);

}  // namespace bern
