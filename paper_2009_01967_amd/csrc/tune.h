// Tile-shape autotuning for the GEMM-shaped kernels.
#pragma once

#include <functional>
#include <string>

#include "internal.h"

namespace kaldo {

// Returns the index of the fastest of `nv` launch variants for a problem
// `key`.  The first time a key is seen each variant is launched once untimed
// (which also loads its code object) and once between events on the context
// stream; the winner is cached in the context.  With tuning disabled the
// variant `fallback` is returned without timing.  Every variant must write the
// same outputs, so the caller runs the chosen one after this returns.
int autotune(kaldo_ctx ctx, const std::string& key, int nv, int fallback, const std::function<void(int)>& launch);

}  // namespace kaldo
