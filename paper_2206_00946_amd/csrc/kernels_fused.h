// Fused single-pass step (placeholder until the fast path lands).
#pragma once

#include "lbm3d.h"
#include "kernels_ref.h"

namespace lbm {

inline bool fused_supported(const lbm_params&) { return false; }

template <typename S>
struct FusedImpl {
  static hipError_t step(const lbm_params&, hipStream_t, const S*, const S*, S*, S*, const double*, bool,
                         const double*, bool, int*) {
    return hipErrorNotSupported;
  }
};

}  // namespace lbm
