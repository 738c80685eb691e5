// Adjoint of the fused step (placeholder state; kernels follow).
#pragma once
#include "scl_common.hpp"

namespace scl {

struct AdjointState {
  void* pool = nullptr;      // checkpoints
  size_t pool_bytes = 0;
};

inline void adjoint_free(AdjointState& a) {
  if (a.pool) (void)hipFree(a.pool);
  a.pool = nullptr;
  a.pool_bytes = 0;
}

}  // namespace scl
