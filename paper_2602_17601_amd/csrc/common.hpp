// Internal helpers shared by the HIP translation units of libgnmpc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "gnmpc.h"

namespace gnmpc {

constexpr int NBX = 6;          // states per node
constexpr int kMaxWidth = 64;   // max blocks in one Jacobian pattern row
constexpr int kInetMaxLayers = 16;   // linear layers of each interaction-network MLP
constexpr int kInetMaxWidth = 256;   // widest hidden layer / message
constexpr int kInetMaxNu = 64;       // global inputs of the interaction network

#define GNMPC_HIP_TRY(plan, expr)                                                   \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess) {                                                         \
      (plan)->last_error = std::string(#expr) + ": " + hipGetErrorString(_e);       \
      return GNMPC_HIP_ERROR;                                                       \
    }                                                                               \
  } while (0)

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace gnmpc
