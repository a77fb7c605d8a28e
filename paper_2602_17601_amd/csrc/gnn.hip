// GNN forward and Jacobian kernels (placeholder until the GNN path lands).
#include "plan.hpp"

namespace gnmpc {

gnmpc_status gnn_set(gnmpc_plan* p, const gnmpc_gnn_desc*, const double*, int64_t) {
  p->last_error = "GNN model not built into this library";
  return GNMPC_UNSUPPORTED;
}
void gnn_free(gnmpc_plan*) {}
gnmpc_status launch_gnn_linearize(gnmpc_plan* p, const void*, const void*, void*, void*, void*, void*, hipStream_t) {
  p->last_error = "GNN model not built into this library";
  return GNMPC_UNSUPPORTED;
}

}  // namespace gnmpc
