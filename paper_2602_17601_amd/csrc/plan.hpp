// Internal definition of gnmpc_plan and the launchers of each kernel file.
#pragma once

#include <string>
#include <vector>

#include "common.hpp"

struct GnnState;   // defined in gnn_state.hpp
struct InetState;  // defined in inet.hip

struct gnmpc_plan {
  int device = 0;
  gnmpc_dims dims{};
  std::string last_error;
  int elem = 4;  // bytes per element of the plan dtype

  // graph and Jacobian pattern
  bool graph_ready = false;
  int M = 0, E = 0, L = 0;
  long nnz = 0;
  int wmax = 0;  // longest pattern row
  std::vector<int32_t> h_row_ptr, h_col, h_prow, h_pcol;
  int32_t *d_row_ptr = nullptr, *d_col = nullptr;
  int32_t *d_prow = nullptr, *d_pcol = nullptr, *d_erow = nullptr, *d_diag = nullptr;
  int32_t *d_cptr = nullptr, *d_cent = nullptr;  // the pattern by column: entries of column node j
  // propagation blocks: pb_nodes consecutive nodes per block; one record of
  // pb_rec_stride words per block (first pattern entry, entry count, union
  // size, node count, row starts, the union of the nodes' pattern columns and,
  // per pattern entry, the position of its column in that union)
  int pb_nodes = 0, pb_count = 0, pb_umax = 0, pb_emax = 0, pb_rec_stride = 0;
  int32_t* d_pb_rec = nullptr;
  // two-stage records of the same blocks (0 = not used): the block's union U1, the
  // union U2 of U1's pattern rows, U1's entries with their positions in U2
  int pb2_stride = 0, pb2_u1max = 0, pb2_u2max = 0, pb2_e1max = 0;
  int32_t* d_pb2_rec = nullptr;
  // propagation variant: -1 the default choice, 0 per-node kernel, 1 one-stage
  // blocks, 2 two-stage blocks where they fit (set by gnmpc_autotune_condense)
  int prop_pref = -1;

  // model
  int model = 0;  // 0 none, 1 mass-spring-damper, 2 GNN, 3 interaction network
  gnmpc_msd_params msd{};
  int n_act = 0;
  std::vector<int32_t> h_act;
  int32_t* d_act_of_node = nullptr;  // [M]: actuator index of the node or -1
  GnnState* gnn = nullptr;
  InetState* inet = nullptr;

  // single-node state rows
  int n_c = 0;
  int32_t *d_row_node = nullptr, *d_row_stage = nullptr;

  // condensing workspace
  void* d_S = nullptr;     // S_k for k = 1..N, stage k stored as [M][6][k nu]
  size_t S_elems = 0;
  void* d_Gx = nullptr;    // [N+1][M][6]
  void* d_part = nullptr;  // split-K partial sums of the Gram kernel
  size_t part_elems = 0;

  // QP workspace
  void* d_qp = nullptr;
  size_t qp_bytes = 0;
  int32_t* d_qp_flag = nullptr;
  void* d_qpdesc = nullptr;  // the QP's solve descriptor, for batched solves (kQpDescBytes)

  // per-block partial counts of the finiteness check of gnmpc_linearize
  void* d_check = nullptr;

  // per-phase timers
  bool timers_on = false;
  std::vector<hipEvent_t> ev_start[GNMPC_PH_COUNT], ev_stop[GNMPC_PH_COUNT];
  int ev_used[GNMPC_PH_COUNT] = {0};
  int ev_open[GNMPC_PH_COUNT] = {0};
};

namespace gnmpc {

constexpr int kTimerRecords = 1024;

// Raise a kernel's dynamic-LDS limit once per (kernel, size): the attribute
// call is slow, so it is not repeated on every launch.
inline hipError_t set_max_lds(const void* fn, hipFuncAttribute attr, int bytes) {
  struct Entry { const void* fn; int bytes; };
  static Entry cache[64];
  static int used = 0;
  for (int t = 0; t < used; ++t)
    if (cache[t].fn == fn && cache[t].bytes >= bytes) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, attr, bytes);
  if (e == hipSuccess) {
    for (int t = 0; t < used; ++t)
      if (cache[t].fn == fn) {
        cache[t].bytes = bytes;
        return e;
      }
    if (used < 64) cache[used++] = Entry{fn, bytes};
  }
  return e;
}

// Record the start / end of a phase on stream s when timers are enabled.
inline void phase_begin(gnmpc_plan* p, int ph, hipStream_t s) {
  if (!p->timers_on || p->ev_used[ph] >= kTimerRecords) return;
  (void)hipEventRecord(p->ev_start[ph][p->ev_used[ph]], s);
  p->ev_open[ph] = 1;
}
inline void phase_end(gnmpc_plan* p, int ph, hipStream_t s) {
  if (!p->timers_on || !p->ev_open[ph]) return;
  (void)hipEventRecord(p->ev_stop[ph][p->ev_used[ph]], s);
  p->ev_open[ph] = 0;
  ++p->ev_used[ph];
}

__host__ __device__ inline size_t S_offset(int k, int M, int nu) {  // element offset of S_k (k >= 1)
  return (size_t)NBX * M * nu * ((size_t)k * (k - 1) / 2);
}

// msd_linearize.hip
gnmpc_status launch_msd_linearize(gnmpc_plan* p, const void* xhat, const void* uhat, void* A, void* B,
                                  void* c, void* fnext, hipStream_t s);
// condense.hip
size_t condense_partial_elems(int M, int nu, int N);
gnmpc_status launch_condense(gnmpc_plan* p, const void* A, const void* B, const void* c, const void* x0,
                             const void* Q, int Q_full, const void* q, const void* R, const void* r,
                             const void* rowC, const void* rowd, void* H, void* g, void* Ct, void* dt,
                             void* Gx, hipStream_t s);
// qp_admm.hip
size_t qp_workspace_bytes(int n, int n_c);
gnmpc_status prop_blocks_build(gnmpc_plan* p);
gnmpc_status prop_blocks_build_nb(gnmpc_plan* p, int nb_max);
void prop_blocks_free(gnmpc_plan* p);
gnmpc_status launch_qp(gnmpc_plan* p, int n, const void* H, const void* g, const void* lb, const void* ub,
                       int n_c, const void* Ct, const void* lc, const void* uc,
                       const gnmpc_admm_settings* st, void* u, gnmpc_qp_info* info, hipStream_t s);
// A QP whose set-up kernel has been enqueued (launch_qp_prep): that kernel also
// stored its solve descriptor at desc (the plan's d_qpdesc); launch_qp_batched
// solves many such QPs in one launch per pass.
constexpr size_t kQpDescBytes = 256;
struct QpPrepared {
  int dtype, n, n_c;
  void* desc;
};
gnmpc_status launch_qp_prep(gnmpc_plan* p, int n, const void* H, const void* g, const void* lb, const void* ub,
                            int n_c, const void* Ct, const void* lc, const void* uc, const gnmpc_admm_settings* st,
                            void* u, gnmpc_qp_info* info, hipStream_t s, QpPrepared* out);
gnmpc_status launch_qp_batched(const QpPrepared* q, int count, hipStream_t s);
// Interior-point solve of the same QP (one workgroup, FP64).
gnmpc_status qp_ipm_check(int n, int n_c);
gnmpc_status launch_qp_ipm(gnmpc_plan* p, int n, const void* H, const void* g, const void* lb, const void* ub,
                           int n_c, const void* Ct, const void* lc, const void* uc, double tol, int max_iter, void* u,
                           gnmpc_qp_info* info, hipStream_t s);
// Allocation-free QP (workspace in a static device array; see qp_admm.hip).
constexpr int kQpNoallocMaxN = 464;
gnmpc_status qp_noalloc_check(int dtype, int n, int n_c);
gnmpc_status launch_qp_noalloc(int dtype, int n, const void* H, const void* g, const void* lb, const void* ub,
                               int n_c, const void* Ct, const void* lc, const void* uc,
                               const gnmpc_admm_settings* st, void* u, gnmpc_qp_info* info, hipStream_t s);
// tangent.hip
gnmpc_status launch_jvp(gnmpc_plan* p, const void* A, const void* B, const void* dx, const void* du, void* out,
                        hipStream_t s);
gnmpc_status launch_vjp(gnmpc_plan* p, const void* A, const void* B, const void* g, void* gx, void* gu,
                        hipStream_t s);
gnmpc_status launch_rollout(gnmpc_plan* p, const void* A, const void* B, const void* c, const void* x0,
                            const void* u, void* x, hipStream_t s);
gnmpc_status launch_rti_shift(gnmpc_plan* p, const void* xpred, const void* u, void* xhat, void* uhat,
                              hipStream_t s);
// check.hip
size_t lin_check_bytes();
gnmpc_status launch_lin_check(gnmpc_plan* p, const void* xhat, const void* uhat, const void* A, const void* B,
                              const void* c, const void* fnext, gnmpc_lin_info* info, hipStream_t s);
// gnn.hip
gnmpc_status gnn_set(gnmpc_plan* p, const gnmpc_gnn_desc* desc, const double* w, int64_t n_w);
void gnn_free(gnmpc_plan* p);
// inet.hip
gnmpc_status inet_set(gnmpc_plan* p, const gnmpc_inet_desc* d, const double* w, int64_t n_w);
void inet_free(gnmpc_plan* p);
gnmpc_status launch_inet_linearize(gnmpc_plan* p, const void* xhat, const void* uhat, void* A, void* B, void* c,
                                   void* fnext, hipStream_t s);
// train.hip
size_t gnn_train_workspace_bytes(const gnmpc_plan* p);
long gnn_param_count(const gnmpc_plan* p);
gnmpc_status launch_gnn_loss_grad(gnmpc_plan* p, const float* theta, const void* x, const void* u, const void* xn,
                                  const float* O, double lambda, void* ws, float* loss, float* grad, hipStream_t s);
gnmpc_status launch_adam(long n, float* theta, const float* grad, float* m, float* v, int step, double lr,
                         double beta1, double beta2, double eps, hipStream_t s);
// msd_sim.hip
bool msd_sim_fits(const gnmpc_plan* p);
gnmpc_status launch_msd_simulate(gnmpc_plan* p, int B, int T, const void* x0, const void* u, void* X, hipStream_t s);
gnmpc_status launch_gnn_forward_only(gnmpc_plan* p, const void* xhat, const void* uhat, void* fnext, hipStream_t s);
gnmpc_status launch_gnn_vjp(gnmpc_plan* p, const void* xhat, const void* uhat, const void* g, void* gx, void* gu,
                            hipStream_t s);
gnmpc_status launch_gnn_linearize(gnmpc_plan* p, const void* xhat, const void* uhat, void* A, void* B,
                                  void* c, void* fnext, hipStream_t s);

}  // namespace gnmpc
