/*
 * gnmpc -- graph-neural MPC hot path on AMD Instinct MI355X (gfx950).
 *
 * C-ABI of the HIP library libgnmpc.so.  Plain pointers and sizes only.
 *
 * The library implements, for one MPC step of Algorithm 1 of
 * "Graph Neural Model Predictive Control for High-Dimensional Systems":
 *   - linearization of the node dynamics into block-sparse Jacobians
 *     A^{ij}_k, B^i_k and offsets c^i_k (Sec. V-A, eq. linearized_dynamics),
 *     either of the message-passing GNN model (Sec. V-A eq. forward_dynamics)
 *     or of an analytic mass-spring-damper chain;
 *   - graph-sparse condensing (Sec. V-B, Thm. 1 proof, eqs. sparse_gamma_i_xb,
 *     sparse_gamma_i_u, H, g and the stacked constraint rows);
 *   - the condensed QP (Sec. III-B eq. condensed_matrices) with box input
 *     bounds, solved by ADMM.
 *
 * Conventions (shared by every entry point)
 *   Layouts are row-major and C-contiguous.  A node state is x^i = [p^i; v^i]
 *   (6 values); stacked states are stage-major then node-major.
 *   Cost convention: stage cost 1/2 x'Qx + q'x + 1/2 u'Ru + r'u and QP
 *   objective 1/2 u'Hu + g'u (the paper's H and g formulas hold exactly in
 *   this convention).
 *   "device" pointers are HIP device allocations on the plan's device, owned
 *   by the caller; "host" pointers are ordinary memory, read during the call
 *   only.  `stream` is a hipStream_t (NULL = the default stream).  Calls that
 *   take a stream enqueue work and return without synchronizing; results are
 *   valid once the stream has been synchronized.
 *   Every call returns a gnmpc_status.  Arguments are validated on the host
 *   before any GPU work is enqueued; on an error nothing is enqueued and
 *   gnmpc_plan_last_error() describes the problem.  Errors found on the GPU
 *   (non-finite data, QP status) are reported in device-side info structs.
 *   A plan is not thread-safe; distinct plans are independent.
 */
#ifndef GNMPC_H
#define GNMPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GNMPC_OK = 0,
  GNMPC_INVALID_ARG = 1,     /* null pointer, non-positive size, bad enum      */
  GNMPC_BAD_GRAPH = 2,       /* malformed CSR: unsorted, duplicate, self loop, out of range */
  GNMPC_SHAPE = 3,           /* size disagrees with the plan                     */
  GNMPC_UNSUPPORTED = 4,     /* valid request outside what the library supports */
  GNMPC_HIP_ERROR = 5,       /* a HIP runtime call failed                       */
  GNMPC_BAD_CONSTRAINT = 6,  /* state row on stage 0 or outside 1..N, bad node  */
  GNMPC_NOT_READY = 7,       /* graph / model / rows not set yet                */
  GNMPC_NO_DEVICE = 8        /* no usable GPU                                   */
} gnmpc_status;

typedef enum { GNMPC_F64 = 0, GNMPC_F32 = 1, GNMPC_BF16 = 2 } gnmpc_dtype;

/* QP status written to gnmpc_qp_info.status on the device. */
typedef enum {
  GNMPC_QP_SOLVED = 0,
  GNMPC_QP_MAXITER = 1,      /* soft: the last iterate is returned              */
  GNMPC_QP_PRIMAL_INFEASIBLE = 2,
  GNMPC_QP_NONFINITE = 3,
  GNMPC_QP_NOT_PD = 4
} gnmpc_qp_status;

typedef struct gnmpc_plan gnmpc_plan;

/* Problem dimensions fixed at plan creation. */
typedef struct {
  int32_t M;        /* nodes |V|                                                */
  int32_t nu;       /* inputs n_u                                               */
  int32_t N;        /* horizon                                                  */
  int32_t n_c_max;  /* maximum number of single-node state rows                  */
  int32_t dtype;    /* GNMPC_F64 or GNMPC_F32: arithmetic of linearize outputs,  */
                    /* condensing and the QP (GNN MLPs may run in BF16, below)  */
} gnmpc_dims;

/* Mass-spring-damper chain (the plain, analytic-Jacobian form).  Springs and
 * dampers act along every graph edge; node `anchor` (or none if -1) is tied to
 * the ground by the same spring and damper.  F(d) = k d + k3 |d|^2 d;
 * a^i = (sum_j F(p^j-p^i) + c (v^j-v^i) + anchor terms + f^i) / m - gravity e_z;
 * v+ = v + dt a, p+ = p + dt v+. */
typedef struct {
  double k, c, m, dt, k3, gravity;
  int32_t anchor;
  int32_t reserved;
} gnmpc_msd_params;

/* Message-passing GNN of Sec. V-A (sum aggregation, ReLU, edge feature from
 * the relative state):
 *   h0_i = relu(W_enc [x^i; P^i u] + b_enc)
 *   m_ij = relu(W_e[l] [h_i; h_i - h_j] + b_e[l]),  j in N_i
 *   h_i <- relu(W_n[l] [h_i; sum_j m_ij] + b_n[l]),  l = 0..L-1
 *   o_i  = W_dec h_i + b_dec;  v+ = v + dt o_i[3:6];  p+ = p + dt v+
 * Weights are passed packed, float64, (out, in) row-major, in the order
 * W_enc[Hd][9], b_enc[Hd], then per layer W_e[Hd][2Hd], b_e[Hd], W_n[Hd][2Hd],
 * b_n[Hd], then W_dec[6][Hd], b_dec[6]. */
typedef struct {
  int32_t Hd;       /* hidden width: 64, 128, 192 or 256                          */
  int32_t L;        /* message-passing rounds (must equal the graph's L)          */
  int32_t dtype;    /* GNMPC_F32, or GNMPC_BF16: weights rounded to bfloat16; the  */
                    /* forward pass keeps activations at FP32 accuracy (so the   */
                    /* ReLU decisions are FP32's), the Jacobian's tangent        */
                    /* products take bfloat16 operands with FP32 accumulation    */
  int32_t reserved;
  double dt;
} gnmpc_gnn_desc;

/* The paper's own model (Sec. V-A eq. forward_dynamics): an interaction network
 * with a global input u shared by every node.  With e^{ij} = x^i - x^j,
 *   v^i+ = v^i + phi([x^i; sum_{j in N_i} psi(e^{ij}); u]),  p^i+ = p^i + dt v^i+,
 * psi: 6 -> psi_hidden layers of psi_width -> d_m, phi: 6 + d_m + nu ->
 * phi_hidden layers of phi_width -> 3, a ReLU after every layer but the last.
 * Weights are passed packed, float64, (out, in) row-major, layer by layer:
 * psi's (W, b) pairs, then phi's.  The paper's robot: psi 4 x 50, phi 8 x 250,
 * nu = 6.  Widths and d_m up to 256, at most 15 hidden layers each, nu <= 64. */
typedef struct {
  int32_t psi_hidden, psi_width, d_m;
  int32_t phi_hidden, phi_width, nu;
  double dt;
} gnmpc_inet_desc;

/* ADMM settings (operator splitting in the form of Stellato et al., OSQP). */
typedef struct {
  double rho;        /* penalty of the inequality rows (> 0)                     */
  double sigma;      /* primal regularization (> 0)                              */
  double alpha;      /* over-relaxation in (0, 2)                                */
  double eps_abs, eps_rel;
  double kappa_fp64; /* condition bound above which the factorization and the   */
                     /* iterations switch to FP64 (e.g. 1e7)                     */
  int32_t max_iter;
  int32_t check_every;
} gnmpc_admm_settings;

/* Device-side QP report. */
typedef struct {
  int32_t status;    /* gnmpc_qp_status                                          */
  int32_t iters;
  int32_t used_fp64; /* 1 if the condition estimate exceeded kappa_fp64          */
  int32_t reserved;
  /* kappa_est: the ADMM's estimate of the 1-norm condition number of K, either the
   * upper bound ||K||_1 ||W||_1 ||W||_inf (W = L^{-1}) when that is at most
   * kappa_fp64, or else Hager's estimate; the interior-point solver reports its
   * last duality measure here instead. */
  double prim_res, dual_res, kappa_est, obj;
} gnmpc_qp_info;

/* Finiteness report of gnmpc_linearize, written on the device (status values). */
typedef enum {
  GNMPC_LIN_FINITE = 0,            /* every input and output entry is finite               */
  GNMPC_LIN_NONFINITE_INPUT = 1,   /* xhat (stages 0..N-1) or uhat holds a NaN or infinity */
  GNMPC_LIN_NONFINITE_OUTPUT = 2   /* inputs finite, but A, B, c or fnext is not (e.g. an   */
                                   /* overflow in the model)                               */
} gnmpc_lin_status;

/* Device-side report of gnmpc_linearize.  Arrays are numbered 0 xhat, 1 uhat,
 * 2 A, 3 B, 4 c, 5 fnext; the "first" entry is the lowest element index of the
 * lowest-numbered array that holds a non-finite value. */
typedef struct {
  int32_t status;       /* gnmpc_lin_status                                          */
  int32_t first_array;  /* array of the first non-finite entry, -1 if none             */
  int32_t first_stage;  /* its stage k, -1 if none                                     */
  int32_t first_node;   /* its node (the row node i of an A block), -1 for uhat or none */
  int64_t nonfinite[6]; /* number of non-finite entries of each array                  */
} gnmpc_lin_info;

const char* gnmpc_version(void);
const char* gnmpc_status_string(int32_t status);

/* ---------------- host-only graph utilities (no GPU needed) ---------------- */

/* Check an incoming-edge CSR: row i lists the senders j of edges j -> i
 * (Sec. III-A: the edge e^{ij} runs from v_j to v_i and N_i is the set of
 * senders).  Rows must be strictly ascending, 0 <= j < M, j != i,
 * row_ptr[0] = 0, row_ptr[M] = E, non-decreasing.  Returns GNMPC_OK or
 * GNMPC_BAD_GRAPH / GNMPC_INVALID_ARG. */
gnmpc_status gnmpc_graph_check(const int32_t* row_ptr, const int32_t* col, int32_t M, int32_t E);

/* Block pattern of the L-round Jacobian (Sec. V-A eq. linearized_dynamics
 * with Assumption 1 applied L times): row i holds every node that reaches i
 * in at most L hops, i included, ascending.  Host arrays; pass col_out =
 * NULL to query the size in *nnz_out; otherwise col_out must hold `cap`
 * entries.  row_ptr_out has M+1 entries. */
gnmpc_status gnmpc_graph_closure(const int32_t* row_ptr, const int32_t* col, int32_t M, int32_t E,
                                 int32_t L, int32_t* row_ptr_out, int32_t* col_out, int64_t cap,
                                 int64_t* nnz_out);

/* ---------------- plans ---------------- */

/* Create a plan on `device`; all workspace for the given dimensions is
 * allocated here so that the per-step calls allocate nothing. */
gnmpc_status gnmpc_plan_create(gnmpc_plan** plan, const gnmpc_dims* dims, int32_t device);
void gnmpc_plan_destroy(gnmpc_plan* plan);
/* Text of the last error on this plan ("" if none).  Owned by the plan. */
const char* gnmpc_plan_last_error(const gnmpc_plan* plan);

/* Set the graph (host CSR of incoming edges, checked as gnmpc_graph_check)
 * and the number of message-passing rounds L that fixes the Jacobian pattern
 * (L = 1 for the mass-spring-damper model).  Builds and uploads the pattern. */
gnmpc_status gnmpc_graph_set(gnmpc_plan* plan, const int32_t* row_ptr, const int32_t* col,
                             int32_t M, int32_t E, int32_t L);
/* Number of Jacobian blocks nnz of the plan's pattern. */
gnmpc_status gnmpc_graph_nnz(const gnmpc_plan* plan, int64_t* nnz);
/* Copy the plan's pattern to host arrays (row_ptr_out[M+1], col_out[nnz]). */
gnmpc_status gnmpc_graph_pattern(const gnmpc_plan* plan, int32_t* row_ptr_out, int32_t* col_out);

/* Choose the mass-spring-damper model.  act[n_act] are the actuated nodes
 * (host, distinct, in [0, M)); u = [f_act[0]; f_act[1]; ...] so nu = 3 n_act. */
gnmpc_status gnmpc_model_set_msd(gnmpc_plan* plan, const gnmpc_msd_params* prm,
                                 const int32_t* act, int32_t n_act);

/* Choose the GNN model; weights are host float64 packed as described at
 * gnmpc_gnn_desc, n_weights their count.  The graph must have been set with
 * the same L. */
gnmpc_status gnmpc_model_set_gnn(gnmpc_plan* plan, const gnmpc_gnn_desc* desc,
                                 const double* weights, int64_t n_weights,
                                 const int32_t* act, int32_t n_act);

/* Choose the interaction-network model (gnmpc_inet_desc); weights host float64
 * packed as described there, n_weights their count.  The graph must have been
 * set with L = 1 and desc->nu must equal the plan's nu.  Linearization then
 * fills every pattern block (the node and its in-neighbours) and B^i for the
 * whole global input; condensing, the QP, the rollout and gnmpc_rti_step are
 * unchanged.  GNMPC_SHAPE for a wrong weight count or nu, GNMPC_UNSUPPORTED
 * when one workgroup's activations exceed LDS. */
gnmpc_status gnmpc_model_set_inet(gnmpc_plan* plan, const gnmpc_inet_desc* desc, const double* weights,
                                  int64_t n_weights);

/* Structure of the single-node state rows C x^{node}_{stage} <= d (Sec. IV-B:
 * half-spaces X^i_k; condensed as in the stacked-constraint formula of
 * Sec. V-B).  Host arrays of n_c entries; 1 <= stage <= N (stage-0 rows do not
 * depend on u and are rejected with GNMPC_BAD_CONSTRAINT).  n_c <= n_c_max. */
gnmpc_status gnmpc_rows_set(gnmpc_plan* plan, int32_t n_c, const int32_t* node, const int32_t* stage);

/* ---------------- the per-step hot path ---------------- */

/* Linearize the plan's model around (xhat, uhat) (Sec. V-A "Linearization";
 * Algorithm 1 "Linearize GNN dynamics").  Device arrays of the plan dtype:
 *   xhat [N+1][M][6] (stage N is unused), uhat [N][nu]
 *   A    [N][nnz][6][6]  A^{ij}_k = d f^i / d x^j at stage k, blocks in pattern order
 *   B    [N][M][6][nu]   B^i_k = d f^i / d u
 *   c    [N][M][6]       c^i_k = f^i - sum_j A^{ij}_k xhat^j_k - B^i_k uhat_k
 *   fnext[N][M][6]       f(xhat_k, uhat_k), may be NULL
 * ReLU uses the subgradient 0 at 0.  info (device, may be NULL): when given, two
 * further launches after the linearization count the non-finite entries of the
 * inputs and outputs and write a gnmpc_lin_info (a fixed-order reduction: no
 * clearing needed, and repeated calls give the same report). */
gnmpc_status gnmpc_linearize(gnmpc_plan* plan, const void* xhat, const void* uhat,
                             void* A, void* B, void* c, void* fnext, gnmpc_lin_info* info, void* stream);

/* Roll the linearized dynamics forward (Sec. III-B, the dynamics constraint of
 * the OCP; Algorithm 1 shifts its trajectory with it): x[0] = x0 and
 * x[k+1] = A_k x[k] + B_k u[k] + c_k for k < N, i.e. the stacked states
 * Gamma_u u + Gamma_x of the condensed form.  Device arrays of the plan dtype:
 * A, B, c as produced by gnmpc_linearize, x0 [M][6], u [N][nu], x [N+1][M][6]
 * (every entry written; x may not alias the inputs).  One launch per stage on
 * `stream`.  GNMPC_NOT_READY before gnmpc_graph_set; GNMPC_INVALID_ARG for a
 * NULL array. */
gnmpc_status gnmpc_rollout_linear(gnmpc_plan* plan, const void* A, const void* B, const void* c,
                                  const void* x0, const void* u, void* x, void* stream);

/* Trajectories of the plan's (nonlinear) mass-spring-damper model: for each of B
 * independent trajectories, X[b][0] = x0[b] and X[b][t+1] = f(X[b][t], u[b][t])
 * for t < T, f being the semi-implicit Euler step of Sec. V-A eq.
 * forward_dynamics with the node accelerations of gnmpc_msd_params (the data a
 * learned GNN surrogate is trained on).  Device arrays of the plan dtype:
 * x0 [B][M][6], u [B][T][nu], X [B][T+1][M][6] (caller-owned; X may not alias
 * the inputs).  GNMPC_NOT_READY unless the graph and a mass-spring-damper model
 * are set; GNMPC_SHAPE for negative B or T; GNMPC_UNSUPPORTED when two states
 * of the graph do not fit one workgroup's LDS (M up to 3413 in FP32, 1706 in
 * FP64). */
gnmpc_status gnmpc_msd_simulate(gnmpc_plan* plan, int32_t B, int32_t T, const void* x0, const void* u,
                                void* X, void* stream);

/* The GNN one-step model of Sec. V-A (eq. forward_dynamics; semi-implicit
 * Euler) at the N stages, without its Jacobians: fnext[k] = f(xhat[k], uhat[k]).
 * xhat [N+1][M][6] (stage N is not read), uhat [N][nu], fnext [N][M][6]: FP32
 * device arrays.  GNMPC_NOT_READY unless the graph and a GNN model are set.
 * Uses the plan's forward-pass workspace (as gnmpc_linearize does). */
gnmpc_status gnmpc_gnn_forward(gnmpc_plan* plan, const void* xhat, const void* uhat, void* fnext,
                               void* stream);

/* Reverse mode through the GNN's layers: the gradient of sum_k g[k] . f(x_k, u_k)
 * at (xhat[k], uhat[k]), i.e. gx[k] = (d f / d x_k)' g[k] and gu[k] = (d f / d u_k)' g[k]
 * (the transposed linearization of Sec. V-A, with ReLU's subgradient 0 at 0),
 * without forming the Jacobian blocks.  The forward pass is recomputed at the
 * given point for its ReLU masks, then the cotangents run back layer by layer.
 * FP32 device arrays: xhat [N+1][M][6], uhat [N][nu], g [N][M][6]; outputs gx
 * [N][M][6], gu [N][nu] (every entry written; outputs may not alias inputs).
 * GNMPC_NOT_READY unless the graph and a GNN model are set; GNMPC_INVALID_ARG
 * for a NULL array.  Uses the plan's forward-pass workspace. */
gnmpc_status gnmpc_gnn_vjp(gnmpc_plan* plan, const void* xhat, const void* uhat, const void* g, void* gx,
                           void* gu, void* stream);

/* Training of the GNN (Sec. V-A "Training"): the loss
 *   L = 1/S sum_t || x_next[t] - F_theta(x[t], u[t]) ||_O^2 + lambda ||theta||^2
 * over S = N samples (the plan's horizon is the batch; ||r||_O^2 = sum over the
 * nodes of r' diag(O) r) and its gradient with respect to theta, by reverse
 * mode through the decoder, the L rounds and the encoder, FP32 on the device.
 * theta: device FP32 array of n_params parameters packed as the weights of
 * gnmpc_model_set_gnn (the plan's own weights are not used, so a training loop
 * never leaves the device; the plan supplies the graph, Hd, L, dt and the
 * actuated nodes).  x, x_next [N][M][6], u [N][nu]: FP32 device; O: host [6],
 * >= 0; workspace: device, workspace_bytes from gnmpc_gnn_train_sizes; loss:
 * device [1]; grad: device [n_params], every entry written.  Deterministic
 * (fixed-order sums).  GNMPC_NOT_READY unless the graph and a GNN model are
 * set; GNMPC_UNSUPPORTED for an FP64 plan. */
gnmpc_status gnmpc_gnn_train_sizes(const gnmpc_plan* plan, int64_t* n_params, int64_t* workspace_bytes);
gnmpc_status gnmpc_gnn_loss_grad(gnmpc_plan* plan, const float* theta, const void* x, const void* u,
                                 const void* x_next, const float* O, double lambda, void* workspace, float* loss,
                                 float* grad, void* stream);
/* One Adam update (Kingma and Ba, with bias correction; step counts from 1) of
 * the n device FP32 parameters theta from grad, with the moment estimates m, v
 * (device, n each, zero before step 1), in place. */
gnmpc_status gnmpc_adam_step(int64_t n, float* theta, const float* grad, float* m, float* v, int32_t step,
                             double lr, double beta1, double beta2, double eps, void* stream);

/* Tangent maps of the linearized one-step model x_{k+1} = f(x_k, u_k) of Sec. V-A,
 * from the blocks gnmpc_linearize produced (A [N][nnz][6][6], B [N][M][6][nu], in
 * the plan's pattern and dtype).  Device arrays of the plan dtype, all N stages:
 *   gnmpc_jvp: out[k] = A_k dx[k] + B_k du[k]       dx, out [N][M][6]; du [N][nu]
 *   gnmpc_vjp: gx[k] = A_k' g[k], gu[k] = B_k' g[k] g, gx [N][M][6]; gu [N][nu]
 * (the directional derivative and the gradient of g . f at the linearization
 * points).  Every output element is one fixed-order sum, so repeated calls give
 * bitwise identical results.  Outputs may not alias inputs.  GNMPC_NOT_READY
 * before gnmpc_graph_set; GNMPC_INVALID_ARG for a NULL array. */
gnmpc_status gnmpc_jvp(gnmpc_plan* plan, const void* A, const void* B, const void* dx, const void* du,
                       void* out, void* stream);
gnmpc_status gnmpc_vjp(gnmpc_plan* plan, const void* A, const void* B, const void* g, void* gx, void* gu,
                       void* stream);

/* Condense the linear time-varying OCP (Sec. V-B): propagate the sensitivities
 * S^i_{k+1} = sum_{j in N~_i} A^{ij}_k S^j_k (+ B^i_k in column block k) and
 * Gx^i_{k+1} = sum_j A^{ij}_k Gx^j_k + c^i_k from S_0 = 0, Gx_0 = x0, then form
 *   H  = sum_k sum_i S^i_k' Q^i_k S^i_k + blkdiag(R_k)            [N nu][N nu], full symmetric
 *   g  = sum_k sum_i S^i_k' (Q^i_k Gx^i_k + q^i_k) + [r_k]         [N nu]
 *   Ct[t] = C_t S^{node_t}_{stage_t},  dt[t] = d_t - C_t Gx^{node_t}_{stage_t}   for each state row.
 * Device arrays of the plan dtype: A, B, c as produced by gnmpc_linearize;
 * x0 [M][6]; Q [N+1][M][6] (diagonal, Q_full = 0) or [N+1][M][6][6] (Q_full = 1);
 * q [N+1][M][6]; R [N][nu][nu]; r [N][nu]; rowC [n_c][6]; rowd [n_c] (n_c as
 * set by gnmpc_rows_set; may be NULL when n_c = 0); outputs H, g, Ct [n_c][N nu],
 * dt [n_c]; Gx [N+1][M][6] may be NULL.  Sums are taken in a fixed order, so
 * repeated calls give bitwise identical results. */
gnmpc_status gnmpc_condense(gnmpc_plan* plan, const void* A, const void* B, const void* c,
                            const void* x0, const void* Q, int32_t Q_full, const void* q,
                            const void* R, const void* r, const void* rowC, const void* rowd,
                            void* H, void* g, void* Ct, void* dt, void* Gx, void* stream);

/* Tile autotuner of the condensing (set-up time, not for graph capture: it
 * synchronizes `stream`).  Times gnmpc_condense on the caller's arrays (the
 * arguments of gnmpc_condense, Gx omitted) `reps` times for every feasible
 * propagation variant -- the per-node kernel, node blocks of 16, 8, 4, 2 or 1 nodes one
 * stage per launch, and the same blocks two stages per launch where their halo
 * fits -- keeps the fastest as the plan's choice for later calls (until the next
 * gnmpc_graph_set) and writes every measurement to `report` (host).  The
 * variants compute the same sums; the per-node kernel may round differently.
 * The outputs hold the last candidate's results. */
#define GNMPC_TUNE_MAX 16
typedef struct {
  int32_t variant;      /* 0 per-node kernel, 1 node blocks one stage per launch, 2 two stages */
  int32_t block_nodes;  /* nodes per block (0 for the per-node kernel) */
  double us;            /* mean time of one gnmpc_condense call, microseconds */
} gnmpc_tune_entry;
typedef struct {
  int32_t count;        /* candidates measured */
  int32_t chosen;       /* index of the fastest: the plan's choice now */
  gnmpc_tune_entry entry[GNMPC_TUNE_MAX];
} gnmpc_tune_report;
gnmpc_status gnmpc_autotune_condense(gnmpc_plan* plan, const void* A, const void* B, const void* c, const void* x0,
                                     const void* Q, int32_t Q_full, const void* q, const void* R, const void* r,
                                     const void* rowC, const void* rowd, void* H, void* g, void* Ct, void* dt,
                                     int32_t reps, gnmpc_tune_report* report, void* stream);
/* Set the propagation variant directly (a recorded tuning result; variant and
 * block_nodes as in gnmpc_tune_entry, -1 for the default choice):
 * GNMPC_UNSUPPORTED, with the default restored, when those blocks do not fit
 * LDS or have no two-stage form.  _get reads the current choice (variant -1 =
 * default; block_nodes = nodes per block of the block records, 0 if none). */
gnmpc_status gnmpc_condense_variant_set(gnmpc_plan* plan, int32_t variant, int32_t block_nodes);
gnmpc_status gnmpc_condense_variant_get(const gnmpc_plan* plan, int32_t* variant, int32_t* block_nodes);

/* Solve  min 1/2 u'Hu + g'u  s.t.  lb <= u <= ub,  lc <= Ct u <= uc
 * (the condensed QP of Sec. III-B with native box bounds, Algorithm 1
 * "Solve QP") by ADMM.  Device arrays of the plan dtype: H [n][n] symmetric
 * positive definite, g, lb, ub [n], Ct [n_c][n], lc, uc [n_c] (lc or uc may be
 * NULL for -inf / +inf; infinite entries are allowed); output u [n];
 * info (device, may be NULL).  n <= N nu and n_c <= n_c_max of the plan.
 * The factorization runs in the plan dtype unless its condition estimate
 * exceeds settings->kappa_fp64, in which case factorization and iterations are
 * redone in FP64 (info->used_fp64 = 1). */
gnmpc_status gnmpc_solve_box_qp(gnmpc_plan* plan, int32_t n, const void* H, const void* g,
                                const void* lb, const void* ub, int32_t n_c, const void* Ct,
                                const void* lc, const void* uc, const gnmpc_admm_settings* settings,
                                void* u, gnmpc_qp_info* info, void* stream);

/* The same QP (box bounds, rows lc <= Ct u <= uc) by an interior-point method, as
 * the paper solves its condensed QP (HPIPM): Mehrotra's predictor-corrector
 * primal-dual method on the inequalities given by every finite bound, FP64 in
 * one workgroup; each iteration forms H + G' diag(lambda / s) G, factors it and
 * solves the reduced Newton system for the predictor and the centring
 * corrector.  Arguments as gnmpc_solve_box_qp (plan dtype, device), with tol
 * the stopping tolerance on the duality measure (the residuals are held to
 * max(tol, 1e-9)), both relative to max(1, |g|_inf, |bounds|_inf), e.g. 1e-12,
 * and max_iter.  Where constraints are nearly degenerate the iterate is
 * O(sqrt(tol)) from the minimizer.  Near the solution the factorization is
 * retried with a small diagonal regularization when it loses definiteness.
 * info (device, may be NULL): status SOLVED / MAXITER / NOT_PD / NONFINITE,
 * iterations, residuals, objective, and the last duality measure in the
 * kappa_est field (used_fp64 = 1).  Uses the plan's QP workspace.  Errors as
 * gnmpc_solve_box_qp, plus GNMPC_INVALID_ARG for tol <= 0 or max_iter < 1, and
 * GNMPC_UNSUPPORTED when the slot arrays exceed one workgroup's LDS (n = 240
 * with 200 rows fits). */
gnmpc_status gnmpc_solve_qp_ipm(gnmpc_plan* plan, int32_t n, const void* H, const void* g, const void* lb,
                                const void* ub, int32_t n_c, const void* Ct, const void* lc, const void* uc, double tol,
                                int32_t max_iter, void* u, gnmpc_qp_info* info, void* stream);

/* Allocation-free variant of gnmpc_solve_box_qp, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It takes no plan: dtype is GNMPC_F32 or
 * GNMPC_F64 (the type of every array), and the arguments, layouts, settings,
 * FP64 fallback and results are those of gnmpc_solve_box_qp (same kernels, so
 * the same bits).  The solver's workspace is a fixed 4 MiB array in device
 * memory, one per GPU, held by the library until the process ends: n may be
 * at most 464 (any n_c the LDS of one workgroup admits).  It runs on the
 * current device, which must own `stream`; the call enqueues a small kernel
 * that clears the solver's flags, then the solve, and never allocates or
 * frees memory.  Every call on a GPU shares that GPU's array, so calls that
 * overlap in time on one GPU (different streams, threads or processes sharing
 * the device's memory) race and give wrong results: serialize them, e.g. on
 * one stream.  Errors: GNMPC_INVALID_ARG (dtype, null arrays, settings),
 * GNMPC_SHAPE (n outside 1..464 or n_c < 0), GNMPC_UNSUPPORTED (the vectors
 * do not fit one workgroup's LDS), GNMPC_HIP_ERROR (symbol lookup or launch);
 * all checked on the host before anything is enqueued. */
gnmpc_status gnmpc_solve_box_qp_noalloc(int32_t dtype, int32_t n, const void* H, const void* g,
                                        const void* lb, const void* ub, int32_t n_c, const void* Ct,
                                        const void* lc, const void* uc,
                                        const gnmpc_admm_settings* settings, void* u,
                                        gnmpc_qp_info* info, void* stream);

/* ---------------- batched steps ---------------- */

/* The device arrays of one instance's condensed MPC step: the arguments of
 * gnmpc_linearize, gnmpc_condense and gnmpc_solve_box_qp for its plan, with
 * the same shapes, dtypes and ownership (the caller owns them).  rowC, rowd,
 * Ct, dt may be NULL when the plan has no state rows; lc, uc may be NULL
 * (-inf / +inf). */
typedef struct {
  gnmpc_plan* plan;
  const void *xhat, *uhat, *x0, *Q, *q, *R, *r, *rowC, *rowd, *lb, *ub, *lc, *uc;
  int32_t Q_full;   /* 0: Q is diagonal [N+1][M][6]; 1: full blocks [N+1][M][6][6] */
  int32_t reserved;
  void *A, *B, *c, *H, *g, *Ct, *dt, *u;
  gnmpc_qp_info* info; /* device, may be NULL */
} gnmpc_step_desc;

/* Batched step: linearize, condense and solve the box QP (Algorithm 1's
 * linearization, condensing and "Solve QP" of one MPC iteration) for `count`
 * independent instances of uneven sizes, each with its own plan on the same
 * device.  Linearization, condensing and the QP set-up run concurrently: the
 * work is forked from `stream` onto up to 4 library-owned streams (instance i
 * on stream i mod 4) and joined back with events; then every instance's QP is
 * solved in one launch per pass on `stream` (one workgroup per instance, up to
 * 16 instances per launch), so `stream` is ordered after every instance and a
 * HIP graph capture of `stream` records the whole batch (the library streams
 * are created on the first call, which must not be captured).  Each instance's
 * results are bitwise those of its single calls.  Settings apply to
 * every QP.  Each instance's arrays are validated as by the single calls; on
 * an error the work already forked is still joined and the first failing
 * status is returned (that plan's last_error names the cause).  Every plan
 * may appear in one descriptor only (GNMPC_INVALID_ARG otherwise, before
 * anything is enqueued): a plan's workspace serves one instance at a time.
 * Concurrent calls from several host threads are serialized while they
 * enqueue. */
gnmpc_status gnmpc_step_batched(const gnmpc_step_desc* descs, int32_t count,
                                const gnmpc_admm_settings* settings, void* stream);

/* One iteration of Algorithm 1 (GNN-MPC, an SQP real-time iteration) for one
 * instance, on `stream`: linearize the plan's model around (d->xhat, d->uhat),
 * condense with the initial state d->x0 (the measured state), solve the box QP
 * into d->u, roll the linearized dynamics forward from x0 with u into
 * xpred [N+1][M][6] (the optimal predicted states x*), and write the shifted
 * trajectory of the next iteration ("update lin. trajectory"):
 *   xhat_next[k] = x*[k+1] (k < N), xhat_next[N] = x*[N];
 *   uhat_next[k] = u*[k+1] (k < N-1), uhat_next[N-1] = u*[N-1].
 * The input to apply is u*[0], the first nu entries of d->u.  xhat_next and
 * uhat_next may be d->xhat and d->uhat (they are written last); xpred may
 * alias neither xhat array.  Arrays as in gnmpc_step_desc, device, plan
 * dtype; the QP status goes to d->info.  Errors as the single calls; the first
 * failing call's status is returned and nothing after it is enqueued. */
gnmpc_status gnmpc_rti_step(const gnmpc_step_desc* d, void* xpred, void* xhat_next, void* uhat_next,
                            const gnmpc_admm_settings* settings, void* stream);

/* The same iteration with the condensed QP solved by the interior-point method
 * (gnmpc_solve_qp_ipm with tol and max_iter; its status and duality measure go
 * to d->info), the kind of QP solver the paper's loop uses (Sec. VI-A).  Other
 * arguments, aliasing rules and errors as gnmpc_rti_step. */
gnmpc_status gnmpc_rti_step_ipm(const gnmpc_step_desc* d, void* xpred, void* xhat_next, void* uhat_next,
                                double tol, int32_t max_iter, void* stream);

/* ---------------- per-phase GPU timers ---------------- */

/* Phases timed by gnmpc_timers_*: hipEvents are recorded on the caller's stream
 * around the kernels of each phase while timers are enabled. */
typedef enum {
  GNMPC_PH_GNN_FORWARD = 0,       /* GNN forward pass at the N linearization points   */
  GNMPC_PH_GNN_JACOBIAN = 1,      /* the forward-mode Jacobian kernel                  */
  GNMPC_PH_GNN_ASSEMBLY = 2,      /* the offsets c (and the B zero fill, where the
                                   * Jacobian kernel runs without stage images)        */
  GNMPC_PH_MSD_LINEARIZE = 3,     /* analytic mass-spring-damper linearization         */
  GNMPC_PH_CONDENSE_PROPAGATE = 4,/* the stage recursion for S_k and Gx_k              */
  GNMPC_PH_CONDENSE_GRAM = 5,     /* H and g                                           */
  GNMPC_PH_CONDENSE_ROWS = 6,     /* condensed state rows                              */
  GNMPC_PH_QP = 7,                /* the QP solve                                      */
  GNMPC_PH_GNN_STAGE_IMAGES = 8,  /* the Jacobian kernel's stage images from the forward pass,
                                   * with the B zero fill in the same launch           */
  GNMPC_PH_COUNT = 9
} gnmpc_phase;

/* Enable (1) or disable (0) the timers; enabling clears earlier records and
 * creates the events (up to 1024 records per phase). */
gnmpc_status gnmpc_timers_enable(gnmpc_plan* plan, int32_t enable);
/* Wait for the recorded events and return, per phase, the summed elapsed
 * milliseconds and the number of records (arrays of GNMPC_PH_COUNT). */
gnmpc_status gnmpc_timers_read(gnmpc_plan* plan, double* total_ms, int32_t* count);

/* Default ADMM settings (rho 0.1, sigma 1e-6, alpha 1.6, eps 1e-6, kappa_fp64 1e7,
 * 4000 iterations, convergence checked every 10). */
void gnmpc_admm_default_settings(gnmpc_admm_settings* s);

#ifdef __cplusplus
}
#endif

#endif /* GNMPC_H */
