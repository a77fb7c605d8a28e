// C-ABI entry points of libgnmpc: argument validation, graph preparation on
// the host, plan workspace and launch sequencing.  Every check runs before any
// HIP call, so invalid requests never touch the GPU.
#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace gnmpc;

namespace {

const char* kVersion = "gnmpc 0.1 (gfx950)";

gnmpc_status fail(gnmpc_plan* p, gnmpc_status s, const std::string& msg) {
  if (p) p->last_error = msg;
  return s;
}

template <typename T>
void dfree(T*& ptr) {
  if (ptr) (void)hipFree((void*)ptr);
  ptr = nullptr;
}

template <typename T>
gnmpc_status upload(gnmpc_plan* p, T*& dst, const T* src, size_t count) {
  dfree(dst);
  if (count == 0) return GNMPC_OK;
  GNMPC_HIP_TRY(p, hipMalloc((void**)&dst, sizeof(T) * count));
  GNMPC_HIP_TRY(p, hipMemcpy(dst, src, sizeof(T) * count, hipMemcpyHostToDevice));
  return GNMPC_OK;
}

// Breadth-first closure over incoming edges: nodes that reach i in <= L hops.
void closure(const int32_t* row_ptr, const int32_t* col, int32_t M, int32_t L, std::vector<int32_t>& prow,
             std::vector<int32_t>& pcol) {
  prow.assign(M + 1, 0);
  pcol.clear();
  std::vector<int32_t> mark(M, -1), frontier, next, found;
  for (int32_t i = 0; i < M; ++i) {
    found.assign(1, i);
    mark[i] = i;
    frontier.assign(1, i);
    for (int32_t h = 0; h < L && !frontier.empty(); ++h) {
      next.clear();
      for (int32_t n : frontier)
        for (int32_t e = row_ptr[n]; e < row_ptr[n + 1]; ++e) {
          int32_t j = col[e];
          if (mark[j] != i) {
            mark[j] = i;
            next.push_back(j);
            found.push_back(j);
          }
        }
      frontier.swap(next);
    }
    std::sort(found.begin(), found.end());
    pcol.insert(pcol.end(), found.begin(), found.end());
    prow[i + 1] = (int32_t)pcol.size();
  }
}

bool dims_ok(const gnmpc_dims* d) {
  return d && d->M > 0 && d->nu > 0 && d->N > 0 && d->n_c_max >= 0 &&
         (d->dtype == GNMPC_F64 || d->dtype == GNMPC_F32) && (long)d->M * 6 < (1L << 30) &&
         (long)d->N * d->nu <= 4096;
}

}  // namespace

extern "C" {

const char* gnmpc_version(void) { return kVersion; }

const char* gnmpc_status_string(int32_t s) {
  switch (s) {
    case GNMPC_OK: return "ok";
    case GNMPC_INVALID_ARG: return "invalid argument";
    case GNMPC_BAD_GRAPH: return "malformed graph";
    case GNMPC_SHAPE: return "shape mismatch";
    case GNMPC_UNSUPPORTED: return "unsupported";
    case GNMPC_HIP_ERROR: return "HIP runtime error";
    case GNMPC_BAD_CONSTRAINT: return "bad constraint row";
    case GNMPC_NOT_READY: return "plan not ready";
    case GNMPC_NO_DEVICE: return "no usable GPU";
    default: return "unknown status";
  }
}

void gnmpc_admm_default_settings(gnmpc_admm_settings* s) {
  if (!s) return;
  s->rho = 0.1;
  s->sigma = 1e-6;
  s->alpha = 1.6;
  s->eps_abs = 1e-6;
  s->eps_rel = 1e-6;
  s->kappa_fp64 = 1e7;
  s->max_iter = 4000;
  s->check_every = 10;
}

gnmpc_status gnmpc_graph_check(const int32_t* row_ptr, const int32_t* col, int32_t M, int32_t E) {
  if (!row_ptr || M <= 0 || E < 0 || (E > 0 && !col)) return GNMPC_INVALID_ARG;
  if (row_ptr[0] != 0 || row_ptr[M] != E) return GNMPC_BAD_GRAPH;
  for (int32_t i = 0; i < M; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) return GNMPC_BAD_GRAPH;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      int32_t j = col[e];
      if (j < 0 || j >= M || j == i) return GNMPC_BAD_GRAPH;
      if (e > row_ptr[i] && col[e - 1] >= j) return GNMPC_BAD_GRAPH;  // unsorted or duplicate
    }
  }
  return GNMPC_OK;
}

gnmpc_status gnmpc_graph_closure(const int32_t* row_ptr, const int32_t* col, int32_t M, int32_t E, int32_t L,
                                 int32_t* row_ptr_out, int32_t* col_out, int64_t cap, int64_t* nnz_out) {
  gnmpc_status s = gnmpc_graph_check(row_ptr, col, M, E);
  if (s != GNMPC_OK) return s;
  if (L < 0 || !nnz_out) return GNMPC_INVALID_ARG;
  std::vector<int32_t> prow, pcol;
  closure(row_ptr, col, M, L, prow, pcol);
  *nnz_out = (int64_t)pcol.size();
  if (!col_out) return GNMPC_OK;
  if (!row_ptr_out || cap < (int64_t)pcol.size()) return GNMPC_INVALID_ARG;
  std::memcpy(row_ptr_out, prow.data(), sizeof(int32_t) * (M + 1));
  std::memcpy(col_out, pcol.data(), sizeof(int32_t) * pcol.size());
  return GNMPC_OK;
}

gnmpc_status gnmpc_plan_create(gnmpc_plan** plan, const gnmpc_dims* dims, int32_t device) {
  if (!plan) return GNMPC_INVALID_ARG;
  *plan = nullptr;
  if (!dims_ok(dims) || device < 0) return GNMPC_INVALID_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= device) return GNMPC_NO_DEVICE;
  gnmpc_plan* p = new gnmpc_plan();
  p->device = device;
  p->dims = *dims;
  p->elem = dims->dtype == GNMPC_F64 ? 8 : 4;
  gnmpc_status st = GNMPC_OK;
  auto alloc = [&](void** ptr, size_t bytes) {
    if (st != GNMPC_OK) return;
    if (hipMalloc(ptr, std::max<size_t>(bytes, 256)) != hipSuccess) {
      p->last_error = "hipMalloc failed";
      st = GNMPC_HIP_ERROR;
    }
  };
  if (hipSetDevice(device) != hipSuccess) {
    delete p;
    return GNMPC_NO_DEVICE;
  }
  const int M = dims->M, nu = dims->nu, N = dims->N;
  p->S_elems = S_offset(N + 1, M, nu);
  alloc(&p->d_S, p->S_elems * p->elem);
  alloc(&p->d_Gx, (size_t)(N + 1) * M * NBX * p->elem);
  p->part_elems = condense_partial_elems(M, nu, N);
  alloc(&p->d_part, p->part_elems * p->elem);
  p->qp_bytes = qp_workspace_bytes(N * nu, dims->n_c_max);
  alloc(&p->d_qp, p->qp_bytes);
  alloc((void**)&p->d_qp_flag, 64);
  alloc(&p->d_check, lin_check_bytes());
  alloc(&p->d_qpdesc, kQpDescBytes);
  if (st == GNMPC_OK && hipMemset(p->d_qp_flag, 0, 64) != hipSuccess) st = GNMPC_HIP_ERROR;
  if (st != GNMPC_OK) {
    gnmpc_plan_destroy(p);
    return st;
  }
  *plan = p;
  return GNMPC_OK;
}

static void destroy_timers(gnmpc_plan* p) {
  for (int ph = 0; ph < GNMPC_PH_COUNT; ++ph) {
    for (hipEvent_t e : p->ev_start[ph]) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->ev_stop[ph]) (void)hipEventDestroy(e);
    p->ev_start[ph].clear();
    p->ev_stop[ph].clear();
    p->ev_used[ph] = 0;
    p->ev_open[ph] = 0;
  }
  p->timers_on = false;
}

gnmpc_status gnmpc_timers_enable(gnmpc_plan* p, int32_t enable) {
  if (!p) return GNMPC_INVALID_ARG;
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  destroy_timers(p);
  if (!enable) return GNMPC_OK;
  for (int ph = 0; ph < GNMPC_PH_COUNT; ++ph) {
    p->ev_start[ph].resize(kTimerRecords);
    p->ev_stop[ph].resize(kTimerRecords);
    for (int t = 0; t < kTimerRecords; ++t) {
      GNMPC_HIP_TRY(p, hipEventCreate(&p->ev_start[ph][t]));
      GNMPC_HIP_TRY(p, hipEventCreate(&p->ev_stop[ph][t]));
    }
  }
  p->timers_on = true;
  return GNMPC_OK;
}

gnmpc_status gnmpc_timers_read(gnmpc_plan* p, double* total_ms, int32_t* count) {
  if (!p || !total_ms || !count) return GNMPC_INVALID_ARG;
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  for (int ph = 0; ph < GNMPC_PH_COUNT; ++ph) {
    double sum = 0.0;
    for (int t = 0; t < p->ev_used[ph]; ++t) {
      GNMPC_HIP_TRY(p, hipEventSynchronize(p->ev_stop[ph][t]));
      float ms = 0.f;
      GNMPC_HIP_TRY(p, hipEventElapsedTime(&ms, p->ev_start[ph][t], p->ev_stop[ph][t]));
      sum += ms;
    }
    total_ms[ph] = sum;
    count[ph] = p->ev_used[ph];
  }
  return GNMPC_OK;
}

void gnmpc_plan_destroy(gnmpc_plan* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  destroy_timers(p);
  gnn_free(p);
  inet_free(p);
  dfree(p->d_row_ptr);
  dfree(p->d_col);
  dfree(p->d_prow);
  dfree(p->d_pcol);
  dfree(p->d_erow);
  dfree(p->d_diag);
  dfree(p->d_cptr);
  dfree(p->d_cent);
  prop_blocks_free(p);
  dfree(p->d_act_of_node);
  dfree(p->d_row_node);
  dfree(p->d_row_stage);
  if (p->d_S) (void)hipFree(p->d_S);
  if (p->d_Gx) (void)hipFree(p->d_Gx);
  if (p->d_part) (void)hipFree(p->d_part);
  if (p->d_qp) (void)hipFree(p->d_qp);
  if (p->d_check) (void)hipFree(p->d_check);
  if (p->d_qpdesc) (void)hipFree(p->d_qpdesc);
  dfree(p->d_qp_flag);
  delete p;
}

const char* gnmpc_plan_last_error(const gnmpc_plan* p) { return p ? p->last_error.c_str() : "null plan"; }

gnmpc_status gnmpc_graph_set(gnmpc_plan* p, const int32_t* row_ptr, const int32_t* col, int32_t M, int32_t E,
                             int32_t L) {
  if (!p) return GNMPC_INVALID_ARG;
  gnmpc_status s = gnmpc_graph_check(row_ptr, col, M, E);
  if (s != GNMPC_OK) return fail(p, s, "graph_set: malformed CSR");
  if (M != p->dims.M) return fail(p, GNMPC_SHAPE, "graph_set: M differs from the plan");
  if (L < 1 || L > 8) return fail(p, GNMPC_INVALID_ARG, "graph_set: L must be in 1..8");
  std::vector<int32_t> prow, pcol;
  closure(row_ptr, col, M, L, prow, pcol);
  int wmax = 0;
  std::vector<int32_t> erow(pcol.size()), diag(M);
  for (int32_t i = 0; i < M; ++i) {
    wmax = std::max(wmax, prow[i + 1] - prow[i]);
    for (int32_t e = prow[i]; e < prow[i + 1]; ++e) {
      erow[e] = i;
      if (pcol[e] == i) diag[i] = e;
    }
  }
  if (wmax > kMaxWidth) return fail(p, GNMPC_UNSUPPORTED, "graph_set: Jacobian pattern row wider than 64 blocks");
  // the pattern by column (entries of column node j in increasing order), for the VJP
  std::vector<int32_t> cptr(M + 1, 0), cent(pcol.size());
  for (int32_t c : pcol) ++cptr[c + 1];
  for (int32_t j = 0; j < M; ++j) cptr[j + 1] += cptr[j];
  {
    std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
    for (size_t e = 0; e < pcol.size(); ++e) cent[fill[pcol[e]]++] = (int32_t)e;
  }
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  p->graph_ready = false;
  p->h_row_ptr.assign(row_ptr, row_ptr + M + 1);
  p->h_col.assign(col, col + E);
  p->h_prow = prow;
  p->h_pcol = pcol;
  p->M = M;
  p->E = E;
  p->L = L;
  p->nnz = (long)pcol.size();
  p->wmax = wmax;
  if ((s = upload(p, p->d_row_ptr, row_ptr, M + 1)) != GNMPC_OK) return s;
  if ((s = upload(p, p->d_col, col, (size_t)E)) != GNMPC_OK) return s;
  if ((s = upload(p, p->d_prow, prow.data(), prow.size())) != GNMPC_OK) return s;
  if ((s = upload(p, p->d_pcol, pcol.data(), pcol.size())) != GNMPC_OK) return s;
  if ((s = upload(p, p->d_erow, erow.data(), erow.size())) != GNMPC_OK) return s;
  if ((s = upload(p, p->d_diag, diag.data(), diag.size())) != GNMPC_OK) return s;
  if ((s = upload(p, p->d_cptr, cptr.data(), cptr.size())) != GNMPC_OK) return s;
  if ((s = upload(p, p->d_cent, cent.data(), cent.size())) != GNMPC_OK) return s;
  p->prop_pref = -1;
  if ((s = prop_blocks_build(p)) != GNMPC_OK) return s;
  p->graph_ready = true;
  p->model = 0;  // a model must be (re)bound to the new graph
  return GNMPC_OK;
}

gnmpc_status gnmpc_graph_nnz(const gnmpc_plan* p, int64_t* nnz) {
  if (!p || !nnz) return GNMPC_INVALID_ARG;
  if (!p->graph_ready) return GNMPC_NOT_READY;
  *nnz = p->nnz;
  return GNMPC_OK;
}

gnmpc_status gnmpc_graph_pattern(const gnmpc_plan* p, int32_t* row_ptr_out, int32_t* col_out) {
  if (!p || !row_ptr_out || !col_out) return GNMPC_INVALID_ARG;
  if (!p->graph_ready) return GNMPC_NOT_READY;
  std::memcpy(row_ptr_out, p->h_prow.data(), sizeof(int32_t) * p->h_prow.size());
  std::memcpy(col_out, p->h_pcol.data(), sizeof(int32_t) * p->h_pcol.size());
  return GNMPC_OK;
}

static gnmpc_status set_actuators(gnmpc_plan* p, const int32_t* act, int32_t n_act) {
  if (n_act < 0 || (n_act > 0 && !act)) return fail(p, GNMPC_INVALID_ARG, "actuators: bad list");
  if (3 * n_act != p->dims.nu) return fail(p, GNMPC_SHAPE, "actuators: nu must equal 3 * n_act");
  std::vector<int32_t> of(p->M, -1);
  for (int32_t a = 0; a < n_act; ++a) {
    if (act[a] < 0 || act[a] >= p->M) return fail(p, GNMPC_INVALID_ARG, "actuators: node out of range");
    if (of[act[a]] >= 0) return fail(p, GNMPC_INVALID_ARG, "actuators: duplicate node");
    of[act[a]] = a;
  }
  p->h_act.assign(act, act + n_act);
  p->n_act = n_act;
  return upload(p, p->d_act_of_node, of.data(), of.size());
}

gnmpc_status gnmpc_model_set_msd(gnmpc_plan* p, const gnmpc_msd_params* prm, const int32_t* act, int32_t n_act) {
  if (!p || !prm) return GNMPC_INVALID_ARG;
  if (!p->graph_ready) return fail(p, GNMPC_NOT_READY, "model_set_msd: set the graph first");
  if (!(prm->m > 0) || !(prm->dt > 0) || !std::isfinite(prm->k) || !std::isfinite(prm->c) ||
      !std::isfinite(prm->k3) || !std::isfinite(prm->gravity) || prm->anchor < -1 || prm->anchor >= p->M)
    return fail(p, GNMPC_INVALID_ARG, "model_set_msd: bad parameters");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  gnmpc_status s = set_actuators(p, act, n_act);
  if (s != GNMPC_OK) return s;
  p->msd = *prm;
  p->model = 1;
  return GNMPC_OK;
}

gnmpc_status gnmpc_model_set_gnn(gnmpc_plan* p, const gnmpc_gnn_desc* desc, const double* weights, int64_t n_weights,
                                 const int32_t* act, int32_t n_act) {
  if (!p || !desc || !weights) return GNMPC_INVALID_ARG;
  if (!p->graph_ready) return fail(p, GNMPC_NOT_READY, "model_set_gnn: set the graph first");
  if (desc->L != p->L) return fail(p, GNMPC_SHAPE, "model_set_gnn: L differs from the graph's L");
  if (desc->Hd <= 0 || desc->Hd % 64 != 0 || desc->Hd > 256 || !(desc->dt > 0) ||
      (desc->dtype != GNMPC_F32 && desc->dtype != GNMPC_BF16))
    return fail(p, GNMPC_INVALID_ARG, "model_set_gnn: Hd must be a multiple of 64 up to 256, dtype F32 or BF16");
  const long Hd = desc->Hd;
  const long expect = Hd * 9 + Hd + desc->L * (2 * (Hd * 2 * Hd + Hd)) + 6 * Hd + 6;
  if (n_weights != expect) return fail(p, GNMPC_SHAPE, "model_set_gnn: wrong number of weights");
  for (int64_t t = 0; t < n_weights; ++t)
    if (!std::isfinite(weights[t])) return fail(p, GNMPC_INVALID_ARG, "model_set_gnn: non-finite weight");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  gnmpc_status s = set_actuators(p, act, n_act);
  if (s != GNMPC_OK) return s;
  s = gnn_set(p, desc, weights, n_weights);
  if (s != GNMPC_OK) return s;
  p->model = 2;
  return GNMPC_OK;
}

gnmpc_status gnmpc_model_set_inet(gnmpc_plan* p, const gnmpc_inet_desc* desc, const double* weights,
                                  int64_t n_weights) {
  if (!p || !desc || !weights) return GNMPC_INVALID_ARG;
  if (!p->graph_ready) return fail(p, GNMPC_NOT_READY, "model_set_inet: set the graph first");
  if (p->L != 1) return fail(p, GNMPC_SHAPE, "model_set_inet: the graph must be set with L = 1");
  if (desc->nu != p->dims.nu) return fail(p, GNMPC_SHAPE, "model_set_inet: nu differs from the plan's nu");
  for (int64_t t = 0; t < n_weights; ++t)
    if (!std::isfinite(weights[t])) return fail(p, GNMPC_INVALID_ARG, "model_set_inet: non-finite weight");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  const gnmpc_status s = inet_set(p, desc, weights, n_weights);
  if (s == GNMPC_INVALID_ARG) return fail(p, s, "model_set_inet: sizes out of range");
  if (s == GNMPC_SHAPE) return fail(p, s, "model_set_inet: wrong number of weights");
  if (s == GNMPC_UNSUPPORTED) return fail(p, s, "model_set_inet: activations exceed one workgroup's LDS");
  if (s != GNMPC_OK) return s;
  p->model = 3;
  return GNMPC_OK;
}

gnmpc_status gnmpc_rows_set(gnmpc_plan* p, int32_t n_c, const int32_t* node, const int32_t* stage) {
  if (!p) return GNMPC_INVALID_ARG;
  if (n_c < 0 || (n_c > 0 && (!node || !stage))) return fail(p, GNMPC_INVALID_ARG, "rows_set: bad arrays");
  if (n_c > p->dims.n_c_max) return fail(p, GNMPC_SHAPE, "rows_set: n_c exceeds n_c_max");
  for (int32_t t = 0; t < n_c; ++t) {
    if (node[t] < 0 || node[t] >= p->dims.M) return fail(p, GNMPC_BAD_CONSTRAINT, "rows_set: node out of range");
    if (stage[t] < 1 || stage[t] > p->dims.N)
      return fail(p, GNMPC_BAD_CONSTRAINT, "rows_set: stage must be in 1..N (stage-0 rows do not depend on u)");
  }
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  gnmpc_status s;
  if ((s = upload(p, p->d_row_node, node, (size_t)n_c)) != GNMPC_OK) return s;
  if ((s = upload(p, p->d_row_stage, stage, (size_t)n_c)) != GNMPC_OK) return s;
  p->n_c = n_c;
  return GNMPC_OK;
}

gnmpc_status gnmpc_linearize(gnmpc_plan* p, const void* xhat, const void* uhat, void* A, void* B, void* c,
                             void* fnext, gnmpc_lin_info* info, void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (!xhat || !uhat || !A || !B || !c) return fail(p, GNMPC_INVALID_ARG, "linearize: null array");
  if (!p->graph_ready || p->model == 0) return fail(p, GNMPC_NOT_READY, "linearize: graph and model must be set");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  hipStream_t s = (hipStream_t)stream;
  const gnmpc_status st = p->model == 1   ? launch_msd_linearize(p, xhat, uhat, A, B, c, fnext, s)
                          : p->model == 3 ? launch_inet_linearize(p, xhat, uhat, A, B, c, fnext, s)
                                          : launch_gnn_linearize(p, xhat, uhat, A, B, c, fnext, s);
  if (st != GNMPC_OK || !info) return st;
  return launch_lin_check(p, xhat, uhat, A, B, c, fnext, info, s);
}

gnmpc_status gnmpc_rollout_linear(gnmpc_plan* p, const void* A, const void* B, const void* c, const void* x0,
                                  const void* u, void* x, void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (!A || !B || !c || !x0 || !u || !x) return fail(p, GNMPC_INVALID_ARG, "rollout_linear: null array");
  if (!p->graph_ready) return fail(p, GNMPC_NOT_READY, "rollout_linear: graph must be set");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  return launch_rollout(p, A, B, c, x0, u, x, (hipStream_t)stream);
}

gnmpc_status gnmpc_msd_simulate(gnmpc_plan* p, int32_t B, int32_t T, const void* x0, const void* u, void* X,
                                void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (B < 0 || T < 0) return fail(p, GNMPC_SHAPE, "msd_simulate: B and T must be >= 0");
  if (!p->graph_ready || p->model != 1)
    return fail(p, GNMPC_NOT_READY, "msd_simulate: graph and mass-spring-damper model must be set");
  if (B == 0) return GNMPC_OK;
  if (!x0 || !X || (T > 0 && p->dims.nu > 0 && !u)) return fail(p, GNMPC_INVALID_ARG, "msd_simulate: null array");
  if (!msd_sim_fits(p)) return fail(p, GNMPC_UNSUPPORTED, "msd_simulate: two states of the graph exceed LDS");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  return launch_msd_simulate(p, B, T, x0, u, X, (hipStream_t)stream);
}

gnmpc_status gnmpc_gnn_forward(gnmpc_plan* p, const void* xhat, const void* uhat, void* fnext, void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (!xhat || !uhat || !fnext) return fail(p, GNMPC_INVALID_ARG, "gnn_forward: null array");
  if (!p->graph_ready || p->model != 2) return fail(p, GNMPC_NOT_READY, "gnn_forward: graph and GNN model must be set");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  return launch_gnn_forward_only(p, xhat, uhat, fnext, (hipStream_t)stream);
}

gnmpc_status gnmpc_gnn_vjp(gnmpc_plan* p, const void* xhat, const void* uhat, const void* g, void* gx, void* gu,
                           void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (!xhat || !uhat || !g || !gx || !gu) return fail(p, GNMPC_INVALID_ARG, "gnn_vjp: null array");
  if (!p->graph_ready || p->model != 2) return fail(p, GNMPC_NOT_READY, "gnn_vjp: graph and GNN model must be set");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  return launch_gnn_vjp(p, xhat, uhat, g, gx, gu, (hipStream_t)stream);
}

gnmpc_status gnmpc_gnn_train_sizes(const gnmpc_plan* p, int64_t* n_params, int64_t* workspace_bytes) {
  if (!p || !n_params || !workspace_bytes) return GNMPC_INVALID_ARG;
  if (!p->graph_ready || p->model != 2) return GNMPC_NOT_READY;
  *n_params = gnn_param_count(p);
  *workspace_bytes = (int64_t)gnn_train_workspace_bytes(p);
  return GNMPC_OK;
}

gnmpc_status gnmpc_gnn_loss_grad(gnmpc_plan* p, const float* theta, const void* x, const void* u, const void* x_next,
                                 const float* O, double lambda, void* workspace, float* loss, float* grad,
                                 void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (!theta || !x || !u || !x_next || !O || !workspace || !loss || !grad)
    return fail(p, GNMPC_INVALID_ARG, "gnn_loss_grad: null array");
  if (!p->graph_ready || p->model != 2) return fail(p, GNMPC_NOT_READY, "gnn_loss_grad: graph and GNN model must be set");
  if (p->dims.dtype != GNMPC_F32) return fail(p, GNMPC_UNSUPPORTED, "gnn_loss_grad: the plan's arrays must be FP32");
  if (!(lambda >= 0) || !std::isfinite(lambda)) return fail(p, GNMPC_INVALID_ARG, "gnn_loss_grad: lambda >= 0");
  for (int c = 0; c < 6; ++c)
    if (!(O[c] >= 0) || !std::isfinite(O[c])) return fail(p, GNMPC_INVALID_ARG, "gnn_loss_grad: O must be >= 0");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  return launch_gnn_loss_grad(p, theta, x, u, x_next, O, lambda, workspace, loss, grad, (hipStream_t)stream);
}

gnmpc_status gnmpc_adam_step(int64_t n, float* theta, const float* grad, float* m, float* v, int32_t step, double lr,
                             double beta1, double beta2, double eps, void* stream) {
  if (n < 0 || (n > 0 && (!theta || !grad || !m || !v)) || step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) ||
      !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return GNMPC_INVALID_ARG;
  if (n == 0) return GNMPC_OK;
  return launch_adam(n, theta, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}

gnmpc_status gnmpc_condense(gnmpc_plan* p, const void* A, const void* B, const void* c, const void* x0,
                            const void* Q, int32_t Q_full, const void* q, const void* R, const void* r,
                            const void* rowC, const void* rowd, void* H, void* g, void* Ct, void* dt, void* Gx,
                            void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (!A || !B || !c || !x0 || !Q || !q || !R || !r || !H || !g)
    return fail(p, GNMPC_INVALID_ARG, "condense: null array");
  if (Q_full != 0 && Q_full != 1) return fail(p, GNMPC_INVALID_ARG, "condense: Q_full must be 0 or 1");
  if (!p->graph_ready) return fail(p, GNMPC_NOT_READY, "condense: graph must be set");
  if (p->n_c > 0 && (!rowC || !rowd || !Ct || !dt)) return fail(p, GNMPC_INVALID_ARG, "condense: null row array");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  return launch_condense(p, A, B, c, x0, Q, Q_full, q, R, r, rowC, rowd, H, g, Ct, dt, Gx, (hipStream_t)stream);
}

static gnmpc_status qp_check(gnmpc_plan* p, int32_t n, const void* H, const void* g, const void* lb, const void* ub,
                             int32_t n_c, const void* Ct, const gnmpc_admm_settings* st, const void* u) {
  if (!H || !g || !lb || !ub || !u || !st) return fail(p, GNMPC_INVALID_ARG, "solve_box_qp: null array");
  if (n <= 0 || n > p->dims.N * p->dims.nu) return fail(p, GNMPC_SHAPE, "solve_box_qp: n outside 1..N*nu");
  if (n_c < 0 || n_c > p->dims.n_c_max) return fail(p, GNMPC_SHAPE, "solve_box_qp: n_c outside 0..n_c_max");
  if (n_c > 0 && !Ct) return fail(p, GNMPC_INVALID_ARG, "solve_box_qp: Ct is null");
  if (!(st->rho > 0) || !(st->sigma > 0) || !(st->alpha > 0 && st->alpha < 2) || !(st->eps_abs >= 0) ||
      !(st->eps_rel >= 0) || st->max_iter < 1 || st->check_every < 1 || !(st->kappa_fp64 > 0))
    return fail(p, GNMPC_INVALID_ARG, "solve_box_qp: bad settings");
  return GNMPC_OK;
}

gnmpc_status gnmpc_condense_variant_set(gnmpc_plan* p, int32_t variant, int32_t block_nodes) {
  if (!p) return GNMPC_INVALID_ARG;
  if (!p->graph_ready) return fail(p, GNMPC_NOT_READY, "condense_variant_set: graph must be set");
  if (variant < -1 || variant > 2 ||
      (variant >= 1 && block_nodes != 1 && block_nodes != 2 && block_nodes != 4 && block_nodes != 8 &&
       block_nodes != 16))
    return fail(p, GNMPC_INVALID_ARG, "condense_variant_set: variant -1..2, blocks of 1, 2, 4, 8 or 16 nodes");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  gnmpc_status st = prop_blocks_build_nb(p, variant >= 1 ? block_nodes : 4);
  if (st != GNMPC_OK) return st;
  if (variant >= 1 && (p->pb_nodes != block_nodes || (variant == 2 && p->pb2_stride == 0))) {
    p->prop_pref = -1;
    const gnmpc_status sb = prop_blocks_build(p);
    return sb != GNMPC_OK ? sb : fail(p, GNMPC_UNSUPPORTED, "condense_variant_set: these blocks do not fit LDS");
  }
  p->prop_pref = variant;
  return GNMPC_OK;
}

gnmpc_status gnmpc_condense_variant_get(const gnmpc_plan* p, int32_t* variant, int32_t* block_nodes) {
  if (!p || !variant || !block_nodes) return GNMPC_INVALID_ARG;
  *variant = p->prop_pref;
  *block_nodes = p->pb_nodes;
  return GNMPC_OK;
}

gnmpc_status gnmpc_autotune_condense(gnmpc_plan* p, const void* A, const void* B, const void* c, const void* x0,
                                     const void* Q, int32_t Q_full, const void* q, const void* R, const void* r,
                                     const void* rowC, const void* rowd, void* H, void* g, void* Ct, void* dt,
                                     int32_t reps, gnmpc_tune_report* rep, void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (!rep || reps < 1) return fail(p, GNMPC_INVALID_ARG, "autotune_condense: report and reps >= 1 required");
  const hipStream_t s = (hipStream_t)stream;
  // validate the arrays once, through the public call
  gnmpc_status st = gnmpc_condense(p, A, B, c, x0, Q, Q_full, q, R, r, rowC, rowd, H, g, Ct, dt, nullptr, stream);
  if (st != GNMPC_OK) return st;
  struct Cand { int variant, nb; };
  std::vector<Cand> cands{{0, 0}};
  for (int nb = 16; nb >= 1; nb /= 2) {
    if ((st = prop_blocks_build_nb(p, nb)) != GNMPC_OK) return st;
    if (p->pb_nodes != nb) continue;  // blocks of nb nodes do not fit LDS
    cands.push_back({1, nb});
    if (p->pb2_stride > 0) cands.push_back({2, nb});
  }
  hipEvent_t e0, e1;
  GNMPC_HIP_TRY(p, hipEventCreate(&e0));
  GNMPC_HIP_TRY(p, hipEventCreate(&e1));
  rep->count = 0;
  rep->chosen = 0;
  double best = 0.0;
  for (const Cand& cd : cands) {
    if (rep->count == GNMPC_TUNE_MAX) break;
    if (cd.nb > 0 && (st = prop_blocks_build_nb(p, cd.nb)) != GNMPC_OK) break;
    p->prop_pref = cd.variant;
    if ((st = launch_condense(p, A, B, c, x0, Q, Q_full, q, R, r, rowC, rowd, H, g, Ct, dt, nullptr, s)) != GNMPC_OK)
      break;
    (void)hipEventRecord(e0, s);
    for (int t = 0; t < reps && st == GNMPC_OK; ++t)
      st = launch_condense(p, A, B, c, x0, Q, Q_full, q, R, r, rowC, rowd, H, g, Ct, dt, nullptr, s);
    (void)hipEventRecord(e1, s);
    if (st != GNMPC_OK || hipEventSynchronize(e1) != hipSuccess) break;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    gnmpc_tune_entry& en = rep->entry[rep->count];
    en.variant = cd.variant;
    en.block_nodes = cd.nb;
    en.us = 1e3 * ms / reps;
    if (rep->count == 0 || en.us < best) {
      best = en.us;
      rep->chosen = rep->count;
    }
    ++rep->count;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // keep the fastest (also after a failure part-way, so the plan stays usable)
  if (rep->count > 0) {
    const gnmpc_tune_entry& ch = rep->entry[rep->chosen];
    const gnmpc_status sb = prop_blocks_build_nb(p, ch.block_nodes > 0 ? ch.block_nodes : 4);
    p->prop_pref = ch.variant;
    if (st == GNMPC_OK) st = sb;
  } else {
    p->prop_pref = -1;
    const gnmpc_status sb = prop_blocks_build(p);
    if (st == GNMPC_OK) st = sb;
  }
  return st;
}

gnmpc_status gnmpc_solve_box_qp(gnmpc_plan* p, int32_t n, const void* H, const void* g, const void* lb,
                                const void* ub, int32_t n_c, const void* Ct, const void* lc, const void* uc,
                                const gnmpc_admm_settings* st, void* u, gnmpc_qp_info* info, void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (const gnmpc_status cs = qp_check(p, n, H, g, lb, ub, n_c, Ct, st, u); cs != GNMPC_OK) return cs;
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  return launch_qp(p, n, H, g, lb, ub, n_c, Ct, lc, uc, st, u, info, (hipStream_t)stream);
}

gnmpc_status gnmpc_solve_qp_ipm(gnmpc_plan* p, int32_t n, const void* H, const void* g, const void* lb,
                                const void* ub, int32_t n_c, const void* Ct, const void* lc, const void* uc, double tol,
                                int32_t max_iter, void* u, gnmpc_qp_info* info, void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (!H || !g || !lb || !ub || !u) return fail(p, GNMPC_INVALID_ARG, "solve_qp_ipm: null array");
  if (n <= 0 || n > p->dims.N * p->dims.nu) return fail(p, GNMPC_SHAPE, "solve_qp_ipm: n outside 1..N*nu");
  if (n_c < 0 || n_c > p->dims.n_c_max) return fail(p, GNMPC_SHAPE, "solve_qp_ipm: n_c outside 0..n_c_max");
  if (n_c > 0 && !Ct) return fail(p, GNMPC_INVALID_ARG, "solve_qp_ipm: Ct is null");
  if (!(tol > 0) || max_iter < 1) return fail(p, GNMPC_INVALID_ARG, "solve_qp_ipm: tol > 0 and max_iter >= 1");
  if (qp_ipm_check(n, n_c) != GNMPC_OK) return fail(p, GNMPC_UNSUPPORTED, "solve_qp_ipm: too large for one workgroup");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  return launch_qp_ipm(p, n, H, g, lb, ub, n_c, Ct, lc, uc, tol, max_iter, u, info, (hipStream_t)stream);
}

gnmpc_status gnmpc_solve_box_qp_noalloc(int32_t dtype, int32_t n, const void* H, const void* g, const void* lb,
                                        const void* ub, int32_t n_c, const void* Ct, const void* lc, const void* uc,
                                        const gnmpc_admm_settings* st, void* u, gnmpc_qp_info* info, void* stream) {
  if (dtype != GNMPC_F32 && dtype != GNMPC_F64) return GNMPC_INVALID_ARG;
  if (!H || !g || !lb || !ub || !u || !st) return GNMPC_INVALID_ARG;
  if (n_c > 0 && !Ct) return GNMPC_INVALID_ARG;
  if (const gnmpc_status cs = qp_noalloc_check(dtype, n, n_c); cs != GNMPC_OK) return cs;
  if (!(st->rho > 0) || !(st->sigma > 0) || !(st->alpha > 0 && st->alpha < 2) || !(st->eps_abs >= 0) ||
      !(st->eps_rel >= 0) || st->max_iter < 1 || st->check_every < 1 || !(st->kappa_fp64 > 0))
    return GNMPC_INVALID_ARG;
  return launch_qp_noalloc(dtype, n, H, g, lb, ub, n_c, Ct, lc, uc, st, u, info, (hipStream_t)stream);
}

gnmpc_status gnmpc_jvp(gnmpc_plan* p, const void* A, const void* B, const void* dx, const void* du, void* out,
                       void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (!A || !B || !dx || !du || !out) return fail(p, GNMPC_INVALID_ARG, "jvp: null array");
  if (!p->graph_ready) return fail(p, GNMPC_NOT_READY, "jvp: graph must be set");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  return launch_jvp(p, A, B, dx, du, out, (hipStream_t)stream);
}

gnmpc_status gnmpc_vjp(gnmpc_plan* p, const void* A, const void* B, const void* g, void* gx, void* gu,
                       void* stream) {
  if (!p) return GNMPC_INVALID_ARG;
  if (!A || !B || !g || !gx || !gu) return fail(p, GNMPC_INVALID_ARG, "vjp: null array");
  if (!p->graph_ready) return fail(p, GNMPC_NOT_READY, "vjp: graph must be set");
  GNMPC_HIP_TRY(p, hipSetDevice(p->device));
  return launch_vjp(p, A, B, g, gx, gu, (hipStream_t)stream);
}

// Library streams of the batched step, per device, created once (default priority).
constexpr int kBatchStreams = 4;
struct BatchStreams {
  bool ready = false;
  hipStream_t s[kBatchStreams];
  hipEvent_t fork, join[kBatchStreams];
};

gnmpc_status gnmpc_step_batched(const gnmpc_step_desc* descs, int32_t count, const gnmpc_admm_settings* st,
                                void* stream) {
  static std::mutex mu;
  static BatchStreams pool[64];
  if (!descs || count < 0 || !st) return GNMPC_INVALID_ARG;
  if (count == 0) return GNMPC_OK;
  for (int32_t i = 0; i < count; ++i)
    if (!descs[i].plan) return GNMPC_INVALID_ARG;
  const int dev = descs[0].plan->device;
  for (int32_t i = 1; i < count; ++i)
    if (descs[i].plan->device != dev) return fail(descs[i].plan, GNMPC_INVALID_ARG, "step_batched: plans on different devices");
  // a plan's workspace serves one instance at a time: a repeated plan would race with itself
  {
    std::vector<const gnmpc_plan*> seen(count);
    for (int32_t i = 0; i < count; ++i) seen[i] = descs[i].plan;
    std::sort(seen.begin(), seen.end());
    for (int32_t i = 1; i < count; ++i)
      if (seen[i] == seen[i - 1])
        return fail(const_cast<gnmpc_plan*>(seen[i]), GNMPC_INVALID_ARG, "step_batched: a plan appears in two descriptors");
  }
  if (dev < 0 || dev >= 64) return GNMPC_INVALID_ARG;
  gnmpc_plan* p0 = descs[0].plan;
  GNMPC_HIP_TRY(p0, hipSetDevice(dev));
  BatchStreams& bs = pool[dev];
  // The fork and join events of a device are shared by every call, so one call's
  // record-then-wait sequence must not interleave with another's: the whole
  // enqueue runs under the lock (enqueueing does not wait for the GPU).
  std::lock_guard<std::mutex> lock(mu);
  if (!bs.ready) {
    for (int t = 0; t < kBatchStreams; ++t) {
      GNMPC_HIP_TRY(p0, hipStreamCreateWithFlags(&bs.s[t], hipStreamNonBlocking));
      GNMPC_HIP_TRY(p0, hipEventCreateWithFlags(&bs.join[t], hipEventDisableTiming));
    }
    GNMPC_HIP_TRY(p0, hipEventCreateWithFlags(&bs.fork, hipEventDisableTiming));
    bs.ready = true;
  }
  const hipStream_t caller = (hipStream_t)stream;
  const int used = std::min<int32_t>(count, kBatchStreams);
  GNMPC_HIP_TRY(p0, hipEventRecord(bs.fork, caller));
  for (int t = 0; t < used; ++t) GNMPC_HIP_TRY(p0, hipStreamWaitEvent(bs.s[t], bs.fork, 0));
  gnmpc_status first = GNMPC_OK;
  std::vector<QpPrepared> prepared(count);
  for (int32_t i = 0; i < count && first == GNMPC_OK; ++i) {
    const gnmpc_step_desc& d = descs[i];
    gnmpc_plan* p = d.plan;
    void* si = (void*)bs.s[i % kBatchStreams];
    const int32_t n = p->dims.N * p->dims.nu;
    gnmpc_status s = gnmpc_linearize(p, d.xhat, d.uhat, d.A, d.B, d.c, nullptr, nullptr, si);
    if (s == GNMPC_OK)
      s = gnmpc_condense(p, d.A, d.B, d.c, d.x0, d.Q, d.Q_full, d.q, d.R, d.r, d.rowC, d.rowd, d.H, d.g, d.Ct,
                         d.dt, nullptr, si);
    if (s == GNMPC_OK) s = qp_check(p, n, d.H, d.g, d.lb, d.ub, p->n_c, d.Ct, st, d.u);
    if (s == GNMPC_OK)
      s = launch_qp_prep(p, n, d.H, d.g, d.lb, d.ub, p->n_c, d.Ct, d.lc, d.uc, st, d.u, d.info, (hipStream_t)si,
                         &prepared[i]);
    first = s;
  }
  // join every forked stream, also after an error
  for (int t = 0; t < used; ++t) {
    GNMPC_HIP_TRY(p0, hipEventRecord(bs.join[t], bs.s[t]));
    GNMPC_HIP_TRY(p0, hipStreamWaitEvent(caller, bs.join[t], 0));
  }
  if (first != GNMPC_OK) return first;
  // every instance's QP in one launch per pass (one workgroup each) on the caller's stream
  const gnmpc_status qs = launch_qp_batched(prepared.data(), count, caller);
  if (qs != GNMPC_OK) return fail(p0, qs, "step_batched: batched QP launch failed");
  return GNMPC_OK;
}

// Algorithm 1's iteration around a QP solve (ADMM or interior point, `qp`).
extern "C++" {
template <typename QpFn>
static gnmpc_status rti_iteration(const gnmpc_step_desc* d, void* xpred, void* xhat_next, void* uhat_next, QpFn qp,
                                  void* stream) {
  gnmpc_plan* p = d->plan;
  if (!xpred || !xhat_next || !uhat_next) return fail(p, GNMPC_INVALID_ARG, "rti_step: null array");
  if (xpred == xhat_next || xpred == d->xhat || xpred == d->x0)
    return fail(p, GNMPC_INVALID_ARG, "rti_step: xpred aliases an input or xhat_next");
  gnmpc_status s = gnmpc_linearize(p, d->xhat, d->uhat, d->A, d->B, d->c, nullptr, nullptr, stream);
  if (s == GNMPC_OK)
    s = gnmpc_condense(p, d->A, d->B, d->c, d->x0, d->Q, d->Q_full, d->q, d->R, d->r, d->rowC, d->rowd, d->H,
                       d->g, d->Ct, d->dt, nullptr, stream);
  if (s == GNMPC_OK) s = qp(p->dims.N * p->dims.nu);
  if (s == GNMPC_OK) s = gnmpc_rollout_linear(p, d->A, d->B, d->c, d->x0, d->u, xpred, stream);
  if (s == GNMPC_OK) s = launch_rti_shift(p, xpred, d->u, xhat_next, uhat_next, (hipStream_t)stream);
  return s;
}
}  // extern "C++"

gnmpc_status gnmpc_rti_step(const gnmpc_step_desc* d, void* xpred, void* xhat_next, void* uhat_next,
                            const gnmpc_admm_settings* st, void* stream) {
  if (!d || !d->plan || !st) return GNMPC_INVALID_ARG;
  gnmpc_plan* p = d->plan;
  return rti_iteration(d, xpred, xhat_next, uhat_next, [&](int32_t n) {
    return gnmpc_solve_box_qp(p, n, d->H, d->g, d->lb, d->ub, p->n_c, d->Ct, d->lc, d->uc, st, d->u, d->info,
                              stream);
  }, stream);
}

gnmpc_status gnmpc_rti_step_ipm(const gnmpc_step_desc* d, void* xpred, void* xhat_next, void* uhat_next, double tol,
                                int32_t max_iter, void* stream) {
  if (!d || !d->plan) return GNMPC_INVALID_ARG;
  gnmpc_plan* p = d->plan;
  if (!(tol > 0) || max_iter < 1) return fail(p, GNMPC_INVALID_ARG, "rti_step_ipm: tol > 0 and max_iter >= 1");
  return rti_iteration(d, xpred, xhat_next, uhat_next, [&](int32_t n) {
    return gnmpc_solve_qp_ipm(p, n, d->H, d->g, d->lb, d->ub, p->n_c, d->Ct, d->lc, d->uc, tol, max_iter, d->u,
                              d->info, stream);
  }, stream);
}

}  // extern "C"
