// Training objective of the plan's GNN and its gradient (Sec. V-A "Training"):
//   L(theta) = 1/S sum_t || x_{t+1} - F_theta(x_t, u_t) ||_O^2 + lambda ||theta||^2
// over the S = N samples of one call (the plan's horizon is the batch), O
// diagonal (one weight per state component), theta every weight and bias in the
// packing of gnmpc_model_set_gnn, as FP32 on the device.  Reverse mode written
// out layer by layer, FP32 throughout:
//   forward     encoder, L rounds (edge messages and node updates) and the decoder
//               per (sample, node), keeping h_l, the sums of messages and the
//               messages (their signs are the edge ReLU masks);
//   decoder     dL/dF = 2 O (F - x+) / S, through p+ = p + dt v+ and
//               v+ = v + dt o[3:6] to o and to h_L;
//   each round  node MLP: z = gh * (h > 0), then W_n' z; edge MLP per in-edge:
//               e = (cotangent of the message sum) * (m > 0), W_e' e split into
//               the parts of h_i and of (h_i - h_j); the sender's part is
//               gathered per node over its out-edges in a fixed order;
//   weights     every layer's gradient is sum over rows (sample, node or edge) of
//               cotangent x input: split-K over fixed row chunks, the chunks then
//               summed in order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "gnn_state.hpp"

namespace gnmpc {
namespace {

constexpr int kTrainChunk = 512;  // rows per split-K chunk of the weight gradients
constexpr int kRedThreads = 256;

struct TrainLayout {
  int Hd, L, S, M, E, nu;
  long n_w;
  // offsets of theta's blocks (elements)
  long o_Wenc, o_benc, o_We[16], o_be[16], o_Wn[16], o_bn[16], o_Wdec, o_bdec;
  // workspace offsets (floats)
  size_t w_t, h, agg, msg, ghA, ghB, ghP, zb, eb, q, od, lossb, erecv, part;
  size_t part_elems, total;
};

TrainLayout train_layout(const GnnState& g, int S) {
  TrainLayout t{};
  t.Hd = g.Hd;
  t.L = g.L;
  t.S = S;
  t.M = g.M;
  t.E = g.E;
  const long Hd = g.Hd;
  long o = 0;
  t.o_Wenc = o;
  o += Hd * 9;
  t.o_benc = o;
  o += Hd;
  for (int l = 0; l < g.L; ++l) {
    t.o_We[l] = o;
    o += Hd * 2 * Hd;
    t.o_be[l] = o;
    o += Hd;
    t.o_Wn[l] = o;
    o += Hd * 2 * Hd;
    t.o_bn[l] = o;
    o += Hd;
  }
  t.o_Wdec = o;
  o += 6 * Hd;
  t.o_bdec = o;
  o += 6;
  t.n_w = o;
  const size_t SM = (size_t)S * g.M, SE = (size_t)S * g.E;
  size_t w = 0;
  auto take = [&](size_t n) {
    const size_t at = w;
    w += (n + 63) / 64 * 64;
    return at;
  };
  t.w_t = take((size_t)o);
  t.h = take((size_t)(g.L + 1) * SM * Hd);
  t.agg = take((size_t)g.L * SM * Hd);
  t.msg = take((size_t)g.L * SE * Hd);
  t.ghA = take(SM * Hd);
  t.ghB = take(SM * Hd);
  t.ghP = take(SM * Hd);
  t.zb = take(SM * Hd);
  t.eb = take(SE * Hd);
  t.q = take(SE * Hd);
  t.od = take(SM * 6);
  t.lossb = take(SM + 1);
  t.erecv = take((size_t)g.E + 1);  // receiver of every edge (int32 stored in the float slots)
  const size_t rows = std::max(SM, SE);
  const size_t chunks = (rows + kTrainChunk - 1) / kTrainChunk;
  t.part_elems = chunks * (size_t)Hd * (2 * Hd + 1);
  t.part = take(t.part_elems);
  t.total = w;
  return t;
}

struct TrainArgs {
  TrainLayout t;
  float dt, lambda;
  float O[6];
  const float* theta;
  const float* x;   // [S][M][6]
  const float* u;   // [S][nu]
  const float* xn;  // [S][M][6]
  const int32_t *row_ptr, *col, *act_of_node, *out_ptr, *out_edge;
  float* ws;
  float* grad;
  float* loss;
};

// transposed copy of every matrix of theta (W [out][in] -> [in][out]); biases copied
__global__ void train_transpose_kernel(TrainArgs a, int out, int in, long off) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)out * in) return;
  const int o = (int)(t / in), c = (int)(t % in);
  a.ws[a.t.w_t + off + (size_t)c * out + o] = a.theta[off + t];
}

// receiver of every edge (its CSR row), one thread per node row
__global__ void train_erecv_kernel(TrainArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.t.M) return;
  int32_t* er = reinterpret_cast<int32_t*>(a.ws + a.t.erecv);
  for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) er[e] = i;
}

__global__ void train_zero_kernel(float* p, long n) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0.f;
}

__device__ inline float relu(float z) { return z > 0.f ? z : 0.f; }

// node input [x^i; P^i u]
__device__ inline float enc_input(const TrainArgs& a, int s, int i, int c) {
  if (c < NBX) return a.x[((size_t)s * a.t.M + i) * NBX + c];
  const int act = a.act_of_node[i];
  return act >= 0 ? a.u[(size_t)s * a.t.nu + 3 * act + (c - NBX)] : 0.f;
}

// ---- forward: one workgroup of Hd lanes per (sample, node)
__global__ void train_fwd_enc_kernel(TrainArgs a) {
  const int s = blockIdx.x / a.t.M, i = blockIdx.x % a.t.M, f = threadIdx.x, Hd = a.t.Hd;
  const float* Wt = a.ws + a.t.w_t + a.t.o_Wenc;  // [9][Hd]
  float z = a.theta[a.t.o_benc + f];
  for (int c = 0; c < 9; ++c) z += Wt[c * Hd + f] * enc_input(a, s, i, c);
  a.ws[a.t.h + ((size_t)s * a.t.M + i) * Hd + f] = relu(z);
}

__global__ void train_fwd_layer_kernel(TrainArgs a, int l) {
  extern __shared__ float tsm[];
  const int Hd = a.t.Hd, M = a.t.M, E = a.t.E;
  const int s = blockIdx.x / M, i = blockIdx.x % M, f = threadIdx.x;
  const size_t SM = (size_t)a.t.S * M;
  float* hi = tsm;          // [Hd]
  float* vin = tsm + Hd;    // [2 Hd]
  const float* h = a.ws + a.t.h + (size_t)l * SM * Hd + (size_t)s * M * Hd;
  hi[f] = h[(size_t)i * Hd + f];
  __syncthreads();
  const float* Wte = a.ws + a.t.w_t + a.t.o_We[l];  // [2 Hd][Hd]
  const float* Wtn = a.ws + a.t.w_t + a.t.o_Wn[l];
  float agg = 0.f;
  for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) {
    const int j = a.col[e];
    vin[f] = hi[f];
    vin[Hd + f] = hi[f] - h[(size_t)j * Hd + f];
    __syncthreads();
    float z = a.theta[a.t.o_be[l] + f];
    for (int c = 0; c < 2 * Hd; ++c) z += Wte[(size_t)c * Hd + f] * vin[c];
    const float m = relu(z);
    a.ws[a.t.msg + ((size_t)l * a.t.S + s) * E * Hd + (size_t)e * Hd + f] = m;
    agg += m;
    __syncthreads();
  }
  vin[f] = hi[f];
  vin[Hd + f] = agg;
  a.ws[a.t.agg + (size_t)l * SM * Hd + ((size_t)s * M + i) * Hd + f] = agg;
  __syncthreads();
  float z = a.theta[a.t.o_bn[l] + f];
  for (int c = 0; c < 2 * Hd; ++c) z += Wtn[(size_t)c * Hd + f] * vin[c];
  a.ws[a.t.h + (size_t)(l + 1) * SM * Hd + ((size_t)s * M + i) * Hd + f] = relu(z);
}

// decoder, loss term and the cotangent of h_L: one workgroup of Hd lanes per (sample, node)
__global__ void train_dec_kernel(TrainArgs a) {
  extern __shared__ float tsm[];
  const int Hd = a.t.Hd, M = a.t.M;
  const int s = blockIdx.x / M, i = blockIdx.x % M, f = threadIdx.x;
  const size_t row = (size_t)s * M + i, SM = (size_t)a.t.S * M;
  const float hL = a.ws[a.t.h + (size_t)a.t.L * SM * Hd + row * Hd + f];
  float* red = tsm;  // [3][Hd]
  const float* Wd = a.theta + a.t.o_Wdec;  // [6][Hd]
  for (int r = 0; r < 3; ++r) red[r * Hd + f] = Wd[(size_t)(3 + r) * Hd + f] * hL;
  __syncthreads();
  int p2 = 1;  // fold to a power of two first (Hd = 192), then halve: a fixed order
  while (2 * p2 <= Hd) p2 *= 2;
  if (f < Hd - p2)
    for (int r = 0; r < 3; ++r) red[r * Hd + f] += red[r * Hd + f + p2];
  __syncthreads();
  for (int hw = p2 / 2; hw > 0; hw >>= 1) {
    if (f < hw)
      for (int r = 0; r < 3; ++r) red[r * Hd + f] += red[r * Hd + f + hw];
    __syncthreads();
  }
  __shared__ float go[6];
  if (f == 0) {
    const float* x = a.x + row * NBX;
    const float* xn = a.xn + row * NBX;
    float F[6];
    for (int r = 0; r < 3; ++r) {
      const float o = red[r * Hd] + a.theta[a.t.o_bdec + 3 + r];
      const float vn = x[3 + r] + a.dt * o;
      F[3 + r] = vn;
      F[r] = x[r] + a.dt * vn;
    }
    float lsum = 0.f;
    float gF[6];
    for (int c = 0; c < 6; ++c) {
      const float rr = F[c] - xn[c];
      lsum += a.O[c] * rr * rr;
      gF[c] = 2.f * a.O[c] * rr / (float)a.t.S;
    }
    a.ws[a.t.lossb + row] = lsum / (float)a.t.S;
    for (int r = 0; r < 3; ++r) {
      go[r] = 0.f;
      go[3 + r] = a.dt * (gF[3 + r] + a.dt * gF[r]);
    }
    for (int c = 0; c < 6; ++c) a.ws[a.t.od + row * 6 + c] = go[c];
  }
  __syncthreads();
  float gh = 0.f;
  for (int r = 3; r < 6; ++r) gh += Wd[(size_t)r * Hd + f] * go[r];
  a.ws[a.t.ghA + row * Hd + f] = gh;
}

// one round backwards, per (sample, node i): node MLP, then the edge MLP of each
// in-edge; writes the node's partial cotangent of h_l (its own terms) and, per
// edge, the sender's term q
__global__ void train_bwd_node_kernel(TrainArgs a, int l, const float* gh_in) {
  extern __shared__ float tsm[];
  const int Hd = a.t.Hd, M = a.t.M, E = a.t.E;
  const int s = blockIdx.x / M, i = blockIdx.x % M, f = threadIdx.x;
  const size_t row = (size_t)s * M + i, SM = (size_t)a.t.S * M;
  float* zs = tsm;       // [Hd] node pre-activation cotangent
  float* ga = tsm + Hd;  // [Hd] cotangent of the message sum
  float* es = ga + Hd;   // [Hd] edge pre-activation cotangent
  const float hnext = a.ws[a.t.h + (size_t)(l + 1) * SM * Hd + row * Hd + f];
  const float z = hnext > 0.f ? gh_in[row * Hd + f] : 0.f;
  zs[f] = z;
  a.ws[a.t.zb + row * Hd + f] = z;
  __syncthreads();
  const float* Wn = a.theta + a.t.o_Wn[l];  // [Hd][2 Hd]
  const float* We = a.theta + a.t.o_We[l];
  float gh = 0.f, gagg = 0.f;
  for (int o = 0; o < Hd; ++o) {
    gh += Wn[(size_t)o * 2 * Hd + f] * zs[o];
    gagg += Wn[(size_t)o * 2 * Hd + Hd + f] * zs[o];
  }
  ga[f] = gagg;
  __syncthreads();
  for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) {
    const size_t er = ((size_t)s * E + e) * Hd;
    const float m = a.ws[a.t.msg + (size_t)l * a.t.S * E * Hd + er + f];
    const float ev = m > 0.f ? ga[f] : 0.f;
    es[f] = ev;
    a.ws[a.t.eb + er + f] = ev;
    __syncthreads();
    float ai = 0.f, bj = 0.f;
    for (int o = 0; o < Hd; ++o) {
      ai += We[(size_t)o * 2 * Hd + f] * es[o];
      bj += We[(size_t)o * 2 * Hd + Hd + f] * es[o];
    }
    gh += ai + bj;
    a.ws[a.t.q + er + f] = bj;
    __syncthreads();
  }
  a.ws[a.t.ghP + row * Hd + f] = gh;
}

// cotangent of h_l for node j: its own terms minus the sender terms of its
// out-edges, in out-edge order
__global__ void train_bwd_gather_kernel(TrainArgs a, float* gh_out) {
  const int Hd = a.t.Hd, M = a.t.M, E = a.t.E;
  const int s = blockIdx.x / M, j = blockIdx.x % M, f = threadIdx.x;
  const size_t row = (size_t)s * M + j;
  float v = a.ws[a.t.ghP + row * Hd + f];
  for (int q = a.out_ptr[j]; q < a.out_ptr[j + 1]; ++q) v -= a.ws[a.t.q + ((size_t)s * E + a.out_edge[q]) * Hd + f];
  gh_out[row * Hd + f] = v;
}

__global__ void train_bwd_enc_kernel(TrainArgs a, const float* gh_in) {
  const int Hd = a.t.Hd, M = a.t.M;
  const size_t row = blockIdx.x;
  const int f = threadIdx.x;
  const float h0 = a.ws[a.t.h + row * Hd + f];
  a.ws[a.t.zb + row * Hd + f] = h0 > 0.f ? gh_in[row * Hd + f] : 0.f;
  (void)M;
}

// Weight gradient of one layer, split-K partials: workgroup (output f, chunk),
// lane c < nin + 1 (c = nin is the bias) sums Z[r][f] X[r][c] over the chunk's
// rows.  kind 0: X = [h_l; agg] (node rows), 1: X = [h_i; h_i - h_j] (edge
// rows), 2: X = h_L (decoder), 3: X = [x^i; P^i u] (encoder).
__global__ void train_wgrad_kernel(TrainArgs a, int kind, int l, const float* Z, int zstride, int R, int nout,
                                   int nin) {
  const int f = blockIdx.x, chunk = blockIdx.y;
  const int Hd = a.t.Hd, M = a.t.M, E = a.t.E;
  const size_t SM = (size_t)a.t.S * M;
  const int r0 = chunk * kTrainChunk, r1 = min(R, r0 + kTrainChunk);
  for (int c = threadIdx.x; c <= nin; c += kRedThreads) {
    float acc = 0.f;
    for (int r = r0; r < r1; ++r) {
      const float zv = Z[(size_t)r * zstride + f];
      float xv = 1.f;
      if (c < nin) {
        if (kind == 0) {
          xv = c < Hd ? a.ws[a.t.h + (size_t)l * SM * Hd + (size_t)r * Hd + c]
                      : a.ws[a.t.agg + (size_t)l * SM * Hd + (size_t)r * Hd + (c - Hd)];
        } else if (kind == 1) {
          const int s = r / E, e = r - s * E;
          const int recv = reinterpret_cast<const int32_t*>(a.ws + a.t.erecv)[e];
          const float* h = a.ws + a.t.h + (size_t)l * SM * Hd + (size_t)s * M * Hd;
          const float hi_c = h[(size_t)recv * Hd + (c < Hd ? c : c - Hd)];
          xv = c < Hd ? hi_c : hi_c - h[(size_t)a.col[e] * Hd + (c - Hd)];
        } else if (kind == 2) {
          xv = a.ws[a.t.h + (size_t)a.t.L * SM * Hd + (size_t)r * Hd + c];
        } else {
          xv = enc_input(a, r / M, r % M, c);
        }
      }
      acc += zv * xv;
    }
    a.ws[a.t.part + ((size_t)chunk * nout + f) * (nin + 1) + c] = acc;
  }
}

// sum the chunks in order: grad[oW + f nin + c], grad[ob + f]
__global__ void train_wgrad_reduce_kernel(TrainArgs a, int nchunk, int nout, int nin, long oW, long ob) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nout * (nin + 1)) return;
  const int f = (int)(t / (nin + 1)), c = (int)(t % (nin + 1));
  float v = 0.f;
  for (int k = 0; k < nchunk; ++k) v += a.ws[a.t.part + ((size_t)k * nout + f) * (nin + 1) + c];
  if (c < nin) a.grad[oW + (long)f * nin + c] = v;
  else a.grad[ob + f] = v;
}

// penalty and loss: grad += 2 lambda theta; loss = sum of the data terms (in
// order) + lambda ||theta||^2, one workgroup
__global__ void __launch_bounds__(kRedThreads) train_finish_kernel(TrainArgs a) {
  __shared__ float red[kRedThreads];
  const size_t SM = (size_t)a.t.S * a.t.M;
  float dsum = 0.f, psum = 0.f;
  for (size_t r = threadIdx.x; r < SM; r += kRedThreads) dsum += a.ws[a.t.lossb + r];
  for (long t = threadIdx.x; t < a.t.n_w; t += kRedThreads) {
    const float th = a.theta[t];
    psum += th * th;
    a.grad[t] += 2.f * a.lambda * th;
  }
  red[threadIdx.x] = dsum + a.lambda * psum;
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *a.loss = red[0];
}

__global__ void adam_kernel(long n, float* theta, const float* g, float* m, float* v, float lr, float b1, float b2,
                            float c1, float c2, float eps) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float mt = b1 * m[t] + (1.f - b1) * g[t];
  const float vt = b2 * v[t] + (1.f - b2) * g[t] * g[t];
  m[t] = mt;
  v[t] = vt;
  theta[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

}  // namespace

size_t gnn_train_workspace_bytes(const gnmpc_plan* p) {
  return train_layout(*p->gnn, p->dims.N).total * sizeof(float);
}

long gnn_param_count(const gnmpc_plan* p) { return train_layout(*p->gnn, p->dims.N).n_w; }

gnmpc_status launch_gnn_loss_grad(gnmpc_plan* p, const float* theta, const void* x, const void* u, const void* xn,
                                  const float* O, double lambda, void* ws, float* loss, float* grad, hipStream_t s) {
  const GnnState& g = *p->gnn;
  TrainArgs a;
  a.t = train_layout(g, p->dims.N);
  a.t.nu = p->dims.nu;
  a.dt = g.dt;
  a.lambda = (float)lambda;
  for (int c = 0; c < 6; ++c) a.O[c] = O[c];
  a.theta = theta;
  a.x = (const float*)x;
  a.u = (const float*)u;
  a.xn = (const float*)xn;
  a.row_ptr = p->d_row_ptr;
  a.col = p->d_col;
  a.act_of_node = p->d_act_of_node;
  a.out_ptr = g.out_ptr;
  a.out_edge = g.out_edge;
  a.ws = (float*)ws;
  a.grad = grad;
  a.loss = loss;
  const TrainLayout& t = a.t;
  const int Hd = t.Hd, S = t.S, M = t.M, E = t.E, L = t.L;
  const int SM = S * M, SE = S * E;
  // transposed matrices for the forward pass
  auto tr = [&](int out, int in, long off) {
    train_transpose_kernel<<<ceil_div((long)out * in, 256), 256, 0, s>>>(a, out, in, off);
  };
  tr(Hd, 9, t.o_Wenc);
  for (int l = 0; l < L; ++l) {
    tr(Hd, 2 * Hd, t.o_We[l]);
    tr(Hd, 2 * Hd, t.o_Wn[l]);
  }
  train_erecv_kernel<<<ceil_div(M, 256), 256, 0, s>>>(a);
  // forward
  train_fwd_enc_kernel<<<SM, Hd, 0, s>>>(a);
  for (int l = 0; l < L; ++l) train_fwd_layer_kernel<<<SM, Hd, 3 * Hd * sizeof(float), s>>>(a, l);
  train_dec_kernel<<<SM, Hd, 3 * Hd * sizeof(float), s>>>(a);
  // weight gradients of the decoder
  auto wgrad = [&](int kind, int l, const float* Z, int zstride, int R, int nout, int nin, long oW, long ob) {
    const int nch = ceil_div(R, kTrainChunk);
    train_wgrad_kernel<<<dim3(nout, nch), kRedThreads, 0, s>>>(a, kind, l, Z, zstride, R, nout, nin);
    train_wgrad_reduce_kernel<<<ceil_div((long)nout * (nin + 1), 256), 256, 0, s>>>(a, nch, nout, nin, oW, ob);
  };
  const float* ws_f = a.ws;
  wgrad(2, 0, ws_f + t.od, 6, SM, 6, Hd, t.o_Wdec, t.o_bdec);
  // rounds backwards
  float* gh_in = a.ws + t.ghA;
  float* gh_out = a.ws + t.ghB;
  for (int l = L - 1; l >= 0; --l) {
    train_bwd_node_kernel<<<SM, Hd, 3 * Hd * sizeof(float), s>>>(a, l, gh_in);
    wgrad(0, l, ws_f + t.zb, Hd, SM, Hd, 2 * Hd, t.o_Wn[l], t.o_bn[l]);
    if (E > 0) wgrad(1, l, ws_f + t.eb, Hd, SE, Hd, 2 * Hd, t.o_We[l], t.o_be[l]);
    else  // no edges: the edge weights get only the penalty below
      train_zero_kernel<<<ceil_div((long)Hd * 2 * Hd + Hd, 256), 256, 0, s>>>(a.grad + t.o_We[l],
                                                                            (long)Hd * 2 * Hd + Hd);
    train_bwd_gather_kernel<<<SM, Hd, 0, s>>>(a, gh_out);
    std::swap(gh_in, gh_out);
  }
  train_bwd_enc_kernel<<<SM, Hd, 0, s>>>(a, gh_in);
  wgrad(3, 0, ws_f + t.zb, Hd, SM, Hd, 9, t.o_Wenc, t.o_benc);
  train_finish_kernel<<<1, kRedThreads, 0, s>>>(a);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

gnmpc_status launch_adam(long n, float* theta, const float* grad, float* m, float* v, int step, double lr,
                         double beta1, double beta2, double eps, hipStream_t s) {
  const float c1 = (float)(1.0 - std::pow(beta1, step)), c2 = (float)(1.0 - std::pow(beta2, step));
  adam_kernel<<<ceil_div(n, 256), 256, 0, s>>>(n, theta, grad, m, v, (float)lr, (float)beta1, (float)beta2, c1, c2,
                                               (float)eps);
  return hipGetLastError() == hipSuccess ? GNMPC_OK : GNMPC_HIP_ERROR;
}

}  // namespace gnmpc
