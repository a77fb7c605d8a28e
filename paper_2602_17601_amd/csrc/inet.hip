// The paper's own dynamics model, an interaction network with a global input
// (Sec. V-A eq. forward_dynamics): with e^{ij} = x^i - x^j and
// a^i = sum_{j in N_i} psi(e^{ij}),
//   v^i+ = v^i + phi([x^i; a^i; u]),   p^i+ = p^i + dt v^i+,
// psi and phi being MLPs with a ReLU after every layer but the last, and its
// linearization (Sec. V-A "Linearization", eq. linearized_dynamics; ReLU
// subgradient 0 at the kink):
//   d v^i+ / d x^j = -G J_psi(e^{ij})                     (j in N_i)
//   d v^i+ / d x^i = [0 I] + J_x + G sum_j J_psi(e^{ij})
//   d v^i+ / d u   = J_u,   d p^i+ / d . = dt d v^i+ / d . (+ [I 0] for x^i)
// where [J_x, G, J_u] = d phi / d [x^i; a^i; u] (3 rows).
//
// One workgroup per (stage, node): psi forward over the in-edges (messages
// summed), phi forward keeping its layer outputs, phi in reverse mode with the
// three output rows as cotangents (the 3 x (6 + d_m + n_u) Jacobian), then per
// in-edge psi again, in reverse mode with the three rows of G as cotangents,
// which gives G J_psi(e^{ij}) directly.  The small matrices of the paper's
// robot (4 nodes, psi 4 x 50, phi 8 x 250) make this latency-bound; every
// workgroup reads the weights from L2 (the forward layers from a transposed
// copy, so a wave reads consecutive words in both directions).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "plan.hpp"

struct InetState {
  int n_psi = 0, n_phi = 0;  // linear layers of psi and phi
  int d_m = 0, nu = 0, in_phi = 0;
  double dt = 0.0;
  int psi_in[gnmpc::kInetMaxLayers], psi_out[gnmpc::kInetMaxLayers];
  int phi_in[gnmpc::kInetMaxLayers], phi_out[gnmpc::kInetMaxLayers];
  long psi_W[gnmpc::kInetMaxLayers], psi_b[gnmpc::kInetMaxLayers];
  long phi_W[gnmpc::kInetMaxLayers], phi_b[gnmpc::kInetMaxLayers];
  int psi_act = 0, phi_act = 0;  // values of all hidden-layer outputs
  long n_w = 0;                  // packed weights; then a copy with every matrix transposed
  void* w = nullptr;             // both, in the plan dtype
};

namespace gnmpc {
namespace {

constexpr int kInetThreads = 256;
constexpr int kInMax = 6 + kInetMaxWidth + kInetMaxNu;  // widest phi input
constexpr int kWMax = kInetMaxWidth;                    // widest psi layer

template <typename T>
struct InetArgs {
  int N, M, nu, n_psi, n_phi, d_m, in_phi, psi_act, phi_act;
  long nnz, wt_off;  // the transposed copy of every matrix starts wt_off elements in
  T dt;
  int psi_in[kInetMaxLayers], psi_out[kInetMaxLayers], phi_in[kInetMaxLayers], phi_out[kInetMaxLayers];
  long psi_W[kInetMaxLayers], psi_b[kInetMaxLayers], phi_W[kInetMaxLayers], phi_b[kInetMaxLayers];
  const T* w;
  const int32_t *row_ptr, *col, *prow, *pcol;
  const T *xhat, *uhat;
  T *A, *B, *c, *fnext;
};

// LDS of one workgroup, in elements of T.
__host__ __device__ constexpr size_t inet_lds_elems(int psi_act, int phi_act) {
  return 32 + kWMax + kInMax + 3 * 3 * (size_t)kInMax + 2 * 3 * (size_t)kWMax + (size_t)kMaxWidth * 18 +
         (size_t)psi_act + (size_t)phi_act;
}

// out = W in + b (then ReLU if relu), one output per thread; Wt is W transposed,
// [nin][nout], so the threads of a wave read consecutive words, and the loop is
// unrolled so several loads are in flight per thread.
template <typename T>
__device__ void dense_fwd(const T* Wt, const T* bias, const T* in, int nin, int nout, T* out, bool relu) {
  for (int o = threadIdx.x; o < nout; o += kInetThreads) {
    T s = T(0);
#pragma unroll 8
    for (int q = 0; q < nin; ++q) s += Wt[(size_t)q * nout + o] * in[q];
    s += bias[o];
    out[o] = relu ? (s > T(0) ? s : T(0)) : s;
  }
  __syncthreads();
}

// Three cotangents through one layer: gin[r][q] = sum_o W[o][q] m_o gout[r][o],
// m_o = (hout[o] > 0) for a ReLU layer (its output is positive exactly where its
// pre-activation is), 1 for a linear one (hout = null).  The mask is applied to
// gout in place first, so the product loop has no branch.  Rows are ld apart.
template <typename T>
__device__ void dense_bwd3(const T* W, int nin, int nout, T* gout, const T* hout, T* gin, int ld) {
  if (hout) {
    for (int o = threadIdx.x; o < nout; o += kInetThreads)
      if (!(hout[o] > T(0))) gout[o] = gout[ld + o] = gout[2 * ld + o] = T(0);
    __syncthreads();
  }
  for (int q = threadIdx.x; q < nin; q += kInetThreads) {
    T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll 8
    for (int o = 0; o < nout; ++o) {
      const T wv = W[(size_t)o * nin + q];
      s0 += wv * gout[o];
      s1 += wv * gout[ld + o];
      s2 += wv * gout[2 * ld + o];
    }
    gin[q] = s0;
    gin[ld + q] = s1;
    gin[2 * ld + q] = s2;
  }
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(kInetThreads) inet_lin_kernel(InetArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char ism[];
  T* sx = reinterpret_cast<T*>(ism);  // x^i [6]
  T* se = sx + 8;                     // e^{ij} [6]
  T* sf = se + 8;                     // phi output [3]
  T* fo = sf + 8;                     // f^i [6]
  T* sa = sx + 32;                    // a^i [d_m]
  T* sin = sa + kWMax;                // phi input [in_phi]
  T* gA = sin + kInMax;               // phi cotangents [3][kInMax], ping
  T* gB = gA + 3 * kInMax;            //                             pong
  T* Jr = gB + 3 * kInMax;            // d phi / d [x; a; u] [3][kInMax]
  T* pA = Jr + 3 * kInMax;            // psi cotangents [3][kWMax], ping
  T* pB = pA + 3 * kWMax;             //                            pong
  T* dvx = pB + 3 * kWMax;            // d v+ / d x^{pcol[e0 + e]} [ne][3][6]
  T* hpsi = dvx + kMaxWidth * 18;     // psi hidden-layer outputs
  T* hphi = hpsi + a.psi_act;         // phi hidden-layer outputs
  const int k = blockIdx.x / a.M, i = blockIdx.x - k * a.M;
  const int tid = threadIdx.x;
  const T* x = a.xhat + (size_t)k * a.M * NBX;
  const T* u = a.uhat + (size_t)k * a.nu;
  const int e0 = a.prow[i], ne = a.prow[i + 1] - e0;
  if (tid < NBX) sx[tid] = x[(size_t)i * NBX + tid];
  for (int t = tid; t < a.d_m; t += kInetThreads) sa[t] = T(0);
  for (int t = tid; t < ne * 18; t += kInetThreads) dvx[t] = T(0);
  __syncthreads();

  // psi on se; hidden outputs to hpsi, the message to `msg`
  auto psi_forward = [&](T* msg) {
    const T* in = se;
    int off = 0;
    for (int l = 0; l < a.n_psi; ++l) {
      const bool last = l == a.n_psi - 1;
      T* out = last ? msg : hpsi + off;
      dense_fwd(a.w + a.wt_off + a.psi_W[l], a.w + a.psi_b[l], in, a.psi_in[l], a.psi_out[l], out, !last);
      in = out;
      if (!last) off += a.psi_out[l];
    }
  };

  // ---- messages: a^i = sum_j psi(x^i - x^j), in-edges in CSR order
  for (int q = a.row_ptr[i]; q < a.row_ptr[i + 1]; ++q) {
    const int j = a.col[q];
    if (tid < NBX) se[tid] = sx[tid] - x[(size_t)j * NBX + tid];
    __syncthreads();
    psi_forward(pA);
    for (int t = tid; t < a.d_m; t += kInetThreads) sa[t] += pA[t];
    __syncthreads();
  }
  // ---- phi forward on [x^i; a^i; u]
  for (int t = tid; t < a.in_phi; t += kInetThreads)
    sin[t] = t < NBX ? sx[t] : (t < NBX + a.d_m ? sa[t - NBX] : u[t - NBX - a.d_m]);
  __syncthreads();
  {
    const T* in = sin;
    int off = 0;
    for (int l = 0; l < a.n_phi; ++l) {
      const bool last = l == a.n_phi - 1;
      T* out = last ? sf : hphi + off;
      dense_fwd(a.w + a.wt_off + a.phi_W[l], a.w + a.phi_b[l], in, a.phi_in[l], a.phi_out[l], out, !last);
      in = out;
      if (!last) off += a.phi_out[l];
    }
  }
  // ---- phi in reverse mode from the three output rows
  for (int t = tid; t < 3 * kInMax; t += kInetThreads) gA[t] = (t % kInMax == t / kInMax) ? T(1) : T(0);
  __syncthreads();
  {
    T* go = gA;
    T* gi = gB;
    int off = a.phi_act;
    for (int l = a.n_phi - 1; l >= 0; --l) {
      const T* hout = nullptr;
      if (l < a.n_phi - 1) {
        off -= a.phi_out[l];
        hout = hphi + off;
      }
      dense_bwd3(a.w + a.phi_W[l], a.phi_in[l], a.phi_out[l], go, hout, gi, kInMax);
      T* tsw = go;
      go = gi;
      gi = tsw;
    }
    for (int t = tid; t < 3 * kInMax; t += kInetThreads) Jr[t] = go[t];
    __syncthreads();
  }
  int ii = 0;  // pattern position of node i
  for (int e = 0; e < ne; ++e)
    if (a.pcol[e0 + e] == i) ii = e;
  if (tid < 18) {
    const int r = tid / 6, q = tid % 6;
    dvx[ii * 18 + tid] = Jr[r * kInMax + q] + ((q == 3 + r) ? T(1) : T(0));  // [0 I] + J_x
  }
  __syncthreads();
  // ---- per in-edge: G J_psi(e^{ij}) by psi in reverse mode from the cotangents G
  for (int q = a.row_ptr[i]; q < a.row_ptr[i + 1]; ++q) {
    const int j = a.col[q];
    if (tid < NBX) se[tid] = sx[tid] - x[(size_t)j * NBX + tid];
    __syncthreads();
    psi_forward(pB);
    for (int t = tid; t < 3 * kWMax; t += kInetThreads) {
      const int r = t / kWMax, o = t - r * kWMax;
      pA[t] = o < a.d_m ? Jr[r * kInMax + NBX + o] : T(0);
    }
    __syncthreads();
    T* go = pA;
    T* gi = pB;
    int off = a.psi_act;
    for (int l = a.n_psi - 1; l >= 0; --l) {
      const T* hout = nullptr;
      if (l < a.n_psi - 1) {
        off -= a.psi_out[l];
        hout = hpsi + off;
      }
      dense_bwd3(a.w + a.psi_W[l], a.psi_in[l], a.psi_out[l], go, hout, gi, kWMax);
      T* tsw = go;
      go = gi;
      gi = tsw;
    }
    int jj = 0;
    for (int e = 0; e < ne; ++e)
      if (a.pcol[e0 + e] == j) jj = e;
    if (tid < 18) {
      const int r = tid / 6, c6 = tid % 6;
      const T h = go[r * kWMax + c6];
      dvx[jj * 18 + tid] -= h;
      dvx[ii * 18 + tid] += h;
    }
    __syncthreads();
  }
  // ---- outputs: f, A blocks of the pattern row, B, c = f - sum A xhat - B uhat
  const T dt = a.dt;
  if (tid < 3) {
    const T vn = sx[3 + tid] + sf[tid];
    fo[3 + tid] = vn;
    fo[tid] = sx[tid] + dt * vn;
  }
  __syncthreads();
  auto a_entry = [&](int e, int rr, int q) {
    const T dv = dvx[e * 18 + (rr % 3) * 6 + q];
    T v = rr < 3 ? dt * dv : dv;
    if (rr < 3 && e == ii && q == rr) v += T(1);
    return v;
  };
  auto b_entry = [&](int rr, int d) {
    const T ju = Jr[(rr % 3) * kInMax + NBX + a.d_m + d];
    return rr < 3 ? dt * ju : ju;
  };
  T* Ak = a.A + ((size_t)k * a.nnz + e0) * 36;
  for (int t = tid; t < ne * 36; t += kInetThreads) Ak[t] = a_entry(t / 36, (t % 36) / 6, t % 6);
  T* Bi = a.B + ((size_t)k * a.M + i) * NBX * a.nu;
  for (int t = tid; t < NBX * a.nu; t += kInetThreads) Bi[t] = b_entry(t / a.nu, t % a.nu);
  if (tid < NBX) {
    T lin = T(0);
    for (int e = 0; e < ne; ++e) {
      const T* xj = x + (size_t)a.pcol[e0 + e] * NBX;
      for (int q = 0; q < NBX; ++q) lin += a_entry(e, tid, q) * xj[q];
    }
    for (int d = 0; d < a.nu; ++d) lin += b_entry(tid, d) * u[d];
    a.c[((size_t)k * a.M + i) * NBX + tid] = fo[tid] - lin;
    if (a.fnext) a.fnext[((size_t)k * a.M + i) * NBX + tid] = fo[tid];
  }
}

template <typename T>
gnmpc_status run_inet(gnmpc_plan* p, const void* xhat, const void* uhat, void* A, void* B, void* c, void* fnext,
                      hipStream_t s) {
  const InetState& g = *p->inet;
  InetArgs<T> a;
  a.N = p->dims.N;
  a.M = p->M;
  a.nu = p->dims.nu;
  a.n_psi = g.n_psi;
  a.n_phi = g.n_phi;
  a.d_m = g.d_m;
  a.in_phi = g.in_phi;
  a.psi_act = g.psi_act;
  a.phi_act = g.phi_act;
  a.nnz = p->nnz;
  a.wt_off = g.n_w;
  a.dt = (T)g.dt;
  for (int l = 0; l < kInetMaxLayers; ++l) {
    a.psi_in[l] = g.psi_in[l];
    a.psi_out[l] = g.psi_out[l];
    a.phi_in[l] = g.phi_in[l];
    a.phi_out[l] = g.phi_out[l];
    a.psi_W[l] = g.psi_W[l];
    a.psi_b[l] = g.psi_b[l];
    a.phi_W[l] = g.phi_W[l];
    a.phi_b[l] = g.phi_b[l];
  }
  a.w = (const T*)g.w;
  a.row_ptr = p->d_row_ptr;
  a.col = p->d_col;
  a.prow = p->d_prow;
  a.pcol = p->d_pcol;
  a.xhat = (const T*)xhat;
  a.uhat = (const T*)uhat;
  a.A = (T*)A;
  a.B = (T*)B;
  a.c = (T*)c;
  a.fnext = (T*)fnext;
  const size_t lds = inet_lds_elems(g.psi_act, g.phi_act) * sizeof(T);
  GNMPC_HIP_TRY(p, set_max_lds((const void*)inet_lin_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  inet_lin_kernel<T><<<a.N * a.M, kInetThreads, lds, s>>>(a);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

}  // namespace

void inet_free(gnmpc_plan* p) {
  if (!p->inet) return;
  if (p->inet->w) (void)hipFree(p->inet->w);
  delete p->inet;
  p->inet = nullptr;
}

gnmpc_status inet_set(gnmpc_plan* p, const gnmpc_inet_desc* d, const double* w, int64_t n_w) {
  const int n_psi = d->psi_hidden + 1, n_phi = d->phi_hidden + 1;
  if (d->psi_hidden < 0 || d->phi_hidden < 0 || n_psi > kInetMaxLayers || n_phi > kInetMaxLayers ||
      d->psi_width < 1 || d->psi_width > kInetMaxWidth || d->phi_width < 1 || d->phi_width > kInetMaxWidth ||
      d->d_m < 1 || d->d_m > kInetMaxWidth || d->nu < 1 || d->nu > kInetMaxNu || !(d->dt > 0))
    return GNMPC_INVALID_ARG;
  InetState g;
  g.n_psi = n_psi;
  g.n_phi = n_phi;
  g.d_m = d->d_m;
  g.nu = d->nu;
  g.in_phi = NBX + d->d_m + d->nu;
  g.dt = d->dt;
  long off = 0;
  for (int l = 0; l < n_psi; ++l) {
    g.psi_in[l] = l == 0 ? NBX : d->psi_width;
    g.psi_out[l] = l == n_psi - 1 ? d->d_m : d->psi_width;
    g.psi_W[l] = off;
    off += (long)g.psi_in[l] * g.psi_out[l];
    g.psi_b[l] = off;
    off += g.psi_out[l];
    if (l < n_psi - 1) g.psi_act += g.psi_out[l];
  }
  for (int l = 0; l < n_phi; ++l) {
    g.phi_in[l] = l == 0 ? g.in_phi : d->phi_width;
    g.phi_out[l] = l == n_phi - 1 ? 3 : d->phi_width;
    g.phi_W[l] = off;
    off += (long)g.phi_in[l] * g.phi_out[l];
    g.phi_b[l] = off;
    off += g.phi_out[l];
    if (l < n_phi - 1) g.phi_act += g.phi_out[l];
  }
  for (int l = n_psi; l < kInetMaxLayers; ++l) g.psi_in[l] = g.psi_out[l] = 0, g.psi_W[l] = g.psi_b[l] = 0;
  for (int l = n_phi; l < kInetMaxLayers; ++l) g.phi_in[l] = g.phi_out[l] = 0, g.phi_W[l] = g.phi_b[l] = 0;
  if (n_w != off) return GNMPC_SHAPE;
  if (inet_lds_elems(g.psi_act, g.phi_act) * (size_t)p->elem > 160 * 1024) return GNMPC_UNSUPPORTED;
  inet_free(p);
  g.n_w = off;
  // the packed weights, then the same layout with every matrix W [out][in]
  // stored as W' [in][out] (biases copied unchanged)
  std::vector<double> both(2 * (size_t)off);
  std::copy(w, w + off, both.begin());
  std::copy(w, w + off, both.begin() + off);
  auto transpose = [&](long at, int nout, int nin) {
    for (int o = 0; o < nout; ++o)
      for (int q = 0; q < nin; ++q) both[off + at + (size_t)q * nout + o] = w[at + (size_t)o * nin + q];
  };
  for (int l = 0; l < n_psi; ++l) transpose(g.psi_W[l], g.psi_out[l], g.psi_in[l]);
  for (int l = 0; l < n_phi; ++l) transpose(g.phi_W[l], g.phi_out[l], g.phi_in[l]);
  const size_t bytes = both.size() * p->elem;
  if (hipMalloc(&g.w, std::max<size_t>(bytes, 256)) != hipSuccess) {
    p->last_error = "model_set_inet: hipMalloc failed";
    return GNMPC_HIP_ERROR;
  }
  hipError_t e;
  if (p->elem == 8) {
    e = hipMemcpy(g.w, both.data(), bytes, hipMemcpyHostToDevice);
  } else {
    std::vector<float> f(both.begin(), both.end());
    e = hipMemcpy(g.w, f.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    (void)hipFree(g.w);
    p->last_error = std::string("model_set_inet: ") + hipGetErrorString(e);
    return GNMPC_HIP_ERROR;
  }
  p->inet = new InetState(g);
  return GNMPC_OK;
}

gnmpc_status launch_inet_linearize(gnmpc_plan* p, const void* xhat, const void* uhat, void* A, void* B, void* c,
                                   void* fnext, hipStream_t s) {
  if (p->dims.dtype == GNMPC_F64) return run_inet<double>(p, xhat, uhat, A, B, c, fnext, s);
  return run_inet<float>(p, xhat, uhat, A, B, c, fnext, s);
}

}  // namespace gnmpc
