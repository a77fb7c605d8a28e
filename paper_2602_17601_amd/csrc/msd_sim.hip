// Trajectories of the nonlinear mass-spring-damper graph (the plant whose
// linearization is the plain form, and the data source of a learned GNN
// surrogate): B independent trajectories of T steps each, from given initial
// states and input sequences, integrated with the semi-implicit Euler step of
// Sec. V-A eq. forward_dynamics (v+ = v + dt a, p+ = p + dt v+).  Node
// acceleration, states being displacements from rest:
//   a^i = 1/m [ sum_{j in N_i} ( F(p^j - p^i) + c (v^j - v^i) )
//               + [i anchored] ( -F(p^i) - c v^i ) + f^i ] - gravity e_z,
//   F(d) = k d + k3 |d|^2 d,  f^i the 3D input force of an actuated node.
//
// One workgroup per trajectory: its state lives in LDS (two buffers, the step
// reads one and writes the other) for all T steps; after each step the new
// state is copied from LDS to HBM with 16-byte stores (consecutive lanes on
// consecutive 16 bytes), while the next step already reads it.  The kernel is
// bound by those writes (B (T + 1) M 6 elements).
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace gnmpc {
namespace {

constexpr int kSimThreads = 512;

template <typename T>
struct SimArgs {
  int B, steps, M, nu, anchor;
  T k, c, m, dt, k3, grav;
  const int32_t *row_ptr, *col, *act_of_node;
  const T* x0;  // [B][M][6]
  const T* u;   // [B][T][nu]
  T* X;         // [B][T+1][M][6]
};

template <typename T>
__device__ inline void spring(const T d[3], T k, T k3, T out[3]) {
  const T n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const T s = k + k3 * n2;
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a] = s * d[a];
}

template <typename T>
__global__ void __launch_bounds__(kSimThreads) msd_sim_kernel(SimArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char sim_smem[];
  T* buf = reinterpret_cast<T*>(sim_smem);  // [2][M][6]
  const int b = blockIdx.x, M = a.M;
  const size_t sz = (size_t)M * NBX;
  const T* x0 = a.x0 + (size_t)b * sz;
  T* Xb = a.X + (size_t)b * (a.steps + 1) * sz;
  // a state is a multiple of 16 bytes when M is even (FP32) or always (FP64)
  const bool vec = (sz * sizeof(T)) % 16 == 0;
  auto store_state = [&](const T* src, T* dst) {
    if (vec) {
      const int n4 = (int)(sz * sizeof(T) / 16);
      for (int t = threadIdx.x; t < n4; t += kSimThreads)
        reinterpret_cast<uint4*>(dst)[t] = reinterpret_cast<const uint4*>(src)[t];
    } else {
      for (int t = threadIdx.x; t < (int)sz; t += kSimThreads) dst[t] = src[t];
    }
  };
  for (int t = threadIdx.x; t < (int)sz; t += kSimThreads) buf[t] = x0[t];
  __syncthreads();
  store_state(buf, Xb);
  const T inv_m = T(1) / a.m;
  for (int step = 0; step < a.steps; ++step) {
    const T* cur = buf + (size_t)(step & 1) * sz;
    T* nxt = buf + (size_t)((step + 1) & 1) * sz;
    const T* ub = a.u + ((size_t)b * a.steps + step) * a.nu;
    for (int i = threadIdx.x; i < M; i += kSimThreads) {
      const T* xi = cur + (size_t)i * NBX;
      T acc[3] = {T(0), T(0), T(0)};
      for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) {
        const T* xj = cur + (size_t)a.col[e] * NBX;
        T d[3], f[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) d[q] = xj[q] - xi[q];
        spring(d, a.k, a.k3, f);
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[q] += f[q] + a.c * (xj[3 + q] - xi[3 + q]);
      }
      if (i == a.anchor) {
        T f[3];
        spring(xi, a.k, a.k3, f);
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[q] += -f[q] - a.c * xi[3 + q];
      }
      const int act = a.act_of_node[i];
      if (act >= 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[q] += ub[3 * act + q];
      }
      T out[6];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        T aq = acc[q] * inv_m;
        if (q == 2) aq -= a.grav;
        const T vn = xi[3 + q] + a.dt * aq;
        out[3 + q] = vn;
        out[q] = xi[q] + a.dt * vn;
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) nxt[(size_t)i * NBX + q] = out[q];
    }
    __syncthreads();
    // the next step reads this state too and writes the other buffer, which every
    // lane finished reading before the barrier above
    store_state(nxt, Xb + (size_t)(step + 1) * sz);
  }
}

size_t sim_lds_bytes(int M, size_t elem) { return 2 * (size_t)M * NBX * elem; }

template <typename T>
gnmpc_status run(gnmpc_plan* p, int B, int steps, const void* x0, const void* u, void* X, hipStream_t s) {
  SimArgs<T> a;
  a.B = B;
  a.steps = steps;
  a.M = p->M;
  a.nu = p->dims.nu;
  a.anchor = p->msd.anchor;
  a.k = (T)p->msd.k;
  a.c = (T)p->msd.c;
  a.m = (T)p->msd.m;
  a.dt = (T)p->msd.dt;
  a.k3 = (T)p->msd.k3;
  a.grav = (T)p->msd.gravity;
  a.row_ptr = p->d_row_ptr;
  a.col = p->d_col;
  a.act_of_node = p->d_act_of_node;
  a.x0 = (const T*)x0;
  a.u = (const T*)u;
  a.X = (T*)X;
  const size_t lds = sim_lds_bytes(p->M, sizeof(T));
  GNMPC_HIP_TRY(p, set_max_lds((const void*)msd_sim_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  msd_sim_kernel<T><<<B, kSimThreads, lds, s>>>(a);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

}  // namespace

bool msd_sim_fits(const gnmpc_plan* p) { return sim_lds_bytes(p->M, (size_t)p->elem) <= 160 * 1024; }

gnmpc_status launch_msd_simulate(gnmpc_plan* p, int B, int T, const void* x0, const void* u, void* X, hipStream_t s) {
  if (p->dims.dtype == GNMPC_F64) return run<double>(p, B, T, x0, u, X, s);
  return run<float>(p, B, T, x0, u, X, s);
}

}  // namespace gnmpc
