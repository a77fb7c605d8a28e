// Analytic linearization of the mass-spring-damper chain (the plain form of
// the linearization step, Sec. V-A eq. linearized_dynamics with an analytic
// model in place of the GNN).
//
// Writes A [N][nnz][6][6], B [N][M][6][nu], c [N][M][6] (and optionally
// f [N][M][6]).  The work is a pure HBM write stream (about 1.2 KB per node
// and stage against a few hundred flops), so each kernel builds its output
// tile in LDS and stores it with consecutive lanes on consecutive addresses.
#include "plan.hpp"

namespace gnmpc {
namespace {

template <typename T>
struct MsdArgs {
  const T* xhat;        // [N+1][M][6]
  const T* uhat;        // [N][nu]
  const int32_t* row_ptr;
  const int32_t* col;
  const int32_t* prow;
  const int32_t* pcol;
  const int32_t* erow;
  const int32_t* act_of_node;
  int M, N, nu;
  long nnz;
  T k, c, m, dt, k3, grav;
  int anchor;
};

// dF/dd for F(d) = k d + k3 |d|^2 d:  k I + k3 (|d|^2 I + 2 d d^T)
template <typename T>
__device__ inline void dforce(const T d[3], T k, T k3, T K[3][3]) {
  T n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) K[a][b] = (a == b ? k + k3 * n2 : T(0)) + T(2) * k3 * d[a] * d[b];
}

// d a^i / d x^j as a 3x6 block [dp | dv]; j == i gives the diagonal block.
template <typename T>
__device__ void dacc_block(const MsdArgs<T>& a, const T* x, int i, int j, T out[3][6]) {
  const T inv_m = T(1) / a.m;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int s = 0; s < 6; ++s) out[r][s] = T(0);
  const T* pi = x + (size_t)i * NBX;
  if (j != i) {
    bool nb = false;
    for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) nb |= (a.col[e] == j);
    if (!nb) return;
    const T* pj = x + (size_t)j * NBX;
    T d[3] = {pj[0] - pi[0], pj[1] - pi[1], pj[2] - pi[2]};
    T K[3][3];
    dforce(d, a.k, a.k3, K);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int s = 0; s < 3; ++s) out[r][s] = K[r][s] * inv_m;
      out[r][3 + r] = a.c * inv_m;
    }
    return;
  }
  T deg = T(0);
  for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) {
    const T* pj = x + (size_t)a.col[e] * NBX;
    T d[3] = {pj[0] - pi[0], pj[1] - pi[1], pj[2] - pi[2]};
    T K[3][3];
    dforce(d, a.k, a.k3, K);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int s = 0; s < 3; ++s) out[r][s] -= K[r][s] * inv_m;
    deg += T(1);
  }
  if (i == a.anchor) {
    T d[3] = {pi[0], pi[1], pi[2]};
    T K[3][3];
    dforce(d, a.k, a.k3, K);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int s = 0; s < 3; ++s) out[r][s] -= K[r][s] * inv_m;
    deg += T(1);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) out[r][3 + r] = -deg * a.c * inv_m;
}

// Semi-implicit Euler Jacobian block: dv+ = [0 I] delta + dt da, dp+ = [I 0] delta + dt dv+.
template <typename T>
__device__ inline void step_block(const T da[3][6], bool diag, T dt, T blk[6][6]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      T dv = dt * da[r][s] + ((diag && s == 3 + r) ? T(1) : T(0));
      blk[3 + r][s] = dv;
      blk[r][s] = dt * dv + ((diag && s == r) ? T(1) : T(0));
    }
}

template <typename T>
__device__ inline T spring_force(const T d[3], T k, T k3, int r) {
  T n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  return k * d[r] + k3 * n2 * d[r];
}

constexpr int kTile = 128;  // (stage, entry) pairs per workgroup

// The three parts of the linearization (A blocks, B, offsets c) read only xhat and
// uhat and write disjoint outputs, so one launch runs all three on disjoint ranges
// of workgroups (msd_lin_kernel below); each part is a device function of its
// workgroup index within its range.
template <typename T>
__device__ inline void msd_A_part(const MsdArgs<T>& a, T* __restrict__ A, long blk, T* tile) {
  const long total = (long)a.N * a.nnz;
  const long base = blk * kTile;
  const long idx = base + threadIdx.x;
  if (idx < total) {
    int k = (int)(idx / a.nnz);
    long e = idx - (long)k * a.nnz;
    int i = a.erow[e], j = a.pcol[e];
    const T* x = a.xhat + (size_t)k * a.M * NBX;
    T da[3][6], blk[6][6];
    dacc_block(a, x, i, j, da);
    step_block(da, i == j, a.dt, blk);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int s = 0; s < 6; ++s) tile[threadIdx.x * 36 + r * 6 + s] = blk[r][s];
  }
  __syncthreads();
  const long n_out = min((long)kTile, total - base) * 36;
  T* dst = A + base * 36;
  for (long t = threadIdx.x; t < n_out; t += kTile) dst[t] = tile[t];
}

// B is constant for this model: node i actuated by input a has B[r][3a + r%3]
// = dt^2/m (positions) or dt/m (velocities).  One lane per output element, grid-stride
// over the nblk workgroups of this part.
template <typename T>
__device__ inline void msd_B_part(const MsdArgs<T>& a, T* __restrict__ B, long blk, long nblk) {
  const long total = (long)a.N * a.M * NBX * a.nu;
  for (long t = blk * kTile + threadIdx.x; t < total; t += nblk * kTile) {
    int col = (int)(t % a.nu);
    long rest = t / a.nu;
    int r = (int)(rest % NBX);
    int i = (int)((rest / NBX) % a.M);
    int act = a.act_of_node[i];
    T v = T(0);
    if (act >= 0 && col == 3 * act + (r % 3)) v = (r < 3 ? a.dt * a.dt : a.dt) / a.m;
    B[t] = v;
  }
}

// c = f(xhat, uhat) - sum_j A^{ij} xhat^j - B uhat, one lane per (stage, node).
template <typename T>
__device__ inline void msd_c_part(const MsdArgs<T>& a, T* __restrict__ c, T* __restrict__ fnext, long blk, T* tc) {
  T* tf = tc + kTile * NBX;
  const long total = (long)a.N * a.M;
  const long base = blk * kTile;
  const long idx = base + threadIdx.x;
  if (idx < total) {
    int k = (int)(idx / a.M);
    int i = (int)(idx - (long)k * a.M);
    const T* x = a.xhat + (size_t)k * a.M * NBX;
    const T* u = a.uhat + (size_t)k * a.nu;
    const T* xi = x + (size_t)i * NBX;
    const T inv_m = T(1) / a.m;
    // nonlinear step at the nominal point
    T acc[3] = {0, 0, 0};
    for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) {
      const T* xj = x + (size_t)a.col[e] * NBX;
      T d[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
#pragma unroll
      for (int r = 0; r < 3; ++r) acc[r] += spring_force(d, a.k, a.k3, r) + a.c * (xj[3 + r] - xi[3 + r]);
    }
    if (i == a.anchor) {
      T d[3] = {xi[0], xi[1], xi[2]};
#pragma unroll
      for (int r = 0; r < 3; ++r) acc[r] -= spring_force(d, a.k, a.k3, r) + a.c * xi[3 + r];
    }
    int act = a.act_of_node[i];
    if (act >= 0) {
#pragma unroll
      for (int r = 0; r < 3; ++r) acc[r] += u[3 * act + r];
    }
    T f[6];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      T ar = acc[r] * inv_m - (r == 2 ? a.grav : T(0));
      T vn = xi[3 + r] + a.dt * ar;
      f[3 + r] = vn;
      f[r] = xi[r] + a.dt * vn;
    }
    // linear part of the model at the nominal point
    T lin[6] = {0, 0, 0, 0, 0, 0};
    for (int e = a.prow[i]; e < a.prow[i + 1]; ++e) {
      int j = a.pcol[e];
      T da[3][6], blk[6][6];
      dacc_block(a, x, i, j, da);
      step_block(da, i == j, a.dt, blk);
      const T* xj = x + (size_t)j * NBX;
#pragma unroll
      for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int s = 0; s < 6; ++s) lin[r] += blk[r][s] * xj[s];
    }
    if (act >= 0) {
#pragma unroll
      for (int r = 0; r < 6; ++r) lin[r] += (r < 3 ? a.dt * a.dt : a.dt) * inv_m * u[3 * act + (r % 3)];
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      tc[threadIdx.x * NBX + r] = f[r] - lin[r];
      tf[threadIdx.x * NBX + r] = f[r];
    }
  }
  __syncthreads();
  const long n_out = min((long)kTile, total - base) * NBX;
  for (long t = threadIdx.x; t < n_out; t += kTile) {
    c[base * NBX + t] = tc[t];
    if (fnext) fnext[base * NBX + t] = tf[t];
  }
}

// Workgroups [0, gA): A blocks; [gA, gA + gC): offsets; the rest: B.
template <typename T>
__global__ void __launch_bounds__(kTile) msd_lin_kernel(MsdArgs<T> a, T* __restrict__ A, T* __restrict__ B,
                                                        T* __restrict__ c, T* __restrict__ fnext, long gA, long gC) {
  __shared__ T smem[kTile * 36];  // the A part's staged blocks, or the c part's two staged rows
  const long b = blockIdx.x;
  if (b < gA) msd_A_part(a, A, b, smem);
  else if (b < gA + gC) msd_c_part(a, c, fnext, b - gA, smem);
  else msd_B_part(a, B, b - gA - gC, (long)gridDim.x - gA - gC);
}

template <typename T>
gnmpc_status run(gnmpc_plan* p, const void* xhat, const void* uhat, void* A, void* B, void* c, void* fnext,
                 hipStream_t s) {
  MsdArgs<T> a;
  a.xhat = (const T*)xhat;
  a.uhat = (const T*)uhat;
  a.row_ptr = p->d_row_ptr;
  a.col = p->d_col;
  a.prow = p->d_prow;
  a.pcol = p->d_pcol;
  a.erow = p->d_erow;
  a.act_of_node = p->d_act_of_node;
  a.M = p->M;
  a.N = p->dims.N;
  a.nu = p->dims.nu;
  a.nnz = p->nnz;
  a.k = (T)p->msd.k;
  a.c = (T)p->msd.c;
  a.m = (T)p->msd.m;
  a.dt = (T)p->msd.dt;
  a.k3 = (T)p->msd.k3;
  a.grav = (T)p->msd.gravity;
  a.anchor = p->msd.anchor;
  const long nA = (long)a.N * a.nnz, nB = (long)a.N * a.M * NBX * a.nu, nc = (long)a.N * a.M;
  const long gA = ceil_div(nA, kTile), gC = ceil_div(nc, kTile), gB = std::min<long>(ceil_div(nB, kTile), 8192);
  phase_begin(p, GNMPC_PH_MSD_LINEARIZE, s);
  msd_lin_kernel<T><<<(unsigned)(gA + gC + gB), kTile, 0, s>>>(a, (T*)A, (T*)B, (T*)c, (T*)fnext, gA, gC);
  phase_end(p, GNMPC_PH_MSD_LINEARIZE, s);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

}  // namespace

gnmpc_status launch_msd_linearize(gnmpc_plan* p, const void* xhat, const void* uhat, void* A, void* B,
                                  void* c, void* fnext, hipStream_t s) {
  if (p->dims.dtype == GNMPC_F64) return run<double>(p, xhat, uhat, A, B, c, fnext, s);
  return run<float>(p, xhat, uhat, A, B, c, fnext, s);
}

}  // namespace gnmpc
