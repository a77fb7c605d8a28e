// Forward- and reverse-mode products of the linearized dynamics (Sec. V-A):
// with the block Jacobians A_k (pattern blocks A^{ij}_k) and B_k (blocks B^i_k)
// of x_{k+1} = f(x_k, u_k), the JVP is t_k = A_k dx_k + B_k du_k and the VJP is
// (A_k' g_k, B_k' g_k).  Every output element is one thread's fixed-order sum, so
// results do not depend on scheduling; the VJP's state part walks the pattern by
// column (the entries of column node j in increasing order).  The linear rollout
// x_{k+1} = A_k x_k + B_k u_k + c_k (Sec. III-B, the dynamics constraint of the
// OCP; the shift of Algorithm 1 needs it) is the JVP's row sum plus the offset,
// one launch per stage since stage k+1 reads stage k.
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace gnmpc {
namespace {

// t[k][i][r] = sum_e sum_c A[k][e][r][c] dx[k][pcol[e]][c] + sum_d B[k][i][r][d] du[k][d]
template <typename T>
__global__ void jvp_kernel(int N, int M, int nu, long nnz, const int32_t* __restrict__ prow,
                           const int32_t* __restrict__ pcol, const T* __restrict__ A, const T* __restrict__ B,
                           const T* __restrict__ dx, const T* __restrict__ du, T* __restrict__ out) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)N * M * NBX) return;
  const int r = (int)(t % NBX);
  const long s = t / NBX;
  const int k = (int)(s / M), i = (int)(s - (long)k * M);
  T v = T(0);
  for (int e = prow[i]; e < prow[i + 1]; ++e) {
    const T* a = A + ((size_t)k * nnz + e) * 36 + r * 6;
    const T* x = dx + ((size_t)k * M + pcol[e]) * NBX;
#pragma unroll
    for (int c = 0; c < 6; ++c) v += a[c] * x[c];
  }
  const T* b = B + ((size_t)s * NBX + r) * nu;
  const T* w = du + (size_t)k * nu;
  for (int d = 0; d < nu; ++d) v += b[d] * w[d];
  out[t] = v;
}

// gx[k][j][c] = sum over entries e of column j (rows erow[e]) of sum_r A[k][e][r][c] g[k][erow[e]][r]
template <typename T>
__global__ void vjp_x_kernel(int N, int M, long nnz, const int32_t* __restrict__ cptr,
                             const int32_t* __restrict__ cent, const int32_t* __restrict__ erow,
                             const T* __restrict__ A, const T* __restrict__ g, T* __restrict__ gx) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)N * M * NBX) return;
  const int c = (int)(t % NBX);
  const long s = t / NBX;
  const int k = (int)(s / M), j = (int)(s - (long)k * M);
  T v = T(0);
  for (int q = cptr[j]; q < cptr[j + 1]; ++q) {
    const int e = cent[q];
    const T* a = A + ((size_t)k * nnz + e) * 36 + c;
    const T* y = g + ((size_t)k * M + erow[e]) * NBX;
#pragma unroll
    for (int r = 0; r < 6; ++r) v += a[r * 6] * y[r];
  }
  gx[t] = v;
}

// gu[k][d] = sum_i sum_r B[k][i][r][d] g[k][i][r]: one workgroup per (k, d); thread
// partial sums over rows (i, r) = threadIdx.x + 256 m, then a fixed pairwise tree
constexpr int kVjpThreads = 256;
template <typename T>
__global__ void __launch_bounds__(kVjpThreads) vjp_u_kernel(int N, int M, int nu, const T* __restrict__ B,
                                                             const T* __restrict__ g, T* __restrict__ gu) {
  __shared__ T red[kVjpThreads];
  const int k = blockIdx.x, d = blockIdx.y;
  const long rows = (long)M * NBX;
  T v = T(0);
  for (long q = threadIdx.x; q < rows; q += kVjpThreads)
    v += B[((size_t)k * rows + q) * nu + d] * g[(size_t)k * rows + q];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = kVjpThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) gu[(size_t)k * nu + d] = red[0];
}

// x[k+1][i][r] = sum_e A[k][e][r][:] x[k][pcol[e]] + B[k][i][r][:] u[k] + c[k][i][r], the same
// fixed order as the oracle's block rollout; the stage-0 launch reads x0 and also
// writes x[0] = x0 (its readers read x0, so no thread waits for another)
template <typename T>
__global__ void rollout_stage_kernel(int k, int M, int nu, long nnz, const int32_t* __restrict__ prow,
                                     const int32_t* __restrict__ pcol, const T* __restrict__ A,
                                     const T* __restrict__ B, const T* __restrict__ c, const T* __restrict__ xk,
                                     const T* __restrict__ u, T* __restrict__ x) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * NBX) return;
  const int r = t % NBX, i = t / NBX;
  const size_t sM = (size_t)M * NBX;
  const T* Ak = A + (size_t)k * nnz * 36;
  T v = T(0);
  for (int e = prow[i]; e < prow[i + 1]; ++e) {
    const T* a = Ak + (size_t)e * 36 + r * 6;
    const T* xj = xk + (size_t)pcol[e] * NBX;
#pragma unroll
    for (int q = 0; q < 6; ++q) v += a[q] * xj[q];
  }
  const T* b = B + (((size_t)k * M + i) * NBX + r) * nu;
  const T* uk = u + (size_t)k * nu;
  for (int d = 0; d < nu; ++d) v += b[d] * uk[d];
  v += c[(size_t)k * sM + t];
  if (k == 0) x[t] = xk[t];
  x[(size_t)(k + 1) * sM + t] = v;
}

template <typename T>
gnmpc_status run_rollout(gnmpc_plan* p, const void* A, const void* B, const void* c, const void* x0,
                         const void* u, void* x, hipStream_t s) {
  const int N = p->dims.N, M = p->M, nu = p->dims.nu;
  const int n = M * NBX;
  for (int k = 0; k < N; ++k) {
    const T* xk = k == 0 ? (const T*)x0 : (const T*)x + (size_t)k * n;
    rollout_stage_kernel<T><<<ceil_div(n, 256), 256, 0, s>>>(k, M, nu, p->nnz, p->d_prow, p->d_pcol, (const T*)A,
                                                            (const T*)B, (const T*)c, xk, (const T*)u, (T*)x);
    GNMPC_HIP_TRY(p, hipGetLastError());
  }
  return GNMPC_OK;
}

// The shift of Algorithm 1 ("update lin. trajectory"): the next linearization
// trajectory is the optimal one advanced by one stage, xhat'[k] = x*[k+1] and
// uhat'[k] = u*[k+1]; the stages that have no successor repeat the last one
// (xhat'[N] = x*[N], uhat'[N-1] = u*[N-1]).  One thread per output element; the
// outputs may be the current linearization trajectory (it is not read here).
template <typename T>
__global__ void rti_shift_kernel(int N, int M, int nu, const T* __restrict__ xpred, const T* __restrict__ u,
                                 T* __restrict__ xhat, T* __restrict__ uhat) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long sM = (long)M * NBX, nx = (long)(N + 1) * sM;
  if (t < nx) {
    const long k = t / sM;
    xhat[t] = xpred[(k < N ? k + 1 : N) * sM + (t - k * sM)];
  } else if (t < nx + (long)N * nu) {
    const long q = t - nx, k = q / nu;
    uhat[q] = u[(k < N - 1 ? k + 1 : N - 1) * nu + (q - k * nu)];
  }
}

template <typename T>
gnmpc_status run_shift(gnmpc_plan* p, const void* xpred, const void* u, void* xhat, void* uhat, hipStream_t s) {
  const int N = p->dims.N, M = p->M, nu = p->dims.nu;
  const long n = (long)(N + 1) * M * NBX + (long)N * nu;
  rti_shift_kernel<T><<<ceil_div(n, 256), 256, 0, s>>>(N, M, nu, (const T*)xpred, (const T*)u, (T*)xhat, (T*)uhat);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

template <typename T>
gnmpc_status run_jvp(gnmpc_plan* p, const void* A, const void* B, const void* dx, const void* du, void* out,
                     hipStream_t s) {
  const int N = p->dims.N, M = p->M, nu = p->dims.nu;
  const long n = (long)N * M * NBX;
  jvp_kernel<T><<<ceil_div(n, 256), 256, 0, s>>>(N, M, nu, p->nnz, p->d_prow, p->d_pcol, (const T*)A, (const T*)B,
                                                 (const T*)dx, (const T*)du, (T*)out);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

template <typename T>
gnmpc_status run_vjp(gnmpc_plan* p, const void* A, const void* B, const void* g, void* gx, void* gu,
                     hipStream_t s) {
  const int N = p->dims.N, M = p->M, nu = p->dims.nu;
  const long n = (long)N * M * NBX;
  vjp_x_kernel<T><<<ceil_div(n, 256), 256, 0, s>>>(N, M, p->nnz, p->d_cptr, p->d_cent, p->d_erow, (const T*)A,
                                                   (const T*)g, (T*)gx);
  vjp_u_kernel<T><<<dim3(N, nu), kVjpThreads, 0, s>>>(N, M, nu, (const T*)B, (const T*)g, (T*)gu);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

}  // namespace

gnmpc_status launch_jvp(gnmpc_plan* p, const void* A, const void* B, const void* dx, const void* du, void* out,
                        hipStream_t s) {
  if (p->dims.dtype == GNMPC_F64) return run_jvp<double>(p, A, B, dx, du, out, s);
  return run_jvp<float>(p, A, B, dx, du, out, s);
}

gnmpc_status launch_vjp(gnmpc_plan* p, const void* A, const void* B, const void* g, void* gx, void* gu,
                        hipStream_t s) {
  if (p->dims.dtype == GNMPC_F64) return run_vjp<double>(p, A, B, g, gx, gu, s);
  return run_vjp<float>(p, A, B, g, gx, gu, s);
}

gnmpc_status launch_rollout(gnmpc_plan* p, const void* A, const void* B, const void* c, const void* x0,
                            const void* u, void* x, hipStream_t s) {
  if (p->dims.dtype == GNMPC_F64) return run_rollout<double>(p, A, B, c, x0, u, x, s);
  return run_rollout<float>(p, A, B, c, x0, u, x, s);
}

gnmpc_status launch_rti_shift(gnmpc_plan* p, const void* xpred, const void* u, void* xhat, void* uhat,
                              hipStream_t s) {
  if (p->dims.dtype == GNMPC_F64) return run_shift<double>(p, xpred, u, xhat, uhat, s);
  return run_shift<float>(p, xpred, u, xhat, uhat, s);
}

}  // namespace gnmpc
