// Graph-sparse condensing (Sec. V-B, proof of Thm. 1).
//
// Stage recursion (eqs. sparse_gamma_i_xb / sparse_gamma_i_u): the last block
// row of Gamma_u^i after k+1 steps is S^i_{k+1} = sum_{j in N~_i} A^{ij}_k S^j_k
// with B^i_k placed in column block k, and Gx^i_{k+1} = sum_j A^{ij}_k Gx^j_k + c^i_k.
// S_k only has k*nu live columns; it is kept for every stage in the plan's
// workspace (stage k at S_offset(k) as [M][6][k nu]) because the Hessian,
// gradient and constraint kernels read it afterwards.
//
// Hessian / gradient (eqs. H and g): H = Rbar + sum_k sum_i S^i_k' Q^i_k S^i_k,
// g = rbar + sum_k sum_i S^i_k' (Q^i_k Gx^i_k + q^i_k), computed as a split-K
// Gram product over 16x16 tiles of H's lower triangle with one partial per
// (tile, stage, node chunk), then reduced in a fixed order (bitwise repeatable).
//
// Constraint rows (stacked-constraint formula of Sec. V-B):
// Ct[t] = C_t S^{i_t}_{k_t}, dt[t] = d_t - C_t Gx^{i_t}_{k_t}.
#include <algorithm>

#include "plan.hpp"

namespace gnmpc {
namespace {

constexpr int kPropThreads = 256;
constexpr int kTileH = 16;        // Gram output tile edge
constexpr int kGramThreads = 256; // one lane per tile element
constexpr int kChunkNodes = 128;  // nodes per split-K chunk
constexpr int kRowsStaged = 48;   // rows (8 nodes) staged in LDS per step

// ---------------------------------------------------------------- propagation
template <typename T>
__global__ void __launch_bounds__(kPropThreads)
sprop_kernel(int k, int M, int nu, int npw, const int32_t* __restrict__ prow, const int32_t* __restrict__ pcol,
             const T* __restrict__ A_k, const T* __restrict__ B_k, const T* __restrict__ c_k,
             const T* __restrict__ S_in, T* __restrict__ S_out, const T* __restrict__ Gx_in,
             T* __restrict__ Gx_out, int wmax) {
  extern __shared__ unsigned char smem_raw[];
  T* As = reinterpret_cast<T*>(smem_raw);  // [npw][wmax][36]
  const int node0 = blockIdx.x * npw;
  const int nn = min(npw, M - node0);
  // stage the pattern rows of this workgroup's nodes
  for (int ln = 0; ln < nn; ++ln) {
    int i = node0 + ln;
    int e0 = prow[i], w = prow[i + 1] - e0;
    const T* src = A_k + (size_t)e0 * 36;
    for (int t = threadIdx.x; t < w * 36; t += kPropThreads) As[(ln * wmax) * 36 + t] = src[t];
  }
  __syncthreads();
  const int cin = k * nu;             // live columns of S_k
  const int cout = (k + 1) * nu;      // live columns of S_{k+1}
  const int ncol = cout + 1;          // + the Gx column
  for (int it = threadIdx.x; it < nn * ncol; it += kPropThreads) {
    int ln = it / ncol;
    int col = it - ln * ncol;
    int i = node0 + ln;
    int e0 = prow[i], w = prow[i + 1] - e0;
    const T* Ab = As + (size_t)(ln * wmax) * 36;
    T o[6] = {0, 0, 0, 0, 0, 0};
    if (col < cin) {
      for (int e = 0; e < w; ++e) {
        const T* Sj = S_in + (size_t)pcol[e0 + e] * NBX * cin + col;
        T sv[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) sv[s] = Sj[(size_t)s * cin];
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int s = 0; s < 6; ++s) o[r] += Ab[e * 36 + r * 6 + s] * sv[s];
      }
#pragma unroll
      for (int r = 0; r < 6; ++r) S_out[((size_t)i * NBX + r) * cout + col] = o[r];
    } else if (col < cout) {
      const T* Bi = B_k + (size_t)i * NBX * nu + (col - cin);
#pragma unroll
      for (int r = 0; r < 6; ++r) S_out[((size_t)i * NBX + r) * cout + col] = Bi[r * nu];
    } else {
      for (int e = 0; e < w; ++e) {
        const T* xj = Gx_in + (size_t)pcol[e0 + e] * NBX;
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int s = 0; s < 6; ++s) o[r] += Ab[e * 36 + r * 6 + s] * xj[s];
      }
#pragma unroll
      for (int r = 0; r < 6; ++r) Gx_out[(size_t)i * NBX + r] = o[r] + c_k[(size_t)i * NBX + r];
    }
  }
}

// ---------------------------------------------------------------- Gram + gradient
struct GramShape {
  int M, nu, N, n, nt, ntiles, nchunks;
};

__host__ __device__ inline int first_stage(int ta, int nu) { return (kTileH * ta) / nu + 1; }

// Decode the linear lower-triangle tile index into (ta, tb), ta >= tb.
__device__ inline void tile_coords(int t, int& ta, int& tb) {
  int a = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  ta = a;
  tb = t - a * (a + 1) / 2;
}

// grid: x = H tiles then g tiles, y = stage k-1, z = node chunk
template <typename T>
__global__ void __launch_bounds__(kGramThreads)
gram_kernel(GramShape sh, const T* __restrict__ S_all, const T* __restrict__ Gx_all, const T* __restrict__ Q,
            int Q_full, const T* __restrict__ q, T* __restrict__ part) {
  __shared__ T Sa[kRowsStaged][kTileH];
  __shared__ T Sb[kRowsStaged][kTileH];  // Q-weighted b operand (or the g vector)
  __shared__ T red[kGramThreads];
  const int k = blockIdx.y + 1;
  const int chunk = blockIdx.z;
  const bool is_g = blockIdx.x >= sh.ntiles;
  int ta, tb;
  if (is_g) {
    ta = blockIdx.x - sh.ntiles;
    tb = 0;
  } else {
    tile_coords(blockIdx.x, ta, tb);
  }
  if (k < first_stage(ta, sh.nu)) return;  // S_k has no live column in this tile
  const int cols = k * sh.nu;
  const T* Sk = S_all + S_offset(k, sh.M, sh.nu);
  const T* Gxk = Gx_all + (size_t)k * sh.M * NBX;
  const T* Qk = Q + (size_t)k * sh.M * NBX * (Q_full ? NBX : 1);
  const T* qk = q + (size_t)k * sh.M * NBX;
  const int a0 = kTileH * ta, b0 = kTileH * tb;
  const int n0 = chunk * kChunkNodes;
  const int n1 = min(sh.M, n0 + kChunkNodes);
  const int la = threadIdx.x / kTileH, lb = threadIdx.x % kTileH;
  T acc = T(0);
  for (int nb = n0; nb < n1; nb += kRowsStaged / NBX) {
    const int nodes = min(kRowsStaged / NBX, n1 - nb);
    const int rows = nodes * NBX;
    __syncthreads();
    // a operand: S_k rows x a-columns
    for (int t = threadIdx.x; t < rows * kTileH; t += kGramThreads) {
      int rr = t / kTileH, cc = t % kTileH;
      int ca = a0 + cc;
      Sa[rr][cc] = (ca < cols) ? Sk[((size_t)nb * NBX + rr) * cols + ca] : T(0);
    }
    // b operand: Q_k S_k (or the gradient weight Q_k Gx_k + q_k in column 0)
    for (int t = threadIdx.x; t < rows * kTileH; t += kGramThreads) {
      int rr = t / kTileH, cc = t % kTileH;
      int node = nb + rr / NBX, r = rr % NBX;
      T v = T(0);
      if (is_g) {
        if (cc == 0) {
          const T* gx = Gxk + (size_t)node * NBX;
          if (Q_full) {
            const T* Qn = Qk + ((size_t)node * NBX + r) * NBX;
            for (int s = 0; s < NBX; ++s) v += Qn[s] * gx[s];
          } else {
            v = Qk[(size_t)node * NBX + r] * gx[r];
          }
          v += qk[(size_t)node * NBX + r];
        }
      } else {
        int cb = b0 + cc;
        if (cb < cols) {
          if (Q_full) {
            const T* Qn = Qk + ((size_t)node * NBX + r) * NBX;
            const T* Sn = Sk + (size_t)node * NBX * cols + cb;
            for (int s = 0; s < NBX; ++s) v += Qn[s] * Sn[(size_t)s * cols];
          } else {
            v = Qk[(size_t)node * NBX + r] * Sk[((size_t)node * NBX + r) * cols + cb];
          }
        }
      }
      Sb[rr][cc] = v;
    }
    __syncthreads();
    if (is_g) {
      // lane (la, lb): column a = la, rows lb, lb+16, ...
      for (int rr = lb; rr < rows; rr += kTileH) acc += Sa[rr][la] * Sb[rr][0];
    } else {
      for (int rr = 0; rr < rows; ++rr) acc += Sa[rr][la] * Sb[rr][lb];
    }
  }
  const size_t slot = (((size_t)blockIdx.x * sh.N) + (k - 1)) * sh.nchunks + chunk;
  if (is_g) {
    red[threadIdx.x] = acc;
    __syncthreads();
    if (lb == 0) {
      T s = T(0);
      for (int t = 0; t < kTileH; ++t) s += red[la * kTileH + t];
      part[slot * (kTileH * kTileH) + la] = s;
    }
  } else {
    part[slot * (kTileH * kTileH) + threadIdx.x] = acc;
  }
}

// One lane per element of the lower triangle (and g): fixed-order sum of the
// partials over stages and chunks, plus R (or r), mirrored to the upper triangle.
template <typename T>
__global__ void gram_reduce_kernel(GramShape sh, const T* __restrict__ part, const T* __restrict__ R,
                                   const T* __restrict__ r, T* __restrict__ H, T* __restrict__ g) {
  const int n = sh.n;
  const long nlow = (long)n * (n + 1) / 2;
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nlow) {
    int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((long)(a + 1) * (a + 2) / 2 <= t) ++a;
    while ((long)a * (a + 1) / 2 > t) --a;
    int b = (int)(t - (long)a * (a + 1) / 2);
    int ta = a / kTileH, tb = b / kTileH;
    int tile = ta * (ta + 1) / 2 + tb;
    int e = (a % kTileH) * kTileH + (b % kTileH);
    T s = T(0);
    for (int k = first_stage(ta, sh.nu); k <= sh.N; ++k)
      for (int ch = 0; ch < sh.nchunks; ++ch)
        s += part[((((size_t)tile * sh.N) + (k - 1)) * sh.nchunks + ch) * (kTileH * kTileH) + e];
    int ka = a / sh.nu, kb = b / sh.nu;
    if (ka == kb) s += R[((size_t)ka * sh.nu + (a % sh.nu)) * sh.nu + (b % sh.nu)];
    H[(size_t)a * n + b] = s;
    H[(size_t)b * n + a] = s;
  } else if (t < nlow + n) {
    int a = (int)(t - nlow);
    int ta = a / kTileH;
    int tile = sh.ntiles + ta;
    T s = T(0);
    for (int k = first_stage(ta, sh.nu); k <= sh.N; ++k)
      for (int ch = 0; ch < sh.nchunks; ++ch)
        s += part[((((size_t)tile * sh.N) + (k - 1)) * sh.nchunks + ch) * (kTileH * kTileH) + (a % kTileH)];
    g[a] = s + r[a];
  }
}

// ---------------------------------------------------------------- constraint rows
template <typename T>
__global__ void cons_kernel(int M, int nu, int N, const int32_t* __restrict__ node, const int32_t* __restrict__ stage,
                            const T* __restrict__ C, const T* __restrict__ d, const T* __restrict__ S_all,
                            const T* __restrict__ Gx_all, T* __restrict__ Ct, T* __restrict__ dt) {
  const int t = blockIdx.x;
  const int i = node[t], k = stage[t];
  const int n = N * nu, cols = k * nu;
  const T* Sk = S_all + S_offset(k, M, nu) + (size_t)i * NBX * cols;
  T Cr[6];
#pragma unroll
  for (int r = 0; r < 6; ++r) Cr[r] = C[(size_t)t * NBX + r];
  for (int col = threadIdx.x; col < n; col += blockDim.x) {
    T v = T(0);
    if (col < cols) {
#pragma unroll
      for (int r = 0; r < 6; ++r) v += Cr[r] * Sk[(size_t)r * cols + col];
    }
    Ct[(size_t)t * n + col] = v;
  }
  if (threadIdx.x == 0) {
    const T* gx = Gx_all + ((size_t)k * M + i) * NBX;
    T v = d[t];
#pragma unroll
    for (int r = 0; r < 6; ++r) v -= Cr[r] * gx[r];
    dt[t] = v;
  }
}

GramShape gram_shape(int M, int nu, int N) {
  GramShape sh;
  sh.M = M;
  sh.nu = nu;
  sh.N = N;
  sh.n = N * nu;
  sh.nt = ceil_div(sh.n, kTileH);
  sh.ntiles = sh.nt * (sh.nt + 1) / 2;
  sh.nchunks = ceil_div(M, kChunkNodes);
  return sh;
}

template <typename T>
gnmpc_status run(gnmpc_plan* p, const void* A, const void* B, const void* c, const void* x0, const void* Q,
                 int Q_full, const void* q, const void* R, const void* r, const void* rowC, const void* rowd,
                 void* H, void* g, void* Ct, void* dt, void* Gx, hipStream_t s) {
  const int M = p->M, nu = p->dims.nu, N = p->dims.N;
  T* S = (T*)p->d_S;
  T* G = (T*)p->d_Gx;
  phase_begin(p, GNMPC_PH_CONDENSE_PROPAGATE, s);
  GNMPC_HIP_TRY(p, hipMemcpyAsync(G, x0, sizeof(T) * M * NBX, hipMemcpyDeviceToDevice, s));
  const int wmax = p->wmax;
  for (int k = 0; k < N; ++k) {
    int ncol = (k + 1) * nu + 1;
    int npw = std::max(1, kPropThreads / ncol);
    int lds_cap = (int)(48 * 1024 / (sizeof(T) * 36 * wmax));
    npw = std::max(1, std::min(npw, lds_cap));
    size_t lds = sizeof(T) * 36 * (size_t)wmax * npw;
    const T* S_in = k ? S + S_offset(k, M, nu) : nullptr;
    sprop_kernel<T><<<ceil_div(M, npw), kPropThreads, lds, s>>>(
        k, M, nu, npw, p->d_prow, p->d_pcol, (const T*)A + (size_t)k * p->nnz * 36,
        (const T*)B + (size_t)k * M * NBX * nu, (const T*)c + (size_t)k * M * NBX, S_in,
        S + S_offset(k + 1, M, nu), G + (size_t)k * M * NBX, G + (size_t)(k + 1) * M * NBX, wmax);
  }
  phase_end(p, GNMPC_PH_CONDENSE_PROPAGATE, s);
  GramShape sh = gram_shape(M, nu, N);
  dim3 grid(sh.ntiles + sh.nt, N, sh.nchunks);
  phase_begin(p, GNMPC_PH_CONDENSE_GRAM, s);
  gram_kernel<T><<<grid, kGramThreads, 0, s>>>(sh, S, G, (const T*)Q, Q_full, (const T*)q, (T*)p->d_part);
  long nred = (long)sh.n * (sh.n + 1) / 2 + sh.n;
  gram_reduce_kernel<T><<<ceil_div(nred, 256), 256, 0, s>>>(sh, (const T*)p->d_part, (const T*)R, (const T*)r,
                                                            (T*)H, (T*)g);
  phase_end(p, GNMPC_PH_CONDENSE_GRAM, s);
  if (p->n_c > 0) {
    phase_begin(p, GNMPC_PH_CONDENSE_ROWS, s);
    cons_kernel<T><<<p->n_c, 256, 0, s>>>(M, nu, N, p->d_row_node, p->d_row_stage, (const T*)rowC,
                                           (const T*)rowd, S, G, (T*)Ct, (T*)dt);
    phase_end(p, GNMPC_PH_CONDENSE_ROWS, s);
  }
  if (Gx)
    GNMPC_HIP_TRY(p, hipMemcpyAsync(Gx, G, sizeof(T) * (size_t)(N + 1) * M * NBX, hipMemcpyDeviceToDevice, s));
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

}  // namespace

size_t condense_partial_elems(int M, int nu, int N) {
  GramShape sh = gram_shape(M, nu, N);
  return (size_t)(sh.ntiles + sh.nt) * N * sh.nchunks * kTileH * kTileH;
}

gnmpc_status launch_condense(gnmpc_plan* p, const void* A, const void* B, const void* c, const void* x0,
                             const void* Q, int Q_full, const void* q, const void* R, const void* r,
                             const void* rowC, const void* rowd, void* H, void* g, void* Ct, void* dt, void* Gx,
                             hipStream_t s) {
  if (p->dims.dtype == GNMPC_F64)
    return run<double>(p, A, B, c, x0, Q, Q_full, q, R, r, rowC, rowd, H, g, Ct, dt, Gx, s);
  return run<float>(p, A, B, c, x0, Q, Q_full, q, R, r, rowC, rowd, H, g, Ct, dt, Gx, s);
}

}  // namespace gnmpc
