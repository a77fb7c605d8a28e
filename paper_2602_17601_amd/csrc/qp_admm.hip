// Condensed QP solve (Algorithm 1 "Solve QP"; the condensed QP of Sec. III-B
// with native box bounds):  min 1/2 u'Hu + g'u  s.t.  l <= A u <= u_b,
// A = [I; Ct].  Operator splitting (ADMM) in the form of Stellato et al.,
// "OSQP: an operator splitting solver for quadratic programs" (2020):
//   x~ = K^{-1} (sigma x - g + A'(rho z - y)),  K = H + sigma I + A' diag(rho) A
//   z~ = A x~,  x <- alpha x~ + (1-alpha) x,  zh = alpha z~ + (1-alpha) z
//   z <- clamp(zh + y/rho, l, u_b),  y <- y + rho (zh - z)
// with the OSQP stopping rule, its primal-infeasibility certificate and its
// rho adaptation (refactorization when the residual balance is off by > 5x).
//
// One workgroup of 1024 lanes solves one instance.  K is factored once per
// rho (right-looking Cholesky on the packed lower triangle, held in LDS when it
// fits) and L is inverted in place, so each iteration costs two packed
// triangular mat-vecs (W = L^{-1}: x~ = W'(W rhs)) plus one pass over Ct that
// fuses z~ = Ct x~, the z/y updates and the next A'(rho z - y).
// The condition number of K is estimated with Hager's 1-norm estimator
// (Hager 1984, Higham 1988) on the explicit W; above kappa_fp64 the FP32
// solver raises a flag and the FP64 instance of the same kernel (launched
// right behind it) redoes factorization and iterations in FP64.
#include <math.h>

#include "plan.hpp"

namespace gnmpc {
namespace {

constexpr int kQpThreads = 1024;
constexpr int kWaves = kQpThreads / 64;

template <typename Tin>
struct QpArgs {
  int n, n_c;
  const Tin *H, *g, *lb, *ub, *Ct, *lc, *uc;
  Tin* u;
  gnmpc_qp_info* info;
  const double* G;   // [n][n]: diag(rho_rel box) + Ct' diag(rho_rel rows) Ct
  double* gmat;      // global fallback storage for the packed factor (doubles)
  int32_t* flag;     // set by the FP32 pass when FP64 is required
  double rho, sigma, alpha, eps_abs, eps_rel, kappa_fp64;
  int max_iter, check_every;
};

__device__ inline double rho_rel(double l, double u) {
  if (!isfinite(l) && !isfinite(u)) return 1e-6;  // free row
  if (l == u) return 1e3;                          // equality row
  return 1.0;
}

// G = diag(rho_rel of the box rows) + Ct' diag(rho_rel of the state rows) Ct, in
// double, fixed summation order.  One lane per element of the lower triangle.
template <typename Tin>
__global__ void qp_gram_kernel(QpArgs<Tin> a, double* G) {
  const int n = a.n;
  const long nlow = (long)n * (n + 1) / 2;
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nlow) return;
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((long)(i + 1) * (i + 2) / 2 <= t) ++i;
  while ((long)i * (i + 1) / 2 > t) --i;
  int j = (int)(t - (long)i * (i + 1) / 2);
  double s = 0.0;
  for (int r = 0; r < a.n_c; ++r) {
    double l = a.lc ? (double)a.lc[r] : -INFINITY;
    double u = a.uc ? (double)a.uc[r] : INFINITY;
    s += rho_rel(l, u) * (double)a.Ct[(size_t)r * n + i] * (double)a.Ct[(size_t)r * n + j];
  }
  if (i == j) s += rho_rel((double)a.lb[i], (double)a.ub[i]);
  G[(size_t)i * n + j] = s;
  G[(size_t)j * n + i] = s;
}

__device__ inline size_t pk(int i, int j) { return (size_t)i * (i + 1) / 2 + j; }  // packed lower, j <= i

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Shared block-wide reductions through a small LDS array.
template <typename T>
__device__ T block_max(T v, T* red) {
  v = wave_max(v);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T r = red[0];
  for (int q = 1; q < kWaves; ++q) r = max(r, red[q]);
  return r;
}
template <typename T>
__device__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T r = red[0];
  for (int q = 1; q < kWaves; ++q) r += red[q];
  return r;
}

template <typename T>
struct Work {
  T* mat;   // packed lower triangle: K, then L, then W = L^{-1}
  T *x, *xt, *rhs, *tv, *ctv, *gv, *hx;   // [n]
  T *z, *y, *lo, *hi, *rho, *yprev;       // [m]
  T* part;  // [kWaves][n]
  T* red;   // [64]
  T* scal;  // [8]
};

// out = W v (W packed lower), 4 lanes per row.
template <typename T>
__device__ void tri_mv(const Work<T>& w, int n, const T* v, T* out) {
  for (int base = 0; base < n; base += kQpThreads / 4) {
    int i = base + threadIdx.x / 4;
    int q = threadIdx.x & 3;
    T s = T(0);
    if (i < n) {
      const T* row = w.mat + pk(i, 0);
      for (int p = q; p <= i; p += 4) s += row[p] * v[p];
    }
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (i < n && q == 0) out[i] = s;
  }
}
// out = W' v, 4 lanes per output.
template <typename T>
__device__ void tri_mv_t(const Work<T>& w, int n, const T* v, T* out) {
  for (int base = 0; base < n; base += kQpThreads / 4) {
    int p = base + threadIdx.x / 4;
    int q = threadIdx.x & 3;
    T s = T(0);
    if (p < n)
      for (int i = p + q; i < n; i += 4) s += w.mat[pk(i, p)] * v[i];
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (p < n && q == 0) out[p] = s;
  }
}
// out = K^{-1} v = W'(W v); uses w.tv as the intermediate.
template <typename T>
__device__ void kinv_apply(const Work<T>& w, int n, const T* v, T* out) {
  tri_mv(w, n, v, w.tv);
  __syncthreads();
  tri_mv_t(w, n, w.tv, out);
  __syncthreads();
}

// K = H + sigma I + s * G into the packed storage; returns ||K||_1.
template <typename T, typename Tin>
__device__ T form_K(const QpArgs<Tin>& a, const Work<T>& w, T s) {
  const int n = a.n;
  const long nlow = (long)n * (n + 1) / 2;
  for (long t = threadIdx.x; t < nlow; t += kQpThreads) {
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((long)(i + 1) * (i + 2) / 2 <= t) ++i;
    while ((long)i * (i + 1) / 2 > t) --i;
    int j = (int)(t - (long)i * (i + 1) / 2);
    T v = (T)a.H[(size_t)i * n + j] + s * (T)a.G[(size_t)i * n + j] + (i == j ? (T)a.sigma : T(0));
    w.mat[t] = v;
  }
  __syncthreads();
  // ||K||_1 = max column abs sum (K symmetric)
  T nrm = T(0);
  for (int c = threadIdx.x; c < n; c += kQpThreads) {
    T cs = T(0);
    for (int r = 0; r < n; ++r) cs += fabs(r >= c ? w.mat[pk(r, c)] : w.mat[pk(c, r)]);
    nrm = max(nrm, cs);
  }
  return block_max(nrm, w.red);
}

// In-place Cholesky of the packed matrix; returns false on a nonpositive pivot.
template <typename T>
__device__ bool cholesky(const Work<T>& w, int n) {
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      T d = w.mat[pk(j, j)];
      w.scal[0] = (d > T(0) && isfinite(d)) ? sqrt(d) : T(-1);
      if (w.scal[0] > T(0)) w.mat[pk(j, j)] = w.scal[0];
    }
    __syncthreads();
    T piv = w.scal[0];
    if (piv <= T(0)) return false;
    for (int i = j + 1 + threadIdx.x; i < n; i += kQpThreads) w.mat[pk(i, j)] /= piv;
    __syncthreads();
    // trailing update: 4 lanes per row i, lane q takes columns l = j+1+q, j+5+q, ...
    for (int i = j + 1 + (int)(threadIdx.x >> 2); i < n; i += kQpThreads / 4) {
      T* rowi = w.mat + pk(i, 0);
      const T lij = rowi[j];
      for (int l = j + 1 + (int)(threadIdx.x & 3); l <= i; l += 4) rowi[l] -= lij * w.mat[pk(l, j)];
    }
    __syncthreads();
  }
  return true;
}

// In-place inverse of the packed lower-triangular factor: column j (right to
// left) of W = L^{-1}: W_jj = 1/L_jj, W_ij = -W_jj sum_{p=j+1..i} W_ip L_pj.
template <typename T>
__device__ void tri_invert(const Work<T>& w, int n) {
  for (int j = n - 1; j >= 0; --j) {
    T wjj = T(1) / w.mat[pk(j, j)];
    for (int base = j + 1; base < n; base += kQpThreads / 4) {
      int i = base + threadIdx.x / 4;
      int q = threadIdx.x & 3;
      T s = T(0);
      if (i < n)
        for (int p = j + 1 + q; p <= i; p += 4) s += w.mat[pk(i, p)] * w.mat[pk(p, j)];
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      if (i < n && q == 0) w.tv[i] = -wjj * s;
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < n; i += kQpThreads) w.mat[pk(i, j)] = w.tv[i];
    if (threadIdx.x == 0) w.mat[pk(j, j)] = wjj;
    __syncthreads();
  }
}

// Hager's estimate of ||K^{-1}||_1 (K symmetric, so K^{-T} = K^{-1}).
template <typename T>
__device__ T inv_norm1_estimate(const Work<T>& w, int n) {
  T* v = w.hx;
  T* y = w.xt;
  for (int i = threadIdx.x; i < n; i += kQpThreads) v[i] = T(1) / T(n);
  __syncthreads();
  T est = T(0);
  for (int it = 0; it < 5; ++it) {
    kinv_apply(w, n, v, y);
    T y1 = T(0);
    for (int i = threadIdx.x; i < n; i += kQpThreads) y1 += fabs(y[i]);
    y1 = block_sum(y1, w.red);
    est = max(est, y1);
    for (int i = threadIdx.x; i < n; i += kQpThreads) w.rhs[i] = y[i] >= T(0) ? T(1) : T(-1);
    __syncthreads();
    kinv_apply(w, n, w.rhs, y);  // z = K^{-1} sign(y)
    T zmax = T(0), ztx = T(0);
    int jmax = 0;
    // argmax |z| (first index on ties), z'v
    for (int i = threadIdx.x; i < n; i += kQpThreads) ztx += y[i] * v[i];
    ztx = block_sum(ztx, w.red);
    if (threadIdx.x == 0) {
      for (int i = 0; i < n; ++i)
        if (fabs(y[i]) > zmax) {
          zmax = fabs(y[i]);
          jmax = i;
        }
      w.scal[1] = zmax;
      w.scal[2] = (T)jmax;
    }
    __syncthreads();
    zmax = w.scal[1];
    jmax = (int)w.scal[2];
    if (zmax <= ztx) break;
    for (int i = threadIdx.x; i < n; i += kQpThreads) v[i] = (i == jmax) ? T(1) : T(0);
    __syncthreads();
  }
  __syncthreads();
  return est;
}

// Factor K(s) and invert; false if K is not positive definite.
template <typename T, typename Tin>
__device__ bool factor(const QpArgs<Tin>& a, const Work<T>& w, T s, T* knorm) {
  *knorm = form_K(a, w, s);
  __syncthreads();
  if (!cholesky(w, a.n)) return false;
  tri_invert(w, a.n);
  return true;
}

template <typename T, typename Tin>
__global__ void __launch_bounds__(kQpThreads) qp_solve_kernel(QpArgs<Tin> a, int mode, int mat_in_lds) {
  // mode 0: primary pass in T (may hand over to FP64); 1: FP64 pass, runs only
  // if the primary pass raised the flag; 2: the only pass.
  if (mode == 1 && *(volatile int32_t*)a.flag == 0) return;
  extern __shared__ unsigned char smem_raw[];
  const int n = a.n, nc = a.n_c, m = n + nc;
  T* sp = reinterpret_cast<T*>(smem_raw);
  Work<T> w;
  size_t off = 0;
  auto take = [&](size_t cnt) {
    T* p = sp + off;
    off += (cnt + 1) & ~(size_t)1;
    return p;
  };
  w.x = take(n); w.xt = take(n); w.rhs = take(n); w.tv = take(n); w.ctv = take(n); w.gv = take(n); w.hx = take(n);
  w.z = take(m); w.y = take(m); w.lo = take(m); w.hi = take(m); w.rho = take(m); w.yprev = take(m);
  w.part = take((size_t)kWaves * n);
  w.red = take(64);
  w.scal = take(8);
  w.mat = mat_in_lds ? take((size_t)n * (n + 1) / 2) : reinterpret_cast<T*>(a.gmat);

  // ---- load problem vectors
  for (int i = threadIdx.x; i < m; i += kQpThreads) {
    T lo, hi;
    if (i < n) {
      lo = (T)a.lb[i];
      hi = (T)a.ub[i];
    } else {
      lo = a.lc ? (T)a.lc[i - n] : -INFINITY;
      hi = a.uc ? (T)a.uc[i - n] : INFINITY;
    }
    w.lo[i] = lo;
    w.hi[i] = hi;
    w.rho[i] = (T)(a.rho * rho_rel((double)lo, (double)hi));
    w.z[i] = T(0);
    w.y[i] = T(0);
    w.yprev[i] = T(0);
  }
  for (int i = threadIdx.x; i < n; i += kQpThreads) {
    w.x[i] = T(0);
    w.gv[i] = (T)a.g[i];
    w.ctv[i] = T(0);
  }
  __syncthreads();
  // ---- finiteness of the data
  {
    int bad = 0;
    for (long t = threadIdx.x; t < (long)n * n; t += kQpThreads) bad |= !isfinite((T)a.H[t]);
    for (long t = threadIdx.x; t < (long)nc * n; t += kQpThreads) bad |= !isfinite((T)a.Ct[t]);
    for (int i = threadIdx.x; i < n; i += kQpThreads) bad |= !isfinite(w.gv[i]);
    T b = block_max((T)bad, w.red);
    if (b > T(0)) {
      if (mode == 0 && threadIdx.x == 0) *a.flag = 0;
      if (threadIdx.x == 0 && a.info) {
        a.info->status = GNMPC_QP_NONFINITE;
        a.info->iters = 0;
      }
      for (int i = threadIdx.x; i < n; i += kQpThreads) a.u[i] = (Tin)NAN;
      return;
    }
  }

  T scale = T(1);  // rho = scale * rho_rel * a.rho
  T knorm;
  bool ok = factor(a, w, (T)a.rho * scale, &knorm);
  if (!ok) {
    if (mode == 0 && sizeof(T) == 4) {  // let the FP64 pass try
      if (threadIdx.x == 0) *a.flag = 1;
      return;
    }
    if (threadIdx.x == 0 && a.info) {
      a.info->status = GNMPC_QP_NOT_PD;
      a.info->iters = 0;
      a.info->used_fp64 = sizeof(T) == 8;
    }
    for (int i = threadIdx.x; i < n; i += kQpThreads) a.u[i] = (Tin)NAN;
    return;
  }
  T kappa = knorm * inv_norm1_estimate(w, n);
  if (mode == 0 && sizeof(T) == 4 && (double)kappa > a.kappa_fp64) {
    if (threadIdx.x == 0) *a.flag = 1;
    return;
  }
  if (mode == 0 && threadIdx.x == 0) *a.flag = 0;

  const T sigma = (T)a.sigma, alpha = (T)a.alpha;
  int status = GNMPC_QP_MAXITER;
  int iter = 0;
  T prim = T(0), dual = T(0);
  int refactors = 0;
  for (iter = 1; iter <= a.max_iter; ++iter) {
    // rhs = sigma x - g + (rho z - y)_box + Ct'(rho z - y)_rows
    for (int i = threadIdx.x; i < n; i += kQpThreads)
      w.rhs[i] = sigma * w.x[i] - w.gv[i] + w.rho[i] * w.z[i] - w.y[i] + w.ctv[i];
    __syncthreads();
    kinv_apply(w, n, w.rhs, w.xt);
    // box rows
    for (int i = threadIdx.x; i < n; i += kQpThreads) {
      T zt = w.xt[i];
      w.x[i] = alpha * zt + (T(1) - alpha) * w.x[i];
      T zh = alpha * zt + (T(1) - alpha) * w.z[i];
      T zn = min(max(zh + w.y[i] / w.rho[i], w.lo[i]), w.hi[i]);
      w.y[i] += w.rho[i] * (zh - zn);
      w.z[i] = zn;
    }
    // state rows: z~ = Ct x~, updates, and the next Ct'(rho z - y)
    {
      const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
      T* pw = w.part + (size_t)wid * n;
      for (int c = lane; c < n; c += 64) pw[c] = T(0);
      for (int r = wid; r < nc; r += kWaves) {
        const Tin* crow = a.Ct + (size_t)r * n;
        T s = T(0);
        for (int c = lane; c < n; c += 64) s += (T)crow[c] * w.xt[c];
        s = wave_sum(s);
        const int ri = n + r;
        T zh = alpha * s + (T(1) - alpha) * w.z[ri];
        T zn = min(max(zh + w.y[ri] / w.rho[ri], w.lo[ri]), w.hi[ri]);
        T yn = w.y[ri] + w.rho[ri] * (zh - zn);
        T v = w.rho[ri] * zn - yn;
        if (lane == 0) {
          w.z[ri] = zn;
          w.y[ri] = yn;
        }
        for (int c = lane; c < n; c += 64) pw[c] += (T)crow[c] * v;
      }
      __syncthreads();
      for (int c = threadIdx.x; c < n; c += kQpThreads) {
        T s = T(0);
        for (int q = 0; q < kWaves; ++q) s += w.part[(size_t)q * n + c];
        w.ctv[c] = s;
      }
      __syncthreads();
    }
    if (iter % a.check_every != 0 && iter != a.max_iter) continue;

    // ---- residuals (OSQP): prim = ||Ax - z||, dual = ||Hx + g + A'y||
    T ax_max = T(0), z_max = T(0), pr = T(0);
    for (int i = threadIdx.x; i < n; i += kQpThreads) {
      pr = max(pr, fabs(w.x[i] - w.z[i]));
      ax_max = max(ax_max, fabs(w.x[i]));
      z_max = max(z_max, fabs(w.z[i]));
    }
    {
      const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
      T* pw = w.part + (size_t)wid * n;
      for (int c = lane; c < n; c += 64) pw[c] = T(0);
      for (int r = wid; r < nc; r += kWaves) {
        const Tin* crow = a.Ct + (size_t)r * n;
        T s = T(0);
        for (int c = lane; c < n; c += 64) s += (T)crow[c] * w.x[c];
        s = wave_sum(s);
        const int ri = n + r;
        if (lane == 0) {
          pr = max(pr, fabs(s - w.z[ri]));
          ax_max = max(ax_max, fabs(s));
          z_max = max(z_max, fabs(w.z[ri]));
        }
        T yv = w.y[ri];
        for (int c = lane; c < n; c += 64) pw[c] += (T)crow[c] * yv;
      }
    }
    __syncthreads();
    T du = T(0), hx_max = T(0), aty_max = T(0), g_max = T(0);
    for (int i = threadIdx.x; i < n; i += kQpThreads) {
      T aty = w.y[i];
      for (int q = 0; q < kWaves; ++q) aty += w.part[(size_t)q * n + i];
      T hx = T(0);
      const Tin* hrow = a.H + (size_t)i * n;
      for (int c = 0; c < n; ++c) hx += (T)hrow[c] * w.x[c];
      du = max(du, fabs(hx + w.gv[i] + aty));
      hx_max = max(hx_max, fabs(hx));
      aty_max = max(aty_max, fabs(aty));
      g_max = max(g_max, fabs(w.gv[i]));
    }
    prim = block_max(pr, w.red);
    ax_max = block_max(ax_max, w.red);
    z_max = block_max(z_max, w.red);
    dual = block_max(du, w.red);
    hx_max = block_max(hx_max, w.red);
    aty_max = block_max(aty_max, w.red);
    g_max = block_max(g_max, w.red);
    const T eps_p = (T)a.eps_abs + (T)a.eps_rel * max(ax_max, z_max);
    const T eps_d = (T)a.eps_abs + (T)a.eps_rel * max(max(hx_max, aty_max), g_max);
    if (!isfinite(prim) || !isfinite(dual)) {
      status = GNMPC_QP_NONFINITE;
      break;
    }
    if (prim <= eps_p && dual <= eps_d) {
      status = GNMPC_QP_SOLVED;
      break;
    }
    // ---- primal infeasibility certificate from dy = y - yprev
    {
      T dy_max = T(0), support = T(0);
      for (int i = threadIdx.x; i < m; i += kQpThreads) {
        T dy = w.y[i] - w.yprev[i];
        dy_max = max(dy_max, fabs(dy));
        T hi = w.hi[i], lo = w.lo[i];
        T sv = T(0);
        if (dy > T(0)) sv = isfinite(hi) ? hi * dy : T(INFINITY);
        else if (dy < T(0)) sv = isfinite(lo) ? lo * dy : T(INFINITY);
        support += sv;
      }
      dy_max = block_max(dy_max, w.red);
      support = block_sum(support, w.red);
      // A' dy: box part plus Ct' dy_rows
      const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
      T* pw = w.part + (size_t)wid * n;
      for (int c = lane; c < n; c += 64) pw[c] = T(0);
      for (int r = wid; r < nc; r += kWaves) {
        const Tin* crow = a.Ct + (size_t)r * n;
        T dy = w.y[n + r] - w.yprev[n + r];
        for (int c = lane; c < n; c += 64) pw[c] += (T)crow[c] * dy;
      }
      __syncthreads();
      T atdy = T(0);
      for (int c = threadIdx.x; c < n; c += kQpThreads) {
        T s = w.y[c] - w.yprev[c];
        for (int q = 0; q < kWaves; ++q) s += w.part[(size_t)q * n + c];
        atdy = max(atdy, fabs(s));
      }
      atdy = block_max(atdy, w.red);
      const T eps_inf = T(1e-5);
      if (dy_max > T(0) && atdy <= eps_inf * dy_max && support <= -eps_inf * dy_max) {
        status = GNMPC_QP_PRIMAL_INFEASIBLE;
        break;
      }
      for (int i = threadIdx.x; i < m; i += kQpThreads) w.yprev[i] = w.y[i];
    }
    // ---- rho adaptation
    {
      T pn = prim / max(max(ax_max, z_max), T(1e-30));
      T dn = dual / max(max(max(hx_max, aty_max), g_max), T(1e-30));
      T ratio = sqrt(pn / max(dn, T(1e-30)));
      if ((ratio > T(5) || ratio < T(0.2)) && refactors < 8 && iter < a.max_iter) {
        T s_new = min(max(scale * ratio, T(1e-6)), T(1e6));
        for (int i = threadIdx.x; i < m; i += kQpThreads) {
          w.rho[i] = w.rho[i] * (s_new / scale);
        }
        scale = s_new;
        __syncthreads();
        T kn;
        if (!factor(a, w, (T)a.rho * scale, &kn)) {
          status = GNMPC_QP_NOT_PD;
          break;
        }
        ++refactors;
        // the cached Ct'(rho z - y) must use the new rho
        const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
        T* pw = w.part + (size_t)wid * n;
        for (int c = lane; c < n; c += 64) pw[c] = T(0);
        for (int r = wid; r < nc; r += kWaves) {
          const Tin* crow = a.Ct + (size_t)r * n;
          T v = w.rho[n + r] * w.z[n + r] - w.y[n + r];
          for (int c = lane; c < n; c += 64) pw[c] += (T)crow[c] * v;
        }
        __syncthreads();
        for (int c = threadIdx.x; c < n; c += kQpThreads) {
          T s = T(0);
          for (int q = 0; q < kWaves; ++q) s += w.part[(size_t)q * n + c];
          w.ctv[c] = s;
        }
      }
    }
    __syncthreads();
  }
  __syncthreads();
  // ---- outputs
  T obj = T(0);
  for (int i = threadIdx.x; i < n; i += kQpThreads) {
    T hx = T(0);
    const Tin* hrow = a.H + (size_t)i * n;
    for (int c = 0; c < n; ++c) hx += (T)hrow[c] * w.x[c];
    obj += w.x[i] * (T(0.5) * hx + w.gv[i]);
    a.u[i] = (Tin)w.x[i];
  }
  obj = block_sum(obj, w.red);
  if (threadIdx.x == 0 && a.info) {
    a.info->status = status;
    a.info->iters = min(iter, a.max_iter);
    a.info->used_fp64 = (sizeof(T) == 8 && mode == 1) ? 1 : 0;
    a.info->prim_res = (double)prim;
    a.info->dual_res = (double)dual;
    a.info->kappa_est = (double)kappa;
    a.info->obj = (double)obj;
  }
}

size_t lds_bytes(int n, int nc, size_t elem, bool mat) {
  const int m = n + nc;
  auto r2 = [](size_t c) { return (c + 1) & ~(size_t)1; };
  size_t e = 7 * r2(n) + 6 * r2(m) + r2((size_t)kWaves * n) + 64 + 8;
  if (mat) e += r2((size_t)n * (n + 1) / 2);
  return e * elem;
}

constexpr size_t kLdsCap = 160 * 1024;

template <typename T, typename Tin>
gnmpc_status launch_pass(gnmpc_plan* p, const QpArgs<Tin>& a, int mode, hipStream_t s) {
  bool in_lds = lds_bytes(a.n, a.n_c, sizeof(T), true) <= kLdsCap;
  size_t lds = lds_bytes(a.n, a.n_c, sizeof(T), in_lds);
  if (lds > kLdsCap) {
    p->last_error = "QP too large for one workgroup's LDS";
    return GNMPC_UNSUPPORTED;
  }
  GNMPC_HIP_TRY(p, hipFuncSetAttribute((const void*)qp_solve_kernel<T, Tin>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  qp_solve_kernel<T, Tin><<<1, kQpThreads, lds, s>>>(a, mode, in_lds ? 1 : 0);
  return GNMPC_OK;
}

template <typename Tin>
gnmpc_status run(gnmpc_plan* p, int n, const void* H, const void* g, const void* lb, const void* ub, int n_c,
                 const void* Ct, const void* lc, const void* uc, const gnmpc_admm_settings* st, void* u,
                 gnmpc_qp_info* info, hipStream_t s) {
  QpArgs<Tin> a;
  a.n = n;
  a.n_c = n_c;
  a.H = (const Tin*)H;
  a.g = (const Tin*)g;
  a.lb = (const Tin*)lb;
  a.ub = (const Tin*)ub;
  a.Ct = (const Tin*)Ct;
  a.lc = (const Tin*)lc;
  a.uc = (const Tin*)uc;
  a.u = (Tin*)u;
  a.info = info;
  unsigned char* ws = (unsigned char*)p->d_qp;
  a.G = (const double*)ws;
  a.gmat = (double*)(ws + sizeof(double) * (size_t)n * n);
  a.flag = p->d_qp_flag;
  a.rho = st->rho;
  a.sigma = st->sigma;
  a.alpha = st->alpha;
  a.eps_abs = st->eps_abs;
  a.eps_rel = st->eps_rel;
  a.kappa_fp64 = st->kappa_fp64;
  a.max_iter = st->max_iter;
  a.check_every = st->check_every;
  long nlow = (long)n * (n + 1) / 2;
  phase_begin(p, GNMPC_PH_QP, s);
  qp_gram_kernel<Tin><<<ceil_div(nlow, 256), 256, 0, s>>>(a, (double*)ws);
  gnmpc_status rc;
  if (sizeof(Tin) == 8) {
    rc = launch_pass<double, Tin>(p, a, 2, s);
  } else {
    rc = launch_pass<float, Tin>(p, a, 0, s);
    if (rc == GNMPC_OK) rc = launch_pass<double, Tin>(p, a, 1, s);
  }
  phase_end(p, GNMPC_PH_QP, s);
  if (rc != GNMPC_OK) return rc;
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

}  // namespace

size_t qp_workspace_bytes(int n, int n_c) {
  (void)n_c;
  return sizeof(double) * ((size_t)n * n + (size_t)n * (n + 1) / 2 + 64);
}

gnmpc_status launch_qp(gnmpc_plan* p, int n, const void* H, const void* g, const void* lb, const void* ub, int n_c,
                       const void* Ct, const void* lc, const void* uc, const gnmpc_admm_settings* st, void* u,
                       gnmpc_qp_info* info, hipStream_t s) {
  if (p->dims.dtype == GNMPC_F64) return run<double>(p, n, H, g, lb, ub, n_c, Ct, lc, uc, st, u, info, s);
  return run<float>(p, n, H, g, lb, ub, n_c, Ct, lc, uc, st, u, info, s);
}

}  // namespace gnmpc
