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
// One workgroup of 512 lanes (8 waves) solves one instance.  K is factored once per
// rho (right-looking Cholesky on the packed lower triangle, held in LDS when it
// fits) and L is inverted in place, so each iteration costs two packed
// triangular mat-vecs (W = L^{-1}: x~ = W'(W rhs)) plus one pass over Ct that
// fuses z~ = Ct x~, the z/y updates and the next A'(rho z - y).
// The condition number of K is first bounded by ||K||_1 ||W||_1 ||W||_inf (one
// pass over W); only when that bound exceeds kappa_fp64 is it estimated with
// Hager's 1-norm estimator (Hager 1984, Higham 1988) on the explicit W.  Above
// kappa_fp64 the FP32 solver raises a flag and the FP64 instance of the same
// kernel (launched right behind it) redoes factorization and iterations in FP64.
#include <math.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "plan.hpp"

namespace gnmpc {
namespace {

constexpr int kQpThreads = 512;
constexpr int kWaves = kQpThreads / 64;
// This lane's wave in the workgroup, as a wave-uniform (scalar) value, so loops
// and tests over waves compile to scalar branches instead of exec-mask updates.
__device__ inline int wave_index() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

template <typename Tin>
struct QpArgs {
  int n, n_c;
  const Tin *H, *g, *lb, *ub, *Ct, *lc, *uc;
  Tin* u;
  gnmpc_qp_info* info;
  const double* G;   // [n][n]: diag(rho_rel box) + Ct' diag(rho_rel rows) Ct
  double* gmat;      // global fallback storage for the packed factor (doubles)
  double* Kp;        // K = H + sigma I + rho G in the block storage, written by qp_prep_kernel
  float* Kf;         // the same K rounded to FP32, for the FP32 pass
  int32_t* flag;     // [0]: FP64 pass required; [1]: non-finite H or Ct seen by qp_prep_kernel
  double rho, sigma, alpha, eps_abs, eps_rel, kappa_fp64;
  int max_iter, check_every;
};

__device__ inline double rho_rel(double l, double u) {
  if (!isfinite(l) && !isfinite(u)) return 1e-6;  // free row
  if (l == u) return 1e3;                          // equality row
  return 1.0;
}

// K, L and W = L^{-1} are kept as the lower triangle of 16x16 blocks, block
// (I, J <= I) row-major at bo(I, J); the order is padded to 16 nb with identity.
constexpr int kBS = 16;
__host__ __device__ inline int nblocks(int n) { return (n + kBS - 1) / kBS; }
__host__ __device__ inline size_t bo(int I, int J) { return ((size_t)I * (I + 1) / 2 + J) * (kBS * kBS); }
// per-wave partial sums of Ct' v
__host__ __device__ inline size_t part_elems(int n) {
  const size_t a = (size_t)(kQpThreads / 64) * n;
  return a > 256 ? a : 256;  // also the 16x16 scratch of the diagonal-block factorization
}
__device__ inline size_t ep(int i, int j) { return bo(i >> 4, j >> 4) + (i & 15) * kBS + (j & 15); }

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

// Order this wave's memory accesses across lanes: a value one lane stores to
// the factor storage (LDS, or global memory when the factor does not fit LDS)
// is read by other lanes of the same wave after this point.  The hardware
// performs a wave's memory operations in order; the wavefront-scope fence
// keeps the compiler from moving loads or stores across the point.
__device__ __attribute__((always_inline)) inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Shared block-wide reductions through a small LDS array.
template <typename T>
__device__ __attribute__((always_inline)) T block_max(T v, T* red) {
  v = wave_max(v);
  int w = wave_index(), l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T r = red[0];
  for (int q = 1; q < kWaves; ++q) r = max(r, red[q]);
  return r;
}
template <typename T>
__device__ __attribute__((always_inline)) T block_sum(T v, T* red) {
  v = wave_sum(v);
  int w = wave_index(), l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T r = red[0];
  for (int q = 1; q < kWaves; ++q) r += red[q];
  return r;
}

// Largest |v[i]| over i < n and its first index (ties: smallest index), for the
// whole block; red needs 2 kWaves entries.
template <typename T>
__device__ void block_argmax_abs(const T* v, int n, T* red, T& vmax, int& imax) {
  T bv = T(-1);
  int bi = 0x7FFFFFFF;
  for (int i = threadIdx.x; i < n; i += kQpThreads) {
    const T a = fabs(v[i]);
    if (a > bv) {  // i increases, so the first maximum of this lane is kept
      bv = a;
      bi = i;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const T ov = __shfl_xor(bv, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  const int w = wave_index(), l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
    red[w] = bv;
    red[kWaves + w] = (T)bi;
  }
  __syncthreads();
  vmax = red[0];
  imax = (int)red[kWaves];
  for (int q = 1; q < kWaves; ++q) {
    const T ov = red[q];
    const int oi = (int)red[kWaves + q];
    if (ov > vmax || (ov == vmax && oi < imax)) {
      vmax = ov;
      imax = oi;
    }
  }
  __syncthreads();
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

typedef float qfloatx4 __attribute__((ext_vector_type(4)));

// 16x16 block products, row layout: lane l holds acc[t] = (A op(B))[l & 15][4 (l >> 4) + t],
// op(B) = B' if TRANS else B; blocks are row-major.  Both types run the transposed
// product on the matrix cores (v_mfma_f32_16x16x4f32, v_mfma_f64_16x16x4f64) with
// the k index permuted (step s takes k = 4 (l >> 4) + s), so A rows, B' rows and
// the result are read and written as 16-byte runs: a lane reads 4 + 4 elements
// per product, which matters where the blocks sit in global memory (the FP64
// factor of a large K).  The FP64 instruction leaves row g + 4 t of its result
// where the FP32 one leaves row 4 g + t (g = l >> 4), so the FP64 product takes
// op(B)'s columns in the order pi(r) = 4 (r & 3) + (r >> 2), which puts the result
// in the same row layout.
template <bool TRANS>
__device__ inline void bmma(float acc[4], const float* A, const float* B) {
  const int l = threadIdx.x & 63, r = l & 15, kq = l >> 4;
  const float4 a4 = *reinterpret_cast<const float4*>(A + r * 16 + 4 * kq);
  float b[4];
  if (TRANS) {
    const float4 b4 = *reinterpret_cast<const float4*>(B + r * 16 + 4 * kq);
    b[0] = b4.x; b[1] = b4.y; b[2] = b4.z; b[3] = b4.w;
  } else {
#pragma unroll
    for (int st = 0; st < 4; ++st) b[st] = B[(4 * kq + st) * 16 + r];
  }
  const float av[4] = {a4.x, a4.y, a4.z, a4.w};
  qfloatx4 c = {acc[0], acc[1], acc[2], acc[3]};
#pragma unroll
  for (int st = 0; st < 4; ++st) c = __builtin_amdgcn_mfma_f32_16x16x4f32(b[st], av[st], c, 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = c[i];
}
typedef double qdoublex4 __attribute__((ext_vector_type(4)));
template <bool TRANS>
__device__ inline void bmma(double acc[4], const double* A, const double* B) {
  const int l = threadIdx.x & 63, r = l & 15, kq = l >> 4;
  const double2 a01 = *reinterpret_cast<const double2*>(A + r * 16 + 4 * kq);
  const double2 a23 = *reinterpret_cast<const double2*>(A + r * 16 + 4 * kq + 2);
  const double av[4] = {a01.x, a01.y, a23.x, a23.y};
  const int pr = 4 * (r & 3) + (r >> 2);
  double b[4];
  if (TRANS) {
    const double2 b01 = *reinterpret_cast<const double2*>(B + pr * 16 + 4 * kq);
    const double2 b23 = *reinterpret_cast<const double2*>(B + pr * 16 + 4 * kq + 2);
    b[0] = b01.x; b[1] = b01.y; b[2] = b23.x; b[3] = b23.y;
  } else {
#pragma unroll
    for (int st = 0; st < 4; ++st) b[st] = B[(4 * kq + st) * 16 + pr];
  }
  qdoublex4 c = {acc[0], acc[1], acc[2], acc[3]};
#pragma unroll
  for (int st = 0; st < 4; ++st) c = __builtin_amdgcn_mfma_f64_16x16x4f64(b[st], av[st], c, 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = c[i];
}

// Set-up over many workgroups, one workgroup per 16x16 block (I, J <= I) of
// the block storage and one lane per element:
// G = diag(rho_rel of the box rows) + Ct' diag(rho_rel of the state rows) Ct
// (FP64, rows summed in order, full symmetric, kept for refactorizations) and
// the first K = H + sigma I + rho G in the block storage; non-finite H or Ct
// raise flag[1].  Column slices of Ct are staged through LDS 64 rows at a time.
constexpr int kPrepRows = 224;  // rows staged per pass (every load of a pass in flight at once)
template <typename Tin>
__global__ void __launch_bounds__(256) qp_prep_kernel(QpArgs<Tin> a, double* G, QpArgs<Tin>* desc_out) {
  __shared__ double ci[kPrepRows][16], cj[kPrepRows][16], rr[kPrepRows];
  // the solve descriptor, for a batched solve that reads it from memory
  if (desc_out && blockIdx.x == 0 && threadIdx.x == 0) *desc_out = a;
  const int n = a.n;
  const int b = blockIdx.x, e = threadIdx.x;
  int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= b) ++I;
  while (I * (I + 1) / 2 > b) --I;
  const int J = b - I * (I + 1) / 2;
  const int i = kBS * I + (e >> 4), j = kBS * J + (e & 15);
  const bool in = j <= i && i < n && j < n;
  const double h = in ? (double)a.H[(size_t)i * n + j] : 0.0;  // issued before the row loop
  double sg = 0.0;
  constexpr int kPer = kPrepRows * 32 / 256;
  for (int r0 = 0; r0 < a.n_c; r0 += kPrepRows) {
    __syncthreads();
    Tin v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = e + 256 * u, rl = t >> 5, c = t & 31, r = r0 + rl;
      const int col = c < 16 ? kBS * I + c : kBS * J + (c - 16);
      v[u] = (r < a.n_c && col < n) ? a.Ct[(size_t)r * n + col] : Tin(0);
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = e + 256 * u, rl = t >> 5, c = t & 31;
      if (c < 16) ci[rl][c] = (double)v[u];
      else cj[rl][c - 16] = (double)v[u];
    }
    for (int t = e; t < kPrepRows; t += 256) {
      const int r = r0 + t;
      double rel = 0.0;
      if (r < a.n_c) {
        const double l = a.lc ? (double)a.lc[r] : -INFINITY;
        const double u = a.uc ? (double)a.uc[r] : INFINITY;
        rel = rho_rel(l, u);
      }
      rr[t] = rel;
    }
    __syncthreads();
    const int nr = min(kPrepRows, a.n_c - r0);
    for (int rl = 0; rl < nr; ++rl) sg += rr[rl] * ci[rl][e >> 4] * cj[rl][e & 15];
  }
  double kv;
  if (j > i) {
    kv = 0.0;
  } else if (i >= n || j >= n) {
    kv = (i == j) ? 1.0 : 0.0;
  } else {
    if (i == j) sg += rho_rel((double)a.lb[i], (double)a.ub[i]);
    G[(size_t)i * n + j] = sg;
    G[(size_t)j * n + i] = sg;
    kv = h + a.rho * sg + (i == j ? a.sigma : 0.0);
    if (!isfinite(kv)) __hip_atomic_fetch_or(a.flag + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  a.Kp[(size_t)b * 256 + e] = kv;
  a.Kf[(size_t)b * 256 + e] = (float)kv;
}

// Four consecutive elements of a 16-byte aligned array.
__device__ inline void ld4(const float* p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
__device__ inline void ld4(const double* p, double (&o)[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  o[0] = a.x;
  o[1] = a.y;
  o[2] = b.x;
  o[3] = b.y;
}

// Triangular mat-vecs with W in the block storage.  A wave reads a whole
// 16x16 block per instruction (lane l: row l >> 2, columns 4 (l & 3) .. +3);
// jobs pair block rows (columns) I and nb-1-I so every wave gets ~nb + 1
// blocks.  Input vectors are zero-padded to 16 nb entries.
// out = W v over the first n rows.
template <typename T>
__device__ void tri_mv(const Work<T>& w, int n, const T* v, T* out) {
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int nb = nblocks(n), r = lane >> 2, c4 = (lane & 3) * 4;
  for (int job = wave; job < (nb + 1) / 2; job += kWaves) {
    for (int half = 0; half < 2; ++half) {
      const int I = half == 0 ? job : nb - 1 - job;
      if (half == 1 && I == job) break;
      const T* brow = w.mat + bo(I, 0) + r * 16 + c4;
      T s = T(0);
#pragma unroll 4
      for (int J = 0; J <= I; ++J) {
        T wv[4], vv[4];
        ld4(brow + (size_t)J * 256, wv);
        ld4(v + 16 * J + c4, vv);
        s += wv[0] * vv[0] + wv[1] * vv[1] + wv[2] * vv[2] + wv[3] * vv[3];
      }
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      if ((lane & 3) == 0 && 16 * I + r < n) out[16 * I + r] = s;
    }
  }
}
// out = W' v over the first n rows.
template <typename T>
__device__ void tri_mv_t(const Work<T>& w, int n, const T* v, T* out) {
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int nb = nblocks(n), r = lane >> 2, c4 = (lane & 3) * 4;
  for (int job = wave; job < (nb + 1) / 2; job += kWaves) {
    for (int half = 0; half < 2; ++half) {
      const int J = half == 0 ? job : nb - 1 - job;
      if (half == 1 && J == job) break;
      T p[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll 4
      for (int I = J; I < nb; ++I) {
        T wv[4];
        ld4(w.mat + bo(I, J) + r * 16 + c4, wv);
        const T uv = v[16 * I + r];
#pragma unroll
        for (int k = 0; k < 4; ++k) p[k] += wv[k] * uv;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        p[k] += __shfl_xor(p[k], 4, 64);
        p[k] += __shfl_xor(p[k], 8, 64);
        p[k] += __shfl_xor(p[k], 16, 64);
        p[k] += __shfl_xor(p[k], 32, 64);
      }
      if (lane < 4) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (16 * J + c4 + k < n) out[16 * J + c4 + k] = p[k];
      }
    }
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

// K = H + sigma I + s * G into the block storage (identity padding); returns ||K||_1.
template <typename T, typename Tin>
__device__ T form_K(const QpArgs<Tin>& a, const Work<T>& w, T s) {
  const int n = a.n, nb = nblocks(n);
  const long total = (long)nb * (nb + 1) / 2 * 256;
  for (long t = threadIdx.x; t < total; t += kQpThreads) {
    const int b = (int)(t >> 8), e = (int)(t & 255);
    int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    while (I * (I + 1) / 2 > b) --I;
    const int J = b - I * (I + 1) / 2;
    const int i = 16 * I + (e >> 4), j = 16 * J + (e & 15);
    T v;
    if (j > i) v = T(0);
    else if (i < n && j < n) v = (T)a.H[(size_t)i * n + j] + s * (T)a.G[(size_t)i * n + j] + (i == j ? (T)a.sigma : T(0));
    else v = (i == j) ? T(1) : T(0);
    w.mat[t] = v;
  }
  __syncthreads();
  T nrm = T(0);
  for (int c = threadIdx.x; c < n; c += kQpThreads) {
    T cs = T(0);
    for (int r = 0; r < n; ++r) cs += fabs(r >= c ? w.mat[ep(r, c)] : w.mat[ep(c, r)]);
    nrm = max(nrm, cs);
  }
  return block_max(nrm, w.red);
}

__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double recip(double x) { return 1.0 / x; }
// 1 / sqrt(x) for x > 0: the hardware reciprocal square root in FP32 (about
// 1 ulp, like the reciprocal above); the correctly rounded quotient in FP64.
__device__ inline float rsqrt_pos(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsqrt_pos(double x) { return 1.0 / sqrt(x); }

// Value of lane J of this lane's 16-lane row (DPP row_newbcast, one VALU op).
template <int J>
__device__ inline float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + J, 0xF, 0xF, false));
}
template <int J>
__device__ inline double row_bcast(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFFll), 0x150 + J, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + J, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Pivot step J of the row-per-lane Cholesky (lane i < 16 holds row i in a).
// Only the lower triangle is meaningful: entries a[k] with k > lane are updated
// too (no per-lane masks) but never read into the lower part, and are zeroed
// when L is written out.
template <int J, typename T>
__device__ inline void chol_step(T (&a)[16], int lane, bool& ok) {
  const T piv = row_bcast<J>(a[J]);
  ok = ok && piv > T(0) && isfinite(piv);
  const T inv = rsqrt_pos(piv > T(0) ? piv : T(1));  // 1 / sqrt(pivot)
  a[J] = lane == J ? piv * inv : a[J] * inv;
  if constexpr (J + 1 < 16) {
    // column J of L is now a[J] across the lanes; lane i updates a[k] for k > J
    T colv[16];
#define GNMPC_BC(K) \
    if constexpr (K > J) colv[K] = row_bcast<K>(a[J]);
    GNMPC_BC(1) GNMPC_BC(2) GNMPC_BC(3) GNMPC_BC(4) GNMPC_BC(5) GNMPC_BC(6) GNMPC_BC(7) GNMPC_BC(8)
    GNMPC_BC(9) GNMPC_BC(10) GNMPC_BC(11) GNMPC_BC(12) GNMPC_BC(13) GNMPC_BC(14) GNMPC_BC(15)
#undef GNMPC_BC
#pragma unroll
    for (int k = J + 1; k < 16; ++k) a[k] -= a[J] * colv[k];
  }
}

// Cholesky factor of the 16x16 diagonal block at Dg (lower part) and its
// inverse, by one wave; tmp is 256 elements of LDS.  Lane i < 16 holds row i;
// pivots and columns move between lanes by row broadcasts (no memory); then L
// goes to tmp and lane c forward-substitutes column c of L^{-1}.  Writes
// L^{-1} (lower, zeros above) to Dg; false on a nonpositive or non-finite pivot.
template <typename T>
__device__ __attribute__((always_inline)) bool diag_factor_invert(T* Dg, T* tmp) {
  const int lane = threadIdx.x & 63;
  const bool act = lane < 16;
  T a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) a[c] = act ? Dg[lane * 16 + c] : T(0);
  bool ok = true;
  chol_step<0>(a, lane, ok);
  chol_step<1>(a, lane, ok);
  chol_step<2>(a, lane, ok);
  chol_step<3>(a, lane, ok);
  chol_step<4>(a, lane, ok);
  chol_step<5>(a, lane, ok);
  chol_step<6>(a, lane, ok);
  chol_step<7>(a, lane, ok);
  chol_step<8>(a, lane, ok);
  chol_step<9>(a, lane, ok);
  chol_step<10>(a, lane, ok);
  chol_step<11>(a, lane, ok);
  chol_step<12>(a, lane, ok);
  chol_step<13>(a, lane, ok);
  chol_step<14>(a, lane, ok);
  chol_step<15>(a, lane, ok);
  // the pivots are read by every lane of row 0; lanes >= 16 carry zeros, so only row 0 decides
  ok = __builtin_amdgcn_readfirstlane((int)ok) != 0;
  if (act) {
#pragma unroll
    for (int c = 0; c < 16; ++c) tmp[lane * 16 + c] = c <= lane ? a[c] : T(0);
  }
  wave_sync();
  T col[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    T sum = (r == lane) ? T(1) : T(0);
#pragma unroll
    for (int k = 0; k < r; ++k) sum -= tmp[r * 16 + k] * col[k];
    col[r] = (r >= lane) ? sum * recip(tmp[r * 16 + r]) : T(0);
  }
  if (act) {
#pragma unroll
    for (int r = 0; r < 16; ++r) Dg[r * 16 + lane] = col[r];
  }
  wave_sync();
  return ok;
}

// C (block, row-major) = sgn * acc in the row layout of bmma, or C -= acc.
template <typename T>
__device__ inline void bstore(T* C, const T acc[4], T sgn) {
  const int lane = threadIdx.x & 63;
  T* p = C + (lane & 15) * 16 + 4 * (lane >> 4);
#pragma unroll
  for (int t = 0; t < 4; ++t) p[t] = sgn * acc[t];
}
template <typename T>
__device__ inline void bsub(T* C, const T acc[4]) {
  const int lane = threadIdx.x & 63;
  T* p = C + (lane & 15) * 16 + 4 * (lane >> 4);
#pragma unroll
  for (int t = 0; t < 4; ++t) p[t] -= acc[t];
}

// In-place blocked Cholesky K = L L' fused with the inverse W = L^{-1}: with
// L = L_0 L_1 ... L_{nb-1} (L_J the identity except block column J of L),
// W = L_{nb-1}^{-1} ... L_0^{-1}, and step J applies L_J^{-1} to the rows J..
// of the partial W while the Schur complement is updated:
//   a. the waves finish the previous column, W_{I,J-1} = -L_{I,J-1} D_{J-1}
//      (D_J = L_JJ^{-1} is already in block (J, J));
//   b. panel L_IJ = K_IJ D' (I > J); W row J: W_JK <- D W_JK (K < J);
//   c. trailing K_IK -= L_IJ L_KJ' (J < K <= I) and W_IK -= L_IJ W_JK (I > J,
//      K < J).  Wave 0 takes the update of block (J+1, J+1) first and then
//      factors and inverts it (lookahead) while the other waves do the rest:
//      strips of up to four target blocks of one block row I, which share the
//      operand L_IJ, so a wave keeps four independent product chains in flight.
// At the end block (I, K) holds W_IK.  False if K is not positive definite.
template <typename T>
__device__ inline void bmma_rt(T acc[4], const T* A, const T* B, bool trans) {
  if (trans) bmma<true>(acc, A, B);
  else bmma<false>(acc, A, B);
}

// C_q -= A op(B_q) for the cnt (1..4, wave-uniform) blocks of a strip: C_q are
// consecutive blocks of one block row (stride 256 elements), B_q given one by one.
// Each block's product is the same as bmma's; FP32 interleaves the four MFMA chains.
template <bool TRANS>
__device__ inline void strip_sub(const float* A, const float* const (&B)[4], float* C, int cnt) {
  const int l = threadIdx.x & 63, r = l & 15, kq = l >> 4;
  const float4 a4 = *reinterpret_cast<const float4*>(A + r * 16 + 4 * kq);
  const float av[4] = {a4.x, a4.y, a4.z, a4.w};
  float b[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < cnt) {
      const float* Bq = B[q];
      if (TRANS) {
        const float4 b4 = *reinterpret_cast<const float4*>(Bq + r * 16 + 4 * kq);
        b[q][0] = b4.x; b[q][1] = b4.y; b[q][2] = b4.z; b[q][3] = b4.w;
      } else {
#pragma unroll
        for (int st = 0; st < 4; ++st) b[q][st] = Bq[(4 * kq + st) * 16 + r];
      }
    }
  }
  qfloatx4 c[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) c[q] = qfloatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < cnt) c[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[q][st], av[st], c[q], 0, 0, 0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < cnt) {
      const float acc[4] = {c[q][0], c[q][1], c[q][2], c[q][3]};
      bsub(C + q * 256, acc);
    }
  }
}
template <bool TRANS>
__device__ inline void strip_sub(const double* A, const double* const (&B)[4], double* C, int cnt) {
  for (int q = 0; q < cnt; ++q) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    bmma<TRANS>(acc, A, B[q]);
    bsub(C + q * 256, acc);
  }
}

template <typename T>
__device__ __attribute__((always_inline)) bool factor_invert(const Work<T>& w, int nb) {
  const int wave = wave_index(), lane = threadIdx.x & 63;
  if (wave == 0) {
    const bool ok = diag_factor_invert(w.mat, w.part);
    if (lane == 0) w.scal[0] = ok ? T(1) : T(-1);
  }
  __syncthreads();
  for (int J = 0; J < nb; ++J) {
    T* D = w.mat + bo(J, J);
    // ---- a
    if (J > 0) {
      const T* Dp = w.mat + bo(J - 1, J - 1);
      for (int I = J + wave; I < nb; I += kWaves) {
        T acc[4] = {T(0), T(0), T(0), T(0)};
        T* B = w.mat + bo(I, J - 1);
        bmma<false>(acc, B, Dp);
        wave_sync();
        bstore(B, acc, T(-1));
      }
    }
    __syncthreads();
    if (w.scal[0] < T(0)) return false;
    const int m = nb - 1 - J;
    // ---- b: panel blocks (I, J), then W row J blocks (J, K < J)
    for (int t = wave; t < m + J; t += kWaves) {
      T acc[4] = {T(0), T(0), T(0), T(0)};
      if (t < m) {
        T* B = w.mat + bo(J + 1 + t, J);
        bmma<true>(acc, B, D);
        wave_sync();
        bstore(B, acc, T(1));
      } else {
        T* B = w.mat + bo(J, t - m);
        bmma<false>(acc, D, B);
        wave_sync();
        bstore(B, acc, T(1));
      }
    }
    __syncthreads();
    if (m == 0) break;
    // ---- c: wave 0 updates (J+1, J+1) and factors it; the other waves take the
    // strips of each block row I > J in turn: trailing blocks K = J+1..I (block
    // (J+1, J+1) excluded), then W blocks K = 0..J-1, four at a time
    if (wave == 0) {
      T acc[4] = {T(0), T(0), T(0), T(0)};
      const T* LJ1 = w.mat + bo(J + 1, J);
      bmma<true>(acc, LJ1, LJ1);
      bsub(w.mat + bo(J + 1, J + 1), acc);
      wave_sync();
      const bool ok = diag_factor_invert(w.mat + bo(J + 1, J + 1), w.part);
      if (lane == 0) w.scal[0] = ok ? T(1) : T(-1);
    } else {
      constexpr int S = kWaves - 1;
      int t = 0;
      for (int I = J + 1; I < nb; ++I) {
        const T* A = w.mat + bo(I, J);
        for (int K = (I == J + 1 ? J + 2 : J + 1); K <= I; K += 4, ++t) {
          if (t % S != wave - 1) continue;
          const int cnt = min(4, I + 1 - K);
          const T* B[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) B[q] = w.mat + bo(q < cnt ? K + q : K, J);
          strip_sub<true>(A, B, w.mat + bo(I, K), cnt);
        }
        for (int K = 0; K < J; K += 4, ++t) {
          if (t % S != wave - 1) continue;
          const int cnt = min(4, J - K);
          const T* B[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) B[q] = w.mat + bo(J, q < cnt ? K + q : K);
          strip_sub<false>(A, B, w.mat + bo(I, K), cnt);
        }
      }
    }
    __syncthreads();
  }
  return true;
}

// Hager's estimate of ||K^{-1}||_1 (K symmetric, so K^{-T} = K^{-1}).
template <typename T>
__device__ T inv_norm1_estimate(const Work<T>& w, int n) {
  T* v = w.hx;
  T* y = w.xt;
  for (int i = threadIdx.x; i < n; i += kQpThreads) v[i] = T(1) / T(n);
  __syncthreads();
  T est = T(0);
  for (int it = 0; it < 2; ++it) {
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
    for (int i = threadIdx.x; i < n; i += kQpThreads) ztx += y[i] * v[i];
    ztx = block_sum(ztx, w.red);
    block_argmax_abs(y, n, w.red, zmax, jmax);
    if (zmax <= ztx) break;
    for (int i = threadIdx.x; i < n; i += kQpThreads) v[i] = (i == jmax) ? T(1) : T(0);
    __syncthreads();
  }
  __syncthreads();
  return est;
}

// Column and row abs sums of one block column / block row of the lower block storage,
// for the 16 columns c = 16 B + (lane & 15) (rows split over the four lane groups, then
// summed across them): col = sum over blocks (I >= B, B) of |X[r][c]|, taking in the
// diagonal block only the entries with take_col(rr, cc); row = sum over blocks (B, J <= B)
// of |X[c][r]|, in the diagonal block only those with take_row(rr, cc).  Four partial
// sums rotate over the blocks, so the loads of several blocks are in flight at once.
template <typename T, typename FC, typename FR>
__device__ inline void block_abs_sums(const Work<T>& w, int nb, int B, FC take_col, FR take_row, T& col, T& row) {
  const int lane = threadIdx.x & 63, cc = lane & 15, rq = lane >> 4;
  T cs[4] = {T(0), T(0), T(0), T(0)}, rs[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll 4
  for (int I = B; I < nb; ++I) {
    const T* blk = w.mat + bo(I, B);
    T p = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int rr = 4 * rq + k;
      if (I > B || take_col(rr, cc)) p += fabs(blk[rr * 16 + cc]);
    }
    cs[(I - B) & 3] += p;
  }
#pragma unroll 4
  for (int J = 0; J <= B; ++J) {
    const T* blk = w.mat + bo(B, J);
    T p = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int rr = 4 * rq + k;  // column index inside the block
      if (J < B || take_row(rr, cc)) p += fabs(blk[cc * 16 + rr]);
    }
    rs[J & 3] += p;
  }
  col = (cs[0] + cs[1]) + (cs[2] + cs[3]);
  row = (rs[0] + rs[1]) + (rs[2] + rs[3]);
  col += __shfl_xor(col, 16, 64);
  col += __shfl_xor(col, 32, 64);
  row += __shfl_xor(row, 16, 64);
  row += __shfl_xor(row, 32, 64);
}

// ||K||_1 (K symmetric: max column abs sum) from the lower block storage: column c
// sums |K_rc| over r >= c (block column c/16) and |K_cr| over r < c (block row c/16).
template <typename T>
__device__ T knorm1(const Work<T>& w, int n) {
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int nb = nblocks(n), cc = lane & 15;
  T nrm = T(0);
  for (int B = wave; B < nb; B += kWaves) {
    T col, row;
    block_abs_sums(w, nb, B, [](int rr, int c) { return rr >= c; }, [](int rr, int c) { return rr < c; }, col, row);
    if (16 * B + cc < n) nrm = max(nrm, col + row);
  }
  return block_max(nrm, w.red);
}

// ||W||_1 and ||W||_inf of the explicit inverse factor W = L^{-1} (lower block storage,
// diagonal blocks lower triangular with zeros above, identity padding): column sums over
// block columns, row sums over block rows.
template <typename T>
__device__ void wnorms(const Work<T>& w, int n, T& n1, T& ninf) {
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int nb = nblocks(n), cc = lane & 15;
  T c1 = T(0), ci = T(0);
  for (int B = wave; B < nb; B += kWaves) {
    T col, row;
    block_abs_sums(w, nb, B, [](int, int) { return true; }, [](int, int) { return true; }, col, row);
    if (16 * B + cc < n) {
      c1 = max(c1, col);
      ci = max(ci, row);
    }
  }
  n1 = block_max(c1, w.red);
  ninf = block_max(ci, w.red);
}

// Factor the K prepared by qp_prep_kernel and invert; false if not positive definite.
// The copy keeps 16 loads of 16 bytes in flight per thread (one CU reads K from L2/MALL).
template <typename T, typename Tin>
__device__ bool factor_prepared(const QpArgs<Tin>& a, const Work<T>& w, T* knorm) {
  const long total = (long)bo(nblocks(a.n), 0);
  if constexpr (sizeof(T) == 4) {
    const float4* src = reinterpret_cast<const float4*>(a.Kf);
#pragma unroll 16
    for (long t = threadIdx.x; t < total / 4; t += kQpThreads) reinterpret_cast<float4*>(w.mat)[t] = src[t];
  } else {
    const double2* src = reinterpret_cast<const double2*>(a.Kp);
#pragma unroll 16
    for (long t = threadIdx.x; t < total / 2; t += kQpThreads) {
      const double2 v = src[t];
      w.mat[2 * t] = (T)v.x;
      w.mat[2 * t + 1] = (T)v.y;
    }
  }
  __syncthreads();
  *knorm = knorm1(w, a.n);
  __syncthreads();
  return factor_invert(w, nblocks(a.n));
}

// Factor K(s) and invert; false if K is not positive definite.
template <typename T, typename Tin>
__device__ __attribute__((always_inline)) bool factor(const QpArgs<Tin>& a, const Work<T>& w, T s, T* knorm) {
  *knorm = form_K(a, w, s);
  __syncthreads();
  return factor_invert(w, nblocks(a.n));
}


// ---------------------------------------------------------------------------
// Row passes over a row-major global matrix (Ct or H) for FP32 instances with
// n, rows <= 256 and n a multiple of 4: every wave takes 4 rows at a time (16
// lanes per row; lane columns c = 4 (lane & 15) + 64 j + e, four consecutive
// columns per 16-byte load), and all of a lane's values are loaded into
// registers at once, so a pass pays one memory latency instead of one per row.
constexpr int kMG = 4;   // row groups per wave held at once
constexpr int kMH = 2;   // passes: kMG * kMH groups cover 4 * kWaves * kMG * kMH rows
constexpr int kMJ = 16;  // columns per lane
constexpr int kMQ = kMJ / 4;  // 4-column chunks per lane

__device__ inline int rp_row(int g, int h) {
  return 4 * (wave_index() + kWaves * (g + kMG * h)) + ((threadIdx.x & 63) >> 4);
}
__device__ inline int rp_col4(int j) { return 4 * (threadIdx.x & 15) + 64 * j; }

template <typename Tin>
__device__ inline void rp_load(float (&R)[kMG][kMJ], const Tin* Mat, int nr, int n, int h) {
#pragma unroll
  for (int g = 0; g < kMG; ++g) {
    const int r = rp_row(g, h);
#pragma unroll
    for (int j = 0; j < kMQ; ++j) {
      const int c = rp_col4(j);
      const bool ok = r < nr && c < n;
      if constexpr (sizeof(Tin) == 4) {
        const float4 v = ok ? *reinterpret_cast<const float4*>(Mat + (size_t)r * n + c) : make_float4(0.f, 0.f, 0.f, 0.f);
        R[g][4 * j] = v.x;
        R[g][4 * j + 1] = v.y;
        R[g][4 * j + 2] = v.z;
        R[g][4 * j + 3] = v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) R[g][4 * j + e] = ok ? (float)Mat[(size_t)r * n + c + e] : 0.f;
      }
    }
  }
}
__device__ inline float seg16_sum(float v) {
  v += __shfl_xor(v, 8, 16);
  v += __shfl_xor(v, 4, 16);
  v += __shfl_xor(v, 2, 16);
  v += __shfl_xor(v, 1, 16);
  return v;
}
// dot of row g with vec (LDS, n entries), the same value in all 16 lanes of the row
__device__ inline float rp_dot(const float (&R)[kMG][kMJ], int g, const float* vec, int n) {
  float sum = 0.f;
#pragma unroll
  for (int j = 0; j < kMQ; ++j) {
    const int c = rp_col4(j);
    const float4 v = c < n ? *reinterpret_cast<const float4*>(vec + c) : make_float4(0.f, 0.f, 0.f, 0.f);
    sum += R[g][4 * j] * v.x + R[g][4 * j + 1] * v.y + R[g][4 * j + 2] * v.z + R[g][4 * j + 3] * v.w;
  }
  return seg16_sum(sum);
}
// contrib (per lane, its columns) += row g * w ; then rp_flush writes the wave's partial Mat' w
__device__ inline void rp_axpy(float (&acc)[kMJ], const float (&R)[kMG][kMJ], int g, float wv) {
#pragma unroll
  for (int j = 0; j < kMJ; ++j) acc[j] += R[g][j] * wv;
}
__device__ inline void rp_flush(float (&acc)[kMJ], float* part, int n) {
  const int wave = wave_index(), lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < kMJ; ++j) {
    float v = acc[j];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    acc[j] = v;
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < kMQ; ++j) {
      const int c = rp_col4(j);
      if (c < n)
        *reinterpret_cast<float4*>(part + (size_t)wave * n + c) =
            make_float4(acc[4 * j], acc[4 * j + 1], acc[4 * j + 2], acc[4 * j + 3]);
    }
  }
}

// MAT_LDS: the block storage of K / L / W lives in LDS (else in the plan's global
// workspace).  A compile-time choice, so the LDS instance addresses it with LDS
// instructions rather than generic ones.
template <typename T, typename Tin, bool MAT_LDS>
__device__ __attribute__((always_inline)) void qp_solve_body(const QpArgs<Tin>& a, int mode) {
  // mode 0: primary pass in T (may hand over to FP64); 1: FP64 pass, runs only
  // if the primary pass raised the flag; 2: the only pass.
  if (mode == 1 && *(volatile int32_t*)a.flag == 0) {
    if (threadIdx.x == 0) a.flag[1] = 0;
    return;
  }
  extern __shared__ unsigned char smem_raw[];
  const int n = a.n, nc = a.n_c, m = n + nc;
  T* sp = reinterpret_cast<T*>(smem_raw);
  Work<T> w;
  size_t off = 0;
  auto take = [&](size_t cnt) {
    T* p = sp + off;
    off += (cnt + 3) & ~(size_t)3;
    return p;
  };
  const int npad = kBS * nblocks(n);  // n-vectors are zero-padded for the block mat-vecs
  w.x = take(npad); w.xt = take(npad); w.rhs = take(npad); w.tv = take(npad); w.ctv = take(npad);
  w.gv = take(npad); w.hx = take(npad);
  w.z = take(m); w.y = take(m); w.lo = take(m); w.hi = take(m); w.rho = take(m); w.yprev = take(m);
  w.part = take(part_elems(n));
  w.red = take(64);
  w.scal = take(8);
  const size_t mat_elems = bo(nblocks(n), 0);
  if constexpr (MAT_LDS) w.mat = take(mat_elems);
  else w.mat = reinterpret_cast<T*>(a.gmat);

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
  for (int i = threadIdx.x; i < 7 * npad; i += kQpThreads) w.x[i] = T(0);  // the 7 n-vectors are contiguous
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kQpThreads) w.gv[i] = (T)a.g[i];
  __syncthreads();
  // ---- finiteness of the data (H and Ct were checked by qp_prep_kernel; the
  // last pass of a solve clears that flag for the next call)
  {
    int bad = *(volatile int32_t*)(a.flag + 1);
    for (int i = threadIdx.x; i < n; i += kQpThreads) bad |= !isfinite(w.gv[i]);
    T b = block_max((T)bad, w.red);
    if (mode != 0 && threadIdx.x == 0) a.flag[1] = 0;
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
  bool ok = factor_prepared(a, w, &knorm);
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
  // kappa_1(K) = ||K||_1 ||W'W||_1 <= ||K||_1 ||W||_1 ||W||_inf: when that bound is at most
  // kappa_fp64 the FP32 factor is kept without Hager's estimate (the same decision, since
  // the estimate never exceeds kappa_1), and the bound is what the info reports
  T kappa;
  {
    T n1, ninf;
    wnorms(w, n, n1, ninf);
    const T bound = knorm * n1 * ninf;
    kappa = (double)bound <= a.kappa_fp64 ? bound : knorm * inv_norm1_estimate(w, n);
  }
  if (mode == 0 && sizeof(T) == 4 && (double)kappa > a.kappa_fp64) {
    if (threadIdx.x == 0) *a.flag = 1;
    return;
  }
  if (mode == 0 && threadIdx.x == 0) *a.flag = 0;

  const T sigma = (T)a.sigma, alpha = (T)a.alpha;
  const bool use_regs = n <= 16 * kMJ && n % 4 == 0 && nc <= 4 * kWaves * kMG * kMH &&
                        ((reinterpret_cast<uintptr_t>(a.H) | reinterpret_cast<uintptr_t>(a.Ct)) & 15) == 0;
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
    bool done_rows = false;
    if constexpr (sizeof(T) == 4) {
      if (use_regs) {
        float R[kMG][kMJ], acc[kMJ];
#pragma unroll
        for (int j = 0; j < kMJ; ++j) acc[j] = 0.f;
        _Pragma("unroll 1") for (int h = 0; h < kMH; ++h) {
        rp_load(R, a.Ct, nc, n, h);
#pragma unroll
        for (int g = 0; g < kMG; ++g) {
          const int r = rp_row(g, h);
          const float sdot = rp_dot(R, g, w.xt, n);
          float v = 0.f;
          if (r < nc) {
            const int ri = n + r;
            const float zh = alpha * sdot + (1.f - alpha) * w.z[ri];
            const float zn = min(max(zh + w.y[ri] / w.rho[ri], w.lo[ri]), w.hi[ri]);
            const float yn = w.y[ri] + w.rho[ri] * (zh - zn);
            v = w.rho[ri] * zn - yn;
            if ((threadIdx.x & 15) == 0) {
              w.z[ri] = zn;
              w.y[ri] = yn;
            }
          }
          rp_axpy(acc, R, g, v);
        }
        }
        rp_flush(acc, w.part, n);
        __syncthreads();
        for (int c = threadIdx.x; c < n; c += kQpThreads) {
          T sum = T(0);
          for (int q = 0; q < kWaves; ++q) sum += w.part[(size_t)q * n + c];
          w.ctv[c] = sum;
        }
        __syncthreads();
        done_rows = true;
      }
    }
    if (!done_rows) {
      const int wid = wave_index(), lane = threadIdx.x & 63;
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
    bool done_res = false;
    if constexpr (sizeof(T) == 4) {
      if (use_regs) {
        float R[kMG][kMJ], acc[kMJ];
#pragma unroll
        for (int j = 0; j < kMJ; ++j) acc[j] = 0.f;
        _Pragma("unroll 1") for (int h = 0; h < kMH; ++h) {
        rp_load(R, a.Ct, nc, n, h);
#pragma unroll
        for (int g = 0; g < kMG; ++g) {
          const int r = rp_row(g, h);
          const float sdot = rp_dot(R, g, w.x, n);
          float yv = 0.f;
          if (r < nc) {
            const int ri = n + r;
            pr = max(pr, fabs(sdot - w.z[ri]));
            ax_max = max(ax_max, fabs(sdot));
            z_max = max(z_max, fabs(w.z[ri]));
            yv = w.y[ri];
          }
          rp_axpy(acc, R, g, yv);
        }
        }
        rp_flush(acc, w.part, n);
        // H x into w.hx, one row per 16 lanes
        _Pragma("unroll 1") for (int h = 0; h < kMH; ++h) {
          rp_load(R, a.H, n, n, h);
#pragma unroll
          for (int g = 0; g < kMG; ++g) {
            const int r = rp_row(g, h);
            const float hv = rp_dot(R, g, w.x, n);
            if (r < n && (threadIdx.x & 15) == 0) w.hx[r] = hv;
          }
        }
        done_res = true;
      }
    }
    if (!done_res) {
      const int wid = wave_index(), lane = threadIdx.x & 63;
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
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += kQpThreads) {
        T hx = T(0);
        const Tin* hrow = a.H + (size_t)i * n;
        for (int c = 0; c < n; ++c) hx += (T)hrow[c] * w.x[c];
        w.hx[i] = hx;
      }
    }
    __syncthreads();
    T du = T(0), hx_max = T(0), aty_max = T(0), g_max = T(0);
    for (int i = threadIdx.x; i < n; i += kQpThreads) {
      T aty = w.y[i];
      for (int q = 0; q < kWaves; ++q) aty += w.part[(size_t)q * n + i];
      const T hx = w.hx[i];
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
      bool done_inf = false;
      if constexpr (sizeof(T) == 4) {
        if (use_regs) {
          float R[kMG][kMJ], acc[kMJ];
#pragma unroll
          for (int j = 0; j < kMJ; ++j) acc[j] = 0.f;
          _Pragma("unroll 1") for (int h = 0; h < kMH; ++h) {
            rp_load(R, a.Ct, nc, n, h);
#pragma unroll
            for (int g = 0; g < kMG; ++g) {
              const int r = rp_row(g, h);
              rp_axpy(acc, R, g, r < nc ? w.y[n + r] - w.yprev[n + r] : 0.f);
            }
          }
          rp_flush(acc, w.part, n);
          done_inf = true;
        }
      }
      if (!done_inf) {
        const int wid = wave_index(), lane = threadIdx.x & 63;
        T* pw = w.part + (size_t)wid * n;
        for (int c = lane; c < n; c += 64) pw[c] = T(0);
        for (int r = wid; r < nc; r += kWaves) {
          const Tin* crow = a.Ct + (size_t)r * n;
          T dy = w.y[n + r] - w.yprev[n + r];
          for (int c = lane; c < n; c += 64) pw[c] += (T)crow[c] * dy;
        }
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
        const int wid = wave_index(), lane = threadIdx.x & 63;
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
  bool done_obj = false;
  if constexpr (sizeof(T) == 4) {
    if (use_regs) {
      float R[kMG][kMJ];
      _Pragma("unroll 1") for (int h = 0; h < kMH; ++h) {
        rp_load(R, a.H, n, n, h);
#pragma unroll
        for (int g = 0; g < kMG; ++g) {
          const int r = rp_row(g, h);
          const float hv = rp_dot(R, g, w.x, n);
          if (r < n && (threadIdx.x & 15) == 0) w.hx[r] = hv;
        }
      }
      done_obj = true;
    }
  }
  if (!done_obj) {
    for (int i = threadIdx.x; i < n; i += kQpThreads) {
      T hx = T(0);
      const Tin* hrow = a.H + (size_t)i * n;
      for (int c = 0; c < n; ++c) hx += (T)hrow[c] * w.x[c];
      w.hx[i] = hx;
    }
  }
  __syncthreads();
  T obj = T(0);
  for (int i = threadIdx.x; i < n; i += kQpThreads) {
    obj += w.x[i] * (T(0.5) * w.hx[i] + w.gv[i]);
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

template <typename T, typename Tin, bool MAT_LDS>
__global__ void __launch_bounds__(kQpThreads) qp_solve_kernel(QpArgs<Tin> a, int mode) {
  qp_solve_body<T, Tin, MAT_LDS>(a, mode);
}

// FP32 pass and, behind it in the same workgroup, the FP64 pass, which returns at
// once unless the FP32 pass raised the flag (thread 0's write is seen by every wave
// after the barrier: the waves of a workgroup share one CU); one launch instead of
// two.  The dynamic LDS is the larger of the two passes' layouts, which share it.
template <typename Tin, bool LDS32, bool LDS64>
__global__ void __launch_bounds__(kQpThreads) qp_solve_two_pass_kernel(QpArgs<Tin> a) {
  qp_solve_body<float, Tin, LDS32>(a, 0);
  __syncthreads();
  qp_solve_body<double, Tin, LDS64>(a, 1);
}

// Many instances' QPs in one launch, one workgroup each: each instance's set-up
// kernel stored its solve descriptor in its plan's memory, and the launch takes
// the addresses (kernel arguments, so the launch needs no copy and a graph can
// capture it).  Each workgroup is the single-instance solve of its own
// descriptor, so results are the same bits.
constexpr int kQpBatchMax = 256;
template <typename Tin>
struct QpBatch {
  const QpArgs<Tin>* a[kQpBatchMax];
};
template <typename T, typename Tin, bool MAT_LDS>
__global__ void __launch_bounds__(kQpThreads) qp_solve_batched_kernel(QpBatch<Tin> b, int mode) {
  const QpArgs<Tin> a = *b.a[blockIdx.x];
  qp_solve_body<T, Tin, MAT_LDS>(a, mode);
}

size_t lds_bytes(int n, int nc, size_t elem, bool mat) {
  const int m = n + nc;
  auto r4 = [](size_t c) { return (c + 3) & ~(size_t)3; };
  size_t e = 7 * r4((size_t)kBS * nblocks(n)) + 6 * r4(m) + r4(part_elems(n)) + 64 + 8;
  if (mat) e += r4(bo(nblocks(n), 0));
  return e * elem;
}

constexpr size_t kLdsCap = 160 * 1024;

template <typename T, typename Tin>
gnmpc_status launch_pass(gnmpc_plan* p, const QpArgs<Tin>& a, int mode, hipStream_t s) {
  bool in_lds = lds_bytes(a.n, a.n_c, sizeof(T), true) <= kLdsCap;
  size_t lds = lds_bytes(a.n, a.n_c, sizeof(T), in_lds);
  if (lds > kLdsCap) {
    if (p) p->last_error = "QP too large for one workgroup's LDS";
    return GNMPC_UNSUPPORTED;
  }
  const void* fn = in_lds ? (const void*)qp_solve_kernel<T, Tin, true> : (const void*)qp_solve_kernel<T, Tin, false>;
  if (set_max_lds(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
    if (p) p->last_error = "QP: could not raise the LDS limit of the solve kernel";
    return GNMPC_HIP_ERROR;
  }
  if (in_lds) qp_solve_kernel<T, Tin, true><<<1, kQpThreads, lds, s>>>(a, mode);
  else qp_solve_kernel<T, Tin, false><<<1, kQpThreads, lds, s>>>(a, mode);
  return GNMPC_OK;
}

// The FP32 pass and its FP64 hand-over in one launch (qp_solve_two_pass_kernel).
template <typename Tin>
gnmpc_status launch_two_pass(gnmpc_plan* p, const QpArgs<Tin>& a, hipStream_t s) {
  const bool l32 = lds_bytes(a.n, a.n_c, sizeof(float), true) <= kLdsCap;
  const bool l64 = lds_bytes(a.n, a.n_c, sizeof(double), true) <= kLdsCap;
  const size_t lds = std::max(lds_bytes(a.n, a.n_c, sizeof(float), l32), lds_bytes(a.n, a.n_c, sizeof(double), l64));
  if (lds > kLdsCap) {
    if (p) p->last_error = "QP too large for one workgroup's LDS";
    return GNMPC_UNSUPPORTED;
  }
  // the FP64 layout fits LDS only where the FP32 one does
  const void* fn = l64 ? (const void*)qp_solve_two_pass_kernel<Tin, true, true>
                       : l32 ? (const void*)qp_solve_two_pass_kernel<Tin, true, false>
                             : (const void*)qp_solve_two_pass_kernel<Tin, false, false>;
  if (set_max_lds(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
    if (p) p->last_error = "QP: could not raise the LDS limit of the solve kernel";
    return GNMPC_HIP_ERROR;
  }
  if (l64) qp_solve_two_pass_kernel<Tin, true, true><<<1, kQpThreads, lds, s>>>(a);
  else if (l32) qp_solve_two_pass_kernel<Tin, true, false><<<1, kQpThreads, lds, s>>>(a);
  else qp_solve_two_pass_kernel<Tin, false, false><<<1, kQpThreads, lds, s>>>(a);
  return GNMPC_OK;
}

__global__ void qp_flag_clear_kernel(int32_t* flag) {
  if (threadIdx.x < 2) flag[threadIdx.x] = 0;
}

// One QP solve with its workspace at `ws` (qp_workspace_bytes(n, n_c) bytes,
// 256-byte aligned) and its two flags at `flag`; p (may be null) receives the
// error text and the phase timer records.
template <typename Tin>
QpArgs<Tin> make_args(unsigned char* ws, int32_t* flag, int n, const void* H, const void* g, const void* lb,
                      const void* ub, int n_c, const void* Ct, const void* lc, const void* uc,
                      const gnmpc_admm_settings* st, void* u, gnmpc_qp_info* info) {
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
  const size_t nbo = bo(nblocks(n), 0);
  a.G = (const double*)ws;
  a.gmat = (double*)(ws + (sizeof(double) * (size_t)n * n + 255) / 256 * 256);  // 256-byte aligned
  a.Kp = a.gmat + nbo;
  a.Kf = reinterpret_cast<float*>(a.Kp + nbo);
  a.flag = flag;
  a.rho = st->rho;
  a.sigma = st->sigma;
  a.alpha = st->alpha;
  a.eps_abs = st->eps_abs;
  a.eps_rel = st->eps_rel;
  a.kappa_fp64 = st->kappa_fp64;
  a.max_iter = st->max_iter;
  a.check_every = st->check_every;
  return a;
}

template <typename Tin>
void launch_prep(const QpArgs<Tin>& a, hipStream_t s, QpArgs<Tin>* desc_out = nullptr) {
  const size_t nbo = bo(nblocks(a.n), 0);
  qp_prep_kernel<Tin><<<(int)(nbo / 256), 256, 0, s>>>(a, const_cast<double*>(a.G), desc_out);
}

template <typename Tin>
gnmpc_status run(gnmpc_plan* p, unsigned char* ws, int32_t* flag, int n, const void* H, const void* g,
                 const void* lb, const void* ub, int n_c, const void* Ct, const void* lc, const void* uc,
                 const gnmpc_admm_settings* st, void* u, gnmpc_qp_info* info, hipStream_t s) {
  const QpArgs<Tin> a = make_args<Tin>(ws, flag, n, H, g, lb, ub, n_c, Ct, lc, uc, st, u, info);
  if (p) phase_begin(p, GNMPC_PH_QP, s);
  launch_prep(a, s);
  gnmpc_status rc;
  if constexpr (sizeof(Tin) == 8) {
    rc = launch_pass<double, Tin>(p, a, 2, s);
  } else {
    rc = launch_two_pass<Tin>(p, a, s);
  }
  if (p) phase_end(p, GNMPC_PH_QP, s);
  if (rc != GNMPC_OK) return rc;
  if (hipGetLastError() != hipSuccess) {
    if (p) p->last_error = "QP: kernel launch failed";
    return GNMPC_HIP_ERROR;
  }
  return GNMPC_OK;
}

// One pass of the batched solve over the prepared instances of one input type:
// T is the pass arithmetic; instances whose factor fits LDS and the others go to
// the two instances of the kernel, up to kQpBatchMax per launch, LDS sized for
// the largest member of each launch.
template <typename T, typename Tin>
gnmpc_status batched_pass(const std::vector<const QpPrepared*>& all, int mode, hipStream_t s) {
  for (int lds_kind = 1; lds_kind >= 0; --lds_kind) {
    std::vector<const QpPrepared*> sel;
    for (const QpPrepared* q : all)
      if ((lds_bytes(q->n, q->n_c, sizeof(T), true) <= kLdsCap) == (lds_kind == 1)) sel.push_back(q);
    for (size_t c0 = 0; c0 < sel.size(); c0 += kQpBatchMax) {
      const int cnt = (int)std::min<size_t>(kQpBatchMax, sel.size() - c0);
      QpBatch<Tin> b;
      size_t lds = 0;
      for (int q = 0; q < cnt; ++q) {
        b.a[q] = static_cast<const QpArgs<Tin>*>(sel[c0 + q]->desc);
        lds = std::max(lds, lds_bytes(sel[c0 + q]->n, sel[c0 + q]->n_c, sizeof(T), lds_kind == 1));
      }
      for (int q = cnt; q < kQpBatchMax; ++q) b.a[q] = b.a[0];  // not launched
      if (lds > kLdsCap) return GNMPC_UNSUPPORTED;
      const void* fn = lds_kind ? (const void*)qp_solve_batched_kernel<T, Tin, true>
                                : (const void*)qp_solve_batched_kernel<T, Tin, false>;
      if (set_max_lds(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return GNMPC_HIP_ERROR;
      if (lds_kind) qp_solve_batched_kernel<T, Tin, true><<<cnt, kQpThreads, lds, s>>>(b, mode);
      else qp_solve_batched_kernel<T, Tin, false><<<cnt, kQpThreads, lds, s>>>(b, mode);
      if (hipGetLastError() != hipSuccess) return GNMPC_HIP_ERROR;
    }
  }
  return GNMPC_OK;
}

// ---------------------------------------------------------------------------
// Interior-point solver of the same QP (the paper solves its condensed QP with an
// interior-point method, HPIPM): Mehrotra's predictor-corrector primal-dual
// method (Mehrotra 1992; Nocedal and Wright, Numerical Optimization, Alg. 16.4) on
//   min 1/2 u'Hu + g'u  s.t.  G u + s = h, s >= 0,
// G's rows being the finite sides of lb <= u <= ub and lc <= Ct u <= uc.  Each
// iteration forms K = H + G' diag(lambda / s) G = H + diag(d_box) + Ct' diag(d_c) Ct
// in the block storage, factors and inverts it (the ADMM's blocked Cholesky),
// and solves the reduced Newton system twice (predictor, then centring
// corrector) with W' W.  FP64, one workgroup.  Inequality slots are fixed:
// 2 i / 2 i + 1 the upper / lower side of u_i, 2 n + 2 r / + 1 those of row r;
// an infinite side is an inactive slot (s = 1, lambda = 0, masked out).
struct IpmArgs {
  int n, n_c, max_iter, f64_in;  // f64_in: the arrays are double (else float)
  double tol;
  const void *H, *g, *lb, *ub, *Ct, *lc, *uc;
  void* u;
  gnmpc_qp_info* info;
  double* gmat;  // block storage of K / L / W (global)
};

// K's row term is formed from kIpmRows rows of Ct at a time, staged in LDS and
// scaled by sqrt(lambda / s) (K_c = W'W); a wave keeps the sums of up to
// kIpmBlk 16x16 blocks in registers per pass over Ct.
constexpr int kIpmRows = 16;
constexpr int kIpmBlk = 4;
__host__ __device__ inline size_t ipm_lds_doubles(int n, int n_c) {
  const size_t npad = (size_t)kBS * nblocks(n), m = 2 * (size_t)n + 2 * (size_t)n_c;
  return 8 * npad + 8 * m + 4 * (size_t)n_c + part_elems(n) + 64 + 8 + (size_t)kIpmRows * npad;
}

__device__ inline double ipm_ld(const void* p, int f64, size_t i) {
  return f64 ? static_cast<const double*>(p)[i] : (double)static_cast<const float*>(p)[i];
}

__global__ void __launch_bounds__(kQpThreads) qp_ipm_kernel(IpmArgs a) {
  extern __shared__ unsigned char ipm_smem[];
  const int n = a.n, nc = a.n_c, f64 = a.f64_in;
  const int nb = nblocks(n), npad = kBS * nb, m = 2 * n + 2 * nc;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_index();
  double* sp = reinterpret_cast<double*>(ipm_smem);
  size_t off = 0;
  auto take = [&](size_t c) {
    double* p = sp + off;
    off += c;
    return p;
  };
  double *u = take(npad), *rd = take(npad), *rhs = take(npad), *du = take(npad), *tv = take(npad);
  double *dbox = take(npad), *gv = take(npad), *tmp = take(npad);
  double *sv = take(m), *lam = take(m), *ds = take(m), *dl = take(m), *rp = take(m), *rc = take(m), *hv = take(m);
  double* act = take(m);
  double *ctu = take(nc), *dctu = take(nc), *dc = take(nc), *wv = take(nc);
  Work<double> w;
  w.mat = a.gmat;
  w.tv = tv;
  w.part = take(part_elems(n));
  w.red = take(64);
  w.scal = take(8);
  double* cs = take((size_t)kIpmRows * npad);  // staged rows of W = diag(sqrt(d_c)) Ct
  // ---- slots, starting point u = 0, s = max(h, 1), lambda = 1 (inactive: s = 1, lambda = 0)
  double hmax = 0.0, gmax = 0.0;
  for (int q = tid; q < m; q += kQpThreads) {
    double bound;
    bool up = (q & 1) == 0;
    if (q < 2 * n) bound = up ? ipm_ld(a.ub, f64, q >> 1) : ipm_ld(a.lb, f64, q >> 1);
    else {
      const int r = (q - 2 * n) >> 1;
      bound = up ? (a.uc ? ipm_ld(a.uc, f64, r) : INFINITY) : (a.lc ? ipm_ld(a.lc, f64, r) : -INFINITY);
    }
    const bool on = isfinite(bound);
    act[q] = on ? 1.0 : 0.0;
    hv[q] = on ? (up ? bound : -bound) : 0.0;
    sv[q] = on ? max(hv[q], 1.0) : 1.0;
    lam[q] = on ? 1.0 : 0.0;
    if (on) hmax = max(hmax, fabs(hv[q]));
  }
  for (int i = tid; i < npad; i += kQpThreads) {
    u[i] = 0.0;
    gv[i] = i < n ? ipm_ld(a.g, f64, i) : 0.0;
    if (i < n) gmax = max(gmax, fabs(gv[i]));
  }
  double nact = 0.0;
  for (int q = tid; q < m; q += kQpThreads) nact += act[q];
  nact = block_sum(nact, w.red);
  const double scale = max(1.0, max(block_max(hmax, w.red), block_max(gmax, w.red)));
  __syncthreads();
  // out[r] = (X v)[r] for the rows r < rows of X [rows][n] (Ct or H): a wave takes
  // eight rows at a time, lanes over the columns, so its loads of the eight rows
  // are in flight together; then one wave reduction per row.
  auto rows_times = [&](const void* X, int rows, const double* v, double* out) {
    for (int r0 = 4 * wave; r0 < rows; r0 += 4 * kWaves) {
      double t[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) t[q] = 0.0;
      for (int c = lane; c < n; c += 64) {
        const double vc = v[c];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (r0 + q < rows) t[q] += ipm_ld(X, f64, (size_t)(r0 + q) * n + c) * vc;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double sq = wave_sum(t[q]);
        if (lane == 0 && r0 + q < rows) out[r0 + q] = sq;
      }
    }
    __syncthreads();
  };
  auto ct_times = [&](const double* v, double* out) { rows_times(a.Ct, nc, v, out); };
  // G' v over the slots: (v_up - v_lo) of u_i plus Ct' (v_up - v_lo) of the rows; into
  // out.  Wave w sums rows w, w + kWaves, ... of Ct scaled by their weights, lanes
  // over the columns (coalesced row reads), into w.part[w][.]; the waves' partial
  // sums are then added in wave order.
  auto gt_times = [&](const double* v, double* out) {
    for (int r = tid; r < nc; r += kQpThreads) wv[r] = v[2 * n + 2 * r] - v[2 * n + 2 * r + 1];
    __syncthreads();
    for (int c0 = 0; c0 < n; c0 += 256) {
      double pc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int r = wave; r < nc; r += kWaves) {
        const double wr = wv[r];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int c = c0 + lane + 64 * t;
          if (c < n) pc[t] += ipm_ld(a.Ct, f64, (size_t)r * n + c) * wr;
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = c0 + lane + 64 * t;
        if (c < n) w.part[(size_t)wave * n + c] = pc[t];
      }
    }
    __syncthreads();
    for (int c = tid; c < npad; c += kQpThreads) {
      double t = 0.0;
      if (c < n) {
        t = v[2 * c] - v[2 * c + 1];
        for (int q = 0; q < kWaves; ++q) t += w.part[(size_t)q * n + c];
      }
      out[c] = t;
    }
    __syncthreads();
  };
  // G x per slot from x (box) and Ct x (rows)
  auto g_slot = [&](int q, const double* x, const double* ctx) {
    const double sg = (q & 1) ? -1.0 : 1.0;
    return sg * (q < 2 * n ? x[q >> 1] : ctx[(q - 2 * n) >> 1]);
  };
  int status = GNMPC_QP_MAXITER, iter = 0;
  double prim = 0.0, dual = 0.0, mu_last = 0.0;
  for (iter = 0; iter < a.max_iter; ++iter) {
    // ---- residuals rd = H u + g + G' lambda, rp = G u + s - h, mu
    ct_times(u, ctu);
    gt_times(lam, tmp);
    rows_times(a.H, n, u, rd);
    for (int i = tid; i < n; i += kQpThreads) rd[i] += gv[i] + tmp[i];
    double pm = 0.0, smu = 0.0;
    for (int q = tid; q < m; q += kQpThreads) {
      rp[q] = act[q] * (g_slot(q, u, ctu) + sv[q] - hv[q]);
      pm = max(pm, fabs(rp[q]));
      smu += sv[q] * lam[q];
    }
    __syncthreads();
    double dm = 0.0;
    for (int i = tid; i < n; i += kQpThreads) dm = max(dm, fabs(rd[i]));
    prim = block_max(pm, w.red);
    dual = block_max(dm, w.red);
    const double mu = nact > 0 ? block_sum(smu, w.red) / nact : 0.0;
    mu_last = mu;
    if (!isfinite(prim) || !isfinite(dual) || !isfinite(mu)) {
      status = GNMPC_QP_NONFINITE;
      break;
    }
    // residuals to max(tol, 1e-9) (below that FP64 rounding of H u + g + G' lambda
    // decides), the duality measure, which sets the distance to the minimizer, to tol
    const double rtol = max(a.tol, 1e-9) * scale;
    if (prim <= rtol && dual <= rtol && mu <= a.tol * scale) {
      status = GNMPC_QP_SOLVED;
      break;
    }
    // ---- K = H + diag(d_box) + Ct' diag(d_c) Ct (+ reg I), then L and W = L^{-1}.
    // Near the solution lambda / s spans many orders of magnitude and K can lose
    // definiteness in FP64; the factorization is then retried with a diagonal
    // regularization reg = 1e-13 (1 + max lambda / s), times 100 per attempt.
    double wmax = 0.0;
    for (int i = tid; i < npad; i += kQpThreads) {
      dbox[i] = i < n ? lam[2 * i] / sv[2 * i] + lam[2 * i + 1] / sv[2 * i + 1] : 0.0;
      wmax = max(wmax, dbox[i]);
    }
    for (int r = tid; r < nc; r += kQpThreads) {
      dc[r] = lam[2 * n + 2 * r] / sv[2 * n + 2 * r] + lam[2 * n + 2 * r + 1] / sv[2 * n + 2 * r + 1];
      wmax = max(wmax, dc[r]);
    }
    wmax = block_max(wmax, w.red);
    bool factored = false;
    for (int attempt = 0; attempt < 4 && !factored; ++attempt) {
    const double reg = attempt == 0 ? 0.0 : 1e-13 * (1.0 + wmax) * pow(100.0, (double)(attempt - 1));
    {
      // K_c = W'W, W = diag(sqrt(d_c)) Ct: passes over blocks (a wave's kIpmBlk blocks
      // b = b0 + wave + kWaves q of the lower triangle), each streaming W through LDS
      // kIpmRows rows at a time; lane (r16, c4) sums K_c[16 I + r16][16 J + c4 + 0..3]
      const int r16 = lane >> 2, c4 = (lane & 3) * 4;
      const int nblk = nb * (nb + 1) / 2;
      for (int b0 = 0; b0 < nblk; b0 += kWaves * kIpmBlk) {
        int bi[kIpmBlk], bj[kIpmBlk];
        double acc[kIpmBlk][4];
#pragma unroll
        for (int q = 0; q < kIpmBlk; ++q) {
          const int b = b0 + wave + kWaves * q;
          int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
          while ((I + 1) * (I + 2) / 2 <= b) ++I;
          while (I * (I + 1) / 2 > b) --I;
          bi[q] = I;
          bj[q] = b - I * (I + 1) / 2;
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[q][k] = 0.0;
        }
        for (int r0 = 0; r0 < nc; r0 += kIpmRows) {
          __syncthreads();  // every wave is done with the previous rows
          for (int t = tid; t < kIpmRows * npad; t += kQpThreads) {
            const int rr = t / npad, c = t - rr * npad, r = r0 + rr;
            cs[t] = (r < nc && c < n) ? sqrt(dc[r]) * ipm_ld(a.Ct, f64, (size_t)r * n + c) : 0.0;
          }
          __syncthreads();
#pragma unroll
          for (int q = 0; q < kIpmBlk; ++q) {
            if (b0 + wave + kWaves * q < nblk) {
              const double* ci = cs + kBS * bi[q] + r16;
              const double* cj = cs + kBS * bj[q] + c4;
#pragma unroll 4
              for (int rr = 0; rr < kIpmRows; ++rr) {
                const double x = ci[rr * npad];
                const double2 y01 = *reinterpret_cast<const double2*>(cj + rr * npad);
                const double2 y23 = *reinterpret_cast<const double2*>(cj + rr * npad + 2);
                acc[q][0] += x * y01.x;
                acc[q][1] += x * y01.y;
                acc[q][2] += x * y23.x;
                acc[q][3] += x * y23.y;
              }
            }
          }
        }
#pragma unroll
        for (int q = 0; q < kIpmBlk; ++q) {
          if (b0 + wave + kWaves * q < nblk) {
            const int i = kBS * bi[q] + r16;
            double* blk = w.mat + bo(bi[q], bj[q]) + r16 * kBS + c4;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int j = kBS * bj[q] + c4 + k;
              double v;
              if (i < n && j < n) v = ipm_ld(a.H, f64, (size_t)i * n + j) + (i == j ? dbox[i] + reg : 0.0) + acc[q][k];
              else v = i == j ? 1.0 : 0.0;
              blk[k] = v;
            }
          }
        }
      }
    }
    __syncthreads();
    factored = factor_invert(w, nb);
    __syncthreads();
    }
    if (!factored) {
      status = GNMPC_QP_NOT_PD;
      break;
    }
    // ---- reduced Newton system: K du = -rd - G'(W rp - rc / s); then dlambda, ds
    auto solve = [&]() {
      // ds holds v = W rp - rc / s until the step is formed
      for (int q = tid; q < m; q += kQpThreads) ds[q] = act[q] * (lam[q] / sv[q] * rp[q] - rc[q] / sv[q]);
      __syncthreads();
      gt_times(ds, tmp);
      for (int i = tid; i < npad; i += kQpThreads) rhs[i] = i < n ? -rd[i] - tmp[i] : 0.0;
      __syncthreads();
      kinv_apply(w, n, rhs, du);
      for (int i = n + tid; i < npad; i += kQpThreads) du[i] = 0.0;
      __syncthreads();
      ct_times(du, dctu);
      for (int q = tid; q < m; q += kQpThreads) {
        const double dlq = act[q] * (lam[q] / sv[q] * (g_slot(q, du, dctu) + rp[q]) - rc[q] / sv[q]);
        dl[q] = dlq;
        ds[q] = act[q] ? -(rc[q] + sv[q] * dlq) / lam[q] : 0.0;
      }
      __syncthreads();
    };
    auto max_step = [&]() {
      double amin = 1.0;
      for (int q = tid; q < m; q += kQpThreads) {
        if (!act[q]) continue;
        if (ds[q] < 0.0) amin = min(amin, -sv[q] / ds[q]);
        if (dl[q] < 0.0) amin = min(amin, -lam[q] / dl[q]);
      }
      return -block_max(-amin, w.red);
    };
    // predictor: rc = s lambda
    for (int q = tid; q < m; q += kQpThreads) rc[q] = act[q] * sv[q] * lam[q];
    __syncthreads();
    solve();
    double al = max_step();
    double smu_aff = 0.0;
    for (int q = tid; q < m; q += kQpThreads) smu_aff += act[q] * (sv[q] + al * ds[q]) * (lam[q] + al * dl[q]);
    const double mu_aff = nact > 0 ? block_sum(smu_aff, w.red) / nact : 0.0;
    const double sig = mu > 0.0 ? (mu_aff / mu) * (mu_aff / mu) * (mu_aff / mu) : 0.0;
    // centring corrector: rc = s lambda + ds_aff dlambda_aff - sigma mu
    for (int q = tid; q < m; q += kQpThreads) rc[q] = act[q] * (sv[q] * lam[q] + ds[q] * dl[q] - sig * mu);
    __syncthreads();
    solve();
    al = min(1.0, 0.995 * max_step());
    if (!(al > 1e-14)) break;
    for (int i = tid; i < n; i += kQpThreads) u[i] += al * du[i];
    for (int q = tid; q < m; q += kQpThreads) {
      if (!act[q]) continue;
      sv[q] += al * ds[q];
      lam[q] += al * dl[q];
    }
    __syncthreads();
  }
  // ---- outputs
  for (int i = tid; i < n; i += kQpThreads) {
    const double v = status == GNMPC_QP_NOT_PD || status == GNMPC_QP_NONFINITE ? NAN : u[i];
    if (f64) static_cast<double*>(a.u)[i] = v;
    else static_cast<float*>(a.u)[i] = (float)v;
  }
  double obj = 0.0;
  if (a.info) {  // the objective 1/2 u'Hu + g'u
    rows_times(a.H, n, u, tmp);
    for (int i = tid; i < n; i += kQpThreads) tmp[i] = u[i] * (0.5 * tmp[i] + gv[i]);
    __syncthreads();
    double o = 0.0;
    for (int i = tid; i < n; i += kQpThreads) o += tmp[i];
    obj = block_sum(o, w.red);
  }
  if (tid == 0 && a.info) {
    a.info->status = status;
    a.info->iters = iter;
    a.info->used_fp64 = 1;
    a.info->prim_res = prim;
    a.info->dual_res = dual;
    a.info->kappa_est = mu_last;  // the interior-point solver reports its duality measure here
    a.info->obj = obj;
  }
}

// Workspace of the allocation-free entry: a file-scope device array (one copy
// per GPU, held until the process ends).  Host code never passes the array's
// name to a kernel: it takes the array's device address on each GPU once, by
// hipGetSymbolAddress, and uses that address.  Layout: 256 bytes of flags, then
// the QP workspace.
constexpr size_t kQpScratchBytes = (size_t)4 << 20;
constexpr size_t kQpScratchFlagBytes = 256;
static __device__ __align__(256) unsigned char scratch[kQpScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
unsigned char* scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t qp_workspace_bytes(int n, int n_c) {
  (void)n_c;
  return (sizeof(double) * (size_t)n * n + 255) / 256 * 256 + sizeof(double) * (2 * bo(nblocks(n), 0) + 64) +
         sizeof(float) * bo(nblocks(n), 0);
}

static_assert(sizeof(QpArgs<double>) <= kQpDescBytes && sizeof(QpArgs<float>) <= kQpDescBytes,
              "a plan's descriptor buffer holds a solve descriptor");

gnmpc_status launch_qp_prep(gnmpc_plan* p, int n, const void* H, const void* g, const void* lb, const void* ub,
                            int n_c, const void* Ct, const void* lc, const void* uc, const gnmpc_admm_settings* st,
                            void* u, gnmpc_qp_info* info, hipStream_t s, QpPrepared* out) {
  unsigned char* ws = (unsigned char*)p->d_qp;
  out->dtype = p->dims.dtype;
  out->n = n;
  out->n_c = n_c;
  out->desc = p->d_qpdesc;
  if (p->dims.dtype == GNMPC_F64)
    launch_prep(make_args<double>(ws, p->d_qp_flag, n, H, g, lb, ub, n_c, Ct, lc, uc, st, u, info), s,
                static_cast<QpArgs<double>*>(p->d_qpdesc));
  else
    launch_prep(make_args<float>(ws, p->d_qp_flag, n, H, g, lb, ub, n_c, Ct, lc, uc, st, u, info), s,
                static_cast<QpArgs<float>*>(p->d_qpdesc));
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

gnmpc_status launch_qp_batched(const QpPrepared* q, int count, hipStream_t s) {
  std::vector<const QpPrepared*> f, d;
  for (int t = 0; t < count; ++t) (q[t].dtype == GNMPC_F64 ? d : f).push_back(&q[t]);
  gnmpc_status rc = GNMPC_OK;
  if (!f.empty()) rc = batched_pass<float, float>(f, 0, s);
  if (rc == GNMPC_OK && !f.empty()) rc = batched_pass<double, float>(f, 1, s);
  if (rc == GNMPC_OK && !d.empty()) rc = batched_pass<double, double>(d, 2, s);
  return rc;
}

gnmpc_status qp_ipm_check(int n, int n_c) {
  return ipm_lds_doubles(n, n_c) * sizeof(double) <= kLdsCap ? GNMPC_OK : GNMPC_UNSUPPORTED;
}

gnmpc_status launch_qp_ipm(gnmpc_plan* p, int n, const void* H, const void* g, const void* lb, const void* ub,
                           int n_c, const void* Ct, const void* lc, const void* uc, double tol, int max_iter, void* u,
                           gnmpc_qp_info* info, hipStream_t s) {
  IpmArgs a;
  a.n = n;
  a.n_c = n_c;
  a.max_iter = max_iter;
  a.f64_in = p->dims.dtype == GNMPC_F64;
  a.tol = tol;
  a.H = H;
  a.g = g;
  a.lb = lb;
  a.ub = ub;
  a.Ct = n_c > 0 ? Ct : nullptr;
  a.lc = lc;
  a.uc = uc;
  a.u = u;
  a.info = info;
  unsigned char* ws = (unsigned char*)p->d_qp;
  a.gmat = (double*)(ws + (sizeof(double) * (size_t)n * n + 255) / 256 * 256);  // the ADMM's factor storage
  const size_t lds = ipm_lds_doubles(n, n_c) * sizeof(double);
  if (lds > kLdsCap) return GNMPC_UNSUPPORTED;
  GNMPC_HIP_TRY(p, set_max_lds((const void*)qp_ipm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (p) phase_begin(p, GNMPC_PH_QP, s);
  qp_ipm_kernel<<<1, kQpThreads, lds, s>>>(a);
  if (p) phase_end(p, GNMPC_PH_QP, s);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

gnmpc_status launch_qp(gnmpc_plan* p, int n, const void* H, const void* g, const void* lb, const void* ub, int n_c,
                       const void* Ct, const void* lc, const void* uc, const gnmpc_admm_settings* st, void* u,
                       gnmpc_qp_info* info, hipStream_t s) {
  unsigned char* ws = (unsigned char*)p->d_qp;
  if (p->dims.dtype == GNMPC_F64)
    return run<double>(p, ws, p->d_qp_flag, n, H, g, lb, ub, n_c, Ct, lc, uc, st, u, info, s);
  return run<float>(p, ws, p->d_qp_flag, n, H, g, lb, ub, n_c, Ct, lc, uc, st, u, info, s);
}

gnmpc_status qp_noalloc_check(int dtype, int n, int n_c) {
  if (n < 1 || n > kQpNoallocMaxN || n_c < 0 || kQpScratchFlagBytes + qp_workspace_bytes(n, n_c) > kQpScratchBytes)
    return GNMPC_SHAPE;
  // the FP64 pass (which an FP32 solve may hand over to) needs the larger LDS
  (void)dtype;
  if (lds_bytes(n, n_c, sizeof(double), false) > kLdsCap) return GNMPC_UNSUPPORTED;
  return GNMPC_OK;
}

gnmpc_status launch_qp_noalloc(int dtype, int n, const void* H, const void* g, const void* lb, const void* ub,
                               int n_c, const void* Ct, const void* lc, const void* uc,
                               const gnmpc_admm_settings* st, void* u, gnmpc_qp_info* info, hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GNMPC_HIP_ERROR;
  unsigned char* base;
  {
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GNMPC_HIP_ERROR;
      scratch_ptr[dev] = (unsigned char*)ptr;
    }
    base = scratch_ptr[dev];
  }
  int32_t* flag = reinterpret_cast<int32_t*>(base);
  unsigned char* ws = base + kQpScratchFlagBytes;
  // the flags must start at zero: the array keeps whatever the last call on this GPU left
  qp_flag_clear_kernel<<<1, 64, 0, s>>>(flag);
  if (dtype == GNMPC_F64) return run<double>(nullptr, ws, flag, n, H, g, lb, ub, n_c, Ct, lc, uc, st, u, info, s);
  return run<float>(nullptr, ws, flag, n, H, g, lb, ub, n_c, Ct, lc, uc, st, u, info, s);
}

}  // namespace gnmpc
