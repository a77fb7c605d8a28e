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
// g = rbar + sum_k sum_i S^i_k' (Q^i_k Gx^i_k + q^i_k), computed as split-K
// reductions with one partial per (tile, stage, row chunk), summed in a fixed
// order (bitwise repeatable).
//
// Constraint rows (stacked-constraint formula of Sec. V-B):
// Ct[t] = C_t S^{i_t}_{k_t}, dt[t] = d_t - C_t Gx^{i_t}_{k_t}.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "plan.hpp"

namespace gnmpc {
namespace {

constexpr int kPropThreads = 256;

// ---------------------------------------------------------------- propagation
template <typename T>
__global__ void __launch_bounds__(kPropThreads)
sprop_kernel(int k, int M, int nu, int npw, const int32_t* __restrict__ prow, const int32_t* __restrict__ pcol,
             const T* __restrict__ A_k, const T* __restrict__ B_k, const T* __restrict__ c_k,
             const T* __restrict__ S_in, T* __restrict__ S_out, const T* __restrict__ Gx_in,
             T* __restrict__ Gx_out, int wmax) {
  extern __shared__ unsigned char smem_raw[];
  T* As = reinterpret_cast<T*>(smem_raw);  // the pattern rows of this workgroup's nodes, contiguous
  const int node0 = blockIdx.x * npw;
  const int nn = min(npw, M - node0);
  const int ebase = prow[node0];
  int32_t* Ps = reinterpret_cast<int32_t*>(As + (size_t)npw * wmax * 36);  // pattern columns
  int32_t* Rs = Ps + npw * wmax;                                            // row starts (relative)
  {
    // the rows of consecutive nodes are consecutive in A and in the pattern: flat copies
    const T* src = A_k + (size_t)ebase * 36;
    const int ne = prow[node0 + nn] - ebase;
    for (int t = threadIdx.x; t < ne * 36; t += kPropThreads) As[t] = src[t];
    for (int t = threadIdx.x; t < ne; t += kPropThreads) Ps[t] = pcol[ebase + t];
    for (int t = threadIdx.x; t <= nn; t += kPropThreads) Rs[t] = prow[node0 + t] - ebase;
  }
  __syncthreads();
  const int cin = k * nu;             // live columns of S_k
  const int cout = (k + 1) * nu;      // live columns of S_{k+1}
  const int ncol = cout + 1;          // + the Gx column
  for (int it = threadIdx.x; it < nn * ncol; it += kPropThreads) {
    int ln = it / ncol;
    int col = it - ln * ncol;
    int i = node0 + ln;
    const int e0 = Rs[ln], w = Rs[ln + 1] - e0;
    const T* Ab = As + (size_t)e0 * 36;
    const int32_t* pc = Ps + e0;
    T o[6] = {0, 0, 0, 0, 0, 0};
    if (col < cin) {
      for (int e = 0; e < w; ++e) {
        const T* Sj = S_in + (size_t)pc[e] * NBX * cin + col;
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
        const T* xj = Gx_in + (size_t)pc[e] * NBX;
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

// Block propagation: a workgroup takes pb_nodes consecutive nodes and a
// slice of kPropCW columns; the S_k rows of the union of their pattern
// columns are staged in LDS once (the rows a chain neighbourhood shares are
// read from L2 once instead of once per node), with the nodes' A blocks.
// Thread: one node and one column.  Slice 0 also does Gx.  The block's static
// data is one fixed-stride record (first pattern entry, entry count, union
// size, node count, row starts, union nodes, union position of every entry),
// so a stage is two dependent reads: the record, then A_k and the S_k rows.
constexpr int kPropCW = 64;
constexpr int kStageBatch = 8;
constexpr int kRowBatch = 32;  // S_k rows in flight per lane: a 4-node block's union (about 16 nodes) in one batch
__device__ inline void ld4v(const float* p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
__device__ inline void ld4v(const double* p, double (&o)[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  o[0] = a.x;
  o[1] = a.y;
  o[2] = b.x;
  o[3] = b.y;
}
template <typename T>
__global__ void __launch_bounds__(256)
sprop_block_kernel(int k, int M, int nu, int nbn, int rstride, int umax, int emax, const int32_t* __restrict__ rec,
                   const T* __restrict__ A_k, const T* __restrict__ B_k,
                   const T* __restrict__ c_k, const T* __restrict__ S_in, T* __restrict__ S_out,
                   const T* __restrict__ Gx_in, T* __restrict__ Gx_out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pb[];
  const int b = blockIdx.x, c0 = blockIdx.y * kPropCW;
  const int node0 = b * nbn;
  const int cin = k * nu, cout = cin + nu;
  const int cw = max(0, min(kPropCW, cin - c0));  // staged columns of S_k
  T* Ss = reinterpret_cast<T*>(smem_pb);          // [umax][6][kPropCW]
  T* As = Ss + (size_t)umax * NBX * kPropCW;      // [emax][36]
  T* Gs = As + (size_t)emax * 36;                 // [umax][6] (chunk 0)
  int32_t* Rr = reinterpret_cast<int32_t*>(Gs + (size_t)umax * NBX);  // the block's record
  for (int t = threadIdx.x; t < rstride; t += 256) Rr[t] = rec[(size_t)b * rstride + t];
  __syncthreads();
  const int e0 = Rr[0], ne = Rr[1], uc = Rr[2], nn = Rr[3];
  const int32_t* Rs = Rr + 4;                // [nn + 1] row starts (relative)
  const int32_t* Us = Rs + nbn + 1;          // [uc] union nodes
  const int32_t* Es = Us + umax;             // [ne] union position of each entry
  // every staging loop keeps kStageBatch loads in flight per lane
  for (int t0 = threadIdx.x; t0 < ne * 36; t0 += 256 * kStageBatch) {
    T v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      const int t = t0 + 256 * u;
      v[u] = t < ne * 36 ? A_k[(size_t)e0 * 36 + t] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u)
      if (t0 + 256 * u < ne * 36) As[t0 + 256 * u] = v[u];
  }
  __syncthreads();
  if (cw > 0) {
    // 4 rows of kPropCW columns per pass of 256 lanes
    const int c = threadIdx.x % kPropCW, rq = threadIdx.x / kPropCW;
    for (int row0 = rq; row0 < uc * NBX; row0 += 4 * kRowBatch) {
      T v[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int row = row0 + 4 * u;
        const bool ok = row < uc * NBX && c < cw;
        const int uu = ok ? row / NBX : 0, sr = ok ? row - uu * NBX : 0;
        v[u] = ok ? S_in[((size_t)Us[uu] * NBX + sr) * cin + c0 + c] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u)
        if (row0 + 4 * u < uc * NBX) Ss[(size_t)(row0 + 4 * u) * kPropCW + c] = v[u];
    }
  }
  if (blockIdx.y == 0)
    for (int t = threadIdx.x; t < uc * NBX; t += 256) Gs[t] = Gx_in[(size_t)Us[t / NBX] * NBX + t % NBX];
  __syncthreads();
  // one thread per (node, column) of the slice
  for (int it = threadIdx.x; it < nn * kPropCW; it += 256) {
    const int ln = it / kPropCW, cl = it - ln * kPropCW, col = c0 + cl, i = node0 + ln;
    if (col >= cout) continue;
    if (col < cin) {
      T o[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
      const int rs = Rs[ln], w = Rs[ln + 1] - rs;
      for (int e = 0; e < w; ++e) {
        const T* Ae = As + (size_t)(rs + e) * 36;
        const T* Su = Ss + (size_t)Es[rs + e] * NBX * kPropCW + cl;
        T sv[6], av[36];
#pragma unroll
        for (int sr = 0; sr < 6; ++sr) sv[sr] = Su[sr * kPropCW];
#pragma unroll
        for (int q = 0; q < 9; ++q) ld4v(Ae + 4 * q, *reinterpret_cast<T(*)[4]>(av + 4 * q));
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int sr = 0; sr < 6; ++sr) o[r] += av[r * 6 + sr] * sv[sr];
      }
#pragma unroll
      for (int r = 0; r < 6; ++r) S_out[((size_t)i * NBX + r) * cout + col] = o[r];
    } else {
#pragma unroll
      for (int r = 0; r < 6; ++r)
        S_out[((size_t)i * NBX + r) * cout + col] = B_k[((size_t)i * NBX + r) * nu + (col - cin)];
    }
  }
  if (blockIdx.y == 0)
    for (int t = threadIdx.x; t < nn * NBX; t += 256) {
      const int ln = t / NBX, r = t - ln * NBX, i = node0 + ln;
      T v = T(0);
      for (int e = Rs[ln]; e < Rs[ln + 1]; ++e) {
        const T* Ae = As + (size_t)e * 36 + r * 6;
        const T* xj = Gs + (size_t)Es[e] * NBX;
#pragma unroll
        for (int sr = 0; sr < 6; ++sr) v += Ae[sr] * xj[sr];
      }
      Gx_out[(size_t)i * NBX + r] = v + c_k[(size_t)i * NBX + r];
    }
}

// Two stages per launch: a block recomputes S_{k+1} (and Gx_{k+1}) on U1, the union of
// its pattern columns, from S_k on U2, in the same order of operations as the one-stage
// kernel (so the values are the same bit for bit), writes the rows of its own nodes, then
// forms S_{k+2} (and Gx_{k+2}) of its nodes from the staged U1 rows.  This halves the
// chain of dependent launches of the recursion.
// LDS a two-stage workgroup may use.  gfx950 allows 160 KB per workgroup, but
// past 64 KB only one 4-wave workgroup fits a CU and the stage pair runs slower
// than two one-stage launches (measured on the 13-wide GNN pattern, ~106 KB:
// 0.56 ms against 0.23 ms for the recursion).
constexpr size_t kProp2LdsCap = 64 * 1024;

struct Prop2Layout {
  int rs, es1, u1, r1, g1, es2, u2, stride;
};
__host__ __device__ inline Prop2Layout prop2_layout(int nb, int emax, int u1max, int e1max, int u2max) {
  Prop2Layout L;
  L.rs = 8;                  // block row starts [nb + 1]
  L.es1 = L.rs + nb + 1;     // block entry -> position of its column in U1 [emax]
  L.u1 = L.es1 + emax;       // U1 nodes [u1max]
  L.r1 = L.u1 + u1max;       // row starts of U1's nodes in the U1 entry list [u1max + 1]
  L.g1 = L.r1 + u1max + 1;   // global pattern entry of each U1 entry [e1max]
  L.es2 = L.g1 + e1max;      // U1 entry -> position of its column in U2 [e1max]
  L.u2 = L.es2 + e1max;      // U2 nodes [u2max]
  L.stride = (L.u2 + u2max + 3) / 4 * 4;
  return L;
}
inline size_t prop2_lds_bytes(const Prop2Layout& L, size_t elem, int emax, int u1max, int e1max, int u2max) {
  return elem * ((size_t)(u1max + u2max) * NBX * kPropCW + (size_t)(e1max + emax) * 36 +
                 (size_t)(u1max + u2max) * NBX) +
         sizeof(int32_t) * (size_t)L.stride;
}

template <typename T>
__global__ void __launch_bounds__(256)
sprop2_block_kernel(int k, int M, int nu, int nbn, int emax, int u1max, int e1max, int u2max,
                    const int32_t* __restrict__ rec, const T* __restrict__ A_k, const T* __restrict__ A_k1,
                    const T* __restrict__ B_k, const T* __restrict__ B_k1, const T* __restrict__ c_k,
                    const T* __restrict__ c_k1, const T* __restrict__ S_in, T* __restrict__ S_mid,
                    T* __restrict__ S_out, const T* __restrict__ Gx_in, T* __restrict__ Gx_mid,
                    T* __restrict__ Gx_out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pb2[];
  const Prop2Layout L = prop2_layout(nbn, emax, u1max, e1max, u2max);
  const int b = blockIdx.x, c0 = blockIdx.y * kPropCW;
  const int node0 = b * nbn;
  const int cin = k * nu, cmid = cin + nu, cout = cmid + nu;
  T* S2s = reinterpret_cast<T*>(smem_pb2);          // [u2max][6][kPropCW]: S_k of U2
  T* S1s = S2s + (size_t)u2max * NBX * kPropCW;     // [u1max][6][kPropCW]: S_{k+1} of U1
  T* A1s = S1s + (size_t)u1max * NBX * kPropCW;     // [e1max][36]: A_k of U1's entries
  T* A2s = A1s + (size_t)e1max * 36;                // [emax][36]: A_{k+1} of the block's entries
  T* G2s = A2s + (size_t)emax * 36;                 // [u2max][6]: Gx_k of U2
  T* G1s = G2s + (size_t)u2max * NBX;               // [u1max][6]: Gx_{k+1} of U1
  int32_t* Rr = reinterpret_cast<int32_t*>(G1s + (size_t)u1max * NBX);
  for (int t = threadIdx.x; t < L.stride; t += 256) Rr[t] = rec[(size_t)b * L.stride + t];
  __syncthreads();
  const int e0 = Rr[0], ne = Rr[1], nn = Rr[2], u1c = Rr[3], u2c = Rr[4], n1e = Rr[5];
  const int32_t* Rs = Rr + L.rs;
  const int32_t* Es1 = Rr + L.es1;
  const int32_t* U1 = Rr + L.u1;
  const int32_t* R1 = Rr + L.r1;
  const int32_t* G1 = Rr + L.g1;
  const int32_t* Es2 = Rr + L.es2;
  const int32_t* U2 = Rr + L.u2;
  for (int t0 = threadIdx.x; t0 < n1e * 36; t0 += 256 * kStageBatch) {
    T v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      const int t = t0 + 256 * u;
      v[u] = t < n1e * 36 ? A_k[(size_t)G1[t / 36] * 36 + t % 36] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u)
      if (t0 + 256 * u < n1e * 36) A1s[t0 + 256 * u] = v[u];
  }
  for (int t0 = threadIdx.x; t0 < ne * 36; t0 += 256 * kStageBatch) {
    T v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      const int t = t0 + 256 * u;
      v[u] = t < ne * 36 ? A_k1[(size_t)e0 * 36 + t] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u)
      if (t0 + 256 * u < ne * 36) A2s[t0 + 256 * u] = v[u];
  }
  const int cw = max(0, min(kPropCW, cin - c0));  // staged columns of S_k
  if (cw > 0) {
    const int c = threadIdx.x % kPropCW, rq = threadIdx.x / kPropCW;
    for (int row0 = rq; row0 < u2c * NBX; row0 += 4 * kRowBatch) {
      T v[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int row = row0 + 4 * u;
        const bool ok = row < u2c * NBX && c < cw;
        const int uu = ok ? row / NBX : 0, sr = ok ? row - uu * NBX : 0;
        v[u] = ok ? S_in[((size_t)U2[uu] * NBX + sr) * cin + c0 + c] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u)
        if (row0 + 4 * u < u2c * NBX) S2s[(size_t)(row0 + 4 * u) * kPropCW + c] = v[u];
    }
  }
  if (blockIdx.y == 0)
    for (int t = threadIdx.x; t < u2c * NBX; t += 256) G2s[t] = Gx_in[(size_t)U2[t / NBX] * NBX + t % NBX];
  __syncthreads();
  // stage k -> k+1 on U1, one thread per (node of U1, column of the slice)
  for (int it = threadIdx.x; it < u1c * kPropCW; it += 256) {
    const int lu = it / kPropCW, cl = it - lu * kPropCW, col = c0 + cl, u = U1[lu];
    T o[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    if (col < cin) {
      for (int e = R1[lu]; e < R1[lu + 1]; ++e) {
        const T* Ae = A1s + (size_t)e * 36;
        const T* Su = S2s + (size_t)Es2[e] * NBX * kPropCW + cl;
        T sv[6], av[36];
#pragma unroll
        for (int sr = 0; sr < 6; ++sr) sv[sr] = Su[sr * kPropCW];
#pragma unroll
        for (int q = 0; q < 9; ++q) ld4v(Ae + 4 * q, *reinterpret_cast<T(*)[4]>(av + 4 * q));
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int sr = 0; sr < 6; ++sr) o[r] += av[r * 6 + sr] * sv[sr];
      }
    } else if (col < cmid) {
#pragma unroll
      for (int r = 0; r < 6; ++r) o[r] = B_k[((size_t)u * NBX + r) * nu + (col - cin)];
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) S1s[((size_t)lu * NBX + r) * kPropCW + cl] = o[r];
    if (u >= node0 && u < node0 + nn && col < cmid) {
#pragma unroll
      for (int r = 0; r < 6; ++r) S_mid[((size_t)u * NBX + r) * cmid + col] = o[r];
    }
  }
  if (blockIdx.y == 0)
    for (int t = threadIdx.x; t < u1c * NBX; t += 256) {
      const int lu = t / NBX, r = t - lu * NBX, u = U1[lu];
      T v = T(0);
      for (int e = R1[lu]; e < R1[lu + 1]; ++e) {
        const T* Ae = A1s + (size_t)e * 36 + r * 6;
        const T* xj = G2s + (size_t)Es2[e] * NBX;
#pragma unroll
        for (int sr = 0; sr < 6; ++sr) v += Ae[sr] * xj[sr];
      }
      v = v + c_k[(size_t)u * NBX + r];
      G1s[t] = v;
      if (u >= node0 && u < node0 + nn) Gx_mid[(size_t)u * NBX + r] = v;
    }
  __syncthreads();
  // stage k+1 -> k+2 on the block
  for (int it = threadIdx.x; it < nn * kPropCW; it += 256) {
    const int ln = it / kPropCW, cl = it - ln * kPropCW, col = c0 + cl, i = node0 + ln;
    if (col >= cout) continue;
    if (col < cmid) {
      T o[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
      const int rs = Rs[ln], w = Rs[ln + 1] - rs;
      for (int e = 0; e < w; ++e) {
        const T* Ae = A2s + (size_t)(rs + e) * 36;
        const T* Su = S1s + (size_t)Es1[rs + e] * NBX * kPropCW + cl;
        T sv[6], av[36];
#pragma unroll
        for (int sr = 0; sr < 6; ++sr) sv[sr] = Su[sr * kPropCW];
#pragma unroll
        for (int q = 0; q < 9; ++q) ld4v(Ae + 4 * q, *reinterpret_cast<T(*)[4]>(av + 4 * q));
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int sr = 0; sr < 6; ++sr) o[r] += av[r * 6 + sr] * sv[sr];
      }
#pragma unroll
      for (int r = 0; r < 6; ++r) S_out[((size_t)i * NBX + r) * cout + col] = o[r];
    } else {
#pragma unroll
      for (int r = 0; r < 6; ++r)
        S_out[((size_t)i * NBX + r) * cout + col] = B_k1[((size_t)i * NBX + r) * nu + (col - cmid)];
    }
  }
  if (blockIdx.y == 0)
    for (int t = threadIdx.x; t < nn * NBX; t += 256) {
      const int ln = t / NBX, r = t - ln * NBX, i = node0 + ln;
      T v = T(0);
      for (int e = Rs[ln]; e < Rs[ln + 1]; ++e) {
        const T* Ae = A2s + (size_t)e * 36 + r * 6;
        const T* xj = G1s + (size_t)Es1[e] * NBX;
#pragma unroll
        for (int sr = 0; sr < 6; ++sr) v += Ae[sr] * xj[sr];
      }
      Gx_out[(size_t)i * NBX + r] = v + c_k1[(size_t)i * NBX + r];
    }
}

// ---------------------------------------------------------------- Gram + gradient
// H: 32x32 output tiles of the lower triangle, one workgroup per (tile, stage,
// row chunk); each of the 4 waves owns a 16x16 quarter and runs
// v_mfma_f32_16x16x4f32 down the rows of S_k (A = S_k columns, B = Q_k S_k
// columns).  g: one workgroup per (stage, row chunk), one lane per column.
// Partials are summed by gram_reduce_kernel in a fixed order.
typedef float cfloatx4 __attribute__((ext_vector_type(4)));
constexpr int kT = 64;             // H output tile edge
constexpr int kChunkRows = 768;    // rows of S_k per split-K chunk (128 nodes)

struct GramShape {
  int M, nu, N, n, nt, ntiles, nchunks, ngchunks;
};

__host__ __device__ inline int first_stage(int ta, int nu) { return (kT * ta) / nu + 1; }

__device__ inline void tile_coords(int t, int& ta, int& tb) {
  int a = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  ta = a;
  tb = t - a * (a + 1) / 2;
}

// Live (tile, stage) pairs: S_k has k nu columns, so the tiles of stage k that
// hold any of them are t < lt(k) = c (c + 1) / 2 with c = ceil(k nu / kT), a
// prefix of the lower triangle.  The Gram grid enumerates only these pairs,
// stage-major, so every launched workgroup has work.
__host__ __device__ inline int live_tiles(int k, int nu, int nt) {
  const int c0 = (k * nu + kT - 1) / kT, c = c0 < nt ? c0 : nt;
  return c * (c + 1) / 2;
}
__host__ inline int live_pairs(const GramShape& sh) {
  int tot = 0;
  for (int k = 1; k <= sh.N; ++k) tot += live_tiles(k, sh.nu, sh.nt);
  return tot;
}
// stage k and tile index of live pair idx (idx < live_pairs)
__device__ inline int live_pair(const GramShape& sh, int idx, int& tile) {
  int k = 1;
  for (int lt = live_tiles(k, sh.nu, sh.nt); idx >= lt && k < sh.N; lt = live_tiles(k, sh.nu, sh.nt)) {
    idx -= lt;
    ++k;
  }
  tile = idx;
  return k;
}

template <typename T>
__device__ inline T qs_value(const T* Sk, const T* Qk, int Q_full, int cols, int row, int cb) {
  const int node = row / NBX, r = row - node * NBX;
  if (!Q_full) return Qk[row] * Sk[(size_t)row * cols + cb];
  const T* Qn = Qk + ((size_t)node * NBX + r) * NBX;
  const T* Sn = Sk + (size_t)node * NBX * cols + cb;
  T v = T(0);
#pragma unroll
  for (int s = 0; s < NBX; ++s) v += Qn[s] * Sn[(size_t)s * cols];
  return v;
}

// FP32 on the matrix cores through bf16 terms.  grid: x = live (tile, stage) pair,
// y = row chunk.  Every FP32 operand v enters as hi = bf16(v), mid = bf16(v - hi),
// lo = bf16(v - hi - mid) (each residual exact in FP32), so hi + mid + lo equals v to
// about 2^-27 relative; a product takes the six terms hi hi, hi mid, mid hi, hi lo,
// lo hi, mid mid (the dropped ones are below 2^-26 of it), each exact, summed in FP32
// by v_mfma_f32_16x16x32_bf16: 6 x 16 cycles per 32-row step of a 16x16 sub-tile
// against 8 x 32 for v_mfma_f32_16x16x4f32.  Rows are staged 32 at a time (the a
// strip and the Q-weighted b strip, 64 columns each) with independent loads issued two
// blocks ahead; thread t owns column t % 64 of the 8 consecutive rows 8 (t / 64) ..,
// so it packs each term of its column into one 16-byte LDS store, and the MFMA
// operand of a lane (8 consecutive rows of one column) is one 16-byte LDS read.
// Each wave owns a 32x32 quarter of the tile (2 x 2 MFMA tiles).
constexpr int kRB = 32;
constexpr int kTS = kRB + 8;       // bf16 per staged column (16-byte pad: conflict-free reads)
typedef __bf16 gbf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 gbf16x2_t __attribute__((ext_vector_type(2)));
typedef float gfloat2_t __attribute__((ext_vector_type(2)));
__device__ inline uint32_t gpack_bf16x2(float a, float b) {  // round to nearest even
  const gfloat2_t f = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, gbf16x2_t));
}
// the three bf16 terms of eight FP32 values, each packed as 8 bf16 (v[0] lowest)
__device__ inline void split3_bf16x8(const float* v, uint4& t0, uint4& t1, uint4& t2) {
  uint32_t w0[4], w1[4], w2[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float a = v[2 * i], b = v[2 * i + 1];
    w0[i] = gpack_bf16x2(a, b);
    const float ra = a - __uint_as_float(w0[i] << 16), rb = b - __uint_as_float(w0[i] & 0xFFFF0000u);
    w1[i] = gpack_bf16x2(ra, rb);
    w2[i] = gpack_bf16x2(ra - __uint_as_float(w1[i] << 16), rb - __uint_as_float(w1[i] & 0xFFFF0000u));
  }
  t0 = make_uint4(w0[0], w0[1], w0[2], w0[3]);
  t1 = make_uint4(w1[0], w1[1], w1[2], w1[3]);
  t2 = make_uint4(w2[0], w2[1], w2[2], w2[3]);
}
// held to 128 registers per lane (no spills), so four waves share each SIMD
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
gram_kernel_f32(GramShape sh, const float* __restrict__ S_all, const float* __restrict__ Q, int Q_full,
                const float* __restrict__ Gx_all, const float* __restrict__ q, float* __restrict__ part,
                float* __restrict__ gpart) {
  // [term][column][row] bf16 terms of the a strip and of the Q-weighted b strip
  __shared__ __attribute__((aligned(16))) __bf16 Ta[3][kT][kTS];
  __shared__ __attribute__((aligned(16))) __bf16 Tb[3][kT][kTS];
  __shared__ float Ws[kRB];        // w = Q_k Gx_k + q_k of the staged rows (diagonal tiles)
  __shared__ float Gp[4][kT];      // gradient partials of the 4 row groups
  // XCD-aware order: workgroups are dealt to the 8 XCDs round robin, so the linear index is
  // remapped to give each XCD a contiguous range of (chunk, pair) items; the live pairs of one
  // row chunk then run on one XCD at once and share its L2 copy of the S_k strips
  int tile;
  const int npairs = gridDim.x, total = npairs * gridDim.y;
  const int gid = blockIdx.x + blockIdx.y * npairs;
  const int xcd = gid % 8, slot = gid / 8, q8 = total / 8, r8 = total % 8;
  const int lin = xcd < r8 ? xcd * (q8 + 1) + slot : r8 * (q8 + 1) + (xcd - r8) * q8 + slot;
  const int k = live_pair(sh, lin % npairs, tile), chunk = lin / npairs;
  int ta, tb;
  tile_coords(tile, ta, tb);
  if (k < first_stage(ta, sh.nu)) return;
  const int cols = k * sh.nu, rows = NBX * sh.M;
  const float* Sk = S_all + S_offset(k, sh.M, sh.nu);
  const float* Qk = Q + (size_t)k * sh.M * NBX * (Q_full ? NBX : 1);
  const float* Gxk = Gx_all + (size_t)k * sh.M * NBX;
  const float* qk = q + (size_t)k * sh.M * NBX;
  const bool diag = ta == tb;
  float gacc = 0.f;  // diagonal tiles: column threadIdx.x % kT over the thread's rows of each block
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int qa = 32 * (wave >> 1), qb = 32 * (wave & 1);
  const int r0 = chunk * kChunkRows, r1 = min(rows, r0 + kChunkRows);
  cfloatx4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = cfloatx4{0.f, 0.f, 0.f, 0.f};
  // this wave's quarter may lie entirely past the live columns
  const bool live = kT * ta + qa < cols && kT * tb + qb < cols;
  constexpr int kPer = kRB * kT / 256;   // rows per thread and block (8)
  const int cc = threadIdx.x % kT, rr0 = threadIdx.x / kT;
  const int ca = kT * ta + cc, cb = kT * tb + cc;
  // two register sets: the block two ahead is in flight while one is multiplied
  float pa[2][kPer], pb[2][kPer], pq[2][kPer], pw[2] = {0.f, 0.f};
  // lanes with threadIdx.x < kRB also fetch w for row rb + threadIdx.x (diagonal tiles)
  auto fetch = [&](int rb, auto slot) {
    constexpr int sl = decltype(slot)::value;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int r = rb + kPer * rr0 + u;
      const bool vr = r < r1;
      pa[sl][u] = (vr && ca < cols) ? Sk[(size_t)r * cols + ca] : 0.f;
      // a diagonal tile's two strips are the same columns: the b strip is not loaded
      pb[sl][u] = (!diag && vr && cb < cols) ? Sk[(size_t)r * cols + cb] : 0.f;
      pq[sl][u] = vr ? Qk[r] : 0.f;
    }
    if (diag && threadIdx.x < kRB) {
      const int r = rb + threadIdx.x;
      pw[sl] = r < r1 ? Qk[r] * Gxk[r] + qk[r] : 0.f;
    }
  };
  auto block = [&](int rb, auto slot) {
    constexpr int sl = decltype(slot)::value;
    float va[kPer], vb[kPer];
    __syncthreads();
    if (!Q_full) {
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        va[u] = pa[sl][u];
        vb[u] = pq[sl][u] * (diag ? pa[sl][u] : pb[sl][u]);
      }
      if (diag && threadIdx.x < kRB) Ws[threadIdx.x] = pw[sl];
    } else {
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int r = rb + kPer * rr0 + u;
        const bool vr = r < r1;
        va[u] = (vr && ca < cols) ? Sk[(size_t)r * cols + ca] : 0.f;
        vb[u] = (vr && cb < cols) ? qs_value(Sk, Qk, Q_full, cols, r, cb) : 0.f;
      }
      if (diag && threadIdx.x < kRB) {
        const int r = rb + threadIdx.x;
        float wv = 0.f;
        if (r < r1) {
          const int node = r / NBX, rr = r - node * NBX;
          const float* Qn = Qk + ((size_t)node * NBX + rr) * NBX;
#pragma unroll
          for (int s2 = 0; s2 < NBX; ++s2) wv += Qn[s2] * Gxk[(size_t)node * NBX + s2];
          wv += qk[r];
        }
        Ws[threadIdx.x] = wv;
      }
    }
    {
      uint4 t0, t1, t2;
      split3_bf16x8(va, t0, t1, t2);
      *reinterpret_cast<uint4*>(&Ta[0][cc][kPer * rr0]) = t0;
      *reinterpret_cast<uint4*>(&Ta[1][cc][kPer * rr0]) = t1;
      *reinterpret_cast<uint4*>(&Ta[2][cc][kPer * rr0]) = t2;
      split3_bf16x8(vb, t0, t1, t2);
      *reinterpret_cast<uint4*>(&Tb[0][cc][kPer * rr0]) = t0;
      *reinterpret_cast<uint4*>(&Tb[1][cc][kPer * rr0]) = t1;
      *reinterpret_cast<uint4*>(&Tb[2][cc][kPer * rr0]) = t2;
    }
    if (!Q_full && rb + 2 * kRB < r1) fetch(rb + 2 * kRB, slot);
    __syncthreads();
    if (diag) {
#pragma unroll
      for (int u = 0; u < kPer; ++u) gacc += va[u] * Ws[kPer * rr0 + u];
    }
    if (live) {
      // lane (n, g): column n of a sub-tile, rows 8 g .. 8 g + 7 of the block
      const int n = lane & 15, g8 = 8 * (lane >> 4);
      gbf16x8_t av[3][2], bv[3][2];
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          av[t][x] = *reinterpret_cast<const gbf16x8_t*>(&Ta[t][qa + 16 * x + n][g8]);
          bv[t][x] = *reinterpret_cast<const gbf16x8_t*>(&Tb[t][qb + 16 * x + n][g8]);
        }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0][x], bv[0][y], acc[x][y], 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0][x], bv[1][y], acc[x][y], 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1][x], bv[0][y], acc[x][y], 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0][x], bv[2][y], acc[x][y], 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[2][x], bv[0][y], acc[x][y], 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1][x], bv[1][y], acc[x][y], 0, 0, 0);
        }
    }
  };
  const std::integral_constant<int, 0> s0;
  const std::integral_constant<int, 1> s1;
  if (!Q_full) {
    fetch(r0, s0);
    if (r0 + kRB < r1) fetch(r0 + kRB, s1);
  }
  for (int rb = r0; rb < r1; rb += 2 * kRB) {
    block(rb, s0);
    if (rb + kRB < r1) block(rb + kRB, s1);
  }
  if (diag) {
    Gp[rr0][cc] = gacc;
    __syncthreads();
    if (threadIdx.x < kT)
      gpart[(((size_t)ta * sh.N + (k - 1)) * sh.nchunks + chunk) * kT + threadIdx.x] =
          ((Gp[0][threadIdx.x] + Gp[1][threadIdx.x]) + Gp[2][threadIdx.x]) + Gp[3][threadIdx.x];
  }
  // C layout: lane holds rows 4 (lane >> 4) + i of each 16x16 tile, column lane & 15
  float* out = part + (((size_t)tile * sh.N + (k - 1)) * sh.nchunks + chunk) * (kT * kT);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        out[(qa + 16 * x + 4 * (lane >> 4) + i) * kT + qb + 16 * y + (lane & 15)] = acc[x][y][i];
}

// FP64: the same tiling on the VALU (one lane per output element).
__global__ void __launch_bounds__(256)
gram_kernel_f64(GramShape sh, const double* __restrict__ S_all, const double* __restrict__ Q, int Q_full,
                double* __restrict__ part) {
  int tile;
  const int k = live_pair(sh, blockIdx.x, tile), chunk = blockIdx.y;
  int ta, tb;
  tile_coords(tile, ta, tb);
  if (k < first_stage(ta, sh.nu)) return;
  const int cols = k * sh.nu, rows = NBX * sh.M;
  const double* Sk = S_all + S_offset(k, sh.M, sh.nu);
  const double* Qk = Q + (size_t)k * sh.M * NBX * (Q_full ? NBX : 1);
  const int r0 = chunk * kChunkRows, r1 = min(rows, r0 + kChunkRows);
  double* out = part + (((size_t)tile * sh.N + (k - 1)) * sh.nchunks + chunk) * (kT * kT);
  for (int e = threadIdx.x; e < kT * kT; e += 256) {
    const int ca = kT * ta + e / kT, cb = kT * tb + e % kT;
    double acc = 0.0;
    if (ca < cols && cb < cols)
      for (int r = r0; r < r1; ++r) acc += Sk[(size_t)r * cols + ca] * qs_value(Sk, Qk, Q_full, cols, r, cb);
    out[e] = acc;
  }
}

// g partials: one lane per column of S_k.  grid: x = stage k-1, y = row chunk
// of kGRows rows (16 nodes), so there are enough workgroups to cover the chip.
constexpr int kGRows = 96;
template <typename T>
__global__ void __launch_bounds__(256)
gvec_kernel(GramShape sh, const T* __restrict__ S_all, const T* __restrict__ Gx_all, const T* __restrict__ Q,
            int Q_full, const T* __restrict__ q, T* __restrict__ gpart) {
  __shared__ T wv[kGRows];
  const int k = blockIdx.x + 1, chunk = blockIdx.y;
  const int cols = k * sh.nu, rows = NBX * sh.M;
  const T* Sk = S_all + S_offset(k, sh.M, sh.nu);
  const T* Gxk = Gx_all + (size_t)k * sh.M * NBX;
  const T* Qk = Q + (size_t)k * sh.M * NBX * (Q_full ? NBX : 1);
  const T* qk = q + (size_t)k * sh.M * NBX;
  const int r0 = chunk * kGRows, r1 = min(rows, r0 + kGRows);
  for (int r = r0 + threadIdx.x; r < r1; r += 256) {  // w = Q_k Gx_k + q_k
    const int node = r / NBX, rr = r - node * NBX;
    T v;
    if (Q_full) {
      v = T(0);
      const T* Qn = Qk + ((size_t)node * NBX + rr) * NBX;
      for (int s2 = 0; s2 < NBX; ++s2) v += Qn[s2] * Gxk[(size_t)node * NBX + s2];
    } else {
      v = Qk[r] * Gxk[r];
    }
    wv[r - r0] = v + qk[r];
  }
  __syncthreads();
  T* out = gpart + ((size_t)(k - 1) * sh.ngchunks + chunk) * sh.n;
  for (int c = threadIdx.x; c < sh.n; c += 256) {
    T acc = T(0);
    if (c < cols)
      for (int r = r0; r < r1; ++r) acc += Sk[(size_t)r * cols + c] * wv[r - r0];
    out[c] = acc;
  }
}

// Fold the gradient partials of all row chunks of one stage (fixed order):
// gstage[k-1][c] = sum over chunks.  One lane per (stage, column).
template <typename T>
__global__ void gvec_fold_kernel(GramShape sh, const T* __restrict__ gpart, T* __restrict__ gstage) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= sh.N * sh.n) return;
  const int k1 = t / sh.n, c = t % sh.n;
  T s = T(0);
  for (int ch = 0; ch < sh.ngchunks; ++ch) s += gpart[((size_t)k1 * sh.ngchunks + ch) * sh.n + c];
  gstage[t] = s;
}

// One lane per element of the lower triangle (and g): fixed-order sum of the
// partials over stages and chunks (chunk loads batched 8 at a time), plus R
// (or r), mirrored to the upper triangle.  g comes from per-stage sums
// (gstage, [N][n]) or, when gtile is set, from the per-(tile, stage, chunk)
// partials of the diagonal Gram tiles ([nt][N][nchunks][kT]).
// One workgroup per 64 consecutive outputs (the lower triangle of H in row order,
// then g); wave q sums the stages k = k0 + q, k0 + q + 4, ... of each output (k0
// its first live stage; each stage's chunk partials in chunk order), and the four
// wave partials are added in wave order: a fixed order, with a quarter of the
// dependent load rounds per thread.
template <typename T>
__global__ void __launch_bounds__(256) gram_reduce_kernel(GramShape sh, const T* __restrict__ part,
                                                          const T* __restrict__ gstage, const T* __restrict__ gtile,
                                                          const T* __restrict__ R, const T* __restrict__ r,
                                                          T* __restrict__ H, T* __restrict__ g) {
  __shared__ T red[4][64];
  const int n = sh.n;
  const long nlow = (long)n * (n + 1) / 2;
  const int q = threadIdx.x >> 6, l = threadIdx.x & 63;
  const long t = (long)blockIdx.x * 64 + l;
  auto chunk_sum = [&](const T* base, size_t stride) {
    T s = T(0);
    for (int c0 = 0; c0 < sh.nchunks; c0 += 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = c0 + u < sh.nchunks ? base[(size_t)(c0 + u) * stride] : T(0);
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    return s;
  };
  int a = 0, b = 0;
  T s = T(0);
  if (t < nlow) {
    a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((long)(a + 1) * (a + 2) / 2 <= t) ++a;
    while ((long)a * (a + 1) / 2 > t) --a;
    b = (int)(t - (long)a * (a + 1) / 2);
    const int ta = a / kT, tb = b / kT;
    const int tile = ta * (ta + 1) / 2 + tb;
    const int e = (a % kT) * kT + (b % kT);
    for (int k = a / sh.nu + 1 + q; k <= sh.N; k += 4)
      s += chunk_sum(part + ((((size_t)tile * sh.N) + (k - 1)) * sh.nchunks) * (kT * kT) + e, (size_t)kT * kT);
  } else if (t < nlow + n) {
    a = (int)(t - nlow);
    if (gtile) {
      const int ta = a / kT;
      for (int k = a / sh.nu + 1 + q; k <= sh.N; k += 4)
        s += chunk_sum(gtile + (((size_t)ta * sh.N + (k - 1)) * sh.nchunks) * kT + a % kT, (size_t)kT);
    } else {
      for (int k = a / sh.nu + 1 + q; k <= sh.N; k += 4) s += gstage[(size_t)(k - 1) * n + a];
    }
  }
  red[q][l] = s;
  __syncthreads();
  if (q != 0) return;
  s = ((red[0][l] + red[1][l]) + red[2][l]) + red[3][l];
  if (t < nlow) {
    const int ka = a / sh.nu, kb = b / sh.nu;
    if (ka == kb) s += R[((size_t)ka * sh.nu + (a % sh.nu)) * sh.nu + (b % sh.nu)];
    H[(size_t)a * n + b] = s;
    H[(size_t)b * n + a] = s;
  } else if (t < nlow + n) {
    g[a] = s + r[a];
  }
}

template <typename T>
__global__ void copy_kernel(const T* __restrict__ src, T* __restrict__ dst, long n) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) dst[t] = src[t];
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
  sh.nt = ceil_div(sh.n, kT);
  sh.ntiles = sh.nt * (sh.nt + 1) / 2;
  sh.nchunks = ceil_div((long)NBX * M, kChunkRows);
  sh.ngchunks = ceil_div((long)NBX * M, kGRows);
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
  // Gx_0 = x0: the first launch reads x0 itself (stage 0 of the workspace is only
  // filled for the optional Gx output below)
  auto gx_in = [&](int k) { return k ? (const T*)(G + (size_t)k * M * NBX) : (const T*)x0; };
  const int wmax = p->wmax;
  const size_t pb_lds = sizeof(T) * ((size_t)p->pb_umax * NBX * (kPropCW + 1) + (size_t)p->pb_emax * 36) +
                        sizeof(int32_t) * (size_t)p->pb_rec_stride;
  const bool use_blocks = p->pb_nodes > 0 && pb_lds <= 64 * 1024 && p->prop_pref != 0;
  if (use_blocks)
    GNMPC_HIP_TRY(p, set_max_lds((const void*)sprop_block_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)pb_lds));
  const bool use2 = use_blocks && p->pb2_stride > 0 && p->prop_pref != 1;
  size_t pb2_lds = 0;
  if (use2) {
    const Prop2Layout L2 = prop2_layout(p->pb_nodes, p->pb_emax, p->pb2_u1max, p->pb2_e1max, p->pb2_u2max);
    pb2_lds = prop2_lds_bytes(L2, sizeof(T), p->pb_emax, p->pb2_u1max, p->pb2_e1max, p->pb2_u2max);
    GNMPC_HIP_TRY(p, set_max_lds((const void*)sprop2_block_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)pb2_lds));
  }
  for (int k = 0; k < N; ++k) {
    const T* S_in = k ? S + S_offset(k, M, nu) : nullptr;
    if (use2 && k + 1 < N) {  // stages k and k + 1 in one launch
      dim3 grid(p->pb_count, ceil_div((k + 2) * nu, kPropCW));
      const size_t sA = (size_t)p->nnz * 36, sB = (size_t)M * NBX * nu, sG = (size_t)M * NBX;
      sprop2_block_kernel<T><<<grid, 256, pb2_lds, s>>>(
          k, M, nu, p->pb_nodes, p->pb_emax, p->pb2_u1max, p->pb2_e1max, p->pb2_u2max, p->d_pb2_rec,
          (const T*)A + k * sA, (const T*)A + (k + 1) * sA, (const T*)B + k * sB, (const T*)B + (k + 1) * sB,
          (const T*)c + k * sG, (const T*)c + (k + 1) * sG, S_in, S + S_offset(k + 1, M, nu),
          S + S_offset(k + 2, M, nu), gx_in(k), G + (k + 1) * sG, G + (k + 2) * sG);
      ++k;
      continue;
    }
    if (use_blocks) {
      dim3 grid(p->pb_count, ceil_div((k + 1) * nu, kPropCW));
      sprop_block_kernel<T><<<grid, 256, pb_lds, s>>>(
          k, M, nu, p->pb_nodes, p->pb_rec_stride, p->pb_umax, p->pb_emax, p->d_pb_rec,
          (const T*)A + (size_t)k * p->nnz * 36, (const T*)B + (size_t)k * M * NBX * nu,
          (const T*)c + (size_t)k * M * NBX, S_in, S + S_offset(k + 1, M, nu), gx_in(k),
          G + (size_t)(k + 1) * M * NBX);
      continue;
    }
    int ncol = (k + 1) * nu + 1;
    int npw = std::max(1, kPropThreads / ncol);
    int lds_cap = (int)(48 * 1024 / (sizeof(T) * 36 * wmax));
    npw = std::max(1, std::min(npw, lds_cap));
    size_t lds = sizeof(T) * 36 * (size_t)wmax * npw + sizeof(int32_t) * ((size_t)wmax * npw + npw + 1);
    sprop_kernel<T><<<ceil_div(M, npw), kPropThreads, lds, s>>>(
        k, M, nu, npw, p->d_prow, p->d_pcol, (const T*)A + (size_t)k * p->nnz * 36,
        (const T*)B + (size_t)k * M * NBX * nu, (const T*)c + (size_t)k * M * NBX, S_in,
        S + S_offset(k + 1, M, nu), gx_in(k), G + (size_t)(k + 1) * M * NBX, wmax);
  }
  phase_end(p, GNMPC_PH_CONDENSE_PROPAGATE, s);
  GramShape sh = gram_shape(M, nu, N);
  phase_begin(p, GNMPC_PH_CONDENSE_GRAM, s);
  T* part = (T*)p->d_part;
  T* gpart = part + (size_t)sh.ntiles * N * sh.nchunks * kT * kT;
  dim3 grid(live_pairs(sh), sh.nchunks);
  T* gstage = gpart + (size_t)N * sh.ngchunks * sh.n;
  const T* gtile = nullptr;
  if (sizeof(T) == 4) {
    // the gradient partials come from the diagonal Gram tiles
    gram_kernel_f32<<<grid, 256, 0, s>>>(sh, (const float*)S, (const float*)Q, Q_full, (const float*)G,
                                         (const float*)q, (float*)part, (float*)gpart);
    gtile = gpart;
  } else {
    gram_kernel_f64<<<grid, 256, 0, s>>>(sh, (const double*)S, (const double*)Q, Q_full, (double*)part);
    gvec_kernel<T><<<dim3(N, sh.ngchunks), 256, 0, s>>>(sh, S, G, (const T*)Q, Q_full, (const T*)q, gpart);
    gvec_fold_kernel<T><<<ceil_div((long)N * sh.n, 256), 256, 0, s>>>(sh, gpart, gstage);
  }
  long nred = (long)sh.n * (sh.n + 1) / 2 + sh.n;
  gram_reduce_kernel<T><<<ceil_div(nred, 64), 256, 0, s>>>(sh, part, gstage, gtile, (const T*)R, (const T*)r,
                                                           (T*)H, (T*)g);
  phase_end(p, GNMPC_PH_CONDENSE_GRAM, s);
  if (p->n_c > 0) {
    phase_begin(p, GNMPC_PH_CONDENSE_ROWS, s);
    cons_kernel<T><<<p->n_c, 256, 0, s>>>(M, nu, N, p->d_row_node, p->d_row_stage, (const T*)rowC,
                                           (const T*)rowd, S, G, (T*)Ct, (T*)dt);
    phase_end(p, GNMPC_PH_CONDENSE_ROWS, s);
  }
  if (Gx) {  // Gx_0 = x0, then stages 1..N from the workspace
    const long n0 = (long)M * NBX, ng = (long)N * M * NBX;
    copy_kernel<T><<<(int)std::min<long>(ceil_div(n0, 256), 2048), 256, 0, s>>>((const T*)x0, (T*)Gx, n0);
    copy_kernel<T><<<(int)std::min<long>(ceil_div(ng, 256), 2048), 256, 0, s>>>(G + n0, (T*)Gx + n0, ng);
  }
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

}  // namespace

void prop_blocks_free(gnmpc_plan* p) {
  if (p->d_pb_rec) {
    (void)hipFree(p->d_pb_rec);
    p->d_pb_rec = nullptr;
  }
  if (p->d_pb2_rec) {
    (void)hipFree(p->d_pb2_rec);
    p->d_pb2_rec = nullptr;
  }
  p->pb2_stride = p->pb2_u1max = p->pb2_u2max = p->pb2_e1max = 0;
  p->pb_nodes = p->pb_count = p->pb_umax = p->pb_emax = p->pb_rec_stride = 0;
}

// Node blocks for the block propagation kernel: the largest block size (up to
// nb_max of 4, 2, 1 nodes: one thread per node and column of a 64-column slice)
// whose staged union and A blocks fit 64 KB of LDS in the plan's precision;
// pb_nodes = 0 if even single nodes do not fit.
gnmpc_status prop_blocks2_build(gnmpc_plan* p);

gnmpc_status prop_blocks_build(gnmpc_plan* p) { return prop_blocks_build_nb(p, 4); }

gnmpc_status prop_blocks_build_nb(gnmpc_plan* p, int nb_max) {
  prop_blocks_free(p);
  const int M = p->M;
  const size_t elem = (size_t)p->elem;
  for (int nb = nb_max; nb >= 1; nb /= 2) {
    std::vector<int32_t> ubeg(1, 0), ulist, epos(p->h_pcol.size());
    int umax = 0, emax = 0;
    for (int node0 = 0; node0 < M; node0 += nb) {
      const int node1 = std::min(M, node0 + nb);
      const int e0 = p->h_prow[node0], e1 = p->h_prow[node1];
      std::vector<int32_t> u(p->h_pcol.begin() + e0, p->h_pcol.begin() + e1);
      std::sort(u.begin(), u.end());
      u.erase(std::unique(u.begin(), u.end()), u.end());
      for (int e = e0; e < e1; ++e)
        epos[e] = (int32_t)(std::lower_bound(u.begin(), u.end(), p->h_pcol[e]) - u.begin());
      ulist.insert(ulist.end(), u.begin(), u.end());
      ubeg.push_back((int32_t)ulist.size());
      umax = std::max(umax, (int)u.size());
      emax = std::max(emax, e1 - e0);
    }
    // record: e0, ne, uc, nn, row starts [nb + 1], union nodes [umax], entry positions [emax]
    const int stride = (4 + (nb + 1) + umax + emax + 3) / 4 * 4;
    if (elem * ((size_t)umax * NBX * (kPropCW + 1) + (size_t)emax * 36) + 4 * (size_t)stride > 64 * 1024) continue;
    const int nblk = (int)ubeg.size() - 1;
    std::vector<int32_t> rec((size_t)nblk * stride, 0);
    for (int b = 0; b < nblk; ++b) {
      int32_t* r = rec.data() + (size_t)b * stride;
      const int node0 = b * nb, node1 = std::min(M, node0 + nb);
      const int e0 = p->h_prow[node0], e1 = p->h_prow[node1];
      r[0] = e0;
      r[1] = e1 - e0;
      r[2] = ubeg[b + 1] - ubeg[b];
      r[3] = node1 - node0;
      for (int t = 0; t <= node1 - node0; ++t) r[4 + t] = p->h_prow[node0 + t] - e0;
      for (int t = 0; t < r[2]; ++t) r[4 + nb + 1 + t] = ulist[ubeg[b] + t];
      for (int e = e0; e < e1; ++e) r[4 + nb + 1 + umax + (e - e0)] = epos[e];
    }
    GNMPC_HIP_TRY(p, hipMalloc((void**)&p->d_pb_rec, sizeof(int32_t) * std::max<size_t>(rec.size(), 1)));
    if (!rec.empty())
      GNMPC_HIP_TRY(p, hipMemcpy(p->d_pb_rec, rec.data(), sizeof(int32_t) * rec.size(), hipMemcpyHostToDevice));
    p->pb_nodes = nb;
    p->pb_count = nblk;
    p->pb_umax = umax;
    p->pb_emax = emax;
    p->pb_rec_stride = stride;
    return prop_blocks2_build(p);
  }
  return GNMPC_OK;
}

// Two-stage records of the propagation blocks: U1 = the union of the block's pattern
// columns (the nodes whose S_{k+1} rows the block's S_{k+2} rows read), U1's pattern
// entries (global index, position of the column in U2) and U2 = the union of U1's
// pattern columns.  Layout per block (int32): e0, ne, nn, |U1|, |U2|, U1 entry count, 0, 0,
// then the arrays at the offsets of Prop2Layout.  Not used (pb2_stride = 0) when the
// staged rows do not fit kProp2LdsCap bytes of LDS.
gnmpc_status prop_blocks2_build(gnmpc_plan* p) {
  if (p->d_pb2_rec) {
    (void)hipFree(p->d_pb2_rec);
    p->d_pb2_rec = nullptr;
  }
  p->pb2_stride = p->pb2_u1max = p->pb2_u2max = p->pb2_e1max = 0;
  const int M = p->M, nb = p->pb_nodes;
  if (nb <= 0) return GNMPC_OK;
  const int nblk = p->pb_count;
  std::vector<std::vector<int32_t>> U1(nblk), U2(nblk), E1(nblk), P2(nblk), R1(nblk);
  int u1max = 0, u2max = 0, e1max = 0;
  for (int b = 0; b < nblk; ++b) {
    const int node0 = b * nb, node1 = std::min(M, node0 + nb);
    const int e0 = p->h_prow[node0], e1 = p->h_prow[node1];
    std::vector<int32_t>& u1 = U1[b];
    u1.assign(p->h_pcol.begin() + e0, p->h_pcol.begin() + e1);
    std::sort(u1.begin(), u1.end());
    u1.erase(std::unique(u1.begin(), u1.end()), u1.end());
    std::vector<int32_t>& u2 = U2[b];
    R1[b].push_back(0);
    for (int32_t u : u1) {
      for (int e = p->h_prow[u]; e < p->h_prow[u + 1]; ++e) {
        E1[b].push_back(e);
        u2.push_back(p->h_pcol[e]);
      }
      R1[b].push_back((int32_t)E1[b].size());
    }
    std::sort(u2.begin(), u2.end());
    u2.erase(std::unique(u2.begin(), u2.end()), u2.end());
    for (int32_t e : E1[b])
      P2[b].push_back((int32_t)(std::lower_bound(u2.begin(), u2.end(), p->h_pcol[e]) - u2.begin()));
    u1max = std::max(u1max, (int)u1.size());
    u2max = std::max(u2max, (int)u2.size());
    e1max = std::max(e1max, (int)E1[b].size());
  }
  const Prop2Layout L = prop2_layout(nb, p->pb_emax, u1max, e1max, u2max);
  const size_t lds = prop2_lds_bytes(L, (size_t)p->elem, p->pb_emax, u1max, e1max, u2max);
  if (lds > kProp2LdsCap) return GNMPC_OK;
  std::vector<int32_t> rec((size_t)nblk * L.stride, 0);
  for (int b = 0; b < nblk; ++b) {
    int32_t* r = rec.data() + (size_t)b * L.stride;
    const int node0 = b * nb, node1 = std::min(M, node0 + nb);
    const int e0 = p->h_prow[node0], e1 = p->h_prow[node1];
    r[0] = e0;
    r[1] = e1 - e0;
    r[2] = node1 - node0;
    r[3] = (int32_t)U1[b].size();
    r[4] = (int32_t)U2[b].size();
    r[5] = (int32_t)E1[b].size();
    for (int t = 0; t <= node1 - node0; ++t) r[L.rs + t] = p->h_prow[node0 + t] - e0;
    for (int e = e0; e < e1; ++e)
      r[L.es1 + (e - e0)] = (int32_t)(std::lower_bound(U1[b].begin(), U1[b].end(), p->h_pcol[e]) - U1[b].begin());
    for (size_t t = 0; t < U1[b].size(); ++t) r[L.u1 + t] = U1[b][t];
    for (size_t t = 0; t < R1[b].size(); ++t) r[L.r1 + t] = R1[b][t];
    for (size_t t = 0; t < E1[b].size(); ++t) {
      r[L.g1 + t] = E1[b][t];
      r[L.es2 + t] = P2[b][t];
    }
    for (size_t t = 0; t < U2[b].size(); ++t) r[L.u2 + t] = U2[b][t];
  }
  GNMPC_HIP_TRY(p, hipMalloc((void**)&p->d_pb2_rec, sizeof(int32_t) * std::max<size_t>(rec.size(), 1)));
  if (!rec.empty())
    GNMPC_HIP_TRY(p, hipMemcpy(p->d_pb2_rec, rec.data(), sizeof(int32_t) * rec.size(), hipMemcpyHostToDevice));
  p->pb2_stride = L.stride;
  p->pb2_u1max = u1max;
  p->pb2_u2max = u2max;
  p->pb2_e1max = e1max;
  return GNMPC_OK;
}

size_t condense_partial_elems(int M, int nu, int N) {
  GramShape sh = gram_shape(M, nu, N);
  // H partials, then either the gradient partials of the diagonal tiles (FP32) or the
  // per-chunk gradient partials and their per-stage sums (FP64)
  const size_t gt = (size_t)sh.nt * N * sh.nchunks * kT;
  const size_t gv = (size_t)N * sh.ngchunks * sh.n + (size_t)N * sh.n;
  return (size_t)sh.ntiles * N * sh.nchunks * kT * kT + std::max(gt, gv);
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
