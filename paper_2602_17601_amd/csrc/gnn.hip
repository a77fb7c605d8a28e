// GNN dynamics model (Sec. V-A eq. forward_dynamics) and its linearization by
// forward-mode differentiation (Sec. V-A "Linearization", eq.
// linearized_dynamics), on the GPU.
//
// Forward pass at the N linearization points: one launch for the encoder, one
// per message-passing round and one for the decoder, each over every
// (stage, node).  The edge MLP is evaluated per node in factored form,
// W_e [h_i; h_i - h_j] = W_a h_i + W_b h_i - W_b h_j, and the ReLU masks of
// the encoder, every edge and every node update are kept as bit masks: they
// are all the Jacobian pass needs from the forward pass.
//
// Jacobian pass (seed-centric forward mode): the tangent columns of one or two
// consecutive "seed" nodes (6 state columns each, plus 3 force columns for an
// actuated node; at most 16 columns) are pushed through all L rounds inside
// one workgroup.  After round l they are nonzero only on the nodes within l
// hops of the seeds, so the workgroup carries exactly those nodes (lists built
// on the host), and after the decoder it owns the blocks A^{is} and B^i of
// every node i reached by its seeds.  No tangent ever leaves the chip.
// In BF16 mode the weights are bfloat16 (round to nearest even).  The forward
// pass keeps the activations in FP32 -- on the matrix cores each FP32 operand
// enters as three bf16 terms hi + mid + lo, so the products are exact and the
// sums FP32 -- and therefore takes every ReLU decision at FP32 accuracy; the
// Jacobian pass rounds the tangents to bfloat16 and accumulates in FP32.
#include <algorithm>
#include <cstring>
#include <vector>

#include "plan.hpp"

#include "gnn_state.hpp"

namespace gnmpc {
namespace {

constexpr int kCols = 16;  // tangent columns per seed tile

// Stage layout of the register-aggregate Jacobian kernel, per round l >= 1
// (32-bit words): one record per node p of round l-1 -- [0] index of p in
// round l (equal to p: each round starts with the previous round's nodes),
// [1] bit set of p's receivers in round l, [2..3] unused,
// [4 + 16 w + q] word w of the ReLU mask of edge (receiver q <- p) or 0,
// [4 + 16 HW + g] four byte counters of p's active in-edges for features
// 4g..4g+3 -- then the node-update masks of the nodes of round l ([q][HW]),
// padded to 4 words; after the last round, one 4-word record per output
// block, then the encoder block: the tile's 16 column-map words and the
// encoder ReLU masks of round 0's nodes ([q][HW]).  The host describes every
// word of a tile's stage by its source, (kind | round << 4, index), and a
// gather kernel writes the stage image of every (tile, stage) to global
// memory after the forward pass, so the Jacobian kernel reads its stage in
// one contiguous copy.
enum GatherKind { kGEdgeMask = 0, kGNodeMask = 1, kGCount = 2, kGConst = 3, kGEncMask = 4 };
__host__ __device__ constexpr int stage_record_words(int Hd) { return 4 + 16 * (Hd / 32) + Hd / 4; }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float float2v_t __attribute__((ext_vector_type(2)));

// Round to bf16, nearest-even (one v_cvt_pk_bf16_f32 on gfx950).
__device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  const float2v_t f = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2_t));
}
__device__ inline float bf16r(float x) { return __uint_as_float(pack_bf16x2(0.f, x) & 0xFFFF0000u); }

float host_bf16r(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  u &= 0xFFFF0000u;
  float r;
  std::memcpy(&r, &u, 4);
  return r;
}

__device__ inline bool mbit(const uint32_t* m, int f) { return (m[f >> 5] >> (f & 31)) & 1u; }

// Store the ReLU mask of the 64 features handled by this wave (z > 0).
__device__ inline void store_mask(uint32_t* words, int f, bool on) {
  unsigned long long b = __ballot(on);
  if ((threadIdx.x & 63) == 0) {
    words[f >> 5] = (uint32_t)(b & 0xFFFFFFFFull);
    words[(f >> 5) + 1] = (uint32_t)(b >> 32);
  }
}

struct FwdArgs {
  int N, M, E, Hd, L, nu, bf16;
  float dt;
  const float *xhat, *uhat;
  const int32_t *row_ptr, *col, *act_of_node;
  const float *encT, *benc, *WaT, *WbT, *be, *Wn1T, *Wn2T, *bn, *decT, *bdec;
  float* h;
  uint32_t *mask_enc, *mask_node, *mask_edge;
  float* fnext;
};

// h0 = relu(W_enc [x; P u] + b); one workgroup of Hd lanes per (stage, node).
__global__ void fwd_enc_kernel(FwdArgs a) {
  const int s = blockIdx.x;  // stage * M + node
  const int k = s / a.M, i = s - k * a.M;
  const int f = threadIdx.x;
  float in[9];
  const float* x = a.xhat + (size_t)s * NBX;
#pragma unroll
  for (int d = 0; d < 6; ++d) in[d] = x[d];
  int act = a.act_of_node[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) in[6 + d] = act >= 0 ? a.uhat[(size_t)k * a.nu + 3 * act + d] : 0.f;
  float z = a.benc[f];
#pragma unroll
  for (int d = 0; d < 9; ++d) z += a.encT[d * a.Hd + f] * in[d];
  bool on = z > 0.f;
  float hv = on ? z : 0.f;
  a.h[(size_t)s * a.Hd + f] = hv;
  store_mask(a.mask_enc + (size_t)s * (a.Hd / 32), f, on);
}

// One message-passing round l; workgroup of Hd lanes per (stage, node).
__global__ void fwd_layer_kernel(FwdArgs a, int l) {
  extern __shared__ float sh[];  // [1 + maxdeg][Hd] inputs, then [Hd] aggregate
  const int s = blockIdx.x;
  const int k = s / a.M, i = s - k * a.M;
  const int f = threadIdx.x, Hd = a.Hd;
  const float* hin = a.h + (size_t)l * a.N * a.M * Hd;
  const int e0 = a.row_ptr[i], deg = a.row_ptr[i + 1] - e0;
  sh[f] = hin[(size_t)s * Hd + f];
  for (int t = 0; t < deg; ++t) sh[(1 + t) * Hd + f] = hin[((size_t)k * a.M + a.col[e0 + t]) * Hd + f];
  __syncthreads();
  const float* WaT = a.WaT + (size_t)l * Hd * Hd;
  const float* WbT = a.WbT + (size_t)l * Hd * Hd;
  float ya = 0.f, ybi = 0.f;
  for (int q = 0; q < Hd; ++q) {
    ya += WaT[q * Hd + f] * sh[q];
    ybi += WbT[q * Hd + f] * sh[q];
  }
  const float base = ya + ybi + a.be[l * Hd + f];
  float agg = 0.f;
  uint32_t* me = a.mask_edge + (((size_t)l * a.N + k) * a.E) * (Hd / 32);
  for (int t = 0; t < deg; ++t) {
    const float* hj = sh + (1 + t) * Hd;
    float ybj = 0.f;
    for (int q = 0; q < Hd; ++q) ybj += WbT[q * Hd + f] * hj[q];
    float z = base - ybj;
    bool on = z > 0.f;
    agg += on ? z : 0.f;
    store_mask(me + (size_t)(e0 + t) * (Hd / 32), f, on);
  }
  float* sagg = sh + (size_t)(1 + deg) * Hd;  // after the inputs
  sagg[f] = agg;
  __syncthreads();
  const float* W1 = a.Wn1T + (size_t)l * Hd * Hd;
  const float* W2 = a.Wn2T + (size_t)l * Hd * Hd;
  float z = a.bn[l * Hd + f];
  for (int q = 0; q < Hd; ++q) z += W1[q * Hd + f] * sh[q] + W2[q * Hd + f] * sagg[q];
  bool on = z > 0.f;
  float hv = on ? z : 0.f;
  a.h[((size_t)(l + 1) * a.N * a.M + s) * Hd + f] = hv;
  store_mask(a.mask_node + ((size_t)l * a.N * a.M + s) * (Hd / 32), f, on);
}

// o = W_dec h + b; v+ = v + dt o[3:6], p+ = p + dt v+ ; one lane per (stage, node).
__global__ void fwd_dec_kernel(FwdArgs a) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.N * a.M) return;
  const float* hL = a.h + ((size_t)a.L * a.N * a.M + s) * a.Hd;
  float o[3] = {a.bdec[3], a.bdec[4], a.bdec[5]};
  for (int q = 0; q < a.Hd; ++q) {
    float hv = hL[q];
#pragma unroll
    for (int r = 0; r < 3; ++r) o[r] += a.decT[q * 6 + 3 + r] * hv;
  }
  const float* x = a.xhat + (size_t)s * NBX;
  float* fo = a.fnext + (size_t)s * NBX;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    float vn = x[3 + r] + a.dt * o[r];
    fo[3 + r] = vn;
    fo[r] = x[r] + a.dt * vn;
  }
}

struct JvpArgs {
  int N, M, E, Hd, L, nu, bf16, meta_stride, bufX;
  float dt;
  const float *encT, *WaT, *WbT, *Wn1T, *Wn2T, *decT;
  const uint32_t *mask_enc, *mask_node, *mask_edge;
  const int32_t *meta, *seed, *seedcol, *seedact, *V, *Vself, *Vebeg, *Vecnt, *Eloc, *Eid, *out3, *bout2;
  float *A, *B;
  long nnz;
};

template <typename S>
struct Store;
template <>
struct Store<float> {
  __device__ static float ld(const float* p) { return *p; }
  __device__ static void st(float* p, float v, int) { *p = v; }
};
template <>
struct Store<uint16_t> {
  __device__ static float ld(const uint16_t* p) { return __uint_as_float((uint32_t)(*p) << 16); }
  __device__ static void st(uint16_t* p, float v, int) { *p = (uint16_t)(__float_as_uint(bf16r(v)) >> 16); }
};

// Seed-centric forward-mode Jacobian, VALU form.  Workgroup (tile, stage),
// 2*Hd lanes: lane t owns feature f = t % Hd and columns c0..c0+7, c0 = 8 (t / Hd).
// Tangent buffers X (rounds 0, 2, ...) and Y (rounds 1, 3, ...) are
// [nodes][Hd][16] in LDS.
template <typename S>
__global__ void jvp_valu_kernel(JvpArgs a) {
  extern __shared__ unsigned char smem_raw[];
  S* X = reinterpret_cast<S*>(smem_raw);
  S* Y = X + (size_t)a.bufX * a.Hd * kCols;
  const int tile = blockIdx.x, k = blockIdx.y;
  const int Hd = a.Hd;
  const int f = threadIdx.x % Hd, c0 = 8 * (threadIdx.x / Hd);
  const int32_t* mt = a.meta + (size_t)tile * a.meta_stride;
  const int sb = mt[0], sc = mt[1], ob = mt[2], oc = mt[3], bb = mt[4], bc = mt[5];
  const int hw = Hd / 32;
  // ---- round 0: encoder tangents on the seeds
  {
    const int vb = mt[6], vc = mt[7];
    for (int q = 0; q < vc; ++q) {
      const int node = a.V[vb + q];
      const int p = a.Vself[vb + q];  // seed index
      const int col0 = a.seedcol[sb + p];
      const bool act = a.seedact[sb + p] >= 0;
      const bool on = mbit(a.mask_enc + ((size_t)k * a.M + node) * hw, f);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        int cc = c0 + c, d = cc - col0;
        float v = 0.f;
        if (on && d >= 0 && (d < 6 || (act && d < 9))) v = a.encT[d * Hd + f];
        Store<S>::st(X + ((size_t)q * Hd + f) * kCols + cc, v, 0);
      }
    }
  }
  __syncthreads();
  for (int l = 1; l <= a.L; ++l) {
    S* in = (l & 1) ? X : Y;
    S* out = (l & 1) ? Y : X;
    const int vb = mt[6 + 2 * l], vc = mt[7 + 2 * l];
    const float* WaT = a.WaT + (size_t)(l - 1) * Hd * Hd;
    const float* WbT = a.WbT + (size_t)(l - 1) * Hd * Hd;
    const float* W1 = a.Wn1T + (size_t)(l - 1) * Hd * Hd;
    const float* W2 = a.Wn2T + (size_t)(l - 1) * Hd * Hd;
    const uint32_t* me = a.mask_edge + ((size_t)(l - 1) * a.N + k) * a.E * hw;
    // phase A: aggregated edge tangents into `out`
    for (int q = 0; q < vc; ++q) {
      const int self = a.Vself[vb + q];
      float P[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) P[c] = 0.f;
      if (self >= 0) {
        const S* t = in + (size_t)self * Hd * kCols + c0;
        for (int r = 0; r < Hd; ++r) {
          float w = WaT[r * Hd + f] + WbT[r * Hd + f];
#pragma unroll
          for (int c = 0; c < 8; ++c) P[c] += w * Store<S>::ld(t + (size_t)r * kCols + c);
        }
      }
      float acc[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] = 0.f;
      const int eb = a.Vebeg[vb + q], ec = a.Vecnt[vb + q];
      for (int t = 0; t < ec; ++t) {
        const int jl = a.Eloc[eb + t], eid = a.Eid[eb + t];
        if (!mbit(me + (size_t)eid * hw, f)) continue;
        float yb[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) yb[c] = 0.f;
        if (jl >= 0) {
          const S* tj = in + (size_t)jl * Hd * kCols + c0;
          for (int r = 0; r < Hd; ++r) {
            float w = WbT[r * Hd + f];
#pragma unroll
            for (int c = 0; c < 8; ++c) yb[c] += w * Store<S>::ld(tj + (size_t)r * kCols + c);
          }
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] += P[c] - yb[c];
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) Store<S>::st(out + ((size_t)q * Hd + f) * kCols + c0 + c, acc[c], 0);
    }
    __syncthreads();
    // phase B: node update tangents, written over the aggregate one node at a time
    const uint32_t* mn = a.mask_node + ((size_t)(l - 1) * a.N + k) * a.M * hw;
    for (int q = 0; q < vc; ++q) {
      const int node = a.V[vb + q];
      const int self = a.Vself[vb + q];
      float z[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) z[c] = 0.f;
      if (mbit(mn + (size_t)node * hw, f)) {
        if (self >= 0) {
          const S* t = in + (size_t)self * Hd * kCols + c0;
          for (int r = 0; r < Hd; ++r) {
            float w = W1[r * Hd + f];
#pragma unroll
            for (int c = 0; c < 8; ++c) z[c] += w * Store<S>::ld(t + (size_t)r * kCols + c);
          }
        }
        const S* ag = out + (size_t)q * Hd * kCols + c0;
        for (int r = 0; r < Hd; ++r) {
          float w = W2[r * Hd + f];
#pragma unroll
          for (int c = 0; c < 8; ++c) z[c] += w * Store<S>::ld(ag + (size_t)r * kCols + c);
        }
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 8; ++c) Store<S>::st(out + ((size_t)q * Hd + f) * kCols + c0 + c, z[c], 0);
      __syncthreads();
    }
  }
  // ---- decoder and the Jacobian blocks
  S* fin = (a.L & 1) ? Y : X;
  const int vbL = mt[6 + 2 * a.L];
  for (int t = threadIdx.x; t < oc * 18; t += blockDim.x) {
    const int o = t / 18, rem = t % 18, r = rem / 6, d = rem % 6;  // r: 0..2 (row pair), d: input column
    const int q = a.out3[3 * (ob + o)], p = a.out3[3 * (ob + o) + 1];
    const long e = a.out3[3 * (ob + o) + 2];
    const int node = a.V[vbL + q];
    const int s_node = a.seed[sb + p];
    const int col = a.seedcol[sb + p] + d;
    float dov = 0.f;
    const S* tq = fin + (size_t)q * Hd * kCols + col;
    for (int ff = 0; ff < Hd; ++ff) dov += a.decT[ff * 6 + 3 + r] * Store<S>::ld(tq + (size_t)ff * kCols);
    const bool diag = node == s_node;
    float dv = (diag && d == 3 + r ? 1.f : 0.f) + a.dt * dov;
    float dp = (diag && d == r ? 1.f : 0.f) + a.dt * dv;
    float* blk = a.A + ((size_t)k * a.nnz + e) * 36;
    blk[r * 6 + d] = dp;
    blk[(3 + r) * 6 + d] = dv;
  }
  for (int t = threadIdx.x; t < bc * 9; t += blockDim.x) {
    const int o = t / 9, rem = t % 9, r = rem / 3, d = rem % 3;
    const int q = a.bout2[2 * (bb + o)], p = a.bout2[2 * (bb + o) + 1];
    const int node = a.V[vbL + q];
    const int act = a.seedact[sb + p];
    const int col = a.seedcol[sb + p] + 6 + d;
    float dov = 0.f;
    const S* tq = fin + (size_t)q * Hd * kCols + col;
    for (int ff = 0; ff < Hd; ++ff) dov += a.decT[ff * 6 + 3 + r] * Store<S>::ld(tq + (size_t)ff * kCols);
    float dv = a.dt * dov;
    float* Bi = a.B + (((size_t)k * a.M + node) * NBX) * a.nu;
    Bi[(3 + r) * a.nu + 3 * act + d] = dv;
    Bi[r * a.nu + 3 * act + d] = a.dt * dv;
  }
  (void)sc;
}


// ---------------------------------------------------------------------------
// Seed-centric forward-mode Jacobian on the matrix cores (BF16 operands, FP32
// accumulation): v_mfma_f32_16x16x32_bf16.  Workgroup (tile, stage) of 4
// waves; wave w owns the output features [w Hd/4, (w+1) Hd/4) of every GEMM,
// so the 16 tangent columns are the MFMA N dimension and the nodes of a round
// are processed one after another.
//   R1: tangents of round l-1, bf16 [node][col][Hd+8]    (MFMA B operands)
//   R2: edge aggregates of round l, fp32 [node][col][Hd+4]
// Round l: for every node p of round l-1, Yb = W_b dh_p and P = W_a dh_p + Yb
// (8 MFMA per 16x16 output tile); P enters p's own aggregate once per in-edge
// whose ReLU is on (a per-feature count), and -Yb enters the aggregate of each
// receiver r of p under the mask of edge (r <- p).  Then per node q of round l:
// dh_q = mask_q (W_n1 dh_q + W_n2 bf16(agg_q)).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

struct MfmaArgs {
  int N, M, E, L, nu, meta_stride, cap1, cap2;
  float dt;
  const float *encT, *decT;
  const uint16_t *Wa, *Wb, *Wn1, *Wn2;
  const uint32_t *mask_enc, *mask_node, *mask_edge;
  const int32_t *meta, *seed, *seedcol, *seedact, *V, *Vself, *prog, *elist, *out3, *bout2;
  float *A, *B;
  long nnz;
};


// LDS columns are XOR-swizzled in 16-byte chunks by (column & 7), so the 16
// lanes that read one k-slice of 16 different columns hit different banks.
__device__ inline int swz(int byte_in_col, int c) { return (((byte_in_col >> 4) ^ (c & 7)) << 4) | (byte_in_col & 15); }
// The same over all 16 chunks of a 256-byte column (16 lanes reading 16 columns
// hit 16 different chunk positions), for columns of 128 bf16 features.
template <int CB>
__device__ inline int swzc(int byte_in_col, int c) {
  constexpr int mask = CB >= 256 ? 15 : 7;
  return (((byte_in_col >> 4) ^ (c & mask)) << 4) | (byte_in_col & 15);
}

template <int MT>
__global__ void __launch_bounds__(256) jvp_mfma_kernel(MfmaArgs a) {
  constexpr int Hd = MT * 64;
  constexpr int KB = Hd / 32;  // 32-deep k-blocks
  constexpr int RW = Hd / 4;   // features per wave
  constexpr int MAXV = 16;     // nodes per round held as output registers
  constexpr int HW = Hd / 32;  // mask words per node or edge
  constexpr int CB1 = Hd * 2;  // bytes per bf16 tangent column
  constexpr int CB2 = Hd * 4;  // bytes per fp32 aggregate column
  extern __shared__ unsigned char smem_raw[];
  unsigned char* R1 = smem_raw;                                            // [cap1][16] bf16 columns
  unsigned char* R2 = smem_raw + (size_t)a.cap1 * kCols * CB1;            // [cap2][16] fp32 columns
  int32_t* SP = reinterpret_cast<int32_t*>(R2 + (size_t)a.cap2 * kCols * CB2);  // staged program + masks
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = lane & 15, grp = lane >> 4;
  const int tile = blockIdx.x, k = blockIdx.y;
  const int32_t* mt = a.meta + (size_t)tile * a.meta_stride;
  const int sb = mt[0], ob = mt[2], oc = mt[3], bb = mt[4], bc = mt[5];

  // ---- round 0: encoder tangents of the seeds (mask x weight, exact in bf16)
  {
    const int vb = mt[6], vc = mt[7];
    for (int t = threadIdx.x; t < vc * kCols * Hd; t += 256) {
      const int q = t / (kCols * Hd), c = (t / Hd) % kCols, f = t % Hd;
      const int node = a.V[vb + q];
      const int p = a.Vself[vb + q];
      const int d = c - a.seedcol[sb + p];
      const bool act = a.seedact[sb + p] >= 0;
      float v = 0.f;
      if (d >= 0 && (d < 6 || (act && d < 9)) && mbit(a.mask_enc + ((size_t)k * a.M + node) * HW, f))
        v = a.encT[d * Hd + f];
      *reinterpret_cast<uint16_t*>(R1 + ((size_t)q * kCols + c) * CB1 + swz(2 * f, c)) =
          (uint16_t)(__float_as_uint(v) >> 16);
    }
  }

  for (int l = 1; l <= a.L; ++l) {
    const int vc0 = mt[7 + 2 * (l - 1)];
    const int vb1 = mt[6 + 2 * l], vc1 = mt[7 + 2 * l];
    const int* pm = mt + 6 + 2 * (a.L + 1) + 4 * (l - 1);
    const int pbeg = pm[0], plen = pm[1], ebeg = pm[2], elen = pm[3];
    const size_t woff = (size_t)(l - 1) * Hd * Hd;
    // stage this round's sender program, the edge masks it reads and the node masks
    const int plen4 = (plen + 3) / 4 * 4;
    uint32_t* SM = reinterpret_cast<uint32_t*>(SP + plen4);   // [elen][HW]
    uint32_t* SN = SM + elen * HW;                             // [vc1][HW]
    {
      for (int t = threadIdx.x; t < plen; t += 256) SP[t] = a.prog[pbeg + t];
      const uint32_t* me = a.mask_edge + ((size_t)(l - 1) * a.N + k) * a.E * HW;
      for (int t = threadIdx.x; t < elen * HW; t += 256) SM[t] = me[(size_t)a.elist[ebeg + t / HW] * HW + t % HW];
      const uint32_t* mn = a.mask_node + ((size_t)(l - 1) * a.N + k) * a.M * HW;
      for (int t = threadIdx.x; t < vc1 * HW; t += 256) SN[t] = mn[(size_t)a.V[vb1 + t / HW] * HW + t % HW];
      for (int t = threadIdx.x; t < vc1 * kCols * CB2 / 16; t += 256)
        reinterpret_cast<uint4*>(R2)[t] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    // ---- phase A: edge GEMMs per sender, masked scatter into the fp32 aggregates
    {
      bf16x8_t wa[MT][KB], wb[MT][KB];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int row = wave * RW + 16 * m + col;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          wa[m][kb] = *reinterpret_cast<const bf16x8_t*>(a.Wa + woff + (size_t)row * Hd + kb * 32 + grp * 8);
          wb[m][kb] = *reinterpret_cast<const bf16x8_t*>(a.Wb + woff + (size_t)row * Hd + kb * 32 + grp * 8);
        }
      }
      int po = 0, mo = 0;
      for (int p = 0; p < vc0; ++p) {
        const unsigned char* Tp = R1 + ((size_t)p * kCols + col) * CB1;
        bf16x8_t bfr[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
          bfr[kb] = *reinterpret_cast<const bf16x8_t*>(Tp + swz(64 * kb + 16 * grp, col));
        floatx4_t ay[MT], ap[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          ay[m] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) ay[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[m][kb], bfr[kb], ay[m], 0, 0, 0);
          ap[m] = ay[m];
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) ap[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[m][kb], bfr[kb], ap[m], 0, 0, 0);
        }
        const int qp = SP[po], nin = SP[po + 1], nout = SP[po + 2];
        po += 3;
        // receiver term: P times the number of in-edges whose ReLU is on, per feature
        float cnt[MT][4];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int i = 0; i < 4; ++i) cnt[m][i] = 0.f;
        for (int e = 0; e < nin; ++e) {
#pragma unroll
          for (int m = 0; m < MT; ++m) {
            const int f0 = wave * RW + 16 * m + 4 * grp;
            const uint32_t bits = SM[mo + e * HW + (f0 >> 5)] >> (f0 & 31);
#pragma unroll
            for (int i = 0; i < 4; ++i) cnt[m][i] += (float)((bits >> i) & 1u);
          }
        }
        mo += nin * HW;
        {
          unsigned char* dq = R2 + ((size_t)qp * kCols + col) * CB2;
#pragma unroll
          for (int m = 0; m < MT; ++m) {
            const int f0 = wave * RW + 16 * m + 4 * grp;
            floatx4_t* ptr = reinterpret_cast<floatx4_t*>(dq + swz(4 * f0, col));
            floatx4_t v = *ptr;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] += cnt[m][i] * ap[m][i];
            *ptr = v;
          }
        }
        // sender term: -mask (r <- p) * Yb into each receiver's aggregate
        for (int t = 0; t < nout; ++t) {
          unsigned char* dr = R2 + ((size_t)SP[po + t] * kCols + col) * CB2;
#pragma unroll
          for (int m = 0; m < MT; ++m) {
            const int f0 = wave * RW + 16 * m + 4 * grp;
            const uint32_t bits = SM[mo + t * HW + (f0 >> 5)] >> (f0 & 31);
            floatx4_t* ptr = reinterpret_cast<floatx4_t*>(dr + swz(4 * f0, col));
            floatx4_t v = *ptr;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] -= ((bits >> i) & 1u) ? ay[m][i] : 0.f;
            *ptr = v;
          }
        }
        po += nout;
        mo += nout * HW;
      }
    }
    __syncthreads();
    // ---- phase B: node GEMMs, outputs held in registers until every wave is done reading
    floatx4_t outv[MAXV][MT];
    {
      bf16x8_t w1[MT][KB], w2[MT][KB];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int row = wave * RW + 16 * m + col;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          w1[m][kb] = *reinterpret_cast<const bf16x8_t*>(a.Wn1 + woff + (size_t)row * Hd + kb * 32 + grp * 8);
          w2[m][kb] = *reinterpret_cast<const bf16x8_t*>(a.Wn2 + woff + (size_t)row * Hd + kb * 32 + grp * 8);
        }
      }
#pragma unroll
      for (int q = 0; q < MAXV; ++q) {
        if (q < vc1) {
          floatx4_t acc[MT];
#pragma unroll
          for (int m = 0; m < MT; ++m) acc[m] = floatx4_t{0.f, 0.f, 0.f, 0.f};
          const int self = a.Vself[vb1 + q];
          if (self >= 0) {
            const unsigned char* Ts = R1 + ((size_t)self * kCols + col) * CB1;
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
              bf16x8_t bfr = *reinterpret_cast<const bf16x8_t*>(Ts + swz(64 * kb + 16 * grp, col));
#pragma unroll
              for (int m = 0; m < MT; ++m) acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[m][kb], bfr, acc[m], 0, 0, 0);
            }
          }
          const unsigned char* Gq = R2 + ((size_t)q * kCols + col) * CB2;
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) {
            const int byte = 4 * (kb * 32 + grp * 8);
            floatx4_t lo = *reinterpret_cast<const floatx4_t*>(Gq + swz(byte, col));
            floatx4_t hi = *reinterpret_cast<const floatx4_t*>(Gq + swz(byte + 16, col));
            uint4 pk;
            pk.x = pack_bf16x2(lo[0], lo[1]);
            pk.y = pack_bf16x2(lo[2], lo[3]);
            pk.z = pack_bf16x2(hi[0], hi[1]);
            pk.w = pack_bf16x2(hi[2], hi[3]);
            bf16x8_t bfr = __builtin_bit_cast(bf16x8_t, pk);
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[m][kb], bfr, acc[m], 0, 0, 0);
          }
#pragma unroll
          for (int m = 0; m < MT; ++m) {
            const int f0 = wave * RW + 16 * m + 4 * grp;
            const uint32_t bits = SN[q * HW + (f0 >> 5)] >> (f0 & 31);
#pragma unroll
            for (int i = 0; i < 4; ++i) outv[q][m][i] = ((bits >> i) & 1u) ? acc[m][i] : 0.f;
          }
        }
      }
    }
    __syncthreads();
    unsigned char* dst = (l < a.L) ? R1 : R2;  // the last round's tangents go where the aggregates were
#pragma unroll
    for (int q = 0; q < MAXV; ++q) {
      if (q < vc1) {
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          const int f0 = wave * RW + 16 * m + 4 * grp;
          uint2 v;
          v.x = pack_bf16x2(outv[q][m][0], outv[q][m][1]);
          v.y = pack_bf16x2(outv[q][m][2], outv[q][m][3]);
          *reinterpret_cast<uint2*>(dst + ((size_t)q * kCols + col) * CB1 + swz(2 * f0, col)) = v;
        }
      }
    }
    __syncthreads();
  }

  // ---- decoder (3 used rows) and the Jacobian blocks
  const int vbL = mt[6 + 2 * a.L];
  for (int t = threadIdx.x; t < oc * 18; t += 256) {
    const int o = t / 18, rem = t % 18, r = rem / 6, d = rem % 6;
    const int q = a.out3[3 * (ob + o)], p = a.out3[3 * (ob + o) + 1];
    const long e = a.out3[3 * (ob + o) + 2];
    const int node = a.V[vbL + q];
    const int cc = a.seedcol[sb + p] + d;
    const unsigned char* tq = R2 + ((size_t)q * kCols + cc) * CB1;
    float dov = 0.f;
    for (int f = 0; f < Hd; ++f)
      dov += a.decT[f * 6 + 3 + r] *
             __uint_as_float((uint32_t)(*reinterpret_cast<const uint16_t*>(tq + swz(2 * f, cc))) << 16);
    const bool diag = node == a.seed[sb + p];
    const float dv = (diag && d == 3 + r ? 1.f : 0.f) + a.dt * dov;
    const float dp = (diag && d == r ? 1.f : 0.f) + a.dt * dv;
    float* blk = a.A + ((size_t)k * a.nnz + e) * 36;
    blk[r * 6 + d] = dp;
    blk[(3 + r) * 6 + d] = dv;
  }
  for (int t = threadIdx.x; t < bc * 9; t += 256) {
    const int o = t / 9, rem = t % 9, r = rem / 3, d = rem % 3;
    const int q = a.bout2[2 * (bb + o)], p = a.bout2[2 * (bb + o) + 1];
    const int node = a.V[vbL + q];
    const int act = a.seedact[sb + p];
    const int cc = a.seedcol[sb + p] + 6 + d;
    const unsigned char* tq = R2 + ((size_t)q * kCols + cc) * CB1;
    float dov = 0.f;
    for (int f = 0; f < Hd; ++f)
      dov += a.decT[f * 6 + 3 + r] *
             __uint_as_float((uint32_t)(*reinterpret_cast<const uint16_t*>(tq + swz(2 * f, cc))) << 16);
    const float dv = a.dt * dov;
    float* Bi = a.B + (((size_t)k * a.M + node) * NBX) * a.nu;
    Bi[(3 + r) * a.nu + 3 * act + d] = dv;
    Bi[r * a.nu + 3 * act + d] = a.dt * dv;
  }
}


// ---------------------------------------------------------------------------
// Seed-centric forward-mode Jacobian with the edge aggregates in registers
// (Hd = 64 or 128).  Workgroup (tile, stage) of Hd/16 waves; wave w owns the 16
// output features [16w, 16w + 16) of every GEMM, so each SIMD runs two waves.
// Round l:
//   A. per node p of round l-1 (tangent dh_p in LDS, bf16): Yb = W_b dh_p and
//      P = W_a dh_p + Yb on the matrix cores; then, in registers, the aggregate
//      of every receiver q of p takes -mask(q <- p) * Yb and p's own aggregate
//      takes cnt_p * P, cnt_p being the number of p's in-edges whose ReLU is on
//      (per feature, from the forward pass).  The aggregates of all nodes of
//      round l (at most 16) stay in registers until every sender is done.
//   B. aggregates go to LDS as bf16 (the GEMM operand precision); per node q of
//      round l: dh_q = mask_q (W_n1 dh_q + W_n2 agg_q).
// Masks, counts and the sender records of every round are gathered from the
// forward pass into an LDS stage, one round ahead.  The decoder's three
// velocity rows are applied to the last round's FP32 tangents in registers and
// reduced across lanes and waves.
struct Mfma2Args {
  int N, M, E, L, nu, meta_stride, cap1, cap2, stage_words;
  float dt;
  const float *encT, *decT;
  const uint16_t *Wa, *Wb, *Wn1, *Wn2;
  const uint32_t *mask_enc, *mask_node, *mask_edge, *cnt;
  const int32_t *meta, *seed, *seedcol, *seedact, *V, *Vself, *out3, *bout2, *colmap;
  const uint32_t* img;  // stage images, [N][img_words]
  long img_words;
  float *A, *B;
  long nnz;
};

// Stage images: word w of (tile, stage k) = its source, read from the forward
// pass's masks and counters of stage k (or a constant).  One thread per word
// and all stages, so each source entry is read once; the source list holds
// (kind | round << 4, index) pairs for every tile.  The workgroups from
// img_blocks on clear the nzero floats at zero instead (B, whose actuated
// entries the Jacobian kernel then writes): an independent fill that shares
// the launch.
template <int Hd>
__global__ void stage_image_kernel(int N, int M, int E, long img_words, const int32_t* __restrict__ src,
                                   const uint32_t* __restrict__ mask_enc, const uint32_t* __restrict__ mask_node,
                                   const uint32_t* __restrict__ mask_edge, const uint32_t* __restrict__ cnt,
                                   uint32_t* __restrict__ img, int img_blocks, float* __restrict__ zero, long nzero) {
  if ((int)blockIdx.x >= img_blocks) {
    const long nb = (long)gridDim.x - img_blocks;
    for (long t = (long)(blockIdx.x - img_blocks) * blockDim.x + threadIdx.x; t < nzero; t += nb * blockDim.x)
      zero[t] = 0.f;
    return;
  }
  constexpr int HW = Hd / 32;
  const long w = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= img_words) return;
  const int2 it = reinterpret_cast<const int2*>(src)[w];
  const int kind = it.x & 15, l = it.x >> 4;
  // stage k's word sits at base + k * step (step 0 for a constant)
  const uint32_t* base = &mask_enc[0];
  size_t step = 0;
  const size_t lo = (size_t)(l > 0 ? l - 1 : 0) * N;
  if (kind == kGEdgeMask) { base = mask_edge + lo * E * HW + it.y; step = (size_t)E * HW; }
  else if (kind == kGNodeMask) { base = mask_node + lo * M * HW + it.y; step = (size_t)M * HW; }
  else if (kind == kGCount) { base = cnt + lo * M * (Hd / 4) + it.y; step = (size_t)M * (Hd / 4); }
  else if (kind == kGEncMask) { base = mask_enc + it.y; step = (size_t)M * HW; }
  const bool cst = kind == kGConst;
  int k = 0;
  for (; k + 4 <= N; k += 4) {
    uint32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = cst ? (uint32_t)it.y : base[(size_t)(k + u) * step];
#pragma unroll
    for (int u = 0; u < 4; ++u) img[(size_t)(k + u) * img_words + w] = v[u];
  }
  for (; k < N; ++k) img[(size_t)k * img_words + w] = cst ? (uint32_t)it.y : base[(size_t)k * step];
}

__device__ inline bf16x8_t ldw(const uint16_t* base, uint32_t off) {
  return *reinterpret_cast<const bf16x8_t*>(base + off);
}

// Weight fragments through buffer resources: one 32-bit lane offset with the
// k-block in the immediate field and the round in the scalar offset.
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__device__ inline __amdgpu_buffer_rsrc_t weight_rsrc(const uint16_t* w, int elems) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(w), (short)0, 2 * elems, 0x00020000);
}
__device__ inline bf16x8_t ldwr(__amdgpu_buffer_rsrc_t r, uint32_t voff_bytes, uint32_t soff_bytes) {
  return __builtin_bit_cast(bf16x8_t, __builtin_amdgcn_raw_buffer_load_b128(r, voff_bytes, soff_bytes, 0));
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also waits for
// every outstanding global load and store of the wave (its release fence covers
// global memory), so each barrier would wait for weight fragments still in flight.
// The kernel below exchanges data between waves through LDS only.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int Hd>
__global__ void __launch_bounds__(Hd * 4) jvp_mfma2_kernel(Mfma2Args a) {
  constexpr int NW = Hd / 16;   // waves
  constexpr int NT = NW * 64;   // threads
  constexpr int KB = Hd / 32;   // 32-deep k-blocks
  constexpr int HW = Hd / 32;   // mask words per node or edge
  constexpr int CB = Hd * 2;    // bytes per bf16 column
  constexpr int MAXV = 16;      // nodes per round
  constexpr int GW = NW / 2;    // waves per node group in phase B
  constexpr int SREC = stage_record_words(Hd);
  extern __shared__ __attribute__((aligned(16))) unsigned char smem2[];
  unsigned char* R1 = smem2;                                         // [cap1][16] bf16 tangent columns
  unsigned char* AG = R1 + (size_t)a.cap1 * kCols * CB;             // [cap2][16] bf16 aggregate columns
  uint32_t* ST = reinterpret_cast<uint32_t*>(AG + (size_t)a.cap2 * kCols * CB);  // stage words
  float* DT = reinterpret_cast<float*>(ST + a.stage_words);                    // decoder rows 3..5, [3][Hd]
  float* ET = DT + 3 * Hd;                                                     // encoder weights [9][Hd]
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = lane & 15, grp = lane >> 4;
  // phase A: wave w owns output features [16 w, 16 w + 16) of every node.  The
  // tangents are the A operand, so lane (n, g) holds feature fA = 16 w + n of
  // tangent columns 4 g .. 4 g + 3 and each edge mask is one bit per lane.
  const int fA = wave * 16 + col;
  const int mw = fA >> 5, mpos = fA & 31;
  // byte offset of feature fA in aggregate column 4 g + i: agb + i CB + ((agc ^ i) << 4)
  const int agb = 4 * grp * CB + (2 * fA & 15);
  const int agc = (2 * fA) >> 4 ^ ((4 * grp) & (CB >= 256 ? 15 : 7));
  // phase B: node group ng takes nodes q = 2 j + ng; its wave wg owns features [32 wg, 32 wg + 32)
  const int ng = wave / GW, wg = wave % GW;
  const int tile = blockIdx.x, k = blockIdx.y;
  const int32_t* mt = a.meta + (size_t)tile * a.meta_stride;
  const int oc = mt[3], bc = mt[5];

  // lane offsets of the weight fragments (rows of the A operands): phase A, then phase B's two row tiles
  const uint32_t woA = (uint32_t)((wave * 16 + col) * Hd + grp * 8);
  const uint32_t woB = (uint32_t)((wg * 32 + col) * Hd + grp * 8);
  const int wel = a.L * Hd * Hd;
  const __amdgpu_buffer_rsrc_t rWa = weight_rsrc(a.Wa, wel), rWb = weight_rsrc(a.Wb, wel);
  const __amdgpu_buffer_rsrc_t rW1 = weight_rsrc(a.Wn1, wel), rW2 = weight_rsrc(a.Wn2, wel);
  bf16x8_t wa[KB], wb[KB], w1[2][KB], w2[2][KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    wa[kb] = ldwr(rWa, 2 * woA + 64 * kb, 0);
    wb[kb] = ldwr(rWb, 2 * woA + 64 * kb, 0);
  }
  // start-up: the stage image (one contiguous read), decoder rows and encoder weights to LDS
  {
    const int ib = mt[6 + 2 * (a.L + 1) + 4 * a.L], nw = mt[6 + 2 * (a.L + 1) + 4 * a.L + 1];
    const uint4* im = reinterpret_cast<const uint4*>(a.img + (size_t)k * a.img_words + ib);
    for (int t = threadIdx.x; t < nw / 4; t += NT) reinterpret_cast<uint4*>(ST)[t] = im[t];
  }
  for (int t = threadIdx.x; t < 3 * Hd; t += NT) DT[t] = a.decT[(t % Hd) * 6 + 3 + t / Hd];
  for (int t = threadIdx.x; t < 9 * Hd / 4; t += NT) reinterpret_cast<float4*>(ET)[t] = reinterpret_cast<const float4*>(a.encT)[t];
  lds_barrier();
  // round 0: encoder tangents of the seeds (mask x weight, exact in bf16), 8 features per item
  {
    const int vc = mt[7];
    const uint32_t* CM = ST + mt[a.meta_stride - 1];  // (seed << 4) | dimension of each column, or -1
    const uint32_t* EM = CM + kCols;                  // encoder masks of round 0's nodes
    for (int t = threadIdx.x; t < vc * kCols * (Hd / 8); t += NT) {
      const int q = t / (kCols * (Hd / 8)), c = (t / (Hd / 8)) % kCols, fc = t % (Hd / 8);
      const int cm = (int)CM[c];
      const bool valid = cm >= 0 && (cm >> 4) == q;
      const int d = cm & 15;
      const uint32_t bits = (EM[q * HW + (fc >> 2)] >> (8 * (fc & 3))) & 0xFFu;
      const float4* e4 = reinterpret_cast<const float4*>(ET + (valid ? d : 0) * Hd + 8 * fc);
      const float4 lo = e4[0], hi = e4[1];
      const float ev[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
      uint32_t pk[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const uint32_t b0 = (valid && ((bits >> (2 * h)) & 1u)) ? (__float_as_uint(ev[2 * h]) >> 16) : 0u;
        const uint32_t b1 = (valid && ((bits >> (2 * h + 1)) & 1u)) ? (__float_as_uint(ev[2 * h + 1]) & 0xFFFF0000u) : 0u;
        pk[h] = b0 | b1;
      }
      *reinterpret_cast<uint4*>(R1 + ((size_t)q * kCols + c) * CB + swzc<CB>(16 * fc, c)) = make_uint4(pk[0], pk[1], pk[2], pk[3]);
    }
  }
  lds_barrier();

  floatx4_t acc[MAXV];
  int so = 0;          // stage offset of the current round
  for (int l = 1; l <= a.L; ++l) {
    const int vc0 = mt[7 + 2 * (l - 1)];
    const int vb1 = mt[6 + 2 * l], vc1 = mt[7 + 2 * l];
    const int nbase = so + vc0 * SREC;
    const size_t woff = (size_t)(l - 1) * Hd * Hd;
    // ---- phase A: edge GEMMs per sender, aggregates of every receiver in registers.
    // Round l-1's nodes lead round l in the same order, so sender p is node p of round l.
#pragma unroll
    for (int q = 0; q < MAXV; ++q) acc[q] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    // The node weights of this round are read two fragments per sender slot, and the
    // next round's edge weights one pair per node slot of phase B: every workgroup
    // reads the same weights from L2, and spreading the requests over the round keeps
    // them from queueing behind each other (issued at once, they stalled the round's
    // first sender by several thousand cycles).
#pragma unroll
    for (int p = 0; p < MAXV; ++p) {
      if (p < 2 * KB) {
        const int m = p / KB, kb = p % KB;
        w1[m][kb] = ldwr(rW1, 2 * woB + 32 * m * Hd + 64 * kb, (uint32_t)(2 * woff));
        w2[m][kb] = ldwr(rW2, 2 * woB + 32 * m * Hd + 64 * kb, (uint32_t)(2 * woff));
      }
      if (p < vc0) {
        const uint32_t* rec = ST + so + p * SREC;
        const uint4* rec4 = reinterpret_cast<const uint4*>(rec);
        const unsigned char* Tp = R1 + ((size_t)p * kCols + col) * CB;
        bf16x8_t bfr[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) bfr[kb] = *reinterpret_cast<const bf16x8_t*>(Tp + swzc<CB>(64 * kb + 16 * grp, col));
        const uint4 t0 = rec4[1 + 4 * mw], t1 = rec4[2 + 4 * mw], t2 = rec4[3 + 4 * mw], t3 = rec4[4 + 4 * mw];
        const float cf = (float)reinterpret_cast<const unsigned char*>(rec + 4 + 16 * HW)[fA];
        const uint32_t rcv = (uint32_t)__builtin_amdgcn_readfirstlane((int)rec[1]);
        // Yb = W_b dh_p, then P = W_a dh_p + Yb accumulated on top of it
        floatx4_t ay = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) ay = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[kb], wb[kb], ay, 0, 0, 0);
        floatx4_t aa = ay;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) aa = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[kb], wa[kb], aa, 0, 0, 0);
        const uint32_t tbl[16] = {t0.x, t0.y, t0.z, t0.w, t1.x, t1.y, t1.z, t1.w,
                                  t2.x, t2.y, t2.z, t2.w, t3.x, t3.y, t3.z, t3.w};
        // receivers tested four at a time: a sender's receivers sit in few groups
#pragma unroll
        for (int q4 = 0; q4 < MAXV; q4 += 4) {
          if ((rcv >> q4) & 15u) {
            // every receiver of the group without a test: a non-receiver's mask word is zero
#pragma unroll
            for (int q = q4; q < q4 + 4; ++q) {
              // 1.0f where the edge's ReLU is on for this lane's feature, else 0
              const float mf = __uint_as_float((uint32_t)__builtin_amdgcn_sbfe((int)tbl[q], mpos, 1) & 0x3F800000u);
#pragma unroll
              for (int i = 0; i < 4; ++i) acc[q][i] = __builtin_fmaf(-mf, ay[i], acc[q][i]);
            }
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[p][i] = __builtin_fmaf(cf, aa[i], acc[p][i]);
      }
    }
    {
      // bf16 aggregates: this lane's feature in four columns
#pragma unroll
      for (int q = 0; q < MAXV; ++q) {
        if (q < vc1) {
          unsigned char* Gq = AG + (size_t)q * kCols * CB;
          const uint32_t lo = pack_bf16x2(acc[q][0], acc[q][1]), hi = pack_bf16x2(acc[q][2], acc[q][3]);
          unsigned char* Gl = Gq + agb + (agc << 4);
          *reinterpret_cast<uint16_t*>(Gl) = (uint16_t)lo;
          *reinterpret_cast<uint16_t*>(Gl + CB + (((agc ^ 1) - agc) << 4)) = (uint16_t)(lo >> 16);
          *reinterpret_cast<uint16_t*>(Gl + 2 * CB + (((agc ^ 2) - agc) << 4)) = (uint16_t)hi;
          *reinterpret_cast<uint16_t*>(Gl + 3 * CB + (((agc ^ 3) - agc) << 4)) = (uint16_t)(hi >> 16);
        }
      }
    }
    lds_barrier();
    const size_t wn = (size_t)l * Hd * Hd;  // next round's weights

    // ---- phase B: node GEMMs, two node groups; results stay in registers until every wave is done reading
    const unsigned char* AGg = AG + ((size_t)ng * kCols + col) * CB;  // node 2 j + ng at + 2 j * kCols * CB
#pragma unroll
    for (int j = 0; j < MAXV / 2; ++j) {
      if (j < KB && l < a.L) {
        wa[j] = ldwr(rWa, 2 * woA + 64 * j, (uint32_t)(2 * wn));
        wb[j] = ldwr(rWb, 2 * woA + 64 * j, (uint32_t)(2 * wn));
      }
      const int q = 2 * j + ng;
      if (q < vc1) {
        floatx4_t c[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) c[m] = floatx4_t{0.f, 0.f, 0.f, 0.f};
        const unsigned char* Gq = AGg + (size_t)(2 * j) * kCols * CB;
        if (q < vc0) {  // node q of round l-1 is node q of round l
          const unsigned char* Ts = R1 + ((size_t)q * kCols + col) * CB;
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) {
            const bf16x8_t bs = *reinterpret_cast<const bf16x8_t*>(Ts + swzc<CB>(64 * kb + 16 * grp, col));
#pragma unroll
            for (int m = 0; m < 2; ++m) c[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[m][kb], bs, c[m], 0, 0, 0);
          }
        }
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const bf16x8_t bg = *reinterpret_cast<const bf16x8_t*>(Gq + swzc<CB>(64 * kb + 16 * grp, col));
#pragma unroll
          for (int m = 0; m < 2; ++m) c[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[m][kb], bg, c[m], 0, 0, 0);
        }
        const int bits = (int)ST[nbase + q * HW + wg];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            acc[2 * j + m][i] = __uint_as_float(__float_as_uint(c[m][i]) &
                                                (uint32_t)__builtin_amdgcn_sbfe(bits, 16 * m + 4 * grp + i, 1));
      }
    }
    lds_barrier();
    if (l < a.L) {
      unsigned char* R1g = R1 + ((size_t)ng * kCols + col) * CB;
      const int sw0 = swzc<CB>(2 * (wg * 32 + 4 * grp), col), sw1 = swzc<CB>(2 * (wg * 32 + 16 + 4 * grp), col);
#pragma unroll
      for (int j = 0; j < MAXV / 2; ++j) {
        const int q = 2 * j + ng;
        if (q < vc1) {
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            uint2 v;
            v.x = pack_bf16x2(acc[2 * j + m][0], acc[2 * j + m][1]);
            v.y = pack_bf16x2(acc[2 * j + m][2], acc[2 * j + m][3]);
            *reinterpret_cast<uint2*>(R1g + (size_t)(2 * j) * kCols * CB + (m ? sw1 : sw0)) = v;
          }
        }
      }
      lds_barrier();
    }
    so = nbase + (vc1 * HW + 3) / 4 * 4;
  }

  // ---- decoder: velocity rows 3..5 of W_dec on the last round's FP32 tangents
  // per-lane partial sums over this lane's 8 features, [q][GW * 4 lanes groups][16 columns][4]
  float4* red = reinterpret_cast<float4*>(AG);
  {
    const int vcL = mt[7 + 2 * a.L];
    float dct[3][2][4];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const float4 d4 = *reinterpret_cast<const float4*>(DT + r * Hd + wg * 32 + 16 * m + 4 * grp);
        dct[r][m][0] = d4.x;
        dct[r][m][1] = d4.y;
        dct[r][m][2] = d4.z;
        dct[r][m][3] = d4.w;
      }
    float4* rw = red + ((size_t)ng * GW * 4 + wg * 4 + grp) * kCols + col;
#pragma unroll
    for (int j = 0; j < MAXV / 2; ++j) {
      if (2 * j + ng < vcL) {
        float v[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          v[r] = 0.f;
#pragma unroll
          for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) v[r] += dct[r][m][i] * acc[2 * j + m][i];
        }
        rw[(size_t)(2 * j) * GW * 4 * kCols] = make_float4(v[0], v[1], v[2], 0.f);
      }
    }
  }
  lds_barrier();
  const int4* orec = reinterpret_cast<const int4*>(ST) + (so >> 2);
  for (int t = threadIdx.x; t < oc * 18; t += NT) {
    const int o = t / 18, rem = t % 18, r = rem / 6, dd = rem % 6;
    const int4 rc = orec[o];  // {block, q, first column, first dim | count << 8 | diagonal << 16}
    if (dd >= ((rc.w >> 8) & 0xFF)) continue;
    const int d = (rc.w & 0xFF) + dd, cc = rc.z + dd;
    float dov = 0.f;
    const float* rq = reinterpret_cast<const float*>(red + (size_t)rc.y * GW * 4 * kCols + cc) + r;
#pragma unroll
    for (int w = 0; w < GW * 4; ++w) dov += rq[w * kCols * 4];
    const bool diag = (rc.w >> 16) != 0;
    const float dv = (diag && d == 3 + r ? 1.f : 0.f) + a.dt * dov;
    const float dp = (diag && d == r ? 1.f : 0.f) + a.dt * dv;
    float* blk = a.A + ((size_t)k * a.nnz + rc.x) * 36;
    blk[r * 6 + d] = dp;
    blk[(3 + r) * 6 + d] = dv;
  }
  for (int t = threadIdx.x; t < bc * 9; t += NT) {
    const int o = t / 9, rem = t % 9, r = rem / 3, dd = rem % 3;
    const int4 rc = orec[oc + o];  // {node, q, first column, 3 actuator + first force dim | count << 8}
    if (dd >= (rc.w >> 8)) continue;
    const int cc = rc.z + dd, bcol = (rc.w & 0xFF) + dd;
    float dov = 0.f;
    const float* rq = reinterpret_cast<const float*>(red + (size_t)rc.y * GW * 4 * kCols + cc) + r;
#pragma unroll
    for (int w = 0; w < GW * 4; ++w) dov += rq[w * kCols * 4];
    const float dv = a.dt * dov;
    float* Bi = a.B + (((size_t)k * a.M + rc.x) * NBX) * a.nu;
    Bi[(3 + r) * a.nu + bcol] = dv;
    Bi[r * a.nu + bcol] = a.dt * dv;
  }
}


// ---------------------------------------------------------------------------
// Forward pass on the matrix cores: bf16 weights, FP32 activations.  An FP32
// operand v enters an MFMA as three bf16 terms, hi = bf16(v), mid =
// bf16(v - hi), lo = bf16(v - hi - mid) (each residual is exact in FP32), so
// hi + mid + lo equals v to about 2^-24 relative; the bf16 x bf16 products
// are exact and the sums FP32, which keeps every ReLU decision at FP32
// accuracy.  One workgroup per (column tile, stage): a tile is 16 or 32 node
// columns -- the target nodes whose next hidden state it produces plus the
// senders of their edges -- so each round is two GEMMs per tile: [W_a; W_b] h
// (edge terms) and [W_n1 W_n2] [h; agg] (node update).  ReLU masks leave as
// 4-bit groups staged in LDS bytes and packed into the same bit layout as the
// VALU path.

// Three-term bf16 split of an FP32 pair, each term packed (a | b << 16).
__device__ inline void split3_bf16x2(float a, float b, uint32_t& p0, uint32_t& p1, uint32_t& p2) {
  p0 = pack_bf16x2(a, b);
  const float ra = a - __uint_as_float(p0 << 16), rb = b - __uint_as_float(p0 & 0xFFFF0000u);
  p1 = pack_bf16x2(ra, rb);
  p2 = pack_bf16x2(ra - __uint_as_float(p1 << 16), rb - __uint_as_float(p1 & 0xFFFF0000u));
}

// Decoder velocity rows on the last hidden state: 16 lanes per (stage, node),
// each taking 8 consecutive features, reduced across the 16 lanes.
__global__ void fwd_dec_coop_kernel(FwdArgs a, const float* hL) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long s = t >> 4;
  const int sub = (int)(t & 15);
  const bool live = s < (long)a.N * a.M;
  float o[3] = {0.f, 0.f, 0.f};
  if (live) {
    for (int f0 = 8 * sub; f0 < a.Hd; f0 += 128) {
      const float4* hp = reinterpret_cast<const float4*>(hL + (size_t)s * a.Hd + f0);
      const float4 h0 = hp[0], h1 = hp[1];
      const float h[8] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w};
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int r = 0; r < 3; ++r) o[r] += a.decT[(f0 + q) * 6 + 3 + r] * h[q];
    }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    o[r] += __shfl_xor(o[r], 8, 16);
    o[r] += __shfl_xor(o[r], 4, 16);
    o[r] += __shfl_xor(o[r], 2, 16);
    o[r] += __shfl_xor(o[r], 1, 16);
  }
  if (!live || sub != 0) return;
  const float* x = a.xhat + (size_t)s * NBX;
  float* fo = a.fnext + (size_t)s * NBX;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float vn = x[3 + r] + a.dt * (o[r] + a.bdec[3 + r]);
    fo[3 + r] = vn;
    fo[r] = x[r] + a.dt * vn;
  }
}

struct FwdMfmaArgs {
  int N, M, E, l, fedge_cap;
  const float* hin;                     // this round's input activations [N][M][Hd]
  float* hout;                          // its output activations
  const uint16_t *Wa, *Wb, *Wn1, *Wn2;  // this round's weights, bf16 row-major (out, in)
  const float *be, *bn;                 // this round's biases
  uint32_t *mask_edge, *mask_node;      // this round, all stages
  uint8_t* cnt;                         // this round, all stages: active in-edges per (node, feature)
  const int32_t *fcols, *fmeta, *fecnt, *fepre, *fesrc, *feid;
};

// Column tiles of the forward pass hold kFwdCT * 16 node columns (Hd <= 128;
// Hd = 256 uses one 16-column group): the weight fragments a wave loads feed
// kFwdCT MFMA column groups.
constexpr int kFwdCT = 2;
__host__ __device__ constexpr int fwd_groups(int Hd) { return Hd <= 128 ? kFwdCT : 1; }
// Dynamic LDS of fwd_mfma_layer_kernel: three bf16 planes of the layer input, one
// region that holds the FP32 W_b h of every column (16-byte chunks XOR-swizzled by
// column, so the 16 columns of a wave read 16 distinct bank groups) until the edge
// terms have read it and the three bf16 planes of the aggregates after that, the
// staged mask groups, then the tile's lists (sender column of each edge; first
// edge, edge count and node of each column).  At Hd = 128 with 32-column tiles this
// is about 52 KB, so three workgroups fit one CU's 160 KB.
__host__ __device__ constexpr size_t fwd_planes_bytes(int Hd) { return (size_t)16 * fwd_groups(Hd) * Hd * 2; }
// W_b h (FP32, until the edge terms have read it) and then the three aggregate planes
// share one region
__host__ __device__ constexpr size_t fwd_union_bytes(int Hd) {
  return (size_t)16 * fwd_groups(Hd) * Hd * 4 > 3 * fwd_planes_bytes(Hd) ? (size_t)16 * fwd_groups(Hd) * Hd * 4
                                                                          : 3 * fwd_planes_bytes(Hd);
}
// Staged mask groups: a lane's 4-bit groups of features 16 m + .. and 16 (m + 1) + ..
// share one byte (Hd >= 128), so a staged row is Hd / 8 bytes (Hd / 4 for Hd = 64).
__host__ __device__ constexpr int fwd_qrow_bytes(int Hd) { return Hd >= 128 ? Hd / 8 : Hd / 4; }
__host__ __device__ constexpr size_t fwd_mask_bytes(int Hd, int fedge_cap) {
  return ((size_t)(fedge_cap + 16 * fwd_groups(Hd)) * fwd_qrow_bytes(Hd) + 15) / 16 * 16;
}
size_t fwd_lds_bytes(int Hd, int fedge_cap) {
  const int NC = 16 * fwd_groups(Hd);
  return 3 * fwd_planes_bytes(Hd) + fwd_union_bytes(Hd) + fwd_mask_bytes(Hd, fedge_cap) +
         (size_t)(fedge_cap + 3 * NC) * 4;
}
// byte and bit offset of 4-bit group g4 in a staged row
__device__ inline int fwd_qbyte(int Hd, int g4) { return Hd >= 128 ? ((g4 >> 3) << 2) | (g4 & 3) : g4; }
__device__ inline int fwd_qshift(int Hd, int g4) { return Hd >= 128 ? 4 * ((g4 >> 2) & 1) : 0; }

// Stage this lane's 4-bit groups of one mask row: group m covers features f_lane + 16 m ..
// + 3 (f_lane = the lane's first feature); for Hd >= 128 groups m and m + 1 share a byte.
template <int Hd, int MT>
__device__ inline void fwd_stage_groups(unsigned char* row, const uint32_t (&nibs)[MT], int f_lane) {
  if constexpr (Hd >= 128) {
#pragma unroll
    for (int m = 0; m < MT; m += 2)
      row[fwd_qbyte(Hd, (f_lane + 16 * m) / 4)] = (unsigned char)(nibs[m] | (nibs[m + 1] << 4));
  } else {
#pragma unroll
    for (int m = 0; m < MT; ++m) row[fwd_qbyte(Hd, (f_lane + 16 * m) / 4)] = (unsigned char)nibs[m];
  }
}

// At most 168 registers per lane (three waves per SIMD), which with the LDS above
// lets three workgroups share a CU: the 720 workgroups of a 1000-node, 20-stage
// layer then run in one round instead of two.
template <int MT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) fwd_mfma_layer_kernel(FwdMfmaArgs a) {
  constexpr int Hd = MT * 64, KB = Hd / 32, RW = Hd / 4, CB = Hd * 2, HW = Hd / 32, NQ = Hd / 4;
  constexpr int CT = fwd_groups(Hd), NC = 16 * CT;
  constexpr int PL = NC * CB;  // bytes of one bf16 plane
  extern __shared__ __attribute__((aligned(16))) unsigned char fsm[];
  constexpr int QB = fwd_qrow_bytes(Hd);
  unsigned char* Hs = fsm;                                 // [3][NC][CB] layer input: hi, mid, lo
  float* Ybs = reinterpret_cast<float*>(Hs + 3 * PL);      // [NC][Hd] W_b h per column, until the edge terms
  unsigned char* Ag = Hs + 3 * PL;                         // [3][NC][CB] aggregates: hi, mid, lo (after them)
  unsigned char* qmask = Hs + 3 * PL + fwd_union_bytes(Hd);  // [edges + NC][QB] 4-bit groups
  int32_t* esrc = reinterpret_cast<int32_t*>(qmask + fwd_mask_bytes(Hd, a.fedge_cap));  // [edges]
  int32_t* epre = esrc + a.fedge_cap;                                                 // [NC]
  int32_t* ecnt = epre + NC;                                                          // [NC]
  int32_t* cnode = ecnt + NC;                                                         // [NC]
  auto ysw = [](int c, int f0) { return c * Hd + ((((f0 >> 2) ^ c) & (NQ - 1)) << 2); };
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = lane & 15, grp = lane >> 4;
  const int tile = blockIdx.x, k = blockIdx.y;
  const int32_t* fm = a.fmeta + (size_t)tile * 4;
  const int nt = fm[0], eb = fm[1], ec = fm[2];
  const int32_t* cols = a.fcols + (size_t)tile * NC;
  // Weight fragments (lane: row 16 m + col of the wave's rows, 8 inputs from
  // 32 kb + 8 grp).  For Hd <= 128 the edge GEMMs' fragments of every k-block are
  // requested first, so they arrive while the columns are gathered, and the node
  // update's before the edge terms; Hd = 256 has no registers for that and loads
  // them per k-block.
  constexpr bool HOIST = MT <= 2;
  constexpr int KH = HOIST ? KB : 1;
  auto load_w = [&](bf16x8_t (&dst)[MT], const uint16_t* W, int kb) {
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int row = wave * RW + 16 * m + col;
      dst[m] = *reinterpret_cast<const bf16x8_t*>(W + (size_t)row * Hd + kb * 32 + grp * 8);
    }
  };
  bf16x8_t wa[KH][MT], wb[KH][MT];
  if constexpr (HOIST) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      load_w(wa[kb], a.Wa, kb);
      load_w(wb[kb], a.Wb, kb);
    }
  }
  for (int t = threadIdx.x; t < ec; t += 256) esrc[t] = a.fesrc[eb + t];
  for (int t = threadIdx.x; t < NC; t += 256) {
    epre[t] = a.fepre[(size_t)tile * NC + t];
    ecnt[t] = t < nt ? a.fecnt[(size_t)tile * NC + t] : 0;
    cnode[t] = cols[t];
  }
  // ---- gather the input columns, 8 features (one 16-byte chunk per plane) per item
  for (int t = threadIdx.x; t < NC * (Hd / 8); t += 256) {
    const int c = t / (Hd / 8), ch = t % (Hd / 8);
    const int node = cols[c];
    float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0;
    if (node >= 0) {
      const float4* src = reinterpret_cast<const float4*>(a.hin + ((size_t)k * a.M + node) * Hd + 8 * ch);
      v0 = src[0];
      v1 = src[1];
    }
    uint4 p0, p1, p2;
    split3_bf16x2(v0.x, v0.y, p0.x, p1.x, p2.x);
    split3_bf16x2(v0.z, v0.w, p0.y, p1.y, p2.y);
    split3_bf16x2(v1.x, v1.y, p0.z, p1.z, p2.z);
    split3_bf16x2(v1.z, v1.w, p0.w, p1.w, p2.w);
    const int off = c * CB + swz(16 * ch, c);
    *reinterpret_cast<uint4*>(Hs + off) = p0;
    *reinterpret_cast<uint4*>(Hs + PL + off) = p1;
    *reinterpret_cast<uint4*>(Hs + 2 * PL + off) = p2;
  }
  __syncthreads();
  // ---- edge GEMMs: Yb = W_b h, P = W_a h + Yb (smallest term first)
  floatx4_t ap[CT][MT], ay[CT][MT];
  {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        ap[ct][m] = floatx4_t{0.f, 0.f, 0.f, 0.f};
        ay[ct][m] = floatx4_t{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int ki = HOIST ? kb : 0;
      if constexpr (!HOIST) {
        load_w(wa[0], a.Wa, kb);
        load_w(wb[0], a.Wb, kb);
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int c = 16 * ct + col;
        const int off = c * CB + swz(64 * kb + 16 * grp, c);
        bf16x8_t bfr[3];
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) bfr[pl] = *reinterpret_cast<const bf16x8_t*>(Hs + pl * PL + off);
#pragma unroll
        for (int pl = 2; pl >= 0; --pl)
#pragma unroll
          for (int m = 0; m < MT; ++m) {
            ay[ct][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[ki][m], bfr[pl], ay[ct][m], 0, 0, 0);
            ap[ct][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[ki][m], bfr[pl], ap[ct][m], 0, 0, 0);
          }
      }
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int f0 = wave * RW + 16 * m + 4 * grp;
        *reinterpret_cast<floatx4_t*>(Ybs + ysw(16 * ct + col, f0)) = ay[ct][m];
#pragma unroll
        for (int i = 0; i < 4; ++i) ap[ct][m][i] += ay[ct][m][i] + a.be[f0 + i];
      }
  }
  bf16x8_t w1[KH][MT], w2[KH][MT];
  if constexpr (HOIST) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      load_w(w1[kb], a.Wn1, kb);
      load_w(w2[kb], a.Wn2, kb);
    }
  }
  __syncthreads();
  // ---- edge terms of the target columns: agg = sum_j relu(P_i - Yb_j); the sums stay in
  // registers until every wave has read W_b h, whose region the aggregate planes take
  float aggv[CT][MT][4];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int c = 16 * ct + col;
    const int e0 = epre[c];
    const int ne = ecnt[c];
    float (&agg)[MT][4] = aggv[ct];
    uint32_t ncnt[MT];  // 4 byte counters: in-edges whose ReLU is on, per feature
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      ncnt[m] = 0u;
#pragma unroll
      for (int i = 0; i < 4; ++i) agg[m][i] = 0.f;
    }
    for (int t = 0; t < ne; ++t) {
      const int sc = esrc[e0 + t];
      uint32_t nibs[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int f0 = wave * RW + 16 * m + 4 * grp;
        const floatx4_t yb = *reinterpret_cast<const floatx4_t*>(Ybs + ysw(sc, f0));
        uint32_t nib = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float z = ap[ct][m][i] - yb[i];
          const bool on = z > 0.f;
          agg[m][i] += on ? z : 0.f;
          nib |= (on ? 1u : 0u) << i;
          ncnt[m] += (on ? 1u : 0u) << (8 * i);
        }
        nibs[m] = nib;
      }
      fwd_stage_groups<Hd, MT>(qmask + (size_t)(e0 + t) * QB, nibs, wave * RW + 4 * grp);
    }
    if (c < nt) {
      const int node = cnode[c];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int f0 = wave * RW + 16 * m + 4 * grp;
        *reinterpret_cast<uint32_t*>(a.cnt + ((size_t)k * a.M + node) * Hd + f0) = ncnt[m];
      }
    }
  }
  __syncthreads();  // W_b h is dead
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int c = 16 * ct + col;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int f0 = wave * RW + 16 * m + 4 * grp;
      uint32_t h0, h1, h2, g0, g1, g2;
      split3_bf16x2(aggv[ct][m][0], aggv[ct][m][1], h0, h1, h2);
      split3_bf16x2(aggv[ct][m][2], aggv[ct][m][3], g0, g1, g2);
      const int off = c * CB + swz(2 * f0, c);
      *reinterpret_cast<uint2*>(Ag + off) = make_uint2(h0, g0);
      *reinterpret_cast<uint2*>(Ag + PL + off) = make_uint2(h1, g1);
      *reinterpret_cast<uint2*>(Ag + 2 * PL + off) = make_uint2(h2, g2);
    }
  }
  __syncthreads();
  // ---- node update: h' = relu(W_n1 h + W_n2 agg + b_n)
  {
    floatx4_t acc[CT][MT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[ct][m] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int ki = HOIST ? kb : 0;
      if constexpr (!HOIST) {
        load_w(w1[0], a.Wn1, kb);
        load_w(w2[0], a.Wn2, kb);
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int c = 16 * ct + col;
        const int off = c * CB + swz(64 * kb + 16 * grp, c);
        bf16x8_t bh[3], bg[3];
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) {
          bh[pl] = *reinterpret_cast<const bf16x8_t*>(Hs + pl * PL + off);
          bg[pl] = *reinterpret_cast<const bf16x8_t*>(Ag + pl * PL + off);
        }
#pragma unroll
        for (int pl = 2; pl >= 0; --pl)
#pragma unroll
          for (int m = 0; m < MT; ++m) {
            acc[ct][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[ki][m], bh[pl], acc[ct][m], 0, 0, 0);
            acc[ct][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[ki][m], bg[pl], acc[ct][m], 0, 0, 0);
          }
      }
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int c = 16 * ct + col;
      if (c < nt) {
        const int node = cnode[c];
        uint32_t nibs[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          const int f0 = wave * RW + 16 * m + 4 * grp;
          float hv[4];
          uint32_t nib = 0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float z = acc[ct][m][i] + a.bn[f0 + i];
            const bool on = z > 0.f;
            hv[i] = on ? z : 0.f;
            nib |= (on ? 1u : 0u) << i;
          }
          *reinterpret_cast<float4*>(a.hout + ((size_t)k * a.M + node) * Hd + f0) = make_float4(hv[0], hv[1], hv[2], hv[3]);
          nibs[m] = nib;
        }
        fwd_stage_groups<Hd, MT>(qmask + (size_t)(a.fedge_cap + c) * QB, nibs, wave * RW + 4 * grp);
      }
    }
  }
  __syncthreads();
  // ---- pack the staged 4-bit groups into mask words
  for (int t = threadIdx.x; t < (ec + nt) * HW; t += 256) {
    const int r = t / HW, wd = t % HW;
    const int srow = r < ec ? r : a.fedge_cap + (r - ec);
    uint32_t word = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int g4 = wd * 8 + q;
      word |= ((uint32_t)(qmask[(size_t)srow * QB + fwd_qbyte(Hd, g4)] >> fwd_qshift(Hd, g4)) & 0xFu) << (4 * q);
    }
    if (r < ec) a.mask_edge[((size_t)k * a.E + a.feid[eb + r]) * HW + wd] = word;
    else a.mask_node[((size_t)k * a.M + cnode[r - ec]) * HW + wd] = word;
  }
}

__global__ void fill_zero_kernel(float* p, long n) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) p[t] = 0.f;
}

// c = f - sum_j A^{ij} xhat^j - B^i uhat (and f copied out); one lane per
// (stage, node, row), pattern blocks taken 4 at a time so their loads overlap.
__global__ void gnn_offset_kernel(int N, int M, int nu, long nnz, const int32_t* prow, const int32_t* pcol,
                                  const float* xhat, const float* uhat, const float* A, const float* B,
                                  const float* fwd, float* c, float* fnext) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)N * M * NBX) return;
  const int r = (int)(t % NBX);
  const long s = t / NBX;
  const int k = (int)(s / M), i = (int)(s - (long)k * M);
  const float* xk = xhat + (size_t)k * M * NBX;
  float lin = 0.f;
  const int e0 = prow[i], e1 = prow[i + 1];
  // row r of a block and a node's state are 6 floats at 8-byte aligned addresses: float2 loads
  for (int e = e0; e < e1; e += 4) {
    float2 av[4][3], xv[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int eu = e + u < e1 ? e + u : e;
      const float2* blk = reinterpret_cast<const float2*>(A + ((size_t)k * nnz + eu) * 36 + r * 6);
      const float2* xj = reinterpret_cast<const float2*>(xk + (size_t)pcol[eu] * NBX);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        av[u][d] = e + u < e1 ? blk[d] : make_float2(0.f, 0.f);
        xv[u][d] = xj[d];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lin += av[u][d].x * xv[u][d].x;
        lin += av[u][d].y * xv[u][d].y;
      }
  }
  const float* Bi = B + ((size_t)s * NBX + r) * nu;
  const float* u = uhat + (size_t)k * nu;
  for (int d = 0; d < nu; ++d) lin += Bi[d] * u[d];
  const float fv = fwd[(size_t)s * NBX + r];
  c[(size_t)s * NBX + r] = fv - lin;
  if (fnext) fnext[(size_t)s * NBX + r] = fv;
}

template <typename T>
gnmpc_status dalloc(gnmpc_plan* p, T*& ptr, size_t count) {
  GNMPC_HIP_TRY(p, hipMalloc((void**)&ptr, sizeof(T) * std::max<size_t>(count, 1)));
  p->gnn->allocs.push_back((void*)ptr);
  return GNMPC_OK;
}

template <typename T>
gnmpc_status dupload(gnmpc_plan* p, T*& ptr, const std::vector<T>& v) {
  gnmpc_status s = dalloc(p, ptr, v.size());
  if (s != GNMPC_OK) return s;
  if (!v.empty()) GNMPC_HIP_TRY(p, hipMemcpy(ptr, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return GNMPC_OK;
}

// Seed tiles and their per-round node lists (host).
struct TilePlan {
  std::vector<int32_t> meta, seed, seedcol, seedact, V, Vself, Vebeg, Vecnt, Eloc, Eid, out3, bout2;
  // per entry of V (round l < L): its index in round l+1 and its out-edges (r <- node) with r's
  // index in round l+1 and the CSR id of the edge in r's row
  // per (tile, round l >= 1): the sender program {qp, n_in, n_out, qr...} of every node of
  // round l-1 and the CSR ids of the edges whose masks it reads (in-edges, then out-edges)
  std::vector<int32_t> prog, elist;
  // per tile and tangent column: (seed index in the tile << 4) | state or force dimension, or -1
  std::vector<int32_t> colmap;
  // stage image sources of the register-aggregate kernel: every word of every
  // tile's stage as a (kind | round << 4, index) pair, tiles at multiples of 4 words
  std::vector<int32_t> img;
  int bufX = 0, bufY = 0, n_tiles = 0, cap1 = 0, cap2 = 0, stage_cap = 0, stage2_cap = 0, vmax = 0;
};


// Seed tiles.  Classic tiles hold whole seeds (one or two, at most 16
// columns).  Packed tiles take the seeds' columns as one stream in node order
// (6 state dimensions, then 3 force dimensions for an actuated node) and cut
// it every 16 columns, so a seed may continue in the next tile; a packed tile
// is shortened to whole seeds only when a round would reach more than 16 nodes.
struct SeedCols {
  int32_t node, c0, d0, cnt;  // first column in the tile, first dimension, number of columns
};

void build_tiles(const gnmpc_plan* p, int L, int max_seeds, TilePlan& tp, bool packed = false) {
  const int M = p->M;
  std::vector<std::vector<int32_t>> outn(M);  // receivers of each sender
  for (int i = 0; i < M; ++i)
    for (int e = p->h_row_ptr[i]; e < p->h_row_ptr[i + 1]; ++e) outn[p->h_col[e]].push_back(i);
  std::vector<int32_t> act_of(M, -1);
  for (int a = 0; a < (int)p->h_act.size(); ++a) act_of[p->h_act[a]] = a;
  const int stride = 6 + 2 * (L + 1) + 4 * L + 2 * L + 1;
  const int Hd = p->gnn ? p->gnn->Hd : 128;
  const int HW = Hd / 32;
  std::vector<int32_t> where(M, -1);
  auto ncols_of = [&](int node) { return 6 + (act_of[node] >= 0 ? 3 : 0); };
  // Round l holds round l-1's nodes first, in their order, then their other
  // receivers sorted by node, so a node keeps its index from round to round.
  auto rounds_of = [&](const std::vector<int32_t>& v0) {
    std::vector<std::vector<int32_t>> Vl(L + 1);
    Vl[0] = v0;
    for (int l = 1; l <= L; ++l) {
      std::vector<int32_t> fresh;
      for (int32_t j : Vl[l - 1])
        for (int32_t r : outn[j])
          if (std::find(Vl[l - 1].begin(), Vl[l - 1].end(), r) == Vl[l - 1].end()) fresh.push_back(r);
      std::sort(fresh.begin(), fresh.end());
      fresh.erase(std::unique(fresh.begin(), fresh.end()), fresh.end());
      Vl[l] = Vl[l - 1];
      Vl[l].insert(Vl[l].end(), fresh.begin(), fresh.end());
    }
    return Vl;
  };
  auto idx_in = [](const std::vector<int32_t>& v, int32_t node) {
    return (int32_t)(std::find(v.begin(), v.end(), node) - v.begin());
  };
  int i = 0, dpos = 0;  // column stream position: node i, its dimension dpos
  while (i < M) {
    std::vector<SeedCols> sc;
    if (!packed) {
      int used = 0;
      while (i < M && (int)sc.size() < max_seeds) {
        const int need = ncols_of(i);
        if (used + need > kCols) break;
        sc.push_back({i, used, 0, need});
        used += need;
        ++i;
      }
    } else {
      const int i0 = i, d0 = dpos;
      int used = 0;
      while (i < M && used < kCols) {
        const int take = std::min(kCols - used, ncols_of(i) - dpos);
        sc.push_back({i, used, dpos, take});
        used += take;
        dpos += take;
        if (dpos == ncols_of(i)) {
          ++i;
          dpos = 0;
        }
      }
      // shorten to whole seeds while a round would hold more than 16 nodes
      auto too_wide = [&]() {
        std::vector<int32_t> v0;
        for (const SeedCols& c : sc) v0.push_back(c.node);
        auto Vl = rounds_of(v0);
        for (auto& v : Vl)
          if (v.size() > 16) return true;
        return false;
      };
      while (sc.size() > 1 && too_wide()) {
        const SeedCols last = sc.back();
        sc.pop_back();
        i = last.node;
        dpos = last.d0;
      }
      (void)i0;
      (void)d0;
    }
    std::vector<int32_t> seeds, cols;
    for (const SeedCols& c : sc) {
      seeds.push_back(c.node);
      cols.push_back(c.c0 - c.d0);  // column of dimension 0 (classic tiles: the seed's first column)
    }
    std::vector<int32_t> m(stride, 0);
    m[0] = (int32_t)tp.seed.size();
    m[1] = (int32_t)seeds.size();
    for (size_t t = 0; t < seeds.size(); ++t) {
      tp.seed.push_back(seeds[t]);
      tp.seedcol.push_back(cols[t]);
      tp.seedact.push_back(act_of[seeds[t]]);
    }
    std::vector<std::vector<int32_t>> Vl = rounds_of(seeds);
    for (int c = 0; c < kCols; ++c) tp.colmap.push_back(-1);
    for (size_t t = 0; t < sc.size(); ++t)
      for (int d = 0; d < sc[t].cnt; ++d) tp.colmap[tp.colmap.size() - kCols + sc[t].c0 + d] = (int32_t)(t << 4) | (sc[t].d0 + d);
    for (int l = 0; l <= L; ++l) {
      tp.vmax = std::max(tp.vmax, (int)Vl[l].size());
      m[6 + 2 * l] = (int32_t)tp.V.size();
      m[7 + 2 * l] = (int32_t)Vl[l].size();
      if (l < L) tp.cap1 = std::max(tp.cap1, (int)Vl[l].size());
      if (l > 0) tp.cap2 = std::max(tp.cap2, (int)Vl[l].size());

      if (l % 2 == 0) tp.bufX = std::max(tp.bufX, (int)Vl[l].size());
      else tp.bufY = std::max(tp.bufY, (int)Vl[l].size());
      if (l > 0) {
        for (size_t q = 0; q < Vl[l - 1].size(); ++q) where[Vl[l - 1][q]] = (int32_t)q;
      }
      for (size_t q = 0; q < Vl[l].size(); ++q) {
        int32_t node = Vl[l][q];
        tp.V.push_back(node);
        if (l == 0) {
          tp.Vself.push_back((int32_t)q);
          tp.Vebeg.push_back((int32_t)tp.Eloc.size());
          tp.Vecnt.push_back(0);
          continue;
        }
        // In-edges whose tangent is nonzero: every edge when the receiver
        // itself carries a tangent (its edge term W_a dh_i + W_b dh_i survives
        // even if the sender's tangent is zero, marked by Eloc = -1), else only
        // the edges from senders that carry one.
        const bool self_on = where[node] >= 0;
        tp.Vself.push_back(where[node]);
        tp.Vebeg.push_back((int32_t)tp.Eloc.size());
        int cnt = 0;
        for (int e = p->h_row_ptr[node]; e < p->h_row_ptr[node + 1]; ++e) {
          int32_t j = p->h_col[e];
          if (where[j] >= 0 || self_on) {
            tp.Eloc.push_back(where[j]);
            tp.Eid.push_back(e);
            ++cnt;
          }
        }
        tp.Vecnt.push_back(cnt);
      }
      if (l > 0)
        for (int32_t n : Vl[l - 1]) where[n] = -1;
    }
    // sender programs for the matrix-core kernel
    for (int l = 1; l <= L; ++l) {
      const std::vector<int32_t>& prv = Vl[l - 1];
      const std::vector<int32_t>& nx = Vl[l];
      const int pb = (int32_t)tp.prog.size(), eb = (int32_t)tp.elist.size();
      for (int32_t node : prv) {
        tp.prog.push_back(idx_in(nx, node));
        const int nin = p->h_row_ptr[node + 1] - p->h_row_ptr[node];
        tp.prog.push_back(nin);
        tp.prog.push_back((int32_t)outn[node].size());
        for (int e = p->h_row_ptr[node]; e < p->h_row_ptr[node + 1]; ++e) tp.elist.push_back(e);
        for (int32_t r : outn[node]) {
          tp.prog.push_back(idx_in(nx, r));
          const int32_t* rb = p->h_col.data() + p->h_row_ptr[r];
          const int32_t* re = p->h_col.data() + p->h_row_ptr[r + 1];
          tp.elist.push_back((int32_t)(std::lower_bound(rb, re, node) - p->h_col.data()));
        }
      }
      const int base = 6 + 2 * (L + 1) + 4 * (l - 1);
      m[base] = pb;
      m[base + 1] = (int32_t)tp.prog.size() - pb;
      m[base + 2] = eb;
      m[base + 3] = (int32_t)tp.elist.size() - eb;
      const int words = (m[base + 1] + 3) / 4 * 4 + m[base + 3] * HW + (int)nx.size() * HW;
      tp.stage_cap = std::max(tp.stage_cap, words);
    }
    // stage image sources of the register-aggregate kernel
    int ocount = 0, bcount = 0;
    {
      const int SREC = stage_record_words(Hd);
      int so = 0;
      std::vector<int32_t> sp;  // (word, kind | round << 4, source) of every sourced word
      for (int l = 1; l <= L; ++l) {
        const std::vector<int32_t>& prv = Vl[l - 1];
        const std::vector<int32_t>& nx = Vl[l];
        auto item = [&](int dst, int kind, int32_t src) {
          sp.push_back(dst);
          sp.push_back(kind | (l << 4));
          sp.push_back(src);
        };
        for (size_t pp = 0; pp < prv.size(); ++pp) {
          const int32_t node = prv[pp];
          const int rec = so + (int)pp * SREC;
          uint32_t rcv = 0;
          for (int32_t r : outn[node]) {
            const int q = idx_in(nx, r);
            if (q >= 16) continue;  // more than 16 nodes in a round: this kernel is not used
            rcv |= 1u << q;
            const int32_t* rb = p->h_col.data() + p->h_row_ptr[r];
            const int32_t* re = p->h_col.data() + p->h_row_ptr[r + 1];
            const int32_t e = (int32_t)(std::lower_bound(rb, re, node) - p->h_col.data());
            for (int w = 0; w < HW; ++w) item(rec + 4 + 16 * w + q, kGEdgeMask, e * HW + w);
          }
          item(rec, kGConst, idx_in(nx, node));
          item(rec + 1, kGConst, (int32_t)rcv);
          for (int g4 = 0; g4 < Hd / 4; ++g4) item(rec + 4 + 16 * HW + g4, kGCount, node * (Hd / 4) + g4);
        }
        const int nb = so + (int)prv.size() * SREC;
        for (size_t q = 0; q < nx.size(); ++q)
          for (int w = 0; w < HW; ++w) item(nb + (int)q * HW + w, kGNodeMask, nx[q] * HW + w);
        so = nb + ((int)nx.size() * HW + 3) / 4 * 4;
        if (l == L) {
          // output records (the tile's columns of each block):
          //   A blocks {CSR block id, node index q, first column, first dim | count << 8 | diagonal << 16},
          //   then B blocks {node, q, first column, 3 actuator + first force dim | count << 8}
          ocount = 0;
          bcount = 0;
          for (size_t q = 0; q < nx.size(); ++q) {
            const int32_t node = nx[q];
            const int32_t* rb = p->h_pcol.data() + p->h_prow[node];
            const int32_t* re = p->h_pcol.data() + p->h_prow[node + 1];
            for (const SeedCols& c : sc) {
              const int s0 = c.d0, s1 = std::min(c.d0 + c.cnt, 6);
              if (s1 <= s0) continue;
              const int32_t* it = std::lower_bound(rb, re, c.node);
              if (it == re || *it != c.node) continue;
              item(so++, kGConst, (int32_t)(it - p->h_pcol.data()));
              item(so++, kGConst, (int32_t)q);
              item(so++, kGConst, c.c0);
              item(so++, kGConst, s0 | ((s1 - s0) << 8) | ((node == c.node ? 1 : 0) << 16));
              ++ocount;
            }
          }
          for (size_t q = 0; q < nx.size(); ++q)
            for (const SeedCols& c : sc) {
              const int f0 = std::max(c.d0, 6), f1 = c.d0 + c.cnt;
              if (act_of[c.node] < 0 || f1 <= f0) continue;
              const int32_t node = nx[q];
              const int32_t* rb = p->h_pcol.data() + p->h_prow[node];
              const int32_t* re = p->h_pcol.data() + p->h_prow[node + 1];
              const int32_t* it = std::lower_bound(rb, re, c.node);
              if (it == re || *it != c.node) continue;
              item(so++, kGConst, node);
              item(so++, kGConst, (int32_t)q);
              item(so++, kGConst, c.c0 + (f0 - c.d0));
              item(so++, kGConst, (3 * act_of[c.node] + (f0 - 6)) | ((f1 - f0) << 8));
              ++bcount;
            }
          // encoder block: the tile's column map, then the encoder masks of round 0's nodes
          m[stride - 1] = so;
          const size_t cmb = tp.colmap.size() - kCols;
          for (int c = 0; c < kCols; ++c) item(so++, kGConst, tp.colmap[cmb + c]);
          for (size_t q = 0; q < Vl[0].size(); ++q)
            for (int w = 0; w < HW; ++w) item(so++, kGEncMask, Vl[0][q] * HW + w);
        }
      }
      // dense image sources: words without a source are constant zeros
      const int words = (so + 3) / 4 * 4;
      const size_t ib = tp.img.size() / 2;
      tp.img.resize(tp.img.size() + 2 * (size_t)words, 0);
      for (int w = 0; w < words; ++w) tp.img[2 * (ib + w)] = kGConst;
      for (size_t t = 0; t < sp.size(); t += 3) {
        tp.img[2 * (ib + sp[t])] = sp[t + 1];
        tp.img[2 * (ib + sp[t]) + 1] = sp[t + 2];
      }
      m[6 + 2 * (L + 1) + 4 * L] = (int32_t)ib;
      m[6 + 2 * (L + 1) + 4 * L + 1] = words;
      tp.stage2_cap = std::max(tp.stage2_cap, words);
    }
    // output blocks: (node of the last round, seed) pairs inside the pattern
    m[2] = (int32_t)(tp.out3.size() / 3);
    m[4] = (int32_t)(tp.bout2.size() / 2);
    int oc = 0, bc = 0;
    for (size_t q = 0; q < (packed ? 0 : Vl[L].size()); ++q) {
      int32_t node = Vl[L][q];
      const int32_t* rb = p->h_pcol.data() + p->h_prow[node];
      const int32_t* re = p->h_pcol.data() + p->h_prow[node + 1];
      for (size_t s = 0; s < seeds.size(); ++s) {
        const int32_t* it = std::lower_bound(rb, re, seeds[s]);
        if (it == re || *it != seeds[s]) continue;
        tp.out3.push_back((int32_t)q);
        tp.out3.push_back((int32_t)s);
        tp.out3.push_back((int32_t)(it - p->h_pcol.data()));
        ++oc;
        if (act_of[seeds[s]] >= 0) {
          tp.bout2.push_back((int32_t)q);
          tp.bout2.push_back((int32_t)s);
          ++bc;
        }
      }
    }
    m[3] = packed ? ocount : oc;
    m[5] = packed ? bcount : bc;
    tp.meta.insert(tp.meta.end(), m.begin(), m.end());
    ++tp.n_tiles;
  }
}

}  // namespace

void gnn_free(gnmpc_plan* p) {
  if (!p->gnn) return;
  for (void* q : p->gnn->allocs) (void)hipFree(q);
  delete p->gnn;
  p->gnn = nullptr;
}

gnmpc_status gnn_set(gnmpc_plan* p, const gnmpc_gnn_desc* desc, const double* w, int64_t n_w) {
  (void)n_w;
  gnn_free(p);
  p->gnn = new GnnState();
  GnnState& g = *p->gnn;
  const int Hd = desc->Hd, L = desc->L;
  g.Hd = Hd;
  g.L = L;
  g.dtype = desc->dtype;
  g.dt = (float)desc->dt;
  g.N = p->dims.N;
  g.M = p->M;
  g.E = p->E;
  if (p->dims.dtype != GNMPC_F32) {
    p->last_error = "model_set_gnn: the GNN path writes FP32 Jacobians (plan dtype must be F32)";
    gnn_free(p);
    return GNMPC_UNSUPPORTED;
  }
  const bool bf = desc->dtype == GNMPC_BF16;
  auto cv = [&](double v) { float f = (float)v; return bf ? host_bf16r(f) : f; };
  // unpack W_enc[Hd][9], b_enc, (W_e[Hd][2Hd], b_e, W_n[Hd][2Hd], b_n) x L, W_dec[6][Hd], b_dec
  size_t o = 0;
  std::vector<float> encT(9 * Hd), benc(Hd), WaT((size_t)L * Hd * Hd), WbT((size_t)L * Hd * Hd), be((size_t)L * Hd),
      Wn1T((size_t)L * Hd * Hd), Wn2T((size_t)L * Hd * Hd), bn((size_t)L * Hd), decT(6 * Hd), bdec(6);
  for (int f = 0; f < Hd; ++f)
    for (int d = 0; d < 9; ++d) encT[d * Hd + f] = cv(w[o + f * 9 + d]);
  o += 9 * Hd;
  for (int f = 0; f < Hd; ++f) benc[f] = (float)w[o + f];  // biases stay FP32 (added to FP32 sums)
  o += Hd;
  for (int l = 0; l < L; ++l) {
    for (int f = 0; f < Hd; ++f)
      for (int q = 0; q < Hd; ++q) {
        WaT[((size_t)l * Hd + q) * Hd + f] = cv(w[o + (size_t)f * 2 * Hd + q]);
        WbT[((size_t)l * Hd + q) * Hd + f] = cv(w[o + (size_t)f * 2 * Hd + Hd + q]);
      }
    o += (size_t)2 * Hd * Hd;
    for (int f = 0; f < Hd; ++f) be[l * Hd + f] = (float)w[o + f];
    o += Hd;
    for (int f = 0; f < Hd; ++f)
      for (int q = 0; q < Hd; ++q) {
        Wn1T[((size_t)l * Hd + q) * Hd + f] = cv(w[o + (size_t)f * 2 * Hd + q]);
        Wn2T[((size_t)l * Hd + q) * Hd + f] = cv(w[o + (size_t)f * 2 * Hd + Hd + q]);
      }
    o += (size_t)2 * Hd * Hd;
    for (int f = 0; f < Hd; ++f) bn[l * Hd + f] = (float)w[o + f];
    o += Hd;
  }
  for (int r = 0; r < 6; ++r)
    for (int f = 0; f < Hd; ++f) decT[f * 6 + r] = cv(w[o + r * Hd + f]);
  o += 6 * Hd;
  for (int r = 0; r < 6; ++r) bdec[r] = (float)w[o + r];
  gnmpc_status s;
#define UP(ptr, vec) \
  if ((s = dupload(p, g.ptr, vec)) != GNMPC_OK) return s;
  UP(encT, encT) UP(benc, benc) UP(WaT, WaT) UP(WbT, WbT) UP(be, be) UP(Wn1T, Wn1T) UP(Wn2T, Wn2T) UP(bn, bn)
  UP(decT, decT) UP(bdec, bdec)
  {
    // reverse mode: W_a + W_b, W_b, W_n1, W_n2 row-major (out f, in q); the transposes above hold [q][f]
    std::vector<float> WabR((size_t)L * Hd * Hd), WbR(WabR.size()), Wn1R(WabR.size()), Wn2R(WabR.size());
    for (int l = 0; l < L; ++l)
      for (int f = 0; f < Hd; ++f)
        for (int q = 0; q < Hd; ++q) {
          const size_t t = ((size_t)l * Hd + q) * Hd + f, r = ((size_t)l * Hd + f) * Hd + q;
          WabR[r] = WaT[t] + WbT[t];
          WbR[r] = WbT[t];
          Wn1R[r] = Wn1T[t];
          Wn2R[r] = Wn2T[t];
        }
    UP(WabR, WabR) UP(WbR, WbR) UP(Wn1R, Wn1R) UP(Wn2R, Wn2R)
    // out-edges of every node j: the receivers i of edges j -> i and the CSR index of each edge
    std::vector<int32_t> optr(p->M + 1, 0), orecv(std::max(p->E, 1)), oedge(std::max(p->E, 1));
    for (int e = 0; e < p->E; ++e) ++optr[p->h_col[e] + 1];
    for (int j = 0; j < p->M; ++j) optr[j + 1] += optr[j];
    std::vector<int32_t> fill(optr.begin(), optr.end() - 1);
    for (int i = 0; i < p->M; ++i)
      for (int e = p->h_row_ptr[i]; e < p->h_row_ptr[i + 1]; ++e) {
        const int q = fill[p->h_col[e]]++;
        orecv[q] = i;
        oedge[q] = e;
      }
    UP(out_ptr, optr) UP(out_recv, orecv) UP(out_edge, oedge)
  }
  const size_t NM = (size_t)g.N * g.M;
  // hidden states of the L + 1 layers; reverse mode reuses this buffer for three
  // cotangent arrays of the same size, so it holds at least three
  if ((s = dalloc(p, g.h, (size_t)std::max(L + 1, 3) * NM * Hd)) != GNMPC_OK) return s;
  if ((s = dalloc(p, g.mask_enc, NM * (Hd / 32))) != GNMPC_OK) return s;
  if ((s = dalloc(p, g.mask_node, (size_t)L * NM * (Hd / 32))) != GNMPC_OK) return s;
  if ((s = dalloc(p, g.mask_edge, (size_t)L * g.N * std::max(g.E, 1) * (Hd / 32))) != GNMPC_OK) return s;
  if ((s = dalloc(p, g.fnext, NM * NBX)) != GNMPC_OK) return s;
  g.maxdeg = 0;
  for (int i = 0; i < p->M; ++i) g.maxdeg = std::max(g.maxdeg, p->h_row_ptr[i + 1] - p->h_row_ptr[i]);
  // seed tiles: two seeds per tile when the tangent buffers fit in LDS, else one
  const size_t elem = bf ? 2 : 4;
  TilePlan tp;
  bool fits = false;
  for (int ms = 2; ms >= 1 && !fits; --ms) {
    tp = TilePlan();
    build_tiles(p, L, ms, tp);
    g.jvp_lds = (size_t)(tp.bufX + tp.bufY) * Hd * kCols * elem;
    fits = g.jvp_lds <= 160 * 1024;
  }
  if (!fits) {
    p->last_error = "model_set_gnn: tangent buffers exceed LDS for this graph";
    gnn_free(p);
    return GNMPC_UNSUPPORTED;
  }
  g.n_tiles = tp.n_tiles;
  g.meta_stride = 6 + 2 * (L + 1) + 4 * L + 2 * L + 1;
  g.bufX = tp.bufX;
  g.bufY = tp.bufY;
  // The matrix-core path needs BF16, a supported width and the round buffers in LDS.
  g.cap1 = tp.cap1;
  g.cap2 = tp.cap2;
  g.stage_cap = tp.stage_cap;
  g.mfma_lds = (size_t)tp.cap1 * kCols * Hd * 2 + (size_t)tp.cap2 * kCols * Hd * 4 + (size_t)tp.stage_cap * 4;
  g.mfma = bf && (Hd == 64 || Hd == 128 || Hd == 256) && tp.cap2 <= 16 && g.mfma_lds <= 160 * 1024;
  // register-aggregate kernel: packed tiles (16 columns from a column stream) when every
  // round stays within 16 nodes, else the classic tiles
  TilePlan tp2;
  auto fits2 = [&](const TilePlan& t, size_t& lds, int& words) {
    words = (t.stage2_cap + 3) / 4 * 4;
    lds = (size_t)(t.cap1 + t.cap2) * kCols * Hd * 2 + (size_t)words * 4 + (size_t)(3 + 9) * Hd * 4;
    return t.vmax <= 16 && lds <= 160 * 1024;
  };
  g.mfma2 = false;
  const TilePlan* t2 = nullptr;
  if (g.mfma && (Hd == 64 || Hd == 128)) {
    build_tiles(p, L, 0, tp2, true);
    if (fits2(tp2, g.mfma2_lds, g.stage2_words)) t2 = &tp2;
    else if (fits2(tp, g.mfma2_lds, g.stage2_words)) t2 = &tp;
    g.mfma2 = t2 != nullptr;
  }
  if (g.mfma) {
    std::vector<uint16_t> wa16((size_t)L * Hd * Hd), wb16(wa16.size()), w1_16(wa16.size()), w2_16(wa16.size());
    auto b16 = [](float v) {
      uint32_t u;
      std::memcpy(&u, &v, 4);
      return (uint16_t)(u >> 16);  // values are already bf16-representable
    };
    for (int l = 0; l < L; ++l)
      for (int f = 0; f < Hd; ++f)
        for (int q = 0; q < Hd; ++q) {
          const size_t src = ((size_t)l * Hd + q) * Hd + f, dst = ((size_t)l * Hd + f) * Hd + q;
          wa16[dst] = b16(WaT[src]);
          wb16[dst] = b16(WbT[src]);
          w1_16[dst] = b16(Wn1T[src]);
          w2_16[dst] = b16(Wn2T[src]);
        }
    UP(Wa16, wa16) UP(Wb16, wb16) UP(Wn1_16, w1_16) UP(Wn2_16, w2_16)
    UP(prog, tp.prog) UP(elist, tp.elist)
    if (t2) {
      UP(img_src, t2->img) UP(t2_meta, t2->meta) UP(t2_V, t2->V) UP(t2_Vself, t2->Vself) UP(t2_colmap, t2->colmap)
      g.t2_tiles = t2->n_tiles;
      g.t2_cap1 = t2->cap1;
      g.t2_cap2 = t2->cap2;
      g.img_words = (long)(t2->img.size() / 2);
      if ((s = dalloc(p, g.img, (size_t)g.N * g.img_words)) != GNMPC_OK) return s;
    }
    // forward column tiles: greedily add target nodes while targets plus their
    // senders fit in NC columns; targets occupy the first columns
    const size_t NC = 16 * (size_t)fwd_groups(Hd);
    std::vector<int32_t> fcols, fmeta, fecnt, fepre, fesrc, feid;
    int i = 0;
    g.fedge_cap = 0;
    while (i < g.M) {
      std::vector<int32_t> tg, hal;
      while (i < g.M) {
        std::vector<int32_t> cand_t = tg, cand_h = hal;
        cand_t.push_back(i);
        for (int e = p->h_row_ptr[i]; e < p->h_row_ptr[i + 1]; ++e) cand_h.push_back(p->h_col[e]);
        std::vector<int32_t> all = cand_h;
        all.erase(std::remove_if(all.begin(), all.end(),
                                 [&](int32_t v) { return std::find(cand_t.begin(), cand_t.end(), v) != cand_t.end(); }),
                  all.end());
        std::sort(all.begin(), all.end());
        all.erase(std::unique(all.begin(), all.end()), all.end());
        if (cand_t.size() + all.size() > NC) break;
        tg = cand_t;
        hal = all;
        ++i;
      }
      if (tg.empty()) {
        p->last_error = "model_set_gnn: a node has too many in-neighbours for a forward column tile";
        gnn_free(p);
        return GNMPC_UNSUPPORTED;
      }
      std::vector<int32_t> colv = tg;
      colv.insert(colv.end(), hal.begin(), hal.end());
      const int eb = (int)fesrc.size();
      for (size_t c = 0; c < NC; ++c) {
        fcols.push_back(c < colv.size() ? colv[c] : -1);
        fepre.push_back((int32_t)fesrc.size() - eb);
        if (c < tg.size()) {
          const int node = tg[c];
          fecnt.push_back(p->h_row_ptr[node + 1] - p->h_row_ptr[node]);
          for (int e = p->h_row_ptr[node]; e < p->h_row_ptr[node + 1]; ++e) {
            fesrc.push_back((int32_t)(std::find(colv.begin(), colv.end(), p->h_col[e]) - colv.begin()));
            feid.push_back(e);
          }
        } else {
          fecnt.push_back(0);
        }
      }
      const int ec = (int)fesrc.size() - eb;
      g.fedge_cap = std::max(g.fedge_cap, ec);
      fmeta.push_back((int32_t)tg.size());
      fmeta.push_back(eb);
      fmeta.push_back(ec);
      fmeta.push_back(0);
      ++g.n_ftiles;
    }
    if (fwd_lds_bytes(Hd, g.fedge_cap) > 160 * 1024) {
      p->last_error = "model_set_gnn: a forward column tile's edges exceed LDS";
      gnn_free(p);
      return GNMPC_UNSUPPORTED;
    }
    UP(fcols, fcols) UP(fmeta, fmeta) UP(fecnt, fecnt) UP(fepre, fepre) UP(fesrc, fesrc) UP(feid, feid)
    if ((s = dalloc(p, g.cnt, (size_t)L * NM * Hd)) != GNMPC_OK) return s;
  }
  UP(meta, tp.meta) UP(seed, tp.seed) UP(seedcol, tp.seedcol) UP(seedact, tp.seedact) UP(V, tp.V)
  UP(Vself, tp.Vself) UP(Vebeg, tp.Vebeg) UP(Vecnt, tp.Vecnt) UP(Eloc, tp.Eloc) UP(Eid, tp.Eid)
  UP(out3, tp.out3) UP(bout2, tp.bout2)
#undef UP
  return GNMPC_OK;
}

// The GNN forward pass at the N stages: hidden states, ReLU masks (and, on the
// matrix-core path, the per-feature active in-edge counts) in the plan's
// workspace, next states in g.fnext.
static gnmpc_status launch_gnn_forward(gnmpc_plan* p, const void* xhat, const void* uhat, FwdArgs& fa,
                                       hipStream_t s) {
  GnnState& g = *p->gnn;
  const int Hd = g.Hd, N = g.N, M = g.M;
  fa.N = N;
  fa.M = M;
  fa.E = g.E;
  fa.Hd = Hd;
  fa.L = g.L;
  fa.nu = p->dims.nu;
  fa.bf16 = g.dtype == GNMPC_BF16;
  fa.dt = g.dt;
  fa.xhat = (const float*)xhat;
  fa.uhat = (const float*)uhat;
  fa.row_ptr = p->d_row_ptr;
  fa.col = p->d_col;
  fa.act_of_node = p->d_act_of_node;
  fa.encT = g.encT;
  fa.benc = g.benc;
  fa.WaT = g.WaT;
  fa.WbT = g.WbT;
  fa.be = g.be;
  fa.Wn1T = g.Wn1T;
  fa.Wn2T = g.Wn2T;
  fa.bn = g.bn;
  fa.decT = g.decT;
  fa.bdec = g.bdec;
  fa.h = g.h;
  fa.mask_enc = g.mask_enc;
  fa.mask_node = g.mask_node;
  fa.mask_edge = g.mask_edge;
  fa.fnext = g.fnext;
  phase_begin(p, GNMPC_PH_GNN_FORWARD, s);
  if (g.mfma) {
    const size_t NM = (size_t)N * M;
    fwd_enc_kernel<<<N * M, Hd, 0, s>>>(fa);
    for (int l = 0; l < g.L; ++l) {
      FwdMfmaArgs f;
      f.N = N;
      f.M = M;
      f.E = g.E;
      f.l = l;
      f.fedge_cap = g.fedge_cap;
      f.hin = g.h + (size_t)l * NM * Hd;
      f.hout = g.h + (size_t)(l + 1) * NM * Hd;
      const size_t wo = (size_t)l * Hd * Hd;
      f.Wa = g.Wa16 + wo;
      f.Wb = g.Wb16 + wo;
      f.Wn1 = g.Wn1_16 + wo;
      f.Wn2 = g.Wn2_16 + wo;
      f.be = g.be + (size_t)l * Hd;
      f.bn = g.bn + (size_t)l * Hd;
      f.mask_edge = g.mask_edge + (size_t)l * N * g.E * (Hd / 32);
      f.mask_node = g.mask_node + (size_t)l * NM * (Hd / 32);
      f.cnt = g.cnt + (size_t)l * NM * Hd;
      f.fcols = g.fcols;
      f.fmeta = g.fmeta;
      f.fecnt = g.fecnt;
      f.fepre = g.fepre;
      f.fesrc = g.fesrc;
      f.feid = g.feid;
      const size_t qbytes = fwd_lds_bytes(Hd, g.fedge_cap);
      dim3 fg(g.n_ftiles, N);
      {
        const void* ffn = Hd == 64 ? (const void*)fwd_mfma_layer_kernel<1>
                        : Hd == 128 ? (const void*)fwd_mfma_layer_kernel<2> : (const void*)fwd_mfma_layer_kernel<4>;
        GNMPC_HIP_TRY(p, set_max_lds(ffn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)qbytes));
      }
      if (Hd == 64) fwd_mfma_layer_kernel<1><<<fg, 256, qbytes, s>>>(f);
      else if (Hd == 128) fwd_mfma_layer_kernel<2><<<fg, 256, qbytes, s>>>(f);
      else fwd_mfma_layer_kernel<4><<<fg, 256, qbytes, s>>>(f);
    }
    fwd_dec_coop_kernel<<<ceil_div((long)N * M * 16, 256), 256, 0, s>>>(fa, g.h + (size_t)g.L * NM * Hd);
  } else {
    fwd_enc_kernel<<<N * M, Hd, 0, s>>>(fa);
    const size_t lds_fwd = sizeof(float) * (size_t)(g.maxdeg + 2) * Hd;
    for (int l = 0; l < g.L; ++l) fwd_layer_kernel<<<N * M, Hd, lds_fwd, s>>>(fa, l);
    fwd_dec_kernel<<<ceil_div((long)N * M, 256), 256, 0, s>>>(fa);
  }
  phase_end(p, GNMPC_PH_GNN_FORWARD, s);
  return GNMPC_OK;
}

gnmpc_status launch_gnn_linearize(gnmpc_plan* p, const void* xhat, const void* uhat, void* A, void* B, void* c,
                                  void* fnext, hipStream_t s) {
  GnnState& g = *p->gnn;
  const int Hd = g.Hd, N = g.N, M = g.M;
  FwdArgs fa;
  {
    const gnmpc_status fs = launch_gnn_forward(p, xhat, uhat, fa, s);
    if (fs != GNMPC_OK) return fs;
  }
  const long nB = (long)N * M * NBX * p->dims.nu;
  const int zero_blocks = (int)std::min<long>(ceil_div(nB, 1024), 2048);
  if (!g.mfma2)  // else the fill shares the stage-image launch
    fill_zero_kernel<<<(int)std::min<long>(ceil_div(nB, 256), 4096), 256, 0, s>>>((float*)B, nB);
  JvpArgs ja;
  ja.N = N;
  ja.M = M;
  ja.E = g.E;
  ja.Hd = Hd;
  ja.L = g.L;
  ja.nu = p->dims.nu;
  ja.bf16 = fa.bf16;
  ja.meta_stride = g.meta_stride;
  ja.bufX = g.bufX;
  ja.dt = g.dt;
  ja.encT = g.encT;
  ja.WaT = g.WaT;
  ja.WbT = g.WbT;
  ja.Wn1T = g.Wn1T;
  ja.Wn2T = g.Wn2T;
  ja.decT = g.decT;
  ja.mask_enc = g.mask_enc;
  ja.mask_node = g.mask_node;
  ja.mask_edge = g.mask_edge;
  ja.meta = g.meta;
  ja.seed = g.seed;
  ja.seedcol = g.seedcol;
  ja.seedact = g.seedact;
  ja.V = g.V;
  ja.Vself = g.Vself;
  ja.Vebeg = g.Vebeg;
  ja.Vecnt = g.Vecnt;
  ja.Eloc = g.Eloc;
  ja.Eid = g.Eid;
  ja.out3 = g.out3;
  ja.bout2 = g.bout2;
  ja.A = (float*)A;
  ja.B = (float*)B;
  ja.nnz = p->nnz;
  dim3 grid(g.n_tiles, N);
  if (g.mfma2) {
    // stage images of every (tile, stage) from this forward pass, and the B fill
    phase_begin(p, GNMPC_PH_GNN_STAGE_IMAGES, s);
    const int img_blocks = (int)((g.img_words + 255) / 256);
    const dim3 gimg((unsigned)(img_blocks + zero_blocks));
    if (Hd == 64)
      stage_image_kernel<64><<<gimg, 256, 0, s>>>(N, M, g.E, g.img_words, g.img_src, g.mask_enc, g.mask_node,
                                                  g.mask_edge, reinterpret_cast<const uint32_t*>(g.cnt), g.img,
                                                  img_blocks, (float*)B, nB);
    else
      stage_image_kernel<128><<<gimg, 256, 0, s>>>(N, M, g.E, g.img_words, g.img_src, g.mask_enc, g.mask_node,
                                                   g.mask_edge, reinterpret_cast<const uint32_t*>(g.cnt), g.img,
                                                   img_blocks, (float*)B, nB);
    phase_end(p, GNMPC_PH_GNN_STAGE_IMAGES, s);
  }
  phase_begin(p, GNMPC_PH_GNN_JACOBIAN, s);
  if (g.mfma2) {
    Mfma2Args ma;
    ma.N = N;
    ma.M = M;
    ma.E = g.E;
    ma.L = g.L;
    ma.nu = p->dims.nu;
    ma.meta_stride = g.meta_stride;
    ma.cap1 = g.t2_cap1;
    ma.cap2 = g.t2_cap2;
    ma.stage_words = g.stage2_words;
    ma.dt = g.dt;
    ma.encT = g.encT;
    ma.decT = g.decT;
    ma.Wa = g.Wa16;
    ma.Wb = g.Wb16;
    ma.Wn1 = g.Wn1_16;
    ma.Wn2 = g.Wn2_16;
    ma.mask_enc = g.mask_enc;
    ma.mask_node = g.mask_node;
    ma.mask_edge = g.mask_edge;
    ma.cnt = reinterpret_cast<const uint32_t*>(g.cnt);
    ma.meta = g.t2_meta;
    ma.seed = g.seed;
    ma.seedcol = g.seedcol;
    ma.seedact = g.seedact;
    ma.V = g.t2_V;
    ma.Vself = g.t2_Vself;
    ma.img = g.img;
    ma.img_words = g.img_words;
    ma.colmap = g.t2_colmap;
    ma.out3 = g.out3;
    ma.bout2 = g.bout2;
    ma.A = (float*)A;
    ma.B = (float*)B;
    ma.nnz = p->nnz;
    const void* kfn = Hd == 64 ? (const void*)jvp_mfma2_kernel<64> : (const void*)jvp_mfma2_kernel<128>;
    GNMPC_HIP_TRY(p, set_max_lds(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.mfma2_lds));
    dim3 grid2(g.t2_tiles, N);
    if (Hd == 64) jvp_mfma2_kernel<64><<<grid2, 256, g.mfma2_lds, s>>>(ma);
    else jvp_mfma2_kernel<128><<<grid2, 512, g.mfma2_lds, s>>>(ma);
  } else if (g.mfma) {
    MfmaArgs ma;
    ma.N = N;
    ma.M = M;
    ma.E = g.E;
    ma.L = g.L;
    ma.nu = p->dims.nu;
    ma.meta_stride = g.meta_stride;
    ma.cap1 = g.cap1;
    ma.cap2 = g.cap2;
    ma.dt = g.dt;
    ma.encT = g.encT;
    ma.decT = g.decT;
    ma.Wa = g.Wa16;
    ma.Wb = g.Wb16;
    ma.Wn1 = g.Wn1_16;
    ma.Wn2 = g.Wn2_16;
    ma.mask_enc = g.mask_enc;
    ma.mask_node = g.mask_node;
    ma.mask_edge = g.mask_edge;
    ma.meta = g.meta;
    ma.seed = g.seed;
    ma.seedcol = g.seedcol;
    ma.seedact = g.seedact;
    ma.V = g.V;
    ma.Vself = g.Vself;
    ma.prog = g.prog;
    ma.elist = g.elist;
    ma.out3 = g.out3;
    ma.bout2 = g.bout2;
    ma.A = (float*)A;
    ma.B = (float*)B;
    ma.nnz = p->nnz;
    const void* kfn = Hd == 64 ? (const void*)jvp_mfma_kernel<1>
                    : Hd == 128 ? (const void*)jvp_mfma_kernel<2> : (const void*)jvp_mfma_kernel<4>;
    GNMPC_HIP_TRY(p, set_max_lds(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.mfma_lds));
    if (Hd == 64) jvp_mfma_kernel<1><<<grid, 256, g.mfma_lds, s>>>(ma);
    else if (Hd == 128) jvp_mfma_kernel<2><<<grid, 256, g.mfma_lds, s>>>(ma);
    else jvp_mfma_kernel<4><<<grid, 256, g.mfma_lds, s>>>(ma);
  } else if (fa.bf16) {
    GNMPC_HIP_TRY(p, set_max_lds((const void*)jvp_valu_kernel<uint16_t>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.jvp_lds));
    jvp_valu_kernel<uint16_t><<<grid, 2 * Hd, g.jvp_lds, s>>>(ja);
  } else {
    GNMPC_HIP_TRY(p, set_max_lds((const void*)jvp_valu_kernel<float>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.jvp_lds));
    jvp_valu_kernel<float><<<grid, 2 * Hd, g.jvp_lds, s>>>(ja);
  }
  phase_end(p, GNMPC_PH_GNN_JACOBIAN, s);
  phase_begin(p, GNMPC_PH_GNN_ASSEMBLY, s);
  gnn_offset_kernel<<<ceil_div((long)N * M * NBX, 256), 256, 0, s>>>(N, M, p->dims.nu, p->nnz, p->d_prow, p->d_pcol,
                                                               (const float*)xhat, (const float*)uhat,
                                                               (const float*)A, (const float*)B, g.fnext,
                                                               (float*)c, (float*)fnext);
  phase_end(p, GNMPC_PH_GNN_ASSEMBLY, s);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

// ---------------------------------------------------------------------------
// Reverse mode through the layers (the gradient of g . f at the N stages,
// Sec. V-A's model f read backwards).  The forward pass is recomputed first, at
// the given point, for its ReLU masks; the backward pass then needs no
// activations, only the masks, and runs layer by layer over every (stage, node)
// with one workgroup of Hd lanes each (lane q owns feature q of the node's
// cotangent).  With W_a, W_b the two halves of the edge MLP's first layer
// (z_ij = W_a h_i + W_b (h_i - h_j) + b_e, m_ij = relu(z_ij)), agg_i = sum_j m_ij,
// and z_i = W_n1 h_i + W_n2 agg_i + b_n, h'_i = relu(z_i), a round backwards is
//   zb_i  = mask_i . hb'_i,   hb_i = W_n1' zb_i,   ab_i = W_n2' zb_i        (node)
//   hb_i += (W_a + W_b)' (cnt_i . ab_i)                 (the receiver side of its in-edges)
//   hb_j -= W_b' sum_{i: j -> i} D_ij . ab_i            (the sender side of its out-edges)
// where D_ij is edge (j -> i)'s ReLU mask and cnt_i = sum_j D_ij per feature.
// Cotangent buffers reuse the forward's hidden-state workspace (the masks carry
// everything the backward pass needs).
namespace {

struct VjpArgs {
  int N, M, E, Hd, L, nu;
  float dt;
  const float *g, *decT, *encT;
  const float *WabR, *WbR, *Wn1R, *Wn2R;          // this round's (for the round kernels)
  const uint32_t *mask_enc, *mask_node, *mask_edge;  // this round's node and edge masks (round kernels)
  const int32_t *row_ptr, *out_ptr, *out_recv, *out_edge, *act_of_node;
  float *hb, *hbt, *ab;  // [N][M][Hd] each
  float *gx, *gu;
};

__device__ inline float mask_on(const uint32_t* words, int f) { return (words[f >> 5] >> (f & 31)) & 1u ? 1.f : 0.f; }

// o = W_dec h^L + b_dec, v+ = v + dt o[3:6], p+ = p + dt v+:
//   vb = g_v + dt g_p,  gx = [g_p; vb] (direct terms),  hb^L = W_dec[3:6]' (dt vb)
__global__ void vjp_dec_kernel(VjpArgs a) {
  const int s = blockIdx.x, q = threadIdx.x;
  const float* gs = a.g + (size_t)s * NBX;
  float vb[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) vb[r] = gs[3 + r] + a.dt * gs[r];
  float h = 0.f;
#pragma unroll
  for (int r = 0; r < 3; ++r) h += a.decT[q * 6 + 3 + r] * (a.dt * vb[r]);
  a.hb[(size_t)s * a.Hd + q] = h;
  if (q < NBX) a.gx[(size_t)s * NBX + q] = q < 3 ? gs[q] : vb[q - 3];
}

// node update and the receiver side of the in-edges of one round
__global__ void vjp_node_kernel(VjpArgs a) {
  extern __shared__ float vs[];  // [Hd] zb, then [Hd] cnt . ab
  const int s = blockIdx.x, q = threadIdx.x, Hd = a.Hd;
  const int k = s / a.M, i = s - k * a.M;
  float* zb = vs;
  float* yb = vs + Hd;
  zb[q] = mask_on(a.mask_node + (size_t)s * (Hd / 32), q) * a.hb[(size_t)s * Hd + q];
  __syncthreads();
  float hn = 0.f, abq = 0.f;
  for (int f = 0; f < Hd; ++f) {
    const float z = zb[f];
    hn += a.Wn1R[(size_t)f * Hd + q] * z;
    abq += a.Wn2R[(size_t)f * Hd + q] * z;
  }
  float cnt = 0.f;
  const uint32_t* me = a.mask_edge + (size_t)k * a.E * (Hd / 32);
  for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) cnt += mask_on(me + (size_t)e * (Hd / 32), q);
  yb[q] = cnt * abq;
  __syncthreads();
  for (int f = 0; f < Hd; ++f) hn += a.WabR[(size_t)f * Hd + q] * yb[f];
  a.hbt[(size_t)s * Hd + q] = hn;
  a.ab[(size_t)s * Hd + q] = abq;
}

// the sender side of the out-edges of one round: hb_j = hbt_j - W_b' sum_i D_ij . ab_i
__global__ void vjp_edge_kernel(VjpArgs a) {
  extern __shared__ float vs[];  // [Hd]
  const int s = blockIdx.x, q = threadIdx.x, Hd = a.Hd;
  const int k = s / a.M, j = s - k * a.M;
  const uint32_t* me = a.mask_edge + (size_t)k * a.E * (Hd / 32);
  float z = 0.f;
  for (int t = a.out_ptr[j]; t < a.out_ptr[j + 1]; ++t)
    z += mask_on(me + (size_t)a.out_edge[t] * (Hd / 32), q) * a.ab[((size_t)k * a.M + a.out_recv[t]) * Hd + q];
  vs[q] = z;
  __syncthreads();
  float h = a.hbt[(size_t)s * Hd + q];
  for (int f = 0; f < Hd; ++f) h -= a.WbR[(size_t)f * Hd + q] * vs[f];
  a.hb[(size_t)s * Hd + q] = h;
}

// encoder h0 = relu(W_enc [x; P u] + b): [xb; ub] = W_enc' (mask . hb^0); gx += xb, gu at the actuator
__global__ void vjp_enc_kernel(VjpArgs a) {
  extern __shared__ float vs[];  // [9][Hd / 64] wave partial sums
  const int s = blockIdx.x, q = threadIdx.x, Hd = a.Hd;
  const int k = s / a.M, i = s - k * a.M;
  const int nwv = Hd / 64, lane = q & 63, wv = q >> 6;
  const float zb = mask_on(a.mask_enc + (size_t)s * (Hd / 32), q) * a.hb[(size_t)s * Hd + q];
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    float v = a.encT[d * Hd + q] * zb;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) vs[d * nwv + wv] = v;
  }
  __syncthreads();
  if (q < 9) {
    float v = 0.f;
    for (int w = 0; w < nwv; ++w) v += vs[q * nwv + w];
    if (q < NBX) {
      a.gx[(size_t)s * NBX + q] += v;
    } else {
      const int act = a.act_of_node[i];
      if (act >= 0) a.gu[(size_t)k * a.nu + 3 * act + (q - NBX)] = v;
    }
  }
}

__global__ void copy_f32_kernel(const float* __restrict__ src, float* __restrict__ dst, long n) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

}  // namespace

gnmpc_status launch_gnn_forward_only(gnmpc_plan* p, const void* xhat, const void* uhat, void* fnext, hipStream_t s) {
  GnnState& g = *p->gnn;
  FwdArgs fa;
  const gnmpc_status fs = launch_gnn_forward(p, xhat, uhat, fa, s);
  if (fs != GNMPC_OK) return fs;
  const long n = (long)g.N * g.M * NBX;
  copy_f32_kernel<<<ceil_div(n, 256), 256, 0, s>>>(g.fnext, (float*)fnext, n);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

gnmpc_status launch_gnn_vjp(gnmpc_plan* p, const void* xhat, const void* uhat, const void* gin, void* gx, void* gu,
                            hipStream_t s) {
  GnnState& g = *p->gnn;
  const int Hd = g.Hd, N = g.N, M = g.M, L = g.L;
  FwdArgs fa;
  const gnmpc_status fs = launch_gnn_forward(p, xhat, uhat, fa, s);
  if (fs != GNMPC_OK) return fs;
  const size_t NM = (size_t)N * M;
  VjpArgs va;
  va.N = N;
  va.M = M;
  va.E = g.E;
  va.Hd = Hd;
  va.L = L;
  va.nu = p->dims.nu;
  va.dt = g.dt;
  va.g = (const float*)gin;
  va.decT = g.decT;
  va.encT = g.encT;
  va.row_ptr = p->d_row_ptr;
  va.out_ptr = g.out_ptr;
  va.out_recv = g.out_recv;
  va.out_edge = g.out_edge;
  va.act_of_node = p->d_act_of_node;
  va.mask_enc = g.mask_enc;
  va.hb = g.h;  // the hidden states are no longer needed (the buffer holds at least three arrays)
  va.hbt = g.h + NM * Hd;
  va.ab = g.h + 2 * NM * Hd;
  va.gx = (float*)gx;
  va.gu = (float*)gu;
  vjp_dec_kernel<<<(unsigned)NM, Hd, 0, s>>>(va);
  for (int l = L - 1; l >= 0; --l) {
    const size_t wo = (size_t)l * Hd * Hd;
    va.WabR = g.WabR + wo;
    va.WbR = g.WbR + wo;
    va.Wn1R = g.Wn1R + wo;
    va.Wn2R = g.Wn2R + wo;
    va.mask_node = g.mask_node + (size_t)l * NM * (Hd / 32);
    va.mask_edge = g.mask_edge + (size_t)l * N * g.E * (Hd / 32);
    vjp_node_kernel<<<(unsigned)NM, Hd, 2 * Hd * sizeof(float), s>>>(va);
    vjp_edge_kernel<<<(unsigned)NM, Hd, Hd * sizeof(float), s>>>(va);
  }
  vjp_enc_kernel<<<(unsigned)NM, Hd, 9 * (Hd / 64) * sizeof(float), s>>>(va);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

}  // namespace gnmpc
