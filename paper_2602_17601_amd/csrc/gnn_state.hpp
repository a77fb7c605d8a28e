// State of the message-passing GNN model of a plan (its weights in the layouts
// the kernels read, forward-pass workspace and tile tables); shared by the GNN
// kernels and the training kernels.
#pragma once

#include <vector>

#include "plan.hpp"

struct GnnState {
  int Hd = 0, L = 0, dtype = GNMPC_F32, N = 0, M = 0, E = 0;
  float dt = 0.f;
  // weights as FP32 values (bf16-representable in BF16 mode), transposed so
  // that lane f of a workgroup reads consecutive addresses
  float *encT = nullptr;           // [9][Hd]
  float *benc = nullptr;           // [Hd]
  float *WaT = nullptr, *WbT = nullptr, *be = nullptr;      // [L][Hd(in)][Hd(out)], [L][Hd]
  float *Wn1T = nullptr, *Wn2T = nullptr, *bn = nullptr;    // [L][Hd][Hd], [L][Hd]
  float *decT = nullptr, *bdec = nullptr;                   // [Hd][6], [6]
  // forward-pass workspace
  float* h = nullptr;              // [max(L+1, 3)][N][M][Hd]
  uint32_t *mask_enc = nullptr;    // [N][M][Hd/32]
  uint32_t *mask_node = nullptr;   // [L][N][M][Hd/32]
  uint32_t *mask_edge = nullptr;   // [L][N][E][Hd/32]
  float* fnext = nullptr;          // [N][M][6]
  int maxdeg = 0;
  // seed tiles
  int n_tiles = 0, meta_stride = 0, bufX = 0, bufY = 0;
  size_t jvp_lds = 0;
  int32_t *meta = nullptr, *seed = nullptr, *seedcol = nullptr, *seedact = nullptr;
  int32_t *V = nullptr, *Vself = nullptr, *Vebeg = nullptr, *Vecnt = nullptr;
  int32_t *Eloc = nullptr, *Eid = nullptr, *out3 = nullptr, *bout2 = nullptr;
  // MFMA Jacobian path (BF16): weights as bf16 row-major (out, in), sender lists
  bool mfma = false;
  int cap1 = 0, cap2 = 0;
  size_t mfma_lds = 0;
  uint16_t *Wa16 = nullptr, *Wb16 = nullptr, *Wn1_16 = nullptr, *Wn2_16 = nullptr;  // [L][Hd][Hd]
  int32_t *prog = nullptr, *elist = nullptr;
  int stage_cap = 0;
  // register-aggregate Jacobian kernel (Hd 64 or 128), on its own (packed) seed tiles
  bool mfma2 = false;
  size_t mfma2_lds = 0;
  int stage2_words = 0, t2_tiles = 0, t2_cap1 = 0, t2_cap2 = 0;
  int32_t *img_src = nullptr, *t2_meta = nullptr, *t2_V = nullptr, *t2_Vself = nullptr, *t2_colmap = nullptr;
  uint32_t* img = nullptr;  // stage images [N][img_words]
  long img_words = 0;
  // matrix-core forward pass (BF16 weights): node column tiles
  uint8_t* cnt = nullptr;         // [L][N][M][Hd] active in-edges of each node per feature
  int n_ftiles = 0, fedge_cap = 0;
  int32_t *fcols = nullptr;       // [n_ftiles][NC] node of each column (-1 = empty)
  int32_t *fmeta = nullptr;       // [n_ftiles][4]: targets, edge begin, edge count, -
  int32_t *fecnt = nullptr;       // [n_ftiles][NC] in-edges of each target column
  int32_t *fepre = nullptr;       // [n_ftiles][NC] edges of the columns before it (exclusive prefix)
  int32_t *fesrc = nullptr, *feid = nullptr;  // per edge: source column, CSR edge id
  // reverse mode (gnmpc_gnn_vjp): FP32 weights row-major (out, in) so lane q reads
  // column q of W (the transposed products), and each node's out-edges
  float *WabR = nullptr, *WbR = nullptr, *Wn1R = nullptr, *Wn2R = nullptr;  // [L][Hd][Hd]; WabR = W_a + W_b
  int32_t *out_ptr = nullptr, *out_recv = nullptr, *out_edge = nullptr;     // [M+1], [E], [E]
  std::vector<void*> allocs;
};
