// Row-block fused step for the BF16 path.
//
// One workgroup owns 16 rows (streams) and runs, without leaving the kernel,
// everything between the FDM product and its adjoint that only involves its
// own rows: LTE up-projection (Eq. 16), every refinement block (Eqs. 9-13),
// the head and softmax (Eq. 1), the integer CDF and the range-coder lane,
// the cross-entropy adjoint (Eq. 2) back through the blocks to dY.  The
// activations of the row block stay in LDS; the weights stream from L2 as
// BF16 "fragment-ordered" copies in which the MFMA operand of one wave for a
// 16-column x 32-k block is a single contiguous 1 KiB chunk.
#pragma once
#include "common.h"
#include "kernels.h"
#include "adam.h"

namespace edpc {

constexpr int kFusedRows = 16;   // rows per workgroup
constexpr int kMaxFusedBlocks = 8;

// Fragment-ordered BF16 copy of a row-major FP32 matrix W [rows][cols].
//   nt: operand of Out = In W^T (k = cols): fragment (nb < rows/16, kb < cols/32),
//       lane l holds W[nb*16 + l%16][kb*32 + 8*(l/16) + 0..7]
//   nn: operand of Out = In W   (k = rows): fragment (nb < cols/16, kb < rows/32),
//       lane l holds W[kb*32 + 8*(l/16) + 0..7][nb*16 + l%16]
// Fragment f = nb * KB + kb is stored as 64 uint4 (one per lane).
struct FragJob {
  const float* src;
  int rows, cols;
  uint4* nt;
  uint4* nn;
  int frag_begin;  // first fragment of this job in the launch (nt and nn counted separately)
};
void k_build_frags(const FragJob* jobs, int n_jobs, int total_frags, hipStream_t s);

// Adam over the jobs' parameters in one launch (adam.h).  The row-block
// step's update takes this pass only when its weight gradients run on a wide
// tile; on a 4-wave tile the weight-gradient launch applies Adam itself.
void k_adam_frags(const StepState* st, const AdamJob* jobs, int n_jobs, int total_items,
                  float* p, float* g, float* m, float* v, AdamCfg ac, hipStream_t s);

struct FusedArgs {
  const StepState* st;
  int n_blocks;  // refinement blocks
  // weights: fragment-ordered BF16 (nt / nn) and FP32 biases / affine
  const uint4 *w2_nt, *w2_nn, *wh_nt, *wh_nn;
  const uint4* wab_nt[kMaxFusedBlocks];
  const uint4* wab_nn[kMaxFusedBlocks];
  const uint4* wo_nt[kMaxFusedBlocks];
  const uint4* wo_nn[kMaxFusedBlocks];
  const float *b2, *bh;
  const float* bab[kMaxFusedBlocks];
  const float* bo[kMaxFusedBlocks];
  const float* gamma[kMaxFusedBlocks];
  const float* beta[kMaxFusedBlocks];
  // activations
  const bf16_t* y16;                    // [rows, L] FDM output
  float* hs[kMaxFusedBlocks + 1];       // [rows, F] block inputs / final
  bf16_t* hn16;                         // [rows, F] BF16 copy of the final H
  bf16_t* z16[kMaxFusedBlocks];         // LayerNorm outputs
  float* mean[kMaxFusedBlocks];
  float* rstd[kMaxFusedBlocks];
  float* abr[kMaxFusedBlocks];          // [rows, 2H] branch values
  bf16_t* g16[kMaxFusedBlocks];         // [rows, H] GeLU outputs
  bf16_t* dz16;                         // [rows, 256]
  bf16_t* dh16[kMaxFusedBlocks + 1];    // [rows, F] adjoints of the block inputs
  bf16_t* da16[kMaxFusedBlocks];        // [rows, 2H] adjoints of the branch values
  float* dy;                            // [rows, L] adjoint of the FDM output
  float* loss_rows;
  // column-sum partials of this step: [row block][cols] (bias / affine grads)
  float* colpart;
  int colpart_cols;
  int off_bh, off_b2;
  int off_bo[kMaxFusedBlocks], off_bab[kMaxFusedBlocks], off_beta[kMaxFusedBlocks],
      off_gamma[kMaxFusedBlocks];
  // head / coder
  HeadArgs head;
  StreamIO io;
};

// Row-block kernel before the FDM: context gather (streams) or staged
// contexts, byte embedding, LTE down-projection (Eq. 14).
struct FusedInArgs {
  StepState* st;
  // sched_mode 0: the step state is already set; 1: the kernel sets it for
  // step sched_step, 2: for step st->base + sched_step (steps of a captured
  // window), from the stream lengths in sched
  int sched_mode, sched_step;
  Schedule sched;
  int gather;             // 1: read the contexts from the streams; 0: use ctx / tgt as staged
  int decoding;
  StreamIO io;
  int C, E;
  const float* emb;       // [256, E] FP32 master
  const uint4* w1_nt;
  const float* b1;
  uint8_t* ctx;           // [rows, C]
  uint8_t* tgt;           // [rows]
  bf16_t* x16;            // [rows, F]
  float* x1;              // [rows, L]
};

// Row-block kernel after the FDM adjoint: dX = dX' W1 (adjoint of Eq. 14),
// the embedding gradient of the block as a one-hot product, and the column
// partial of b1.
struct FusedOutArgs {
  const StepState* st;
  int C, E;
  const uint4* w1_nn;
  const bf16_t* dx1_16;   // [rows, L]
  const float* dx1_32;    // [rows, L]
  const uint8_t* ctx;     // [rows, C]
  float* emb_partial;     // [row block][256 * E]
  float* colpart;
  int colpart_cols, off_b1;
};

// F, L, H combinations compiled for the fused path.
bool fused_supported(int F, int L, int H, int branches, int blocks);
hipError_t launch_fused(int F, int L, int H, const FusedArgs& a, int grid_rows, hipStream_t s);
hipError_t launch_fused_in(int F, int L, const FusedInArgs& a, int grid_rows, hipStream_t s);
hipError_t launch_fused_out(int F, int L, const FusedOutArgs& a, int grid_rows, hipStream_t s);

}  // namespace edpc
