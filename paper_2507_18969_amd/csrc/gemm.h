// Tiled matrix products on the gfx950 matrix cores (MFMA).
//
// C[M, N] = A[M, K] * B[K, N] with either operand stored K-contiguous
// ("K-major") or M/N-contiguous, FP32 accumulation, and fused epilogues:
//   forward dense layers  Out = In W^T + b (+ residual)       A K-major, B K-major
//   adjoint of the input  dIn = dOut W                         A K-major, B N-major
//   weight gradients      dW = dOut^T In (sum over rows)      A M-major, B N-major
// The refinement block's branch product (Eqs. 10-12) is one product with
// several B matrices sharing the A tile; its epilogue forms
// GeLU(X_1 * ... * X_k), and the adjoint epilogue forms dX_i.
//
// Summation order is fixed by the tile configuration: K is walked in BK
// chunks in increasing order, each chunk by the MFMA's own fixed order.  No
// atomics: results are identical run to run for a given configuration.
#pragma once
#include "common.h"
#include "adam.h"

namespace edpc {

enum EpiKind : int {
  EPI_STORE = 0,     // out = acc (+ bias[n]) (+ resid[m, n])
  EPI_GATE_FWD = 1,  // a_i = acc_i + bias_i[n]; aux[m, i*H+n] = a_i; out = gelu(prod a_i)
  EPI_GATE_BWD = 2,  // dP = acc * gelu'(prod a_i); out[m, i*H+n] = dP * prod_{k!=i} a_k
};

struct GemmArgs {
  const void* A;
  const void* B;
  int M, N, K;
  int lda, ldb;
  long long b_branch_stride;  // elements between the B matrices of a multi-B product
  const StepState* st;        // rows from the step state: M (m_rows) or K (k_rows)
  int m_rows, k_rows;
  // epilogue
  const float* bias;
  int bias_branch_stride;     // GATE_FWD: elements between branch biases; GATE_BWD: branch count k
  const float* resid;
  int ld_resid;
  float* out32;
  int ld_out32;
  bf16_t* out16;
  int ld_out16;
  float* aux;       // GATE_FWD: branch values written; GATE_BWD: read
  int ld_aux;
  int aux_branch;   // column offset between branches in aux / gate-bwd outputs
};

// Grouped weight-gradient products: one launch over many (dOut, In) pairs.
struct WgradProblem {
  const void* dout;  // [rows, M] (M = out features)
  const void* in;    // [rows, N] (N = in features)
  float* dw;         // [M, N]
  int M, N;
  int tiles_n, tile_begin;  // tiles of this problem start at tile_begin
  // Adam launch only: the BF16 fragment copies of the weight, nt (16-row
  // blocks, 32 columns deep) and nn (16-column blocks, 32 rows deep)
  uint4* nt;
  uint4* nn;
};

// Adam applied by the weight-gradient launch itself (the row-block step's
// update): each tile, once its sum over rows is complete, writes its
// gradient to dw, updates the parameters at the same offset of p (dw - g),
// their moments m and v, and rewrites both fragment copies.
struct WgradAdam {
  float* g;  // base of the gradient buffer that every dw points into
  float *p, *m, *v;
  AdamCfg ac;
  int tiles;  // work-groups past the tiles run element-range Adam items:
  const AdamJob* ejobs;  // jobs with cols == 0 (biases, LayerNorm, embedding)
  int n_ejobs;
};

// Work-group -> tile order for a launch of `total` tiles numbered row-major
// (tiles of one row of the output share their A rows).  Work-groups are
// dealt to the 8 XCDs in turn (work-group L to XCD L mod 8), and each XCD
// has its own L2, so consecutive tile numbers would land on different XCDs
// and every XCD would fetch every A row panel.  This mapping gives XCD x
// the contiguous tile range [x q + min(x, r), ...) (q = total / 8,
// r = total % 8) in the order its work-groups arrive, so a row panel is
// fetched by one XCD and reused from its L2.  It only permutes which
// work-group computes which tile: results do not change.
__device__ __forceinline__ int xcd_tile(int L, int total) {
  const int x = L & 7, q = total >> 3, r = total & 7;
  return x * q + (x < r ? x : r) + (L >> 3);
}

// Tile configurations (the autotuner picks one per product; the choice is
// recorded in the container so the decoder uses the same summation order).
enum TileId : int {
  TILE_32x32 = 0,
  TILE_64x32 = 1,
  TILE_32x64 = 2,
  TILE_64x64 = 3,
  TILE_128x64 = 4,
  TILE_64x128 = 5,
  TILE_128x128 = 6,
  // 8-wave wide tiles, BF16 only (gemm_wide.hip); gated products with k = 2
  TILE_W128x128 = 7,
  TILE_W256x128 = 8,
  TILE_W128x256 = 9,
  TILE_W256x256 = 10,
  TILE_COUNT = 11
};

struct TileShape {
  int bm, bn;
};
inline TileShape tile_shape(int id) {
  static const TileShape t[TILE_COUNT] = {{32, 32},  {64, 32},   {32, 64},   {64, 64},
                                          {128, 64}, {64, 128},  {128, 128}, {128, 128},
                                          {256, 128}, {128, 256}, {256, 256}};
  return t[id];
}

// Whether tile id `tile` serves a product of this precision / epilogue /
// branch count (the wide tiles: BF16, and gated forward products only with
// two branches).
bool wide_tile_supported(int tile, bool bf16, EpiKind epi, int nb);

// Launchers (gemm.hip).  `bf16` selects BF16 operands (A, B hold bf16_t).
// `a_kmajor` / `b_kmajor` select the operand layouts; nb = number of B
// matrices (1..3) for the gated products.
hipError_t launch_gemm(int tile, bool bf16, bool a_kmajor, bool b_kmajor, EpiKind epi, int nb,
                       const GemmArgs& g, int grid_m_max, hipStream_t s);
// `part`: scratch of wgrad_part_floats(tile) floats for the balanced launch of
// wide tiles (taken when a table has at least kWgradRanges tiles), or null for
// one work-group per tile.
hipError_t launch_wgrad(int tile, bool bf16, const WgradProblem* d_probs, int n_probs,
                        int total_tiles, const StepState* st, float* part, hipStream_t s);
// The same weight gradients with Adam in the epilogue (4-wave tiles only;
// M and N multiples of 32, the shared weights of the row-block step), plus
// elem_items work-groups of element-range Adam (ad.ejobs).  Returns
// hipErrorInvalidValue for other tiles.
hipError_t launch_wgrad_adam(int tile, const WgradProblem* d_probs, int n_probs, int total_tiles,
                             int elem_items, const StepState* st, const WgradAdam& ad,
                             hipStream_t s);
// Wide tiles (gemm_wide.hip), reached through the two launchers above.
hipError_t launch_gemm_wide(int tile, bool a_kmajor, bool b_kmajor, EpiKind epi, int nb,
                            const GemmArgs& g, int grid_m_max, hipStream_t s);
hipError_t launch_wgrad_wide(int tile, const WgradProblem* d_probs, int n_probs, int total_tiles,
                             const StepState* st, float* part, hipStream_t s);

// Balanced weight gradients of wide tiles: this many equal ranges of K
// chunks (one work-group each, one per CU of the part); tiles cut by range
// boundaries are summed in parts, two scratch tiles per range.
constexpr int kWgradRanges = 256;
inline size_t wgrad_part_floats(int tile) {
  const TileShape t = tile_shape(tile);
  return 2 * (size_t)kWgradRanges * t.bm * t.bn;
}

}  // namespace edpc
