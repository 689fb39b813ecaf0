// Row-wise and element-wise kernels of one model step, and the coder lanes.
#pragma once
#include "common.h"
#include "rangecoder.h"

namespace edpc {

// Schedule of a multi-stream run: streams sorted by decreasing length so
// that the active streams at step i are rows 0 .. rows(i)-1.
struct Schedule {
  const int64_t* lens_sorted;  // [n] decreasing
  int n;
  int context;
  float beta1, beta2;
};

// Where each row's bytes live in a multi-stream run.
struct StreamIO {
  const uint32_t* slot;       // row -> stream index (original order)
  const uint8_t* src;         // encoder input (concatenated streams)
  uint8_t* dst;               // decoder output (concatenated streams)
  const uint64_t* off;        // stream -> offset in src / dst
  const uint64_t* lens;       // stream -> length
  uint8_t* pay;               // encoder payload region base
  const uint8_t* pay_in;      // decoder payload base
  const uint64_t* pay_off;    // stream -> payload offset
  const uint64_t* pay_cap;    // stream -> payload capacity (encoder) / length (decoder)
  RcEnc* enc;                 // [n_streams]
  RcDec* dec;                 // [n_streams]
  uint32_t ring;              // 0: a stream's bytes are contiguous from off[s];
                              // else each stream has a window of `ring` bytes
                              // and position p lives at off[s] + p % ring
};

// Address of position p of the stream whose bytes start at `off`.
__device__ __forceinline__ uint64_t io_at(const StreamIO& io, uint64_t off, uint64_t p) {
  return off + (io.ring ? (uint64_t)((uint32_t)p % io.ring) : p);
}

struct HeadArgs {
  const float* logits;  // [rows, 256]
  const uint8_t* target;  // [rows] (encode / plain step)
  uint8_t* target_out;    // decoded symbol per row (decode)
  float* dz32;            // [rows, 256]
  bf16_t* dz16;
  float* loss_rows;       // [rows]
  float* probs;           // optional [rows, 256]
  uint32_t* cum_out;      // optional [rows, 257]
  int mode;               // 0 plain step, 1 encode, 2 decode
  int want_grad;
};

// Number of streams longer than `step`, the active rows of that step (Alg. 1:
// a stream takes part while it has bytes left).  A blockDim.x-way search of
// the decreasing lengths; every thread of the workgroup must call it, and each
// gets the count.
__device__ inline int active_rows(const Schedule& sc, int step) {
  const int64_t nt = blockDim.x, t = threadIdx.x;
  int64_t lo = 0, hi = sc.n;  // the count lies in [lo, hi]
  while (lo < hi) {
    const int64_t chunk = (hi - lo + nt - 1) / nt;
    const int64_t i = lo + t * chunk;
    const int c = __syncthreads_count(i < hi && sc.lens_sorted[i] > (int64_t)step);
    const int64_t nlo = c == 0 ? lo : lo + (c - 1) * chunk + 1;
    hi = min(lo + c * chunk, hi);
    lo = nlo;
  }
  return (int)lo;
}

// The step state of step `step` with `rows` active rows (one thread writes).
__device__ inline void write_step_state(StepState* st, const Schedule& sc, int step, int rows) {
  st->step = step;
  st->rows = rows;
  st->inv_rows = rows > 0 ? 1.0f / (float)rows : 0.0f;
  st->model = step >= sc.context ? 1 : 0;
  const uint32_t tau = step >= sc.context ? (uint32_t)(step - sc.context + 1) : 0u;
  st->tau = tau;
  st->bc1 = adam_bias_correction(sc.beta1, tau);
  st->bc2 = adam_bias_correction(sc.beta2, tau);
}

// step >= 0: state for that step; step < 0: the step after st->step.
void k_step_schedule(StepState* st, Schedule sc, int step, hipStream_t s);
// st->step = st->base = step (the step before a window of relative steps)
void k_step_set(StepState* st, int step, hipStream_t s);
void k_step_explicit(StepState* st, int rows, uint32_t tau, float beta1, float beta2, hipStream_t s);

void k_gather(const StepState* st, StreamIO io, int C, uint8_t* ctx, uint8_t* tgt, int max_rows,
              bool decoding, hipStream_t s);
void k_embed(const StepState* st, const uint8_t* ctx, const float* emb, int C, int E, float* x32,
             bf16_t* x16, int max_rows, hipStream_t s);
// Per-stream [Lin, Lout] matrix: Lin <= 256, Lout a power of two in 4..256.
void k_fdm_fwd(const StepState* st, const float* x1, const float* U, const uint32_t* slot, int Lin,
               int Lout, float* y32, bf16_t* y16, int max_rows, hipStream_t s);
void k_fdm_bwd(const StepState* st, const float* x1, const float* dy, float* U, float* mU,
               float* vU, float* dU_keep, const uint32_t* slot, int Lin, int Lout, AdamCfg ac,
               bool update, float* dx1_32, bf16_t* dx1_16, int max_rows, hipStream_t s);
void k_ln_fwd(const StepState* st, const float* h, const float* gamma, const float* beta, int F,
              float* z32, bf16_t* z16, float* mean, float* rstd, int max_rows, hipStream_t s);
// LayerNorm adjoint (Eq. 9) plus the residual adjoint dh_next.  With `part`
// (only where ln_bwd_folds(F)) it also forms, per group of kLnFoldRows rows in
// row order, the column sums of the block's LayerNorm affine gradients and of
// dh_next (the gradient of the output bias of the block before): part[group]
// holds [beta | gamma | dh_next] sums, 3F floats.
constexpr int kLnFoldRows = 16;
bool ln_bwd_folds(int F);
size_t ln_fold_part_elems(int max_rows, int F);
void k_ln_bwd(const StepState* st, const float* h, const float* mean, const float* rstd,
              const float* gamma, const float* dz, const float* dh_next, int F, float* dh32,
              bf16_t* dh16, float* part, int max_rows, hipStream_t s);
void k_head(const StepState* st, HeadArgs a, StreamIO io, int max_rows, hipStream_t s);

// Column sums over the active rows (bias and LayerNorm gradients, loss).
struct ColsumJob {
  const float* src;    // [rows, cols] with leading dimension ld
  const float* h;      // LN gamma jobs: the block input; xhat = (h - mean) * rstd
  const float* mean;
  const float* rstd;
  float* dst;          // [cols]
  int cols, ld;
  int col_block_begin; // first 64-column block of this job
  int col_offset;      // first column of this job in the partial buffer
  float scale;         // 0: scale by 1/rows
  // sums formed elsewhere (the LayerNorm adjoint's row groups): the job's
  // column c is the in-order sum of part[k * part_ld + c] over the
  // ceil(rows / part_rows) groups, and the first pass skips the job (such
  // jobs follow the others, with col_block_begin past the first pass's grid)
  const float* part;
  int part_ld, part_rows;
};
size_t colsum_partial_elems(int max_rows, int total_cols);
void k_colsum(const StepState* st, const ColsumJob* jobs, int n_jobs, int total_blocks,
              int total_cols, float* partial, int max_rows, hipStream_t s);

// Second pass only: partial[k][col] over chunks of chunk_rows rows.
void k_colsum_reduce(const StepState* st, const ColsumJob* jobs, int n_jobs, int total_cols,
                     const float* partial, int chunk_rows, hipStream_t s);

// Second pass of the embedding gradient: partial[chunk][256*E] over chunks of chunk_rows.
void k_emb_grad_reduce(const StepState* st, const float* partial, int chunk_rows, int E,
                       float* demb, hipStream_t s);

void emb_grad_plan(int max_rows, int C, int E, int* chunk_rows, int* sub_rows);
void k_emb_grad(const StepState* st, const uint8_t* ctx, const float* dx, int C, int E,
                float* partial, int chunk_rows, int sub_rows, int max_rows, float* demb,
                hipStream_t s);
void k_adam(const StepState* st, float* p, const float* g, float* m, float* v, bf16_t* p16,
            size_t n, AdamCfg ac, hipStream_t s);

// Counter-based initialisation: dst[j] = fl32(a_j * bound), a_j from
// SplitMix64(seed + (tid << 40) + start + j).
void k_init_uniform(float* dst, size_t n, uint64_t seed, uint32_t tid, uint64_t start, float bound,
                    hipStream_t s);
void k_fill(float* dst, size_t n, float v, hipStream_t s);
void k_to_bf16(const float* src, bf16_t* dst, size_t n, hipStream_t s);

// Coder lanes.
void k_uniform_prefix(StreamIO io, int n_streams, int C, bool decoding, hipStream_t s);
void k_rc_finish(StreamIO io, int n_streams, hipStream_t s);
void k_rc_table_encode(const uint32_t* cum, const uint8_t* sym, size_t n_steps, size_t n_streams,
                       uint8_t* out, size_t cap, uint64_t* out_lens, hipStream_t s);
void k_rc_table_decode(const uint32_t* cum, const uint8_t* in, const uint64_t* in_lens, size_t cap,
                       size_t n_steps, size_t n_streams, uint8_t* sym, hipStream_t s);
void k_crc32(const uint8_t* data, const uint64_t* off, const uint64_t* lens, int n, uint32_t* crc,
             hipStream_t s);
void k_gather_payloads(const uint8_t* pay, const uint64_t* pay_off, const uint64_t* len,
                       const uint64_t* dst_off, uint8_t* dst, int n, hipStream_t s);

// Streaming encoder: per stream, move the payload bytes that no later carry
// can change (all written bytes if `all`) from the payload region to
// out + s * stride, at most `stride` bytes past done[s]; out_len[s] gets the
// count and done[s] advances by it.
void k_pay_drain(const RcEnc* enc, const uint8_t* pay, const uint64_t* pay_off, uint64_t* done,
                 int n, bool all, uint8_t* out, uint32_t stride, uint32_t* out_len, hipStream_t s);

}  // namespace edpc
