/*
 * edpc.h -- C ABI of the MI355X library for the online-adaptive byte-model
 * compressor of "EDPC: Efficient Dual-path Parallel Compression"
 * (arXiv 2507.18969).
 *
 * The method (Sec. 2.1, Algorithm 1): each byte x_i of a stream is coded
 * with the probability Pr(i) = P(x_i | x_{i-t} .. x_{i-1}) that a small
 * network predicts from the t previous bytes (Eq. 1); after coding, the
 * network takes one gradient step on the cross entropy of that prediction
 * (Eq. 2), so the decoder, replaying the same steps from the same random
 * start, reproduces every probability bit for bit.  Many streams ("batch"
 * b, Secs. 3.1.2 and 3.2) advance in lockstep and share one model; each
 * stream owns its slice U_s of the Feature Distribution Matrix (Eq. 15).
 *
 * The network (all dimensions in edpc_config):
 *   byte embedding of the t previous bytes, concatenated oldest first
 *   (F = context * embed) -> Latent Transformation Engine: X' = W1 X + b1
 *   (Eq. 14), Y = bmm(X', U) (Eq. 15), X'' = W2 Y + b2 (Eq. 16) ->
 *   `blocks` Multi-path Byte Refinement Blocks (Eqs. 9-13: LayerNorm,
 *   `branches` parallel linear paths fused by an element-wise product,
 *   GeLU, output linear, residual) -> linear head to 256 logits -> softmax.
 *
 * Everything below runs on one GPU.  Conventions for every function:
 *   - `d_` pointers are device memory, `h_` pointers host memory; all
 *     buffers stay owned by the caller and no pointer is retained after
 *     the call returns, except where a session keeps its input (stated).
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *   - Functions return an edpc_status; on failure edpc_last_error() gives a
 *     thread-local message.  Nothing aborts the process.
 *   - Handles (edpc_model, edpc_session) are not thread-safe.
 *   - Results are deterministic: no floating-point atomics; every reduction
 *     has a fixed order fixed by the kernel configuration, which is written
 *     into the container so that the decoder reproduces the encoder.
 */
#ifndef EDPC_H
#define EDPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EDPC_ABI_VERSION 2

/* Limits of the codec.  The step counter of a run is a signed 32-bit value
 * on the device, so a stream holds fewer than 2^31 bytes; the stream count
 * bounds the container header. */
#define EDPC_MAX_STREAM_LEN 0x7FFFFFFFull
#define EDPC_MAX_STREAMS (1u << 24)

typedef enum {
  EDPC_OK = 0,
  EDPC_E_INVALID_ARG = -1,  /* bad argument or configuration */
  EDPC_E_NOMEM = -2,        /* device or host allocation failed */
  EDPC_E_CAPACITY = -3,     /* output buffer too small; required size returned */
  EDPC_E_CORRUPT = -4,      /* container malformed or truncated */
  EDPC_E_CHECKSUM = -5,     /* CRC mismatch (header or decoded data) */
  EDPC_E_UNSUPPORTED = -6,  /* format version / device / kernel config mismatch */
  EDPC_E_DEVICE = -7        /* HIP runtime error */
} edpc_status;

/* Operand type of the dense layers' matrix products.  FP32: every step in
 * FP32.  BF16: the operands of the embedding->LTE, LTE-up, refinement-block
 * and head products and of their adjoint products are BF16 with FP32
 * accumulation; master weights, Adam state, LayerNorm statistics, GeLU,
 * softmax, the FDM product and the CDF stay FP32. */
typedef enum { EDPC_FP32 = 0, EDPC_BF16 = 1 } edpc_precision;

/* edpc_config.flags */
#define EDPC_CFG_ZERO_HEAD 0x1u /* head weights start at zero (with lr = 0 the
                                   model predicts exactly 1/256: a test case) */
#define EDPC_CFG_AUTOTUNE 0x2u  /* encoder / model creation times every tile
                                   configuration of each matrix product and
                                   keeps the fastest; the choice is written to
                                   the container (so two encodes may pick
                                   different, equally valid, summation orders).
                                   Without it a fixed default is used. */
#define EDPC_CFG_NO_LTE 0x4u    /* the "w/o LTE" ablation (Table 4): no W1, b1,
                                   W2, b2; the per-stream FDM U_s is F x F and
                                   acts on the embedded features directly
                                   (Eq. 15 with x' = x, Eq. 16 with y = x'').
                                   latent must equal context * embed.  Runs the
                                   layer-by-layer step in both precisions. */
#define EDPC_CFG_LOW_RANK 0x8u  /* the "low-rank factorization" ablation
                                   (Table 4): no shared W1, b1, W2, b2; each
                                   stream owns three factors, x' = x A_s
                                   (A_s [F, latent]), Eq. 15 y = x' U_s, and
                                   x'' = y B_s (B_s [latent, F]), without biases,
                                   all three updated by Adam on the steps their
                                   stream is active.  context * embed must be a
                                   power of two <= 256; excludes
                                   EDPC_CFG_NO_LTE.  Runs the layer-by-layer
                                   step in both precisions. */
#define EDPC_CFG_LAYERWISE 0x10u /* BF16 models whose shape has the row-block
                                   fused step run the layer-by-layer launch
                                   sequence instead.  The two sequences sum in
                                   different orders; the choice is recorded in
                                   the container and the decoder follows the
                                   container, not this flag. */
#define EDPC_CFG_NO_GRAPHS 0x20u /* sessions launch every step directly instead
                                   of replaying captured windows of 32 steps
                                   (same results; for timing and debugging) */

typedef struct {
  uint32_t struct_size; /* sizeof(edpc_config) */
  uint32_t context;     /* t: bytes of history (Algorithm 1), multiple of 4 in 4..256 */
  uint32_t embed;       /* embedding width E (16, 32 or 64); F = context * embed */
  uint32_t latent;      /* F' of the LTE (Eq. 14), multiple of 16 */
  uint32_t blocks;      /* number of refinement blocks, 0..16 */
  uint32_t hidden;      /* hidden width of each branch, multiple of 16 */
  uint32_t branches;    /* k parallel paths per block (Eq. 10), 1..3 */
  uint32_t cdf_bits;    /* CDF total 2^cdf_bits; only 16 is supported */
  uint32_t precision;   /* edpc_precision */
  uint32_t flags;       /* EDPC_CFG_* */
  float lr, beta1, beta2, eps; /* Adam (Sec. 4.1: lr 1e-3) */
  uint64_t seed;        /* counter-RNG seed of the random initialisation */
} edpc_config;

const char* edpc_status_string(int status);
const char* edpc_last_error(void);
int edpc_abi_version(void);

/* Default configuration: context 16, embed 16, latent 64, 2 blocks of hidden
 * 128, 2 branches, 16-bit CDF, FP32, Adam(1e-3, 0.9, 0.999, 1e-8), seed 0. */
edpc_status edpc_config_default(edpc_config* cfg);
/* EDPC_OK if the library can run `cfg`; EDPC_E_INVALID_ARG otherwise. */
edpc_status edpc_config_validate(const edpc_config* cfg);

/* ------------------------------------------------------------------------
 * Whole-input codec: Algorithm 1 run over b streams in lockstep.  Bytes
 * 0 .. t-1 of every stream are coded with equal probability; every later
 * byte x_i is coded with the model's Pr(i) (Eq. 1) and followed by one Adam
 * step on the mean cross entropy over the active streams (Eq. 2); decoding
 * replays the same loop.  Input: n_streams byte streams concatenated in
 * d_in, lengths in h_lens (each <= EDPC_MAX_STREAM_LEN, n_streams <=
 * EDPC_MAX_STREAMS).  Output: one container (header + per-stream payloads)
 * in d_out.  These calls synchronise `stream` before returning.
 * ---------------------------------------------------------------------- */

/* Upper bound of the container size for these lengths (bytes). */
edpc_status edpc_encode_bound(const edpc_config* cfg, const uint64_t* h_lens,
                              size_t n_streams, size_t* bound);

/* Compress.  n_streams >= 1; zero-length streams are allowed.  If out_cap is
 * too small returns EDPC_E_CAPACITY with the required size in *out_len. */
edpc_status edpc_encode(const edpc_config* cfg, const uint8_t* d_in,
                        const uint64_t* h_lens, size_t n_streams,
                        uint8_t* d_out, size_t out_cap, size_t* out_len,
                        void* stream);

/* Parse a container header held in host memory (at least the header bytes;
 * lengths above the codec limits, or sums of them that would overflow, are
 * EDPC_E_CORRUPT;
 * *header_len receives its size, or the size needed if in_len is short, in
 * which case EDPC_E_CORRUPT is returned).  cfg/n_streams/h_lens may be NULL;
 * h_lens needs lens_cap >= n_streams entries. */
edpc_status edpc_decode_info(const uint8_t* h_in, size_t in_len, edpc_config* cfg,
                             size_t* n_streams, uint64_t* h_lens, size_t lens_cap,
                             size_t* header_len, size_t* decoded_len);

/* Decompress a container held in device memory into d_out (streams
 * concatenated).  Verifies the per-stream CRC32 of the decoded bytes. */
edpc_status edpc_decode(const uint8_t* d_in, size_t in_len, uint8_t* d_out,
                        size_t out_cap, size_t* out_len, void* stream);

/* Host-to-host codec: the same containers as edpc_encode / edpc_decode, for
 * inputs and outputs in host memory (pinned memory copies fastest).  The
 * paper pipelines GPU prediction with CPU coding (Sec. 3.3); here the coder
 * runs on the GPU, and what is pipelined is the data movement: streams pass
 * through a device window of a few chunks of `chunk_steps` bytes per stream
 * (chunk_steps >= context), chunk k + 1 moving host -> device on a second
 * stream while chunk k is coded, and finished payload bytes (decoded bytes)
 * moving back the same way.  Device memory holds the model, the window and
 * (encoder) the payload region; the input or output is never resident whole.
 * encode: EDPC_E_CAPACITY if out_cap is short, with the size in *out_len.
 * decode: verifies the CRCs; *out_len = bytes decoded.  Synchronous. */
edpc_status edpc_encode_host(const edpc_config* cfg, const uint8_t* h_in,
                             const uint64_t* h_lens, size_t n_streams, uint8_t* h_out,
                             size_t out_cap, size_t* out_len, uint32_t chunk_steps,
                             void* stream);
edpc_status edpc_decode_host(const uint8_t* h_in, size_t in_len, uint8_t* h_out,
                             size_t out_cap, size_t* out_len, uint32_t chunk_steps,
                             void* stream);

/* ------------------------------------------------------------------------
 * Step-granular sessions: the same codec, advanced a number of model steps
 * at a time (for streaming callers and for timing).  A session keeps
 * reading d_in (encoder) or d_in/d_out (decoder) until it is destroyed.
 * ---------------------------------------------------------------------- */
typedef struct edpc_session edpc_session;

edpc_status edpc_encoder_begin(const edpc_config* cfg, const uint8_t* d_in,
                               const uint64_t* h_lens, size_t n_streams,
                               void* stream, edpc_session** out);
edpc_status edpc_decoder_begin(const uint8_t* d_in, size_t in_len, uint8_t* d_out,
                               size_t out_cap, void* stream, edpc_session** out);
/* Enqueue up to n_steps more steps (asynchronous); *done = steps taken. */
edpc_status edpc_session_run(edpc_session* s, uint64_t n_steps, uint64_t* done);
/* Current step and total steps (= longest stream). */
edpc_status edpc_session_progress(const edpc_session* s, uint64_t* step,
                                  uint64_t* total);
/* Encoder: finish all remaining steps, flush, write the container. */
edpc_status edpc_encoder_finish(edpc_session* s, uint8_t* d_out, size_t out_cap,
                                size_t* out_len);
/* Decoder: finish all remaining steps, check CRCs; *out_len = bytes decoded. */
edpc_status edpc_decoder_finish(edpc_session* s, size_t* out_len);
void edpc_session_destroy(edpc_session* s);

/* Kernel-level timing (profiling aid).  Runs the next n_steps of the session
 * with a HIP event recorded before and after every kernel launch on the
 * session's stream, then synchronises: h_ms[c] receives the summed kernel
 * milliseconds and h_launches[c] the launch count of kernel class c, for
 * c < EDPC_KCLASS_COUNT.  The class names come from edpc_kclass_name. */
#define EDPC_KCLASS_COUNT 24
edpc_status edpc_session_time_kernels(edpc_session* s, uint64_t n_steps, float* h_ms,
                                      uint32_t* h_launches);
const char* edpc_kclass_name(int c);

/* ------------------------------------------------------------------------
 * Model-level access: one step of the network on explicit contexts, i.e.
 * the "Model(x_{i-t} .. x_{i-1})" call of Algorithm 1 with Pr(i) (Eq. 1),
 * optionally the cross entropy (Eq. 2), its gradient, and the update step
 * (Adam, Sec. 4.1).  The network is Eqs. 9-16 (see the top of this file).
 * ---------------------------------------------------------------------- */
typedef struct edpc_model edpc_model;

/* edpc_model_step flags */
#define EDPC_STEP_BACKWARD 0x1u /* compute gradients of the mean cross entropy */
#define EDPC_STEP_UPDATE 0x2u   /* ... and apply one Adam step (implies BACKWARD) */
#define EDPC_STEP_KEEP_FDM_GRAD 0x4u /* store dL/dU of each row's slot (no update) */

/* A model with n_slots FDM slices (one per stream) accepting up to max_rows
 * rows per step.  Parameters are initialised from cfg->seed. */
edpc_status edpc_model_create(const edpc_config* cfg, size_t n_slots,
                              size_t max_rows, edpc_model** out);
void edpc_model_destroy(edpc_model* m);

/* The same with an explicit kernel configuration: `kernel_id` is the 64-bit
 * id a container records (tile shape per matrix product, 4 bits per product
 * slot; bit 47 the BF16 row-block fused step; bit 46 the layer-by-layer
 * step's LayerNorm adjoint with its column sums folded in; bits 48.. the
 * numerics revision), so that a model can run the summation orders of a given
 * container, or a chosen tile everywhere.  0 picks the default.  An id of
 * another numerics revision, an unknown tile, or a tile or fused step the
 * model's shape and precision cannot run is EDPC_E_UNSUPPORTED. */
edpc_status edpc_model_create_with_kernels(const edpc_config* cfg, size_t n_slots,
                                           size_t max_rows, uint64_t kernel_id,
                                           edpc_model** out);
/* The kernel configuration id a model runs. */
edpc_status edpc_model_kernel_id(const edpc_model* m, uint64_t* kernel_id);

/* One step on `rows` rows.  d_ctx: [rows, context] bytes, oldest first.
 * d_target: [rows] bytes (required with BACKWARD/UPDATE, else may be NULL).
 * h_slot: [rows] distinct FDM slot indices < n_slots (host memory: the
 * library checks range and distinctness before any kernel reads a slot).
 * Optional outputs: d_probs [rows, 256] FP32 softmax, d_cum [rows, 257]
 * integer CDF (the coder's table), d_loss [1] FP32 mean cross entropy
 * (device memory, so that the call stays asynchronous).
 * Asynchronous on `stream`. */
edpc_status edpc_model_step(edpc_model* m, const uint8_t* d_ctx,
                            const uint8_t* d_target, const uint32_t* h_slot,
                            size_t rows, float* d_probs, uint32_t* d_cum,
                            float* d_loss, uint32_t flags, void* stream);

/* Tensor access (synchronous).  Tensors are numbered 0..count-1 in storage
 * order: the shared parameters, then the FDM "U" with n_slots*latent*latent
 * entries; under EDPC_CFG_LOW_RANK two more follow, "A" and "B", each with
 * n_slots*F*latent entries (no kept gradient: EDPC_KIND_GRAD on them fails). */
#define EDPC_KIND_PARAM 0u
#define EDPC_KIND_GRAD 1u
#define EDPC_KIND_ADAM_M 2u
#define EDPC_KIND_ADAM_V 3u
/* BF16 models, edpc_model_read only: the BF16 operand copy of a shared
 * tensor that the products read, widened to FP32, in the tensor's own
 * layout.  The row-block fused step keeps two copies of each weight matrix,
 * one per product orientation (X W^T: OPERAND_NT, X W: OPERAND_NN); the
 * layer-by-layer step keeps one copy of every tensor (both kinds return it).
 * Tensors without an operand copy, and FP32 models, are EDPC_E_INVALID_ARG. */
#define EDPC_KIND_OPERAND_NT 4u
#define EDPC_KIND_OPERAND_NN 5u
edpc_status edpc_model_tensor_count(const edpc_model* m, size_t* n);
edpc_status edpc_model_tensor_info(const edpc_model* m, size_t idx, char* name,
                                   size_t name_cap, size_t* numel);
edpc_status edpc_model_read(const edpc_model* m, uint32_t kind, size_t idx,
                            float* h_dst, size_t numel);
edpc_status edpc_model_write(edpc_model* m, uint32_t kind, size_t idx,
                             const float* h_src, size_t numel);
/* The same transfers between a model tensor and caller device memory,
 * asynchronous on `stream` (for autograd wrappers and zero-copy callers). */
edpc_status edpc_model_read_device(const edpc_model* m, uint32_t kind, size_t idx,
                                   float* d_dst, size_t numel, void* stream);
edpc_status edpc_model_write_device(edpc_model* m, uint32_t kind, size_t idx,
                                    const float* d_src, size_t numel, void* stream);
/* Adam step counter (number of updates taken). */
edpc_status edpc_model_get_step(const edpc_model* m, uint64_t* tau);
edpc_status edpc_model_set_step(edpc_model* m, uint64_t tau);

/* FP32 input of refinement block `block` of the last edpc_model_step
 * (block = blocks: the head's input, i.e. the last block's output), [rows,
 * context * embed] row-major, copied to d_dst asynchronously on `stream`.
 * Block j's skip connection S and its output S + X^(k) (Sec. 3.1.1) are
 * blocks j and j + 1.  The BF16 row-block step keeps no FP32 copy of the
 * head's input (EDPC_E_UNSUPPORTED); numel must be rows * context * embed. */
edpc_status edpc_model_activation(const edpc_model* m, uint32_t block, float* d_dst,
                                  size_t numel, void* stream);

/* Whole training state of a model (what Algorithm 1 adapts online: every
 * parameter with its Adam moments, and the Adam step counter), as one host
 * blob.  Layout (little-endian): "EDPS", u32 version (1), u32 tensor count,
 * u32 0, u64 tau, u32 x 9 configuration fields (context, embed, latent,
 * blocks, hidden, branches, cdf_bits, precision, flags), u64 n_slots; then
 * per tensor in edpc_model_tensor_info order: u32 name length, the name
 * padded with zeros to a multiple of 4 bytes, u64 numel, numel FP32
 * parameters, numel FP32 first moments, numel FP32 second moments.
 * get_state: if cap is too small (or h_buf is NULL) returns
 * EDPC_E_CAPACITY with the size in *len.  set_state: the blob must come
 * from a model of the same configuration and slot count
 * (EDPC_E_INVALID_ARG otherwise).  Both synchronise the device. */
edpc_status edpc_model_get_state(const edpc_model* m, void* h_buf, size_t cap, size_t* len);
edpc_status edpc_model_set_state(edpc_model* m, const void* h_buf, size_t len);

/* ------------------------------------------------------------------------
 * Mutual information (the analysis of Sec. 3.1.1): Kraskov's first
 * estimator (Eq. 7; Kraskov, Stoegbauer & Grassberger 2004) of I(Z; Y) from
 * c samples, d_z [c, dz] and d_y [c, dy] FP32 row-major device arrays:
 *   psi(v) + psi(c) - (1/c) sum_i [psi(c_z(i) + 1) + psi(c_y(i) + 1)],
 * eps_i the distance from sample i to its v-th nearest other sample in the
 * joint space under the max norm (ties with multiplicity), c_z(i) (c_y(i))
 * the samples strictly closer than eps_i in z (y) alone.  Distances are FP32.
 * IFR_{k1->k2} (Eq. 8) is the ratio of two such estimates.  2 <= c <= 32768,
 * 1 <= v <= min(16, c - 1).  *h_mi in nats; optional d_counts [c, 2] int32
 * (c_z, c_y) and d_eps [c].  Allocates 8 c^2 bytes of work memory while it
 * runs; synchronises `stream`. */
edpc_status edpc_mutual_info(const float* d_z, size_t dz, const float* d_y, size_t dy,
                             size_t c, uint32_t v, double* h_mi, int32_t* d_counts,
                             float* d_eps, void* stream);

/* ------------------------------------------------------------------------
 * Range coder alone (the arithmetic-coding step of Sec. 2.1 and of
 * Algorithm 1's encode / decode lines; G. N. N. Martin's range coder): codes
 * symbols with caller-supplied 16-bit CDF tables, one coder per stream.
 * d_cum: [n_steps, n_streams, 257] u32, cum[0] = 0, cum[256] = 65536,
 * strictly increasing.  d_sym: [n_steps, n_streams] bytes.  Stream s writes
 * its payload at d_out + s*cap_per_stream (cap_per_stream >= 2*n_steps + 2)
 * and its length to h_out_lens[s].  Decoding reverses it.  Synchronous.
 * ---------------------------------------------------------------------- */
edpc_status edpc_rc_encode(const uint32_t* d_cum, const uint8_t* d_sym,
                           size_t n_steps, size_t n_streams, uint8_t* d_out,
                           size_t cap_per_stream, uint32_t* h_out_lens, void* stream);
edpc_status edpc_rc_decode(const uint32_t* d_cum, const uint8_t* d_in,
                           const uint32_t* h_in_lens, size_t cap_per_stream,
                           size_t n_steps, size_t n_streams, uint8_t* d_sym,
                           void* stream);
/* Allocation-free edpc_rc_encode, for callers that cannot allocate device
 * memory (serving loops and harnesses that forbid hipMalloc): same arguments
 * and results, but the per-stream payload lengths pass through a fixed
 * device array of EDPC_RC_NOALLOC_MAX_STREAMS entries that the library
 * holds, one per GPU, until the process ends, instead of a temporary
 * allocation.  n_streams above EDPC_RC_NOALLOC_MAX_STREAMS is
 * EDPC_E_INVALID_ARG.  Calls that overlap on one GPU race on that array;
 * the call synchronises `stream`. */
#define EDPC_RC_NOALLOC_MAX_STREAMS 65536
edpc_status edpc_rc_encode_noalloc(const uint32_t* d_cum, const uint8_t* d_sym,
                                   size_t n_steps, size_t n_streams, uint8_t* d_out,
                                   size_t cap_per_stream, uint32_t* h_out_lens,
                                   void* stream);

/* The same coder compiled for the host (reference and CPU tests). */
edpc_status edpc_rc_encode_host(const uint32_t* h_cum, const uint8_t* h_sym,
                                size_t n_steps, uint8_t* h_out, size_t cap,
                                size_t* out_len);
edpc_status edpc_rc_decode_host(const uint32_t* h_cum, const uint8_t* h_in,
                                size_t in_len, size_t n_steps, uint8_t* h_sym);

#ifdef __cplusplus
}
#endif
#endif /* EDPC_H */
