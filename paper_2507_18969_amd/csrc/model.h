// The model object: parameters, Adam state, per-stream FDM slices,
// activation workspace, and the launch sequence of one step.
#pragma once
#include <string>
#include <vector>

#include "../../include/edpc.h"
#include "fused.h"
#include "gemm.h"
#include "kernels.h"

namespace edpc {

// Kraskov mutual-information estimate (ksg.hip); see edpc_mutual_info.
double mutual_info(const float* d_z, size_t dz, const float* d_y, size_t dy, size_t c, uint32_t v,
                   int32_t* d_counts, float* d_eps, hipStream_t s);

// Thrown inside the library, turned into an edpc_status at the C boundary.
struct Error {
  edpc_status status;
  std::string msg;
};
[[noreturn]] void fail(edpc_status st, const std::string& msg);
void hip_check(hipError_t e, const char* what);

// Product slots that carry their own tile configuration.
enum ProductSlot : int {
  PS_LTE_DOWN = 0,
  PS_LTE_UP,
  PS_GATE,
  PS_OUT,
  PS_HEAD,
  PS_HEAD_BWD,
  PS_GATE_BWD,
  PS_DZ,
  PS_LTE_UP_BWD,
  PS_LTE_DOWN_BWD,
  PS_WGRAD,
  PS_COUNT
};

// Kernel configuration: one tile id per product slot, plus the numerics
// revision of the kernels.  Encoded into 64 bits for the container.
constexpr uint32_t kNumericsRevision = 7;
struct KernelConfig {
  int tile[PS_COUNT];
  bool fused = false;  // BF16 row-block fused step (bit 47 of the id)
  bool ln_fold = false;  // layer-by-layer step: LayerNorm adjoint with its column sums (bit 46)
  uint64_t encode() const;
  static bool decode(uint64_t id, KernelConfig* out);
};

struct TensorInfo {
  std::string name;
  size_t off;    // element offset in the flat shared buffers
  size_t numel;
  uint32_t tid;  // counter-RNG tensor id (0: constant)
  float bound;   // RNG bound or constant value
};

// Kernel classes for per-kernel timing: the product slots, then the rest.
enum KClass : int {
  KC_SCHEDULE = PS_COUNT,
  KC_GATHER,
  KC_EMBED,
  KC_FDM_FWD,
  KC_LN_FWD,
  KC_HEAD,
  KC_LN_BWD,
  KC_FDM_BWD,
  KC_EMB_GRAD,
  KC_COLSUM,
  KC_ADAM,
  KC_FUSED,
  KC_FRAGS,
  KC_COUNT
};
static_assert(KC_COUNT == EDPC_KCLASS_COUNT, "kernel class count");
const char* kclass_name(int c);

// HIP events around every launch (profiling aid; off unless installed).
struct KTimer {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Span { int cls; hipEvent_t a, b; };
  std::vector<Span> spans;
  int cur = -1;
  hipEvent_t cur_ev = nullptr;
  void begin(int cls, hipStream_t s);
  void end(hipStream_t s);
  void collect(float* ms, uint32_t* launches);
  ~KTimer();
};

enum StepMode : int { MODE_PLAIN = 0, MODE_ENCODE = 1, MODE_DECODE = 2 };

// Step state to be set inside the step: mode 1 for step `step`, mode 2 for
// step st->base + step.
struct StepSched {
  Schedule sc;
  int mode;
  int step;
};

struct StepOutputs {
  float* probs = nullptr;
  uint32_t* cum = nullptr;
  float* loss = nullptr;
  bool backward = false;
  bool update = false;
  bool keep_fdm_grad = false;
  bool has_target = true;  // plain steps: targets staged in tgt
};

struct Model {
  edpc_config cfg;
  int C, E, F, L, N, H, K;
  bool bf16;
  bool lte = true;  // false: no shared W1, b1, W2, b2 (EDPC_CFG_NO_LTE or EDPC_CFG_LOW_RANK)
  bool low_rank = false;  // per-stream factors A_s, U_s, B_s (EDPC_CFG_LOW_RANK)
  size_t n_slots, max_rows;
  KernelConfig kc;
  std::vector<TensorInfo> tens;
  size_t P = 0;  // shared parameter count (with alignment padding)
  uint64_t tau = 0;
  int last_rows = 0;  // rows of the last step (activation read-back)

  // device state
  float *param = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  bf16_t* p16 = nullptr;
  float *U = nullptr, *mU = nullptr, *vU = nullptr, *dUkeep = nullptr;
  // low-rank ablation: A [n_slots, F, L] and B [n_slots, L, F] with Adam moments
  float *A = nullptr, *mA = nullptr, *vA = nullptr, *B = nullptr, *mB = nullptr, *vB = nullptr;
  StepState* st = nullptr;

  // workspace
  uint8_t *ctx = nullptr, *tgt = nullptr;
  uint32_t* slot = nullptr;
  float* X32 = nullptr;
  bf16_t* X16 = nullptr;
  float* X1 = nullptr;
  float* Y32 = nullptr;
  bf16_t* Y16 = nullptr;
  std::vector<float*> Hs;
  bf16_t* HN16 = nullptr;
  std::vector<float*> Z32, mean, rstd, Abr, G32, dA32, dZ, dH32;
  std::vector<bf16_t*> Z16, G16, dA16, dH16;
  float *logits = nullptr, *dz32 = nullptr, *loss_rows = nullptr, *loss_out = nullptr;
  bf16_t* dz16 = nullptr;
  float *dY = nullptr, *dX1_32 = nullptr, *dX = nullptr, *emb_partial = nullptr;
  bf16_t* dX1_16 = nullptr;
  struct WgTable {
    WgradProblem* d = nullptr;
    int n = 0, tiles = 0;
    std::vector<WgradProblem> host;
    WgradProblem* d_adam = nullptr;  // row-block step: the same with fragment copies (Adam launch)
  } wg_tab[TILE_COUNT];
  float* wg_part = nullptr;  // scratch of the balanced wide-tile weight-gradient launch
  size_t wg_part_floats = 0;
  ColsumJob* d_cs = nullptr;
  int n_cs = 0, cs_blocks = 0, cs_cols = 0;
  float* cs_partial = nullptr;
  std::vector<float*> ln_part;  // LayerNorm adjoint's row-group column sums, per block (or empty)
  ColsumJob* d_loss_job = nullptr;
  float* loss_partial = nullptr;
  int emb_chunk = 16, emb_sub = 16;
  KTimer* timer = nullptr;
  // fused BF16 path: fragment-ordered weight copies and column-sum partials
  uint4* frags = nullptr;
  FragJob* d_frag_jobs = nullptr;
  int n_frag_jobs = 0, total_frags = 0;
  FusedArgs fa;
  FusedInArgs fin{};
  FusedOutArgs fout;
  float* fused_emb_partial = nullptr;
  AdamJob* d_adam_jobs = nullptr;
  int n_adam_jobs = 0, adam_items = 0;
  // the element-range jobs alone (the matrices take Adam in the weight-gradient launch)
  AdamJob* d_adam_elem_jobs = nullptr;
  int n_adam_elem_jobs = 0, adam_elem_items = 0;
  float* fused_colpart = nullptr;
  ColsumJob* d_fcs = nullptr;
  int n_fcs = 0, fcs_cols = 0;
  ColsumJob* d_b1_job = nullptr;
  int b1_blocks = 0;
  float* b1_partial = nullptr;
  void build_frags(hipStream_t s) { k_build_frags(d_frag_jobs, n_frag_jobs, total_frags, s); }
  // matrices with fragment copies: element offset in the flat buffers, shape
  // and the two copies (for read-back)
  struct FragMat {
    size_t off;
    int rows, cols;
    const uint4* nt;
    const uint4* nn;
  };
  std::vector<FragMat> frag_mats;
  std::vector<void*> allocs;

  Model(const edpc_config& c, size_t n_slots, size_t max_rows, const KernelConfig* kc);
  ~Model();
  Model(const Model&) = delete;
  Model& operator=(const Model&) = delete;

  const TensorInfo& tensor(const std::string& name) const;
  float* P_(const std::string& name) { return param + tensor(name).off; }
  float* G_(const std::string& name) { return grad + tensor(name).off; }
  const void* W_(const std::string& name) const;  // weight operand (fp32 or bf16 shadow)

  void init_params(hipStream_t s);
  void build_tables(hipStream_t s);
  // One step on rows already staged in ctx/tgt/slot with st set; grid_rows
  // bounds the launch grids (>= st->rows).
  // sched: when given, the row-block step's first kernel sets the step state
  // itself (see FusedInArgs); other steps take it as already set.
  void step(StepMode mode, const StreamIO& io, const StepOutputs& out, int grid_rows,
            hipStream_t s, const StepSched* sched = nullptr);

  void product(int ps, int j, int R, hipStream_t s);
  void setup_fused(hipStream_t s);
  void autotune(hipStream_t s);
  static KernelConfig default_config(const edpc_config& c, size_t rows);
  // FP32 input of refinement block j (j = N: the head's input) of the last
  // step, [last_rows, F]; null where the launch sequence keeps none.
  const float* block_input(int j) const;
  static void validate(const edpc_config& c);

 private:
  template <class T>
  T* dalloc(size_t n);
  void gemm(int slot, bool ak, bool bk, EpiKind epi, int nb, GemmArgs g, int grid_rows,
            hipStream_t s);
};

}  // namespace edpc
