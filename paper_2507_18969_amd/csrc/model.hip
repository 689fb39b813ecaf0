// Model object and the launch sequence of one step (Algorithm 1, lines
// "Model", "Encode/Decode", "loss", "backward", "update").
#include "model.h"
#include "trace.h"

#include <cmath>
#include <cstdlib>
#include <cstring>

namespace edpc {

[[noreturn]] void fail(edpc_status st, const std::string& msg) { throw Error{st, msg}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) fail(EDPC_E_NOMEM, std::string(what) + ": out of device memory");
    fail(EDPC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}

uint64_t KernelConfig::encode() const {
  uint64_t id = (uint64_t)kNumericsRevision << 48;
  for (int i = 0; i < PS_COUNT; ++i) id |= (uint64_t)(tile[i] & 15) << (4 * i);
  if (fused) id |= 1ull << 47;
  if (ln_fold) id |= 1ull << 46;
  return id;
}

bool KernelConfig::decode(uint64_t id, KernelConfig* out) {
  static_assert(4 * PS_COUNT <= 46, "tile ids overlap the flag bits");
  if ((id >> 48) != kNumericsRevision) return false;
  if ((id >> (4 * PS_COUNT)) & ((1ull << (46 - 4 * PS_COUNT)) - 1)) return false;
  out->fused = ((id >> 47) & 1) != 0;
  out->ln_fold = ((id >> 46) & 1) != 0;
  for (int i = 0; i < PS_COUNT; ++i) {
    const int t = (int)((id >> (4 * i)) & 15);
    if (t >= TILE_COUNT) return false;
    out->tile[i] = t;
  }
  return true;
}

const char* kclass_name(int c) {
  static const char* names[KC_COUNT] = {
      "gemm_lte_down", "gemm_lte_up", "gemm_branches_gelu", "gemm_block_out", "gemm_head",
      "gemm_head_bwd", "gemm_gelu_bwd", "gemm_branches_bwd", "gemm_lte_up_bwd",
      "gemm_lte_down_bwd", "gemm_weight_grads", "step_schedule", "gather", "embed", "fdm_fwd",
      "layernorm_fwd", "head_softmax_cdf_coder", "layernorm_bwd", "fdm_bwd_adam", "emb_grad",
      "colsum_bias_grads", "adam_shared", "fused_rowblock_step", "weight_fragments"};
  return (c >= 0 && c < KC_COUNT) ? names[c] : "unknown";
}

void KTimer::begin(int cls, hipStream_t s) {
  if (used == pool.size()) {
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    pool.push_back(e);
  }
  cur = cls;
  cur_ev = pool[used++];
  hip_check(hipEventRecord(cur_ev, s), "hipEventRecord");
}

void KTimer::end(hipStream_t s) {
  if (used == pool.size()) {
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    pool.push_back(e);
  }
  hipEvent_t b = pool[used++];
  hip_check(hipEventRecord(b, s), "hipEventRecord");
  spans.push_back(Span{cur, cur_ev, b});
}

void KTimer::collect(float* ms, uint32_t* launches) {
  for (int c = 0; c < KC_COUNT; ++c) { ms[c] = 0.f; launches[c] = 0; }
  for (auto& sp : spans) {
    hip_check(hipEventSynchronize(sp.b), "hipEventSynchronize");
    float t = 0.f;
    hip_check(hipEventElapsedTime(&t, sp.a, sp.b), "hipEventElapsedTime");
    ms[sp.cls] += t;
    launches[sp.cls] += 1;
  }
}

KTimer::~KTimer() {
  for (auto e : pool) (void)hipEventDestroy(e);
}

#define TIMED(cls, call)                  \
  do {                                    \
    if (timer) timer->begin((cls), s);    \
    call;                                 \
    if (timer) timer->end(s);             \
  } while (0)

static bool pow2(uint32_t x) { return x && !(x & (x - 1)); }

void Model::validate(const edpc_config& c) {
  if (c.struct_size != sizeof(edpc_config)) fail(EDPC_E_INVALID_ARG, "edpc_config.struct_size mismatch");
  if (c.context < 4 || c.context > 256) fail(EDPC_E_INVALID_ARG, "context must be in 4..256");
  if (!pow2(c.embed) || c.embed < 16 || c.embed > 64) fail(EDPC_E_INVALID_ARG, "embed must be a power of two in 16..64");
  if (c.context % 4) fail(EDPC_E_INVALID_ARG, "context must be a multiple of 4");
  if (!pow2(c.latent) || c.latent < 16 || c.latent > 256) fail(EDPC_E_INVALID_ARG, "latent must be a power of two in 16..256");
  if (c.blocks > 16) fail(EDPC_E_INVALID_ARG, "blocks must be <= 16");
  if (c.hidden < 16 || c.hidden % 16 || c.hidden > 8192) fail(EDPC_E_INVALID_ARG, "hidden must be a multiple of 16 in 16..8192");
  if (c.branches < 1 || c.branches > 3) fail(EDPC_E_INVALID_ARG, "branches must be 1..3");
  if (c.cdf_bits != 16) fail(EDPC_E_INVALID_ARG, "only 16-bit CDFs are supported");
  if (c.precision != EDPC_FP32 && c.precision != EDPC_BF16) fail(EDPC_E_INVALID_ARG, "unknown precision");
  if (c.flags & ~(EDPC_CFG_ZERO_HEAD | EDPC_CFG_AUTOTUNE | EDPC_CFG_NO_LTE | EDPC_CFG_LOW_RANK |
                  EDPC_CFG_LAYERWISE | EDPC_CFG_NO_GRAPHS))
    fail(EDPC_E_INVALID_ARG, "unknown config flags");
  if ((c.flags & EDPC_CFG_NO_LTE) && (c.flags & EDPC_CFG_LOW_RANK))
    fail(EDPC_E_INVALID_ARG, "EDPC_CFG_NO_LTE and EDPC_CFG_LOW_RANK exclude each other");
  if ((c.flags & EDPC_CFG_LOW_RANK) && (!pow2((uint32_t)(c.context * c.embed)) || c.context * c.embed > 256))
    fail(EDPC_E_INVALID_ARG, "the low-rank factors need context * embed a power of two <= 256");
  if ((c.flags & EDPC_CFG_NO_LTE) && c.latent != c.context * c.embed)
    fail(EDPC_E_INVALID_ARG, "without the LTE the FDM is F x F: latent must equal context * embed");
  if ((c.context * c.embed) % 8) fail(EDPC_E_INVALID_ARG, "context * embed must be a multiple of 8");
  if ((uint64_t)c.context * c.embed > 16384) fail(EDPC_E_INVALID_ARG, "context * embed must be <= 16384");
  if (!(c.lr >= 0.f) || !(c.beta1 >= 0.f && c.beta1 < 1.f) || !(c.beta2 >= 0.f && c.beta2 < 1.f) || !(c.eps > 0.f))
    fail(EDPC_E_INVALID_ARG, "invalid Adam constants");
}

// Largest tile whose grid still has >= `want` tiles; the smallest otherwise.
// The wide 8-wave tiles serve BF16 products (and gated ones with k = 2).
static int pick_tile(size_t M, const std::vector<std::pair<int, int>>& shapes, size_t want,
                     bool bf16, EpiKind epi = EPI_STORE, int nb = 1) {
  static const int order[] = {TILE_W256x256, TILE_W256x128, TILE_W128x256, TILE_W128x128,
                              TILE_128x64,   TILE_64x128,   TILE_64x64,    TILE_64x32,
                              TILE_32x64,    TILE_32x32};
  for (int t : order) {
    if (!wide_tile_supported(t, bf16, epi, nb)) continue;
    const TileShape ts = tile_shape(t);
    // a wide gated tile holds bn / 2 outputs of each of the two branches
    const int bn = (epi == EPI_GATE_FWD && t >= TILE_W128x128) ? ts.bn / 2 : ts.bn;
    size_t n = 0;
    for (auto& mn : shapes) {
      const size_t m = mn.first ? (size_t)mn.first : M;
      n += ((m + ts.bm - 1) / ts.bm) * ((mn.second + bn - 1) / bn);
    }
    if (n >= want) return t;
  }
  return TILE_32x32;
}

KernelConfig Model::default_config(const edpc_config& c, size_t rows) {
  KernelConfig k;
  const int F = c.context * c.embed, L = c.latent, H = c.hidden;
  const int KH = c.branches * H;
  const bool bf = c.precision == EDPC_BF16;
  // tiles wanted per product: the FP32 autotuner took 32 x 32 tiles for every
  // product at 1024 rows of the 1024-stream model (512 of them for 512
  // outputs), where 256 tiles would give 64 x 32 (515 against 495 us a step)
  const size_t want = bf ? 256 : 512;
  auto one = [&](int n) { return pick_tile(rows, {{0, n}}, want, bf); };
  k.tile[PS_LTE_DOWN] = one(L);
  k.tile[PS_LTE_UP] = one(F);
  // gated products: a wide tile's columns hold both branches of H / 2 outputs
  k.tile[PS_GATE] = pick_tile(rows, {{0, H}}, want, bf, EPI_GATE_FWD, (int)c.branches);
  k.tile[PS_OUT] = one(F);
  k.tile[PS_HEAD] = one(256);
  k.tile[PS_HEAD_BWD] = one(F);
  k.tile[PS_GATE_BWD] = one(H);
  k.tile[PS_DZ] = one(F);
  k.tile[PS_LTE_UP_BWD] = one(L);
  k.tile[PS_LTE_DOWN_BWD] = one(F);
  std::vector<std::pair<int, int>> wg = {{256, F}, {F, L}, {L, F}};
  for (uint32_t j = 0; j < c.blocks; ++j) {
    wg.push_back({F, H});
    wg.push_back({KH, F});
  }
  // Weight gradients: fewer, larger tiles than the other products.  At 1024
  // rows of the 1024-stream model the general rule's 512 tiles took 62 us
  // per BF16 step against 25 us on the autotuner's choice, and 55 against 50
  // us in FP32, whose autotuner takes 64 x 64 tiles at every size measured.
  auto wg_tiles = [&](int t) {
    const TileShape ts = tile_shape(t);
    size_t n = 0;
    for (auto& mn : wg) n += ((mn.first + ts.bm - 1) / ts.bm) * ((mn.second + ts.bn - 1) / ts.bn);
    return n;
  };
  if (bf)
    k.tile[PS_WGRAD] = pick_tile(rows, wg, 192, bf);
  else
    k.tile[PS_WGRAD] = wg_tiles(TILE_64x64) >= 192 ? TILE_64x64 : pick_tile(rows, wg, 512, bf);
  if (rows >= 4096) {
    // Many rows: the autotuner's choices at 16384 rows of the large model,
    // as rules of the product's shape.
    if (bf) {
      // weight gradients: the balanced launch of 256 x 256 tiles once that
      // table covers every CU (0.85 against 1.21 ms per step); the output
      // product, short in K with a residual epilogue, on more and smaller
      // tiles (0.57 against 0.62 ms)
      if (wg_tiles(TILE_W256x256) >= (size_t)kWgradRanges) k.tile[PS_WGRAD] = TILE_W256x256;
      if (H <= 512) k.tile[PS_OUT] = TILE_W128x128;
    } else {
      // FP32 (35.5 against 30.0 ms per step with the general rule): forward
      // products on 128 x 128 tiles for at most 256 outputs, 64 x 64 when
      // K <= 512, else 128 x 64; every input adjoint on 64 x 128; the
      // weight gradients on 64 x 64
      auto fwd = [&](int n, int kk) {
        return n <= 256 ? TILE_128x128 : kk <= 512 ? TILE_64x64 : TILE_128x64;
      };
      k.tile[PS_LTE_DOWN] = fwd(L, F);
      k.tile[PS_LTE_UP] = fwd(F, L);
      k.tile[PS_OUT] = fwd(F, H);
      k.tile[PS_HEAD] = fwd(256, F);
      for (int ps : {PS_HEAD_BWD, PS_GATE_BWD, PS_DZ, PS_LTE_UP_BWD, PS_LTE_DOWN_BWD})
        k.tile[ps] = TILE_64x128;
    }
  }
  // BF16 shapes with a row-block kernel take the fused step (one workgroup per
  // 16 rows runs LTE up .. head .. coder .. adjoint) unless EDPC_CFG_LAYERWISE
  // asks for the layer-by-layer products.  The row-block kernels index
  // activations with 32-bit offsets.
  k.fused = !(c.flags & EDPC_CFG_LAYERWISE) && c.precision == EDPC_BF16 && rows <= (1u << 20) &&
            !(c.flags & (EDPC_CFG_NO_LTE | EDPC_CFG_LOW_RANK)) &&
            fused_supported(F, L, H, (int)c.branches, (int)c.blocks);
  // The row-block step's update applies Adam in the epilogue of a 4-wave
  // weight-gradient tile (a wide tile would need a separate Adam pass).  That
  // epilogue favours larger tiles over more of them: at 1024 rows of the
  // 1024-stream model an update step took 248 us on 64 x 128 or 128 x 64
  // tiles (224 of them) against 284 us on the 64 x 32 ones the general rule
  // picks for 512 tiles (896); the 192-tile rule above gives 128 x 64.
  if (k.fused && k.tile[PS_WGRAD] >= TILE_W128x128) k.tile[PS_WGRAD] = TILE_64x128;
  // from 4096 rows the LayerNorm adjoint forms its block's column sums itself
  // (16 rows a workgroup in turn); below that its workgroups would be too few
  k.ln_fold = !k.fused && c.blocks > 0 && ln_bwd_folds(F) && rows >= 4096;
  return k;
}

template <class T>
T* Model::dalloc(size_t n) {
  void* p = nullptr;
  if (n == 0) n = 1;
  hip_check(hipMalloc(&p, n * sizeof(T)), "hipMalloc");
  allocs.push_back(p);
  return (T*)p;
}

static size_t align64(size_t x) { return (x + 63) & ~(size_t)63; }

Model::Model(const edpc_config& c, size_t nslots, size_t rows, const KernelConfig* kcfg)
    : cfg(c), n_slots(nslots), max_rows(rows) {
  validate(c);
  if (nslots == 0 || rows == 0) fail(EDPC_E_INVALID_ARG, "n_slots and max_rows must be >= 1");
  if (rows > (1u << 24)) fail(EDPC_E_INVALID_ARG, "max_rows too large");
  C = c.context;
  E = c.embed;
  F = C * E;
  L = c.latent;
  N = c.blocks;
  H = c.hidden;
  K = c.branches;
  bf16 = c.precision == EDPC_BF16;
  kc = kcfg ? *kcfg : default_config(c, rows);
  low_rank = (c.flags & EDPC_CFG_LOW_RANK) != 0;
  lte = !(c.flags & EDPC_CFG_NO_LTE) && !low_rank;
  if (kc.fused && !(bf16 && lte && fused_supported(F, L, H, K, N) && rows <= (1u << 20)))
    fail(EDPC_E_UNSUPPORTED, "fused step requested for an unsupported shape");
  if (kc.ln_fold && (kc.fused || N == 0 || !ln_bwd_folds(F)))
    fail(EDPC_E_UNSUPPORTED, "LayerNorm adjoint with column sums requested for an unsupported shape");

  // Flat layout of the shared parameters; each tensor starts 64-aligned.
  auto add = [&](const std::string& n, size_t numel, uint32_t tid, double bound) {
    tens.push_back(TensorInfo{n, P, numel, tid, (float)bound});
    P = align64(P + numel);
  };
  const double bF = 1.0 / std::sqrt((double)F), bL = 1.0 / std::sqrt((double)L),
               bH = 1.0 / std::sqrt((double)H);
  add("emb", 256 * (size_t)E, 1, std::sqrt(3.0));
  if (lte) {
    add("w1", (size_t)L * F, 2, bF);
    add("b1", L, 3, bF);
    add("w2", (size_t)F * L, 5, bL);
    add("b2", F, 6, bL);
  }
  for (int j = 0; j < N; ++j) {
    add("ln" + std::to_string(j) + ".gamma", F, 0, 1.0);
    add("ln" + std::to_string(j) + ".beta", F, 0, 0.0);
    // branch weights contiguous ([K*H, F]) so one product covers all paths
    const size_t wbase = P;
    for (int i = 0; i < K; ++i) {
      tens.push_back(TensorInfo{"blk" + std::to_string(j) + ".w" + std::to_string(i),
                                wbase + (size_t)i * H * F, (size_t)H * F, 16u + 16u * j + 2u * i,
                                (float)bF});
    }
    P = align64(wbase + (size_t)K * H * F);
    const size_t bbase = P;
    for (int i = 0; i < K; ++i) {
      tens.push_back(TensorInfo{"blk" + std::to_string(j) + ".b" + std::to_string(i),
                                bbase + (size_t)i * H, (size_t)H, 17u + 16u * j + 2u * i,
                                (float)bF});
    }
    P = align64(bbase + (size_t)K * H);
    add("blk" + std::to_string(j) + ".wo", (size_t)F * H, 16u + 16u * j + 14u, bH);
    add("blk" + std::to_string(j) + ".bo", F, 16u + 16u * j + 15u, bH);
  }
  const bool zh = (c.flags & EDPC_CFG_ZERO_HEAD) != 0;
  add("wh", 256 * (size_t)F, zh ? 0 : 7, zh ? 0.0 : bF);
  add("bh", 256, zh ? 0 : 8, zh ? 0.0 : bF);

  param = dalloc<float>(P);
  grad = dalloc<float>(P);
  m = dalloc<float>(P);
  v = dalloc<float>(P);
  if (bf16) p16 = dalloc<bf16_t>(P);
  const size_t fdm = n_slots * (size_t)L * L;
  U = dalloc<float>(fdm);
  mU = dalloc<float>(fdm);
  vU = dalloc<float>(fdm);
  if (low_rank) {
    const size_t fac = n_slots * (size_t)F * L;
    A = dalloc<float>(fac);
    mA = dalloc<float>(fac);
    vA = dalloc<float>(fac);
    B = dalloc<float>(fac);
    mB = dalloc<float>(fac);
    vB = dalloc<float>(fac);
  }
  st = dalloc<StepState>(1);

  const size_t R = max_rows;
  ctx = dalloc<uint8_t>(R * C);
  tgt = dalloc<uint8_t>(R);
  slot = dalloc<uint32_t>(R);
  // without the LTE the FDM reads the FP32 embedding (x' = x) and writes the
  // first block's input (x'' = y) directly
  if (bf16 && lte) X16 = dalloc<bf16_t>(R * F);
  if (!bf16 || !lte) X32 = dalloc<float>(R * F);
  X1 = (lte || low_rank) ? dalloc<float>(R * L) : X32;
  for (int j = 0; j <= N; ++j) Hs.push_back(dalloc<float>(R * F));
  if (lte) {
    if (bf16) Y16 = dalloc<bf16_t>(R * L); else Y32 = dalloc<float>(R * L);
  } else if (low_rank) {  // y = x' U_s in FP32, then x'' = y B_s writes the first block's input
    Y32 = dalloc<float>(R * L);
  } else {
    Y32 = Hs[0];
  }
  if (bf16) HN16 = dalloc<bf16_t>(R * F);
  for (int j = 0; j < N; ++j) {
    if (bf16) Z16.push_back(dalloc<bf16_t>(R * F)); else Z32.push_back(dalloc<float>(R * F));
    mean.push_back(dalloc<float>(R));
    rstd.push_back(dalloc<float>(R));
    Abr.push_back(dalloc<float>(R * K * H));
    if (bf16) G16.push_back(dalloc<bf16_t>(R * H)); else G32.push_back(dalloc<float>(R * H));
    dA32.push_back(dalloc<float>(R * K * H));
    if (bf16) dA16.push_back(dalloc<bf16_t>(R * K * H));
    dZ.push_back(dalloc<float>(R * F));
  }
  for (int j = 0; j <= N; ++j) {
    dH32.push_back(dalloc<float>(R * F));
    if (bf16) dH16.push_back(dalloc<bf16_t>(R * F));
  }
  logits = dalloc<float>(R * 256);
  dz32 = dalloc<float>(R * 256);
  if (bf16) dz16 = dalloc<bf16_t>(R * 256);
  loss_rows = dalloc<float>(R);
  loss_out = dalloc<float>(1);
  dX = dalloc<float>(R * F);
  if (lte) {
    dY = dalloc<float>(R * L);
    dX1_32 = dalloc<float>(R * L);
    if (bf16) dX1_16 = dalloc<bf16_t>(R * L);
  } else if (low_rank) {
    dY = dalloc<float>(R * L);
    dX1_32 = dalloc<float>(R * L);
  } else {  // dy = dx'' and dx = dx'
    dY = dH32[0];
    dX1_32 = dX;
  }
  emb_grad_plan((int)R, C, E, &emb_chunk, &emb_sub);
  emb_partial = dalloc<float>(((R + emb_chunk - 1) / emb_chunk) * 256 * (size_t)E);
}

Model::~Model() {
  for (void* p : allocs) (void)hipFree(p);
}

const TensorInfo& Model::tensor(const std::string& name) const {
  for (const auto& t : tens)
    if (t.name == name) return t;
  fail(EDPC_E_INVALID_ARG, "no tensor " + name);
}

const void* Model::W_(const std::string& name) const {
  const TensorInfo& t = tensor(name);
  return bf16 ? (const void*)(p16 + t.off) : (const void*)(param + t.off);
}

void Model::init_params(hipStream_t s) {
  hip_check(hipMemsetAsync(param, 0, P * sizeof(float), s), "memset");
  for (const auto& t : tens) {
    if (t.tid) k_init_uniform(param + t.off, t.numel, cfg.seed, t.tid, 0, t.bound, s);
    else k_fill(param + t.off, t.numel, t.bound, s);
  }
  k_init_uniform(U, n_slots * (size_t)L * L, cfg.seed, 4, 0,
                 (float)(1.0 / std::sqrt((double)L)), s);
  hip_check(hipMemsetAsync(m, 0, P * sizeof(float), s), "memset");
  hip_check(hipMemsetAsync(v, 0, P * sizeof(float), s), "memset");
  hip_check(hipMemsetAsync(grad, 0, P * sizeof(float), s), "memset");
  hip_check(hipMemsetAsync(mU, 0, n_slots * (size_t)L * L * sizeof(float), s), "memset");
  hip_check(hipMemsetAsync(vU, 0, n_slots * (size_t)L * L * sizeof(float), s), "memset");
  if (low_rank) {  // slot s draws the counter range starting at s * F * L, like U
    const size_t fac = n_slots * (size_t)F * L;
    k_init_uniform(A, fac, cfg.seed, 9, 0, (float)(1.0 / std::sqrt((double)F)), s);
    k_init_uniform(B, fac, cfg.seed, 10, 0, (float)(1.0 / std::sqrt((double)L)), s);
    for (float* z : {mA, vA, mB, vB}) hip_check(hipMemsetAsync(z, 0, fac * sizeof(float), s), "memset");
  }
  if (bf16) k_to_bf16(param, p16, P, s);
  if (kc.fused) build_frags(s);
  hip_check(hipGetLastError(), "init");
  tau = 0;
}

void Model::build_tables(hipStream_t s) {
  // weight-gradient products (sum over rows), one table per tile shape
  const void* dz_op = bf16 ? (const void*)dz16 : (const void*)dz32;
  const void* hN_op = bf16 ? (const void*)HN16 : (const void*)Hs[N];
  for (int tile = 0; tile < TILE_COUNT; ++tile) {
    std::vector<WgradProblem> wg;
    const TileShape ts = tile_shape(tile);
    int tiles = 0;
    auto addw = [&](const void* dout, const void* in, float* dw, int Mo, int Ni) {
      WgradProblem p{};
      p.dout = dout;
      p.in = in;
      p.dw = dw;
      p.M = Mo;
      p.N = Ni;
      p.tiles_n = (Ni + ts.bn - 1) / ts.bn;
      p.tile_begin = tiles;
      tiles += p.tiles_n * ((Mo + ts.bm - 1) / ts.bm);
      wg.push_back(p);
    };
    addw(dz_op, hN_op, G_("wh"), 256, F);
    for (int j = 0; j < N; ++j) {
      const std::string b = "blk" + std::to_string(j);
      addw(bf16 ? (const void*)dH16[j + 1] : (const void*)dH32[j + 1],
           bf16 ? (const void*)G16[j] : (const void*)G32[j], G_(b + ".wo"), F, H);
      addw(bf16 ? (const void*)dA16[j] : (const void*)dA32[j],
           bf16 ? (const void*)Z16[j] : (const void*)Z32[j], G_(b + ".w0"), K * H, F);
    }
    if (lte) {
      addw(bf16 ? (const void*)dH16[0] : (const void*)dH32[0],
           bf16 ? (const void*)Y16 : (const void*)Y32, G_("w2"), F, L);
      addw(bf16 ? (const void*)dX1_16 : (const void*)dX1_32,
           bf16 ? (const void*)X16 : (const void*)X32, G_("w1"), L, F);
    }
    WgTable& t = wg_tab[tile];
    t.n = (int)wg.size();
    t.tiles = tiles;
    t.host = wg;
    t.d = dalloc<WgradProblem>(wg.size());
    hip_check(hipMemcpyAsync(t.d, wg.data(), wg.size() * sizeof(WgradProblem),
                             hipMemcpyHostToDevice, s), "copy");
  }

  // scratch of the balanced weight-gradient launch (wide tiles, large tables)
  if (bf16 && kc.tile[PS_WGRAD] >= TILE_W128x128 &&
      wg_tab[kc.tile[PS_WGRAD]].tiles >= kWgradRanges) {
    wg_part_floats = wgrad_part_floats(kc.tile[PS_WGRAD]);
    wg_part = dalloc<float>(wg_part_floats);
  }

  // column sums: bias gradients, LayerNorm affine gradients.  Where the
  // LayerNorm adjoint folds them in (kernel configuration bit 46), each block's beta, gamma
  // and output-bias sums come from its row-group partials; those jobs follow
  // the others, past the first pass's grid.
  std::vector<ColsumJob> cs;
  const bool fold = kc.ln_fold;
  auto addc = [&](const float* src, int cols, int ld, float* dst, const float* h,
                  const float* mu, const float* rs) {
    ColsumJob j{};
    j.src = src;
    j.h = h;
    j.mean = mu;
    j.rstd = rs;
    j.dst = dst;
    j.cols = cols;
    j.ld = ld;
    j.col_block_begin = cs_blocks;
    j.col_offset = cs_cols;
    cs_cols += cols;
    j.scale = 1.0f;
    cs_blocks += (cols + 63) / 64;
    cs.push_back(j);
  };
  addc(dz32, 256, 256, G_("bh"), nullptr, nullptr, nullptr);
  for (int j = 0; j < N; ++j) {
    const std::string b = "blk" + std::to_string(j);
    if (!fold) addc(dH32[j + 1], F, F, G_(b + ".bo"), nullptr, nullptr, nullptr);
    addc(dA32[j], K * H, K * H, G_(b + ".b0"), nullptr, nullptr, nullptr);
    if (!fold) {
      addc(dZ[j], F, F, G_("ln" + std::to_string(j) + ".beta"), nullptr, nullptr, nullptr);
      addc(dZ[j], F, F, G_("ln" + std::to_string(j) + ".gamma"), Hs[j], mean[j], rstd[j]);
    }
  }
  if (lte) {
    addc(dH32[0], F, F, G_("b2"), nullptr, nullptr, nullptr);
    addc(dX1_32, L, L, G_("b1"), nullptr, nullptr, nullptr);
  }
  ln_part.assign(fold ? N : 0, nullptr);
  if (fold) {
    for (int j = 0; j < N; ++j) {
      ln_part[j] = dalloc<float>(ln_fold_part_elems((int)max_rows, F));
      const std::string b = "blk" + std::to_string(j), ln = "ln" + std::to_string(j);
      float* dsts[3] = {G_(ln + ".beta"), G_(ln + ".gamma"), G_(b + ".bo")};
      for (int q = 0; q < 3; ++q) {
        ColsumJob jb{};
        jb.dst = dsts[q];
        jb.cols = F;
        jb.col_block_begin = cs_blocks;  // past the first pass's grid
        jb.col_offset = cs_cols;
        cs_cols += F;
        jb.scale = 1.0f;
        jb.part = ln_part[j] + (size_t)q * F;
        jb.part_ld = 3 * F;
        jb.part_rows = kLnFoldRows;
        cs.push_back(jb);
      }
    }
  }
  n_cs = (int)cs.size();
  d_cs = dalloc<ColsumJob>(cs.size());
  cs_partial = dalloc<float>(colsum_partial_elems((int)max_rows, cs_cols));
  hip_check(hipMemcpyAsync(d_cs, cs.data(), cs.size() * sizeof(ColsumJob), hipMemcpyHostToDevice, s),
            "copy");
  ColsumJob lj{};
  lj.src = loss_rows;
  lj.h = nullptr;
  lj.mean = lj.rstd = nullptr;
  lj.dst = loss_out;
  lj.cols = 1;
  lj.ld = 1;
  lj.col_block_begin = 0;
  lj.col_offset = 0;
  lj.scale = 0.0f;  // scale by 1/rows
  loss_partial = dalloc<float>(colsum_partial_elems((int)max_rows, 1));
  d_loss_job = dalloc<ColsumJob>(1);
  hip_check(hipMemcpyAsync(d_loss_job, &lj, sizeof(lj), hipMemcpyHostToDevice, s), "copy");
  if (kc.fused) setup_fused(s);
  hip_check(hipStreamSynchronize(s), "sync");
}

void Model::setup_fused(hipStream_t s) {
  // fragment-ordered BF16 copies of every matrix the row-block kernel streams
  struct Mat { const char* name; int rows, cols; };
  std::vector<FragJob> jobs;
  std::vector<std::pair<std::string, size_t>> where;  // matrix -> uint4 offset of its nt copy
  size_t off = 0;
  int fr = 0;
  auto add = [&](const std::string& name, int rows, int cols) {
    FragJob j;
    j.src = param + tensor(name).off;
    j.rows = rows;
    j.cols = cols;
    j.frag_begin = fr;
    j.nt = (uint4*)(size_t)off;  // offsets for now
    j.nn = (uint4*)(size_t)(off + (size_t)rows * cols / 8);
    where.push_back({name, off});
    off += 2 * (size_t)rows * cols / 8;
    fr += 2 * rows * cols / 512;
    jobs.push_back(j);
  };
  add("w1", L, F);
  add("w2", F, L);
  for (int j = 0; j < N; ++j) {
    add("blk" + std::to_string(j) + ".w0", K * H, F);
    add("blk" + std::to_string(j) + ".wo", F, H);
  }
  add("wh", 256, F);
  frags = dalloc<uint4>(off);
  for (auto& j : jobs) {
    j.nt = frags + (size_t)j.nt;
    j.nn = frags + (size_t)j.nn;
    frag_mats.push_back(FragMat{(size_t)(j.src - param), j.rows, j.cols, j.nt, j.nn});
  }
  n_frag_jobs = (int)jobs.size();
  total_frags = fr;
  std::vector<AdamJob> aj;
  std::vector<std::string> aj_name;  // tensor of each element-range job
  {  // Adam jobs: matrices with fragment copies by tiles, the other tensors by element

    int items = 0;
    std::vector<char> covered(tens.size(), 0);
    for (const auto& fj : jobs) {
      AdamJob a;
      a.off = (size_t)(fj.src - param);
      a.rows = fj.rows;
      a.cols = fj.cols;
      a.nt = fj.nt;
      a.nn = fj.nn;
      a.red = nullptr;
      a.red_ld = 0;
      a.red_block = kFusedRows;
      a.item_begin = items;
      if (fj.rows % kAdamTileRows || fj.cols % kAdamTileCols)
        fail(EDPC_E_UNSUPPORTED, "matrix shape of the fused step's Adam tiles");
      items += (fj.rows / kAdamTileRows) * (fj.cols / kAdamTileCols);
      aj.push_back(a);
      aj_name.push_back("");
      for (size_t t = 0; t < tens.size(); ++t)
        if (tens[t].off >= a.off && tens[t].off < a.off + (size_t)a.rows * a.cols) covered[t] = 1;
    }
    for (size_t t = 0; t < tens.size(); ++t) {
      if (covered[t]) continue;
      AdamJob a;
      a.off = tens[t].off;
      a.rows = (int)tens[t].numel;
      a.cols = 0;
      a.nt = a.nn = nullptr;
      a.red = nullptr;
      a.red_ld = 0;
      a.red_block = kFusedRows;
      a.item_begin = items;
      items += (a.rows + kAdamVecItem - 1) / kAdamVecItem;
      aj.push_back(a);
      aj_name.push_back(tens[t].name);
    }
    n_adam_jobs = (int)aj.size();
    adam_items = items;
  }
  d_frag_jobs = dalloc<FragJob>(jobs.size());
  hip_check(hipMemcpyAsync(d_frag_jobs, jobs.data(), jobs.size() * sizeof(FragJob),
                           hipMemcpyHostToDevice, s), "copy");
  auto nt = [&](const std::string& n) -> const uint4* {
    for (auto& w : where) if (w.first == n) return frags + w.second;
    fail(EDPC_E_DEVICE, "fragment table");
  };
  auto nn = [&](const std::string& n, int numel) -> const uint4* { return nt(n) + numel / 8; };

  std::memset(&fa, 0, sizeof(fa));
  fa.st = st;
  fa.n_blocks = N;
  fa.w2_nt = nt("w2");
  fa.w2_nn = nn("w2", F * L);
  fa.wh_nt = nt("wh");
  fa.wh_nn = nn("wh", 256 * F);
  fa.b2 = P_("b2");
  fa.bh = P_("bh");
  for (int j = 0; j < N; ++j) {
    const std::string b = "blk" + std::to_string(j), ln = "ln" + std::to_string(j);
    fa.wab_nt[j] = nt(b + ".w0");
    fa.wab_nn[j] = nn(b + ".w0", K * H * F);
    fa.wo_nt[j] = nt(b + ".wo");
    fa.wo_nn[j] = nn(b + ".wo", F * H);
    fa.bab[j] = P_(b + ".b0");
    fa.bo[j] = P_(b + ".bo");
    fa.gamma[j] = P_(ln + ".gamma");
    fa.beta[j] = P_(ln + ".beta");
    fa.z16[j] = Z16[j];
    fa.mean[j] = mean[j];
    fa.rstd[j] = rstd[j];
    fa.abr[j] = Abr[j];
    fa.g16[j] = G16[j];
    fa.da16[j] = dA16[j];
  }
  for (int j = 0; j <= N; ++j) {
    fa.hs[j] = Hs[j];
    fa.dh16[j] = dH16[j];
  }
  fa.y16 = Y16;
  fa.hn16 = HN16;
  fa.dz16 = dz16;
  fa.dy = dY;
  fa.loss_rows = loss_rows;

  // column-sum partials: [row block][bh | per block: bo, bab, beta, gamma | b2]
  std::vector<ColsumJob> cs;
  int cols = 0;
  auto addc = [&](float* dst, int n) {
    ColsumJob j;
    std::memset(&j, 0, sizeof(j));
    j.dst = dst;
    j.cols = n;
    j.col_offset = cols;
    j.scale = 1.0f;
    cols += n;
    cs.push_back(j);
    return j.col_offset;
  };
  fa.off_bh = addc(G_("bh"), 256);
  for (int j = 0; j < N; ++j) {
    const std::string b = "blk" + std::to_string(j), ln = "ln" + std::to_string(j);
    fa.off_bo[j] = addc(G_(b + ".bo"), F);
    fa.off_bab[j] = addc(G_(b + ".b0"), K * H);
    fa.off_beta[j] = addc(G_(ln + ".beta"), F);
    fa.off_gamma[j] = addc(G_(ln + ".gamma"), F);
  }
  fa.off_b2 = addc(G_("b2"), F);
  const int off_b1 = addc(G_("b1"), L);
  fcs_cols = cols;
  n_fcs = (int)cs.size();
  fa.colpart_cols = cols;
  fused_colpart = dalloc<float>(((max_rows + kFusedRows - 1) / kFusedRows) * (size_t)cols);
  fa.colpart = fused_colpart;
  d_fcs = dalloc<ColsumJob>(cs.size());
  hip_check(hipMemcpyAsync(d_fcs, cs.data(), cs.size() * sizeof(ColsumJob), hipMemcpyHostToDevice, s),
            "copy");
  std::memset(&fin, 0, sizeof(fin));
  fin.st = st;
  fin.C = C;
  fin.E = E;
  fin.emb = P_("emb");
  fin.w1_nt = nt("w1");
  fin.b1 = P_("b1");
  fin.ctx = ctx;
  fin.tgt = tgt;
  fin.x16 = X16;
  fin.x1 = X1;
  std::memset(&fout, 0, sizeof(fout));
  fout.st = st;
  fout.C = C;
  fout.E = E;
  fout.w1_nn = nn("w1", L * F);
  fout.dx1_16 = dX1_16;
  fout.dx1_32 = dX1_32;
  fout.ctx = ctx;
  fused_emb_partial = dalloc<float>(((max_rows + kFusedRows - 1) / kFusedRows) * 256 * (size_t)E);
  fout.emb_partial = fused_emb_partial;
  fout.colpart = fused_colpart;
  // element-range Adam jobs take their gradients from the row-block partials
  for (size_t k = 0; k < aj.size(); ++k) {
    if (aj[k].cols != 0) continue;
    if (aj_name[k] == "emb") {
      aj[k].red = fused_emb_partial;
      aj[k].red_ld = 256 * E;
      continue;
    }
    const float* dst = G_(aj_name[k]);
    for (const ColsumJob& j : cs)  // a job may span several tensors (the branch biases)
      if (dst >= j.dst && dst + aj[k].rows <= j.dst + j.cols) {
        aj[k].red = fused_colpart + j.col_offset + (dst - j.dst);
        aj[k].red_ld = fcs_cols;
      }
    if (!aj[k].red) fail(EDPC_E_DEVICE, "no gradient partials for " + aj_name[k]);
  }
  d_adam_jobs = dalloc<AdamJob>(aj.size());
  hip_check(hipMemcpyAsync(d_adam_jobs, aj.data(), aj.size() * sizeof(AdamJob),
                           hipMemcpyHostToDevice, s), "copy");
  {  // the element-range jobs alone, and weight-gradient tables that apply Adam
    std::vector<AdamJob> ae;
    int items = 0;
    for (AdamJob a : aj) {
      if (a.cols != 0) continue;
      a.item_begin = items;
      items += (a.rows + kAdamVecItem - 1) / kAdamVecItem;
      ae.push_back(a);
    }
    n_adam_elem_jobs = (int)ae.size();
    adam_elem_items = items;
    d_adam_elem_jobs = dalloc<AdamJob>(ae.size());
    hip_check(hipMemcpyAsync(d_adam_elem_jobs, ae.data(), ae.size() * sizeof(AdamJob),
                             hipMemcpyHostToDevice, s), "copy");
    for (int tile = 0; tile < TILE_W128x128; ++tile) {
      std::vector<WgradProblem> wp = wg_tab[tile].host;
      bool ok = !wp.empty();
      for (WgradProblem& p : wp) {
        p.nt = p.nn = nullptr;
        for (const FragMat& fm : frag_mats)
          if (p.dw == grad + fm.off && fm.rows == p.M && fm.cols == p.N) {
            p.nt = const_cast<uint4*>(fm.nt);
            p.nn = const_cast<uint4*>(fm.nn);
          }
        if (!p.nt || p.M % 32 || p.N % 32) ok = false;
      }
      if (!ok) continue;
      wg_tab[tile].d_adam = dalloc<WgradProblem>(wp.size());
      hip_check(hipMemcpyAsync(wg_tab[tile].d_adam, wp.data(), wp.size() * sizeof(WgradProblem),
                               hipMemcpyHostToDevice, s), "copy");
    }
  }
  fout.colpart_cols = cols;
  fout.off_b1 = off_b1;
  build_frags(s);
}

void Model::gemm(int ps, bool ak, bool bk, EpiKind epi, int nb, GemmArgs g, int grid_rows,
                 hipStream_t s) {
  g.st = st;
  TIMED(ps, hip_check(launch_gemm(kc.tile[ps], bf16, ak, bk, epi, nb, g, grid_rows, s), "gemm launch"));
}

static GemmArgs ga() {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  return g;
}

// One dense product of the step; j = block index where it applies.
void Model::product(int ps, int j, int R, hipStream_t s) {
  const std::string b = "blk" + std::to_string(j);
  GemmArgs g = ga();
  g.M = R;
  g.m_rows = 1;
  switch (ps) {
    case PS_LTE_DOWN:  // Eq. 14
      g.A = bf16 ? (const void*)X16 : (const void*)X32; g.lda = F; g.B = W_("w1"); g.ldb = F;
      g.N = L; g.K = F; g.bias = P_("b1"); g.out32 = X1; g.ld_out32 = L;
      return gemm(ps, true, true, EPI_STORE, 1, g, R, s);
    case PS_LTE_UP:  // Eq. 16
      g.A = bf16 ? (const void*)Y16 : (const void*)Y32; g.lda = L; g.B = W_("w2"); g.ldb = L;
      g.N = F; g.K = L; g.bias = P_("b2"); g.out32 = Hs[0]; g.ld_out32 = F;
      if (N == 0 && bf16) { g.out16 = HN16; g.ld_out16 = F; }
      return gemm(ps, true, true, EPI_STORE, 1, g, R, s);
    case PS_GATE:  // Eqs. 10-12: k branch products sharing the LayerNorm output
      g.A = bf16 ? (const void*)Z16[j] : (const void*)Z32[j]; g.lda = F;
      g.B = W_(b + ".w0"); g.ldb = F; g.b_branch_stride = (long long)H * F;
      g.N = H; g.K = F; g.bias = P_(b + ".b0"); g.bias_branch_stride = H;
      g.aux = Abr[j]; g.ld_aux = K * H; g.aux_branch = H;
      if (bf16) { g.out16 = G16[j]; g.ld_out16 = H; } else { g.out32 = G32[j]; g.ld_out32 = H; }
      return gemm(ps, true, true, EPI_GATE_FWD, K, g, R, s);
    case PS_OUT:  // Eq. 13: output linear + residual
      g.A = bf16 ? (const void*)G16[j] : (const void*)G32[j]; g.lda = H;
      g.B = W_(b + ".wo"); g.ldb = H; g.N = F; g.K = H;
      g.bias = P_(b + ".bo"); g.resid = Hs[j]; g.ld_resid = F;
      g.out32 = Hs[j + 1]; g.ld_out32 = F;
      if (j == N - 1 && bf16) { g.out16 = HN16; g.ld_out16 = F; }
      return gemm(ps, true, true, EPI_STORE, 1, g, R, s);
    case PS_HEAD:
      g.A = bf16 ? (const void*)HN16 : (const void*)Hs[N]; g.lda = F; g.B = W_("wh"); g.ldb = F;
      g.N = 256; g.K = F; g.bias = P_("bh"); g.out32 = logits; g.ld_out32 = 256;
      return gemm(ps, true, true, EPI_STORE, 1, g, R, s);
    case PS_HEAD_BWD:
      g.A = bf16 ? (const void*)dz16 : (const void*)dz32; g.lda = 256; g.B = W_("wh"); g.ldb = F;
      g.N = F; g.K = 256; g.out32 = dH32[N]; g.ld_out32 = F;
      if (bf16) { g.out16 = dH16[N]; g.ld_out16 = F; }
      return gemm(ps, true, false, EPI_STORE, 1, g, R, s);
    case PS_GATE_BWD:  // dX_ff = dH Wo, then dX_i through GeLU and the product
      g.A = bf16 ? (const void*)dH16[j + 1] : (const void*)dH32[j + 1]; g.lda = F;
      g.B = W_(b + ".wo"); g.ldb = H; g.N = H; g.K = F;
      g.aux = Abr[j]; g.ld_aux = K * H; g.aux_branch = H; g.bias_branch_stride = K;
      g.out32 = dA32[j]; g.ld_out32 = K * H;
      if (bf16) { g.out16 = dA16[j]; g.ld_out16 = K * H; }
      return gemm(ps, true, false, EPI_GATE_BWD, 1, g, R, s);
    case PS_DZ:  // dX0 = sum_i dX_i W_i
      g.A = bf16 ? (const void*)dA16[j] : (const void*)dA32[j]; g.lda = K * H;
      g.B = W_(b + ".w0"); g.ldb = F; g.N = F; g.K = K * H;
      g.out32 = dZ[j]; g.ld_out32 = F;
      return gemm(ps, true, false, EPI_STORE, 1, g, R, s);
    case PS_LTE_UP_BWD:
      g.A = bf16 ? (const void*)dH16[0] : (const void*)dH32[0]; g.lda = F;
      g.B = W_("w2"); g.ldb = L; g.N = L; g.K = F; g.out32 = dY; g.ld_out32 = L;
      return gemm(ps, true, false, EPI_STORE, 1, g, R, s);
    case PS_LTE_DOWN_BWD:
      g.A = bf16 ? (const void*)dX1_16 : (const void*)dX1_32; g.lda = L;
      g.B = W_("w1"); g.ldb = F; g.N = F; g.K = L; g.out32 = dX; g.ld_out32 = F;
      return gemm(ps, true, false, EPI_STORE, 1, g, R, s);
    case PS_WGRAD: {
      const WgTable& t = wg_tab[kc.tile[PS_WGRAD]];
      TIMED(PS_WGRAD, hip_check(launch_wgrad(kc.tile[PS_WGRAD], bf16, t.d, t.n, t.tiles, st,
                                             wg_part, s),
                                "wgrad launch"));
      return;
    }
  }
}

const float* Model::block_input(int j) const {
  if (j < 0 || j > N) return nullptr;
  if (kc.fused && j == N) return nullptr;  // the row-block step keeps only a BF16 copy
  return Hs[j];
}

void Model::step(StepMode mode, const StreamIO& io, const StepOutputs& out, int grid_rows,
                 hipStream_t s, const StepSched* sched) {
  TraceRange range(kc.fused ? "step (row-block)" : "step (layer by layer)");
  const int R = grid_rows;
  last_rows = grid_rows;
  // ---- forward: Eq. 1 through Eqs. 14-16 and 9-13 -------------------------
  const bool backward = out.backward || out.update || out.keep_fdm_grad;
  HeadArgs ha;
  std::memset(&ha, 0, sizeof(ha));
  ha.logits = logits;
  ha.target = (mode == MODE_DECODE || (mode == MODE_PLAIN && !out.has_target)) ? nullptr : tgt;
  ha.target_out = mode == MODE_DECODE ? tgt : nullptr;
  ha.dz32 = dz32;
  ha.dz16 = dz16;
  ha.loss_rows = loss_rows;
  ha.probs = out.probs;
  ha.cum_out = out.cum;
  ha.mode = mode;
  ha.want_grad = backward ? 1 : 0;
  StreamIO hio = io;
  if (mode == MODE_PLAIN) hio.slot = nullptr;
  AdamCfg ac{cfg.lr, cfg.beta1, cfg.beta2, cfg.eps};
  if (kc.fused) {
    // before the FDM: gather (coding modes), embedding, LTE down (Eq. 14)
    FusedInArgs fi = fin;
    fi.gather = mode == MODE_PLAIN ? 0 : 1;
    fi.decoding = mode == MODE_DECODE ? 1 : 0;
    fi.io = io;
    if (sched) {  // the step state is formed here, not by a launch of its own
      fi.sched = sched->sc;
      fi.sched_mode = sched->mode;
      fi.sched_step = sched->step;
    }
    TIMED(KC_EMBED, hip_check(launch_fused_in(F, L, fi, R, s), "fused in launch"));
    TIMED(KC_FDM_FWD, k_fdm_fwd(st, X1, U, slot, L, L, Y32, Y16, R, s));  // Eq. 15
    // LTE up .. head .. coder .. adjoint back to dY, one workgroup per 16 rows
    FusedArgs a = fa;
    a.head = ha;
    a.io = hio;
    TIMED(KC_FUSED, hip_check(launch_fused(F, L, H, a, R, s), "fused launch"));
    if (out.loss) {
      TIMED(KC_COLSUM, k_colsum(st, d_loss_job, 1, 1, 1, loss_partial, R, s));
      hip_check(hipMemcpyAsync(out.loss, loss_out, sizeof(float), hipMemcpyDeviceToDevice, s), "copy");
    }
    if (!backward) return;
    TIMED(KC_FDM_BWD, k_fdm_bwd(st, X1, dY, U, mU, vU, out.keep_fdm_grad ? dUkeep : nullptr, slot,
                                L, L, ac, out.update, dX1_32, dX1_16, R, s));
    TIMED(KC_EMB_GRAD, hip_check(launch_fused_out(F, L, fout, R, s), "fused out launch"));
    const int wt = kc.tile[PS_WGRAD];
    if (out.update && wt < TILE_W128x128 && wg_tab[wt].d_adam) {
      // each weight tile takes Adam and its fragment rewrite as soon as its
      // gradient is summed; work-groups past the tiles take the biases,
      // LayerNorm and embedding (their partials are complete by now)
      const WgTable& t = wg_tab[wt];
      const WgradAdam ad{grad, param, m, v, ac, 0, d_adam_elem_jobs, n_adam_elem_jobs};
      TIMED(PS_WGRAD, hip_check(launch_wgrad_adam(wt, t.d_adam, t.n, t.tiles, adam_elem_items, st,
                                                  ad, s),
                                "wgrad launch"));
      return;
    }
    product(PS_WGRAD, 0, R, s);
    if (out.update) {
      // Adam fused with the refresh of the fragment copies and with the sums
      // of the bias / embedding gradient partials
      TIMED(KC_ADAM, k_adam_frags(st, d_adam_jobs, n_adam_jobs, adam_items, param, grad, m, v, ac, s));
    } else {
      TIMED(KC_EMB_GRAD, k_emb_grad_reduce(st, fused_emb_partial, kFusedRows, E, G_("emb"), s));
      TIMED(KC_COLSUM, k_colsum_reduce(st, d_fcs, n_fcs, fcs_cols, fused_colpart, kFusedRows, s));
    }
    hip_check(hipGetLastError(), "step launch");
    return;
  }
  TIMED(KC_EMBED, k_embed(st, ctx, P_("emb"), C, E, X32, X16, R, s));
  if (lte) product(PS_LTE_DOWN, 0, R, s);
  if (low_rank) TIMED(KC_FDM_FWD, k_fdm_fwd(st, X32, A, slot, F, L, X1, nullptr, R, s));  // x' = x A_s
  TIMED(KC_FDM_FWD, k_fdm_fwd(st, X1, U, slot, L, L, Y32, Y16, R, s));  // Eq. 15
  if (lte) product(PS_LTE_UP, 0, R, s);
  if (low_rank) TIMED(KC_FDM_FWD, k_fdm_fwd(st, Y32, B, slot, L, F, Hs[0], nullptr, R, s));  // x'' = y B_s
  for (int j = 0; j < N; ++j) {
    const std::string ln = "ln" + std::to_string(j);
    TIMED(KC_LN_FWD, k_ln_fwd(st, Hs[j], P_(ln + ".gamma"), P_(ln + ".beta"), F,
                              bf16 ? nullptr : Z32[j], bf16 ? Z16[j] : nullptr, mean[j],
                              rstd[j], R, s));
    product(PS_GATE, j, R, s);
    product(PS_OUT, j, R, s);
  }
  product(PS_HEAD, 0, R, s);
  TIMED(KC_HEAD, k_head(st, ha, hio, R, s));
  if (out.loss) {
    TIMED(KC_COLSUM, k_colsum(st, d_loss_job, 1, 1, 1, loss_partial, R, s));
    hip_check(hipMemcpyAsync(out.loss, loss_out, sizeof(float), hipMemcpyDeviceToDevice, s), "copy");
  }
  if (!backward) return;

  // ---- adjoint of the mean cross entropy (Eq. 2) -------------------------
  product(PS_HEAD_BWD, 0, R, s);
  for (int j = N - 1; j >= 0; --j) {
    const std::string ln = "ln" + std::to_string(j);
    product(PS_GATE_BWD, j, R, s);
    product(PS_DZ, j, R, s);
    TIMED(KC_LN_BWD, k_ln_bwd(st, Hs[j], mean[j], rstd[j], P_(ln + ".gamma"), dZ[j],
                              dH32[j + 1], F, dH32[j], bf16 ? dH16[j] : nullptr,
                              ln_part.empty() ? nullptr : ln_part[j], R, s));
  }
  if (lte) product(PS_LTE_UP_BWD, 0, R, s);
  // low rank: dy = B_s dx'', dB_s = y (x) dx'' (B before its update), Adam on B_s
  if (low_rank)
    TIMED(KC_FDM_BWD, k_fdm_bwd(st, Y32, dH32[0], B, mB, vB, nullptr, slot, L, F, ac, out.update,
                                dY, nullptr, R, s));
  // adjoint of Eq. 15, fused with Adam on U_s
  TIMED(KC_FDM_BWD, k_fdm_bwd(st, X1, dY, U, mU, vU, out.keep_fdm_grad ? dUkeep : nullptr, slot,
                              L, L, ac, out.update, dX1_32, dX1_16, R, s));
  if (lte) product(PS_LTE_DOWN_BWD, 0, R, s);
  // low rank: dx = A_s dx', dA_s = x (x) dx', Adam on A_s
  if (low_rank)
    TIMED(KC_FDM_BWD, k_fdm_bwd(st, X32, dX1_32, A, mA, vA, nullptr, slot, F, L, ac, out.update,
                                dX, nullptr, R, s));
  TIMED(KC_EMB_GRAD, k_emb_grad(st, ctx, dX, C, E, emb_partial, emb_chunk, emb_sub, R, G_("emb"), s));
  product(PS_WGRAD, 0, R, s);
  TIMED(KC_COLSUM, k_colsum(st, d_cs, n_cs, cs_blocks, cs_cols, cs_partial, R, s));
  if (out.update) TIMED(KC_ADAM, k_adam(st, param, grad, m, v, p16, P, ac, s));
  hip_check(hipGetLastError(), "step launch");
}

// Time every tile configuration of every product on the model's own buffers
// (rows = max_rows) and keep the fastest.  Outputs of the trial launches are
// scratch: every buffer they write is rewritten by the first real step.
void Model::autotune(hipStream_t s) {
  const int R = (int)max_rows;
  k_step_explicit(st, R, 1, cfg.beta1, cfg.beta2, s);
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  KTimer* saved = timer;
  timer = nullptr;
  // the wide weight-gradient candidates run the balanced launch: scratch for
  // the largest of them during the trials, then for the tile chosen
  struct Scratch {
    void* p = nullptr;
    hipStream_t s;
    ~Scratch() {
      if (p) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(p);
      }
    }
  } trial;
  trial.s = s;
  float* const kept_part = wg_part;
  if (bf16) {
    size_t most = 0;
    for (int t = TILE_W128x128; t < TILE_COUNT; ++t) most = std::max(most, wgrad_part_floats(t));
    hip_check(hipMalloc(&trial.p, most * sizeof(float)), "hipMalloc");
    wg_part = (float*)trial.p;
  }
  for (int ps = 0; ps < PS_COUNT; ++ps) {
    const bool per_block = ps == PS_GATE || ps == PS_OUT || ps == PS_GATE_BWD || ps == PS_DZ;
    if (per_block && N == 0) continue;
    const bool lte_ps = ps == PS_LTE_DOWN || ps == PS_LTE_UP || ps == PS_LTE_UP_BWD ||
                        ps == PS_LTE_DOWN_BWD;
    if (lte_ps && !lte) continue;
    // row-block step: the weight-gradient tile also carries Adam in its
    // epilogue, whose cost the trials (the products alone) cannot see: the
    // 128 x 128 tile timed best here but took 45 against 34 us with Adam (112
    // work-groups move the Adam traffic).  It keeps its default.
    if (ps == PS_WGRAD && kc.fused) continue;
    int best = kc.tile[ps];
    float best_ms = 1e30f;
    const EpiKind epi = ps == PS_GATE ? EPI_GATE_FWD : ps == PS_GATE_BWD ? EPI_GATE_BWD : EPI_STORE;
    const int nb = ps == PS_GATE ? K : 1;
    for (int t = 0; t < TILE_COUNT; ++t) {
      const TileShape sh = tile_shape(t);
      if (!wide_tile_supported(t, bf16, epi, nb)) continue;
      if (ps != PS_WGRAD && sh.bm > 2 * R && t != TILE_32x32) continue;
      kc.tile[ps] = t;
      product(ps, 0, R, s);  // warm-up (first launch may set attributes)
      hip_check(hipEventRecord(e0, s), "event");
      for (int rep = 0; rep < 3; ++rep) product(ps, 0, R, s);
      hip_check(hipEventRecord(e1, s), "event");
      hip_check(hipEventSynchronize(e1), "event");
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
      if (ms < best_ms) { best_ms = ms; best = t; }
    }
    kc.tile[ps] = best;
  }
  wg_part = kept_part;
  if (bf16 && kc.tile[PS_WGRAD] >= TILE_W128x128 &&
      wg_tab[kc.tile[PS_WGRAD]].tiles >= kWgradRanges &&
      wgrad_part_floats(kc.tile[PS_WGRAD]) > wg_part_floats) {
    wg_part_floats = wgrad_part_floats(kc.tile[PS_WGRAD]);
    wg_part = dalloc<float>(wg_part_floats);
  }
  timer = saved;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

}  // namespace edpc
