// Row-block fused step (BF16 operands, FP32 accumulation); see fused.h.
#include "fused.h"
#include "head_row.h"

namespace edpc {

// ---------------------------------------------------------------------------
// Fragment-ordered BF16 weight copies
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) build_frags_kernel(const FragJob* __restrict__ jobs,
                                                          int n_jobs, int total_frags) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = gid & 63;
  const int f = gid >> 6;
  if (f >= total_frags) return;
  int j = 0;
  while (j + 1 < n_jobs && f >= jobs[j + 1].frag_begin) ++j;
  const FragJob jb = jobs[j];
  const int nfr = jb.rows * jb.cols / 512;  // 16 x 32 elements per fragment
  int local = f - jb.frag_begin;
  uint32_t w[4];
  if (local < nfr) {  // nt
    const int KB = jb.cols / 32;
    const int nb = local / KB, kb = local % KB;
    const float* s = jb.src + (size_t)(nb * 16 + (lane & 15)) * jb.cols + kb * 32 + 8 * (lane >> 4);
    const float4 a = __builtin_bit_cast(float4, ld_global16(s));
    const float4 b = __builtin_bit_cast(float4, ld_global16(s + 4));
    w[0] = (uint32_t)f2bf(a.x) | ((uint32_t)f2bf(a.y) << 16);
    w[1] = (uint32_t)f2bf(a.z) | ((uint32_t)f2bf(a.w) << 16);
    w[2] = (uint32_t)f2bf(b.x) | ((uint32_t)f2bf(b.y) << 16);
    w[3] = (uint32_t)f2bf(b.z) | ((uint32_t)f2bf(b.w) << 16);
    st_global16(jb.nt + (size_t)local * 64 + lane, make_uint4(w[0], w[1], w[2], w[3]));
  } else {  // nn
    local -= nfr;
    const int KB = jb.rows / 32;
    const int nb = local / KB, kb = local % KB;
    const int col = nb * 16 + (lane & 15);
    const int k0 = kb * 32 + 8 * (lane >> 4);
    bf16_t h[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) h[v] = f2bf(gl(jb.src)[(size_t)(k0 + v) * jb.cols + col]);
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = (uint32_t)h[2 * q] | ((uint32_t)h[2 * q + 1] << 16);
    st_global16(jb.nn + (size_t)local * 64 + lane, make_uint4(w[0], w[1], w[2], w[3]));
  }
}

void k_build_frags(const FragJob* jobs, int n_jobs, int total_frags, hipStream_t s) {
  if (total_frags == 0) return;
  const size_t threads = (size_t)total_frags * 64;
  hipLaunchKernelGGL(build_frags_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                     jobs, n_jobs, total_frags);
}

// in[i] holds 8 bf16 of row i; out[j] receives column j
__device__ __forceinline__ void transpose8x8(const uint4* in, uint4* out) {
  const uint32_t* w = (const uint32_t*)in;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int q = j >> 1;
    const uint32_t sel = (j & 1) ? 0x07060302u : 0x05040100u;
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      o[k] = __builtin_amdgcn_perm(w[4 * (2 * k + 1) + q], w[4 * (2 * k) + q], sel);
    out[j] = make_uint4(o[0], o[1], o[2], o[3]);
  }
}

// One workgroup per work item: a 32 x 64 tile of a matrix (one thread per
// row chunk of 8; the nt copy is written straight from registers, the nn copy
// after a transpose through LDS) or 256 elements of another tensor.
__global__ void __launch_bounds__(256) adam_frags_kernel(const StepState* __restrict__ st,
                                                         const AdamJob* __restrict__ jobs, int n_jobs,
                                                         float* __restrict__ p,
                                                         float* __restrict__ g,
                                                         float* __restrict__ m, float* __restrict__ v,
                                                         AdamCfg ac) {
  __shared__ __align__(16) bf16_t tile[kAdamTileRows][kAdamTileCols + 8];
  const int it = blockIdx.x;
  int j = 0;
  while (j + 1 < n_jobs && it >= jobs[j + 1].item_begin) ++j;
  const AdamJob jb = jobs[j];
  const int local = it - jb.item_begin;
  const float lr_bc = ac.lr / st->bc1;
  const float inv_bc2 = 1.0f / st->bc2;
  const int t = threadIdx.x;
  float gv[8], nv[8];
  if (jb.cols == 0) {  // element range, one element a thread
    adam_elements(st, jb, local, p, g, m, v, ac, lr_bc, inv_bc2);
    return;
  }
  const int tiles_c = jb.cols / kAdamTileCols;
  const int r0 = (local / tiles_c) * kAdamTileRows, c0 = (local % tiles_c) * kAdamTileCols;
  const int tr = t >> 3, tc = 8 * (t & 7);
  const int row = r0 + tr, col = c0 + tc;
  const size_t o = jb.off + (size_t)row * jb.cols + col;
  load8(g + o, gv);
  adam8(p + o, gv, m + o, v + o, lr_bc, inv_bc2, ac, nv);
  const uint4 pk = pack_bf16x8(nv);
  // nt fragment (nb = row/16, kb = col/32), lane = row%16 + 16*((col%32)/8)
  st_global16(jb.nt + ((size_t)(row >> 4) * (jb.cols / 32) + (col >> 5)) * 64 + (row & 15) +
                  16 * ((col & 31) >> 3), pk);
  *(uint4*)&tile[tr][tc] = pk;
  __syncthreads();
  // nn fragment (nb = col/16, kb = row/32), lane = col%16 + 16*((row%32)/8):
  // the tile holds kb = r0/32 of column blocks c0/16 .. c0/16 + 3
  const int f = t >> 6, l = t & 63;
  const int cc = 16 * f + (l & 15), rr = 8 * (l >> 4);
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    w[k] = (uint32_t)tile[rr + 2 * k][cc] | ((uint32_t)tile[rr + 2 * k + 1][cc] << 16);
  st_global16(jb.nn + ((size_t)((c0 + cc) >> 4) * (jb.rows / 32) + (r0 >> 5)) * 64 + l,
              make_uint4(w[0], w[1], w[2], w[3]));
}

void k_adam_frags(const StepState* st, const AdamJob* jobs, int n_jobs, int total_items, float* p,
                  float* g, float* m, float* v, AdamCfg ac, hipStream_t s) {
  if (total_items == 0) return;
  hipLaunchKernelGGL(adam_frags_kernel, dim3(total_items), dim3(256), 0, s, st, jobs, n_jobs, p, g,
                     m, v, ac);
}

// ---------------------------------------------------------------------------
// Row-block products
// ---------------------------------------------------------------------------
// Word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format,
// no swizzle, no index stride).
constexpr int kBufferWord3 = 0x00020000;

__device__ __forceinline__ f32x4 mfma16(uint4 a, uint4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// acc[t] = A (16 rows in LDS, bf16, row stride lda, K columns) x fragments of
// column block cb[t] (fragment base + cb*K/32*64 uint4), for the NT column
// blocks of this wave (cb must be wave-uniform).  The wave's fragments, taken
// in the order i = kb * NT + t, stream in batches of B buffer loads issued back
// to back; batch b + 1 is issued before batch b feeds the MFMAs, so up to 2B
// loads are in flight.  Each load takes the lane offset from one VGPR and the
// fragment offset from an SGPR, so in-flight loads cost no address registers.
// The scheduling barriers keep the compiler from sinking the loads next to
// their uses.
template <int K, int NT, int B>
struct MmShape {
  static constexpr int KB = K / 32;
  static constexpr int TOT = KB * NT;
  static constexpr int BB = B < TOT ? B : TOT;
  static constexpr int NBT = (TOT + BB - 1) / BB;
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t frag_rsrc(const uint4* base) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7FFFFFFF, kBufferWord3);
}

// First batch of a product's fragment loads, into buf[0 .. BB-1]; issued
// ahead of the product (before the previous stage's epilogue) so that its
// latency overlaps that work.
template <int K, int NT, int B>
__device__ __forceinline__ void mm_first(const uint4* __restrict__ base, const int (&cb)[NT],
                                         uint4 (&buf)[B]) {
  typedef MmShape<K, NT, B> S;
  const __amdgpu_buffer_rsrc_t rs = frag_rsrc(base);
  const int voff = (threadIdx.x & 63) * 16;
#pragma unroll
  for (int q = 0; q < S::BB; ++q) {
    const int soff = (cb[q % NT] * S::KB + q / NT) * 1024;
    buf[q] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
  }
}

// The product, its first batch already in first[] (see mm_first).
template <int K, int NT, int B, typename Between>
__device__ __forceinline__ void mm_rest(const bf16_t* sA, int lda, const uint4* __restrict__ base,
                                        const int (&cb)[NT], f32x4 (&acc)[NT],
                                        const uint4 (&first)[B], Between&& between) {
  typedef MmShape<K, NT, B> S;
  constexpr int KB = S::KB, TOT = S::TOT, BB = S::BB, NBT = S::NBT;
  const int lane = threadIdx.x & 63;
  const __amdgpu_buffer_rsrc_t rs = frag_rsrc(base);
  const int voff = lane * 16;
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto frag = [&](int i) -> uint4 {
    const int soff = (cb[i % NT] * KB + i / NT) * 1024;
    return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
  };
  const bf16_t* arow = sA + (lane & 15) * lda + 8 * (lane >> 4);
  uint4 buf[2][BB];
#pragma unroll
  for (int q = 0; q < BB; ++q) buf[0][q] = first[q];
  // work that only needs the LDS state left by the previous stage (copies of
  // its results to global memory) goes behind the first batch, so the
  // fragment waits do not include its stores
  __builtin_amdgcn_sched_barrier(0);
  between();
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int b = 0; b < NBT; ++b) {
    if (b + 1 < NBT) {
#pragma unroll
      for (int q = 0; q < BB; ++q) {
        const int i = (b + 1) * BB + q;
        if (i < TOT) buf[(b + 1) & 1][q] = frag(i);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < BB; ++q) {
      const int i = b * BB + q;
      if (i < TOT) {
        const uint4 av = *(const uint4*)(arow + (i / NT) * 32);
        acc[i % NT] = mfma16(av, buf[b & 1][q], acc[i % NT]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// acc[t] = A (16 rows in LDS, bf16, row stride lda, K columns) x fragments of
// column block cb[t] (fragment base + cb*K/32*64 uint4), for the NT column
// blocks of this wave (cb must be wave-uniform).  The wave's fragments, taken
// in the order i = kb * NT + t, stream in batches of B buffer loads issued back
// to back; batch b + 1 is issued before batch b feeds the MFMAs, so up to 2B
// loads are in flight.  Each load takes the lane offset from one VGPR and the
// fragment offset from an SGPR, so in-flight loads cost no address registers.
// The scheduling barriers keep the compiler from sinking the loads next to
// their uses.
template <int K, int NT, int B, typename Between>
__device__ __forceinline__ void mm(const bf16_t* sA, int lda, const uint4* __restrict__ base,
                                   const int (&cb)[NT], f32x4 (&acc)[NT], Between&& between) {
  uint4 first[B];
  mm_first<K, NT, B>(base, cb, first);
  mm_rest<K, NT, B>(sA, lda, base, cb, acc, first, between);
}

template <int K, int NT, int B>
__device__ __forceinline__ void mm(const bf16_t* sA, int lda, const uint4* __restrict__ base,
                                   const int (&cb)[NT], f32x4 (&acc)[NT]) {
  mm<K, NT, B>(sA, lda, base, cb, acc, [] {});
}

// Barrier for LDS traffic only: waits for the wave's LDS accesses, not for its
// outstanding global loads and stores.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kFusedWaves = 8;  // waves of a row-block workgroup

// Coder inputs of one row, staged in LDS at the start of the fused step.
struct RowCoder {
  RcEnc enc;       // encoder state (encode)
  RcDec dec;       // decoder state (decode)
  uint64_t poff;   // payload offset
  uint64_t pcap;   // payload capacity / length
  uint64_t off;    // stream offset (decoder output)
  uint32_t s;      // stream index
  int32_t tgt;     // target byte (encode / plain step)
};
constexpr int kFusedThreads = 64 * kFusedWaves;
constexpr int kFusedBatch = 8;  // weight fragments per load batch and wave

template <int F, int L, int H>
struct FusedDims {
  static constexpr int BM = kFusedRows;
  static constexpr int NW = kFusedWaves;
  static constexpr int RPW = BM / NW;  // rows per wave in the row-wise stages
  static constexpr int H2 = 2 * H;
  static constexpr int KM0 = F > H2 ? F : H2;
  static constexpr int KMAX = KM0 > 256 ? KM0 : 256;
  static constexpr int LDA = KMAX + 8;   // bf16 row stride
  static constexpr int LDF = KMAX + 4;   // fp32 row stride
  static constexpr int LDH = F + 4;
  static constexpr size_t OFF_H = 0;
  static constexpr size_t OFF_F = OFF_H + (size_t)BM * LDH * 4;
  static constexpr size_t OFF_A = OFF_F + (size_t)BM * LDF * 4;
  static constexpr size_t OFF_B = OFF_A + (size_t)BM * LDA * 2;
  static constexpr size_t OFF_RED = OFF_B + (size_t)BM * LDA * 2;
  static constexpr size_t OFF_STAT = OFF_RED + (size_t)NW * BM * 2 * 4;
  static constexpr size_t OFF_GB = OFF_STAT + (size_t)kMaxFusedBlocks * BM * 2 * 4;
  static constexpr size_t OFF_CODE = OFF_GB + (size_t)2 * F * 4;
  static constexpr size_t BYTES = OFF_CODE + (size_t)BM * sizeof(RowCoder);
  static_assert(BM % NW == 0, "rows per wave");
};

// Column blocks (16 outputs each) of a product with N outputs, dealt to the
// waves: wave w takes blocks w, w + NW, ...; a product with fewer blocks than
// waves leaves the last waves idle.
template <int N>
struct ColSplit {
  static constexpr int NCB = N / 16;
  static_assert(N % 16 == 0 && (NCB % kFusedWaves == 0 || NCB < kFusedWaves), "column split");
  static constexpr int NT = NCB >= kFusedWaves ? NCB / kFusedWaves : 1;
  __device__ static bool active(int w) { return NCB >= kFusedWaves || w < NCB; }
};

// Rows [0, nr) of an LDS tile (row stride ld_l elements) to global rows
// r0 .. r0 + nr - 1 (row stride ld_g), in 16-byte pieces over the workgroup.
template <int COLS, typename T>
__device__ __forceinline__ void copy_rows(const T* lds, int ld_l, T* g, int ld_g, int r0, int nr) {
  constexpr int V = 16 / sizeof(T);
  constexpr int CH = COLS / V;
  for (int idx = threadIdx.x; idx < nr * CH; idx += kFusedThreads) {
    const int i = idx / CH, q = idx - i * CH;
    *(uint4*)(g + (r0 + i) * ld_g + q * V) = *(const uint4*)(lds + i * ld_l + q * V);
  }
}

// Column sums over rows [0, nr) of an LDS tile -> one row of partials.
template <int COLS>
__device__ __forceinline__ void col_sums(const float* lds, int ld_l, int nr, float* out) {
  for (int c = threadIdx.x; c < COLS; c += kFusedThreads) {
    float v[kFusedRows];
#pragma unroll
    for (int i = 0; i < kFusedRows; ++i) v[i] = i < nr ? lds[i * ld_l + c] : 0.f;
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kFusedRows; ++i) s += v[i];  // rows in order
    out[c] = s;
  }
}

template <int F, int L, int H>
__global__ void __launch_bounds__(kFusedThreads, 1) fused_kernel(FusedArgs a) {
  typedef FusedDims<F, L, H> D;
  constexpr int BM = D::BM, NW = D::NW, RPW = D::RPW, H2 = D::H2, LDA = D::LDA, LDF = D::LDF,
                LDH = D::LDH;
  static_assert((H / 16) % NW == 0, "branch columns per wave");
  extern __shared__ __align__(16) char smem[];
  float (*sH)[LDH] = (float (*)[LDH])(smem + D::OFF_H);      // residual stream / its adjoint
  float (*sF)[LDF] = (float (*)[LDF])(smem + D::OFF_F);      // fp32 scratch (branches, logits, dz, dA)
  bf16_t (*sA)[LDA] = (bf16_t (*)[LDA])(smem + D::OFF_A);    // product operand
  bf16_t (*sB)[LDA] = (bf16_t (*)[LDA])(smem + D::OFF_B);    // second product operand
  float (*sRed)[BM][2] = (float (*)[BM][2])(smem + D::OFF_RED);
  float (*sStat)[BM][2] = (float (*)[BM][2])(smem + D::OFF_STAT);
  float (*sGB)[F] = (float (*)[F])(smem + D::OFF_GB);         // LayerNorm affine gradients
  RowCoder* sCode = (RowCoder*)(smem + D::OFF_CODE);

  const StepState* st = a.st;
  const int rows = st->rows;
  const int r0 = blockIdx.x * BM;
  if (r0 >= rows) return;
  const int nr = min(BM, rows - r0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index (uniform)
  const int li = 4 * (lane >> 4), lc = lane & 15;
  float* colp = a.colpart + (size_t)blockIdx.x * a.colpart_cols;
  const int NB = a.n_blocks;
  const int mode = a.head.mode;
  // next product's first batch of weight fragments, issued before the
  // current stage's epilogue
  uint4 pf[kFusedBatch];
  constexpr int NTF = ColSplit<F>::NT, NHH = ColSplit<H>::NT;
  auto cb_cols = [&](auto& cb) {  // column blocks w, w + NW, ...
#pragma unroll
    for (int t = 0; t < (int)(sizeof(cb) / sizeof(cb[0])); ++t) cb[t] = w + NW * t;
  };
  auto cb_branches = [&](int (&cb)[2 * NHH]) {  // both branches' blocks
#pragma unroll
    for (int t = 0; t < NHH; ++t) {
      cb[t] = w + NW * t;
      cb[NHH + t] = H / 16 + w + NW * t;
    }
  };

  // ---- LTE up-projection (Eq. 16): X'' = W2 Y + b2 -------------------------
  if (w == NW - 1) {
    // the last wave stages the coder inputs of the block's rows
    if (lane < BM) {
      // field by field into LDS (a local RowCoder filled under these
      // branches is kept in scratch memory by the compiler)
      RowCoder& rc = sCode[lane];
      uint32_t s = 0u;
      int32_t tgt = 0;
      uint64_t poff = 0, pcap = 0, off = 0;
      if (lane < nr) {
        const int r = r0 + lane;
        s = a.io.slot ? a.io.slot[r] : 0u;
        if (mode != 2 && a.head.target) tgt = a.head.target[r];
        if (mode != 0) {
          poff = a.io.pay_off[s];
          pcap = a.io.pay_cap[s];
        }
        if (mode == 2) off = a.io.off[s];
      }
      const bool live = lane < nr;
      rc.enc = live && mode == 1 ? a.io.enc[s] : RcEnc{};
      rc.dec = live && mode == 2 ? a.io.dec[s] : RcDec{};
      rc.poff = poff;
      rc.pcap = pcap;
      rc.off = off;
      rc.s = s;
      rc.tgt = tgt;
    }
  } else {
    // the others stage the FDM output
    for (int idx = tid; idx < BM * (L / 8); idx += kFusedThreads - 64) {
      const int i = idx / (L / 8), q = idx % (L / 8);
      uint4 v = make_uint4(0, 0, 0, 0);
      if (i < nr) v = *(const uint4*)(a.y16 + (r0 + i) * L + 8 * q);
      *(uint4*)(&sA[i][8 * q]) = v;
    }
  }
  __syncthreads();
  {
    constexpr int NT = ColSplit<F>::NT;
    int cb[NT];
    f32x4 acc[NT];
    float bias[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      cb[t] = w + NW * t;
      bias[t] = a.b2[cb[t] * 16 + lc];
    }
    mm<L, NT, kFusedBatch>(&sA[0][0], LDA, a.w2_nt, cb, acc);
    {
      int cbn[2 * NHH];
      cb_branches(cbn);
      mm_first<F, 2 * NHH, kFusedBatch>(a.wab_nt[0], cbn, pf);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int c = cb[t] * 16 + lc;
#pragma unroll
      for (int r = 0; r < 4; ++r) sH[li + r][c] = acc[t][r] + bias[t];
    }
  }
  lds_barrier();

  // ---- refinement blocks (Eqs. 9-13) ----------------------------------------
  for (int j = 0; j < NB; ++j) {
    // LayerNorm (Eq. 9): wave w normalises rows RPW w .. RPW w + RPW - 1
    constexpr int FV = F / 64;
    float gmr[FV], btr[FV];
#pragma unroll
    for (int k = 0; k < FV; ++k) {
      gmr[k] = a.gamma[j][lane + 64 * k];
      btr[k] = a.beta[j][lane + 64 * k];
    }
    for (int q = 0; q < RPW; ++q) {
      const int i = RPW * w + q;
      float s = 0.f;
#pragma unroll
      for (int k = 0; k < FV; ++k) s += sH[i][lane + 64 * k];
      const float mu = wave_sum(s) / (float)F;
      float v2 = 0.f;
#pragma unroll
      for (int k = 0; k < FV; ++k) {
        const float d = sH[i][lane + 64 * k] - mu;
        v2 += d * d;
      }
      const float rs = 1.0f / sqrtf(wave_sum(v2) / (float)F + 1e-5f);
#pragma unroll
      for (int k = 0; k < FV; ++k) {
        const int f = lane + 64 * k;
        sA[i][f] = f2bf((sH[i][f] - mu) * rs * gmr[k] + btr[k]);
      }
      if (lane == 0) {
        sStat[j][i][0] = mu;
        sStat[j][i][1] = rs;
      }
    }
    lds_barrier();
    {  // branches (Eq. 10), product fusion (Eq. 11), GeLU (Eq. 12)
      constexpr int NH = ColSplit<H>::NT;
      constexpr int NT = 2 * NH;
      int cb[NT];
      f32x4 acc[NT];
      float bias0[NH], bias1[NH];
#pragma unroll
      for (int t = 0; t < NH; ++t) {
        cb[t] = w + NW * t;
        cb[NH + t] = H / 16 + w + NW * t;
        bias0[t] = a.bab[j][cb[t] * 16 + lc];
        bias1[t] = a.bab[j][H + cb[t] * 16 + lc];
      }
      mm_rest<F, NT, kFusedBatch>(&sA[0][0], LDA, a.wab_nt[j], cb, acc, pf, [&] {
        copy_rows<F>(&sA[0][0], LDA, a.z16[j], F, r0, nr);   // LayerNorm output
        copy_rows<F>(&sH[0][0], LDH, a.hs[j], F, r0, nr);    // block input
      });
      {
        int cbn[NTF];
        cb_cols(cbn);
        mm_first<H, NTF, kFusedBatch>(a.wo_nt[j], cbn, pf);
      }
#pragma unroll
      for (int t = 0; t < NH; ++t) {
        const int c = cb[t] * 16 + lc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = li + r;
          const float a0 = acc[t][r] + bias0[t];
          const float a1 = acc[NH + t][r] + bias1[t];
          sB[i][c] = f2bf(gelu_f(a0 * a1));
          sF[i][c] = a0;
          sF[i][H + c] = a1;
        }
      }
    }
    lds_barrier();
    {  // output linear + residual (Eq. 13)
      constexpr int NT = ColSplit<F>::NT;
      int cb[NT];
      f32x4 acc[NT];
      float bias[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        cb[t] = w + NW * t;
        bias[t] = a.bo[j][cb[t] * 16 + lc];
      }
      mm_rest<H, NT, kFusedBatch>(&sB[0][0], LDA, a.wo_nt[j], cb, acc, pf, [&] {
        copy_rows<H>(&sB[0][0], LDA, a.g16[j], H, r0, nr);     // GeLU output
        copy_rows<H2>(&sF[0][0], LDF, a.abr[j], H2, r0, nr);   // branch values
      });
      if (j + 1 < NB) {
        int cbn[2 * NHH];
        cb_branches(cbn);
        mm_first<F, 2 * NHH, kFusedBatch>(a.wab_nt[j + 1], cbn, pf);
      } else {
        int cbn[ColSplit<256>::NT];
        cb_cols(cbn);
        mm_first<F, ColSplit<256>::NT, kFusedBatch>(a.wh_nt, cbn, pf);
      }
      const bool last = j == NB - 1;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int c = cb[t] * 16 + lc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = li + r;
          const float v = acc[t][r] + bias[t] + sH[i][c];
          sH[i][c] = v;
          if (last) sA[i][c] = f2bf(v);
        }
      }
    }
    lds_barrier();
  }

  // ---- head logits ------------------------------------------------------------
  {
    constexpr int NT = ColSplit<256>::NT;
    int cb[NT];
    f32x4 acc[NT];
    float bias[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      cb[t] = w + NW * t;
      bias[t] = a.bh[cb[t] * 16 + lc];
    }
    mm_rest<F, NT, kFusedBatch>(&sA[0][0], LDA, a.wh_nt, cb, acc, pf, [&] {
      copy_rows<F>(&sA[0][0], LDA, a.hn16, F, r0, nr);  // final features
    });
    if (a.head.want_grad) {
      int cbn[NTF];
      cb_cols(cbn);
      mm_first<256, NTF, kFusedBatch>(a.wh_nn, cbn, pf);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int c = cb[t] * 16 + lc;
#pragma unroll
      for (int r = 0; r < 4; ++r) sF[li + r][c] = acc[t][r] + bias[t];
    }
  }
  lds_barrier();

  // ---- softmax, CDF, coder, cross-entropy adjoint (Eqs. 1-2) ------------------
  const bool grad = a.head.want_grad != 0;
  const bool have_target = mode != 0 || a.head.target != nullptr;
  int my_cx = 0, my_qx = 0, my_x = 0;
  for (int q = 0; q < RPW; ++q) {
    const int i = RPW * w + q;
    float d[4] = {0.f, 0.f, 0.f, 0.f};
    if (i < nr) {
      const float z[4] = {sF[i][4 * lane], sF[i][4 * lane + 1], sF[i][4 * lane + 2],
                          sF[i][4 * lane + 3]};
      RowCdf c;
      row_cdf(lane, z, c);
      const int x = mode == 2 ? row_decode_symbol(c, sCode[i].dec.d, sCode[i].dec.range) : sCode[i].tgt;
      int cx, qx;
      float zx;
      row_pick(c, z, x, &cx, &qx, &zx);
      if (lane == q) {
        my_cx = cx;
        my_qx = qx;
        my_x = x;
        if (have_target && a.head.loss_rows) a.head.loss_rows[r0 + i] = logf(c.S) - (zx - c.m);
      }
      row_outputs(a.head, r0 + i, lane, c);
      if (have_target && grad) {
        const float ir = st->inv_rows;
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k] = (c.p[k] - (4 * lane + k == x ? 1.0f : 0.0f)) * ir;
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sF[i][4 * lane + k] = d[k];
      sA[i][4 * lane + k] = f2bf(d[k]);
    }
  }
  // range-coder lanes: lane q of wave w codes row RPW w + q
  const int my_i = RPW * w + lane;
  if (lane < RPW && my_i < nr && mode != 0) {
    const RowCoder& rc = sCode[my_i];
    if (mode == 1) {
      RcEnc en = rc.enc;
      rc_encode(en, a.io.pay + rc.poff, rc.pcap, (uint32_t)my_cx, (uint32_t)my_qx);
      a.io.enc[rc.s] = en;
    } else {
      RcDec de = rc.dec;
      rc_consume(de, a.io.pay_in + rc.poff, rc.pcap, (uint32_t)my_cx, (uint32_t)(my_cx + my_qx));
      a.io.dec[rc.s] = de;
      a.io.dst[io_at(a.io, rc.off, (uint64_t)st->step)] = (uint8_t)my_x;
      if (a.head.target_out) a.head.target_out[r0 + my_i] = (uint8_t)my_x;
    }
  }
  if (!grad) return;
  __syncthreads();
  {  // dH_N = dz Wh
    constexpr int NT = ColSplit<F>::NT;
    int cb[NT];
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) cb[t] = w + NW * t;
    mm_rest<256, NT, kFusedBatch>(&sA[0][0], LDA, a.wh_nn, cb, acc, pf, [&] {
      copy_rows<256>(&sA[0][0], LDA, a.dz16, 256, r0, nr);      // logit adjoint
      col_sums<256>(&sF[0][0], LDF, nr, colp + a.off_bh);       // head bias gradient
    });
    {
      int cbn[NHH];
      cb_cols(cbn);
      mm_first<F, NHH, kFusedBatch>(a.wo_nn[NB - 1], cbn, pf);
    }
    lds_barrier();  // every wave is done reading sA / sF
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int c = cb[t] * 16 + lc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = li + r;
        sH[i][c] = acc[t][r];
        sA[i][c] = f2bf(acc[t][r]);
      }
    }
  }
  lds_barrier();

  for (int j = NB - 1; j >= 0; --j) {
    {  // dX_ff = dH Wo; through GeLU and the branch product (adjoint of Eqs. 11-13)
      constexpr int NH = ColSplit<H>::NT;
      int cb[NH];
      f32x4 acc[NH];
      float sa0[NH][4], sa1[NH][4];  // saved branch values (Eq. 10)
#pragma unroll
      for (int t = 0; t < NH; ++t) {
        cb[t] = w + NW * t;
        const int c = cb[t] * 16 + lc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = li + r;
          sa0[t][r] = 0.f;
          sa1[t][r] = 0.f;
          if (i < nr) {
            sa0[t][r] = a.abr[j][(r0 + i) * H2 + c];
            sa1[t][r] = a.abr[j][(r0 + i) * H2 + H + c];
          }
        }
      }
      mm_rest<F, NH, kFusedBatch>(&sA[0][0], LDA, a.wo_nn[j], cb, acc, pf, [&] {
        copy_rows<F>(&sA[0][0], LDA, a.dh16[j + 1], F, r0, nr);  // adjoint of the block output
        col_sums<F>(&sH[0][0], LDH, nr, colp + a.off_bo[j]);     // output bias gradient
        if (j + 1 < NB) {  // affine gradients of the LayerNorm of block j + 1
          for (int c = tid; c < F; c += kFusedThreads) {
            colp[a.off_beta[j + 1] + c] = sGB[0][c];
            colp[a.off_gamma[j + 1] + c] = sGB[1][c];
          }
        }
      });
      {
        int cbn[NTF];
        cb_cols(cbn);
        mm_first<H2, NTF, kFusedBatch>(a.wab_nn[j], cbn, pf);
      }
#pragma unroll
      for (int t = 0; t < NH; ++t) {
        const int c = cb[t] * 16 + lc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = li + r;
          const float a0 = sa0[t][r], a1 = sa1[t][r];
          const float dp = acc[t][r] * gelu_grad_f(a0 * a1);
          const float d0 = dp * a1, d1 = dp * a0;
          sF[i][c] = d0;
          sF[i][H + c] = d1;
          sB[i][c] = f2bf(d0);
          sB[i][H + c] = f2bf(d1);
        }
      }
    }
    lds_barrier();
    {  // dX0 = sum_i dX_i W_i, then the LayerNorm adjoint (Eq. 9)
      constexpr int NT = ColSplit<F>::NT;
      int cb[NT];
      f32x4 acc[NT];
      float xh[NT][4], gmr[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        cb[t] = w + NW * t;
        const int c = cb[t] * 16 + lc;
        gmr[t] = a.gamma[j][c];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = li + r;
          xh[t][r] = i < nr ? a.hs[j][(r0 + i) * F + c] : 0.f;
        }
      }
      mm_rest<H2, NT, kFusedBatch>(&sB[0][0], LDA, a.wab_nn[j], cb, acc, pf, [&] {
        copy_rows<H2>(&sB[0][0], LDA, a.da16[j], H2, r0, nr);  // branch adjoints
        col_sums<H2>(&sF[0][0], LDF, nr, colp + a.off_bab[j]);  // branch bias gradients
      });
      if (j > 0) {
        int cbn[NHH];
        cb_cols(cbn);
        mm_first<F, NHH, kFusedBatch>(a.wo_nn[j - 1], cbn, pf);
      } else if (ColSplit<L>::active(w)) {
        int cbn[ColSplit<L>::NT];
        cb_cols(cbn);
        mm_first<F, ColSplit<L>::NT, kFusedBatch>(a.w2_nn, cbn, pf);
      }
      float s1[4] = {0.f, 0.f, 0.f, 0.f}, s2[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int c = cb[t] * 16 + lc;
        float cz = 0.f, czx = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = li + r;
          float x = 0.f, dz = 0.f;
          if (i < nr) {
            x = (xh[t][r] - sStat[j][i][0]) * sStat[j][i][1];
            dz = acc[t][r];
          }
          xh[t][r] = x;
          acc[t][r] = dz * gmr[t];  // dxhat
          s1[r] += acc[t][r];
          s2[r] += acc[t][r] * x;
          cz += dz;
          czx += dz * x;
        }
        // LayerNorm affine gradients: column sums over the 16 rows
        cz += __shfl_xor(cz, 16, 64);
        cz += __shfl_xor(cz, 32, 64);
        czx += __shfl_xor(czx, 16, 64);
        czx += __shfl_xor(czx, 32, 64);
        if (lane < 16) {
          sGB[0][c] = cz;
          sGB[1][c] = czx;
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) {
          s1[r] += __shfl_xor(s1[r], o, 64);
          s2[r] += __shfl_xor(s2[r], o, 64);
        }
        if (lc == 0) {
          sRed[w][li + r][0] = s1[r];
          sRed[w][li + r][1] = s2[r];
        }
      }
      lds_barrier();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = li + r;
        float m1 = 0.f, m2 = 0.f;
#pragma unroll
        for (int u = 0; u < NW; ++u) {  // waves in a fixed order
          m1 += sRed[u][i][0];
          m2 += sRed[u][i][1];
        }
        m1 /= (float)F;
        m2 /= (float)F;
        const float rs = sStat[j][i][1];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int c = cb[t] * 16 + lc;
          float dh = 0.f;
          if (i < nr) dh = sH[i][c] + rs * (acc[t][r] - m1 - xh[t][r] * m2);
          sH[i][c] = dh;
          sA[i][c] = f2bf(dh);
        }
      }
    }
    lds_barrier();
  }

  // ---- adjoint of Eq. 16 ---------------------------------------------------------
  auto tail = [&] {
    copy_rows<F>(&sA[0][0], LDA, a.dh16[0], F, r0, nr);  // adjoint of the LTE output
    col_sums<F>(&sH[0][0], LDH, nr, colp + a.off_b2);    // b2 gradient
    for (int c = tid; c < F; c += kFusedThreads) {       // LayerNorm of block 0
      colp[a.off_beta[0] + c] = sGB[0][c];
      colp[a.off_gamma[0] + c] = sGB[1][c];
    }
  };
  if (ColSplit<L>::active(w)) {
    constexpr int NT = ColSplit<L>::NT;
    int cb[NT];
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) cb[t] = w + NW * t;
    mm_rest<F, NT, kFusedBatch>(&sA[0][0], LDA, a.w2_nn, cb, acc, pf, tail);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int c = cb[t] * 16 + lc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = li + r;
        if (i < nr) a.dy[(r0 + i) * L + c] = acc[t][r];
      }
    }
  } else {
    tail();
  }
}

// ---------------------------------------------------------------------------
// Before the FDM: gather, embedding, LTE down-projection
// ---------------------------------------------------------------------------
template <int F, int L, int E>
__global__ void __launch_bounds__(256) fused_in_kernel(FusedInArgs a) {
  constexpr int C = F / E;
  constexpr int BM = kFusedRows, LDA = F + 8;
  __shared__ __align__(16) bf16_t sA[BM][LDA];
  __shared__ uint8_t sC[BM][256];
  StepState* st = a.st;
  int step, rows;
  if (a.sched_mode == 0) {
    step = st->step;
    rows = st->rows;
  } else {
    // every workgroup finds the step's rows; the first one records the step
    // state for the later kernels (none of this launch reads st->step)
    step = a.sched_mode == 1 ? a.sched_step : st->base + a.sched_step;
    rows = active_rows(a.sched, step);
    if (blockIdx.x == 0 && threadIdx.x == 0) write_step_state(st, a.sched, step, rows);
  }
  const int r0 = blockIdx.x * BM;
  if (r0 >= rows) return;
  const int nr = min(BM, rows - r0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index (uniform)
  // the product's first batch of W1 fragments goes out before the gather, so
  // its latency overlaps the dependent loads of the context bytes
  constexpr int NT = L / 64;
  int cb[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) cb[t] = w + 4 * t;
  uint4 first[8];
  mm_first<F, NT, 8>(a.w1_nt, cb, first);
  for (int idx = tid; idx < BM * C; idx += 256) {
    const int i = idx / C, c = idx % C;
    uint8_t v = 0;
    if (i < nr) {
      const int r = r0 + i;
      if (a.gather) {
        const uint32_t sidx = a.io.slot[r];
        const uint8_t* base = a.decoding ? a.io.dst : a.io.src;
        const uint64_t o = a.io.off[sidx];
        v = base[io_at(a.io, o, (uint64_t)(step - C + c))];
        a.ctx[(size_t)r * C + c] = v;
        if (!a.decoding && c == 0) a.tgt[r] = a.io.src[io_at(a.io, o, (uint64_t)step)];
      } else {
        v = a.ctx[(size_t)r * C + c];
      }
    }
    sC[i][c] = v;
  }
  __syncthreads();
  // byte embedding, oldest byte first: X[i][c*E + e] = Emb[ctx[i][c]][e]
  for (int idx = tid; idx < BM * F / 4; idx += 256) {
    const int i = idx / (F / 4), f = (idx % (F / 4)) * 4;
    const int c = f / E, e = f % E;
    const float4 v = *(const float4*)(a.emb + (size_t)sC[i][c] * E + e);
    const ushort4 h = make_ushort4(f2bf(v.x), f2bf(v.y), f2bf(v.z), f2bf(v.w));
    *(ushort4*)(&sA[i][f]) = h;
    if (i < nr) *(ushort4*)(a.x16 + (size_t)(r0 + i) * F + f) = h;
  }
  __syncthreads();
  f32x4 acc[NT];
  float bias[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) bias[t] = a.b1[cb[t] * 16 + (lane & 15)];
  mm_rest<F, NT, 8>(&sA[0][0], LDA, a.w1_nt, cb, acc, first, [] {});
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = cb[t] * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * (lane >> 4) + r;
      if (i < nr) a.x1[(size_t)(r0 + i) * L + c] = acc[t][r] + bias[t];
    }
  }
}

// ---------------------------------------------------------------------------
// After the FDM adjoint: dX = dX' W1, embedding gradient partial, b1 partial
// ---------------------------------------------------------------------------
template <int F, int L, int E>
__global__ void __launch_bounds__(256) fused_out_kernel(FusedOutArgs a) {
  constexpr int C = F / E;
  constexpr int BM = kFusedRows, LDA = L + 8, LDX = F + 4;
  __shared__ __align__(16) bf16_t sA[BM][LDA];
  __shared__ __align__(16) float sX[BM][LDX];
  __shared__ __align__(16) uint8_t sC[BM * 256 + 16];
  const StepState* st = a.st;
  const int rows = st->rows;
  const int r0 = blockIdx.x * BM;
  if (r0 >= rows) return;
  const int nr = min(BM, rows - r0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index (uniform)
  // the product's first batch of W1 fragments goes out before the loads of
  // dX' and the b1 partial, so their latencies overlap
  constexpr int NTO = F / 64;
  int cbo[NTO];
#pragma unroll
  for (int t = 0; t < NTO; ++t) cbo[t] = w + 4 * t;
  uint4 first[8];
  mm_first<L, NTO, 8>(a.w1_nn, cbo, first);
  for (int idx = tid; idx < BM * (L / 8); idx += 256) {
    const int i = idx / (L / 8), q = idx % (L / 8);
    uint4 v = make_uint4(0, 0, 0, 0);
    if (i < nr) v = *(const uint4*)(a.dx1_16 + (size_t)(r0 + i) * L + 8 * q);
    *(uint4*)(&sA[i][8 * q]) = v;
  }
  for (int idx = tid; idx < BM * C; idx += 256)
    sC[idx] = (idx / C) < nr ? a.ctx[(size_t)r0 * C + idx] : 0;
  float* colp = a.colpart + (size_t)blockIdx.x * a.colpart_cols;
  for (int c = tid; c < L; c += 256) {  // b1 gradient partial, rows in order
    float v[BM];
#pragma unroll
    for (int i = 0; i < BM; ++i) v[i] = i < nr ? a.dx1_32[(size_t)(r0 + i) * L + c] : 0.f;
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < BM; ++i) s += v[i];
    colp[a.off_b1 + c] = s;
  }
  __syncthreads();
  {
    f32x4 acc[NTO];
    mm_rest<L, NTO, 8>(&sA[0][0], LDA, a.w1_nn, cbo, acc, first, [] {});
#pragma unroll
    for (int t = 0; t < NTO; ++t) {
      const int c = cbo[t] * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) sX[4 * (lane >> 4) + r][c] = acc[t][r];
    }
  }
  __syncthreads();
  // dEmb_block[v][e] = sum over pairs p = (i, c), i < nr, of [ctx = v] dX[i][c E + e]:
  // BF16 one-hot product, pairs in increasing order in 32-pair MFMA steps.
  // Wave w owns byte values 64w .. 64w+63 (4 blocks of 16), E/16 column blocks.
  const int np = nr * C;
  const int NE = E / 16;
  f32x4 acc[4][4];
#pragma unroll
  for (int vb = 0; vb < 4; ++vb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[vb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  // With C a multiple of 32 every 32-pair step lies inside one row, so the
  // row bound is the only (wave-uniform) guard.
  constexpr bool kRowSteps = C % 32 == 0;
  for (int k0 = 0; k0 < np; k0 += 32) {
    const int p0 = k0 + 8 * (lane >> 4);
    uint32_t bytes[8];
    if constexpr (kRowSteps) {
      const uint2 b8 = *(const uint2*)&sC[p0];
#pragma unroll
      for (int v = 0; v < 8; ++v) bytes[v] = ((v < 4 ? b8.x : b8.y) >> (8 * (v & 3))) & 0xFFu;
    } else {
#pragma unroll
      for (int v = 0; v < 8; ++v) bytes[v] = (p0 + v < np) ? (uint32_t)sC[p0 + v] : 0xFFFFu;
    }
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      if (nb >= NE) break;
      bf16_t bv[8];
      if constexpr (kRowSteps) {
        const float* xr = &sX[k0 / C][(p0 % C) * E + 16 * nb + (lane & 15)];
#pragma unroll
        for (int v = 0; v < 8; ++v) bv[v] = f2bf(xr[v * E]);
      } else {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int p = p0 + v;
          bv[v] = p < np ? f2bf(sX[p / C][(p % C) * E + 16 * nb + (lane & 15)]) : (bf16_t)0;
        }
      }
      const uint4 b = make_uint4((uint32_t)bv[0] | ((uint32_t)bv[1] << 16),
                                 (uint32_t)bv[2] | ((uint32_t)bv[3] << 16),
                                 (uint32_t)bv[4] | ((uint32_t)bv[5] << 16),
                                 (uint32_t)bv[6] | ((uint32_t)bv[7] << 16));
#pragma unroll
      for (int vb = 0; vb < 4; ++vb) {
        const uint32_t me = (uint32_t)(64 * w + 16 * vb + (lane & 15));
        uint32_t q[4];
#pragma unroll
        for (int h = 0; h < 4; ++h)
          q[h] = (bytes[2 * h] == me ? 0x3F80u : 0u) | ((bytes[2 * h + 1] == me ? 0x3F80u : 0u) << 16);
        acc[vb][nb] = mfma16(make_uint4(q[0], q[1], q[2], q[3]), b, acc[vb][nb]);
      }
    }
  }
  float* out = a.emb_partial + (size_t)blockIdx.x * 256 * E;
#pragma unroll
  for (int vb = 0; vb < 4; ++vb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      if (nb >= NE) break;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int v = 64 * w + 16 * vb + 4 * (lane >> 4) + r;
        out[(size_t)v * E + 16 * nb + (lane & 15)] = acc[vb][nb][r];
      }
    }
}

bool fused_supported(int F, int L, int H, int branches, int blocks) {
  if (branches != 2 || blocks < 1 || blocks > kMaxFusedBlocks) return false;
  return (F == 512 && L == 128 && H == 256) || (F == 256 && L == 64 && H == 128);
}

template <int F, int L, int H>
static hipError_t launch_t(const FusedArgs& a, int grid_rows, hipStream_t s) {
  typedef FusedDims<F, L, H> D;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)fused_kernel<F, L, H>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)D::BYTES);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int blocks = (grid_rows + kFusedRows - 1) / kFusedRows;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((fused_kernel<F, L, H>), dim3(blocks), dim3(kFusedThreads), D::BYTES, s, a);
  return hipGetLastError();
}

// (F, L) of the fused shapes and the byte-embedding width E: C = F / E
// context bytes, known at compile time.
#define EDPC_FUSED_IO_SHAPES(X) \
  X(512, 128, 16) X(512, 128, 32) X(512, 128, 64) X(256, 64, 16) X(256, 64, 32) X(256, 64, 64)

hipError_t launch_fused_in(int F, int L, const FusedInArgs& a, int grid_rows, hipStream_t s) {
  const int blocks = (grid_rows + kFusedRows - 1) / kFusedRows;
  if (blocks == 0) return hipSuccess;
  if (a.C * a.E != F) return hipErrorInvalidValue;
#define X(FF, LL, EE)                                                                         \
  if (F == FF && L == LL && a.E == EE) {                                                      \
    hipLaunchKernelGGL((fused_in_kernel<FF, LL, EE>), dim3(blocks), dim3(256), 0, s, a);      \
    return hipGetLastError();                                                                 \
  }
  EDPC_FUSED_IO_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_fused_out(int F, int L, const FusedOutArgs& a, int grid_rows, hipStream_t s) {
  const int blocks = (grid_rows + kFusedRows - 1) / kFusedRows;
  if (blocks == 0) return hipSuccess;
  if (a.C * a.E != F) return hipErrorInvalidValue;
#define X(FF, LL, EE)                                                                         \
  if (F == FF && L == LL && a.E == EE) {                                                      \
    hipLaunchKernelGGL((fused_out_kernel<FF, LL, EE>), dim3(blocks), dim3(256), 0, s, a);     \
    return hipGetLastError();                                                                 \
  }
  EDPC_FUSED_IO_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_fused(int F, int L, int H, const FusedArgs& a, int grid_rows, hipStream_t s) {
  if (F == 512 && L == 128 && H == 256) return launch_t<512, 128, 256>(a, grid_rows, s);
  if (F == 256 && L == 64 && H == 128) return launch_t<256, 64, 128>(a, grid_rows, s);
  return hipErrorInvalidValue;
}

}  // namespace edpc
