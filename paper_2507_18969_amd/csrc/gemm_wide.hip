// Wide-tile BF16 matrix products for the large models (gfx950 MFMA).
//
// The 4-wave tiles of gemm.hip move 64 KiB of operands per 128 x 128 x 128
// chunk for 4.2 MFLOP: 64 flops per byte, which at one CU's share of the
// BF16 peak (about 4 kflop per clock) asks ~64 bytes per clock from L2, the
// most a CU's vector cache can take.  These kernels use 8 waves on tiles of
// up to 256 x 256 outputs (128 flops per byte), K in chunks of 64 staged
// through a double-buffered LDS tile (one barrier per chunk, the next
// chunk's global loads in flight under the current chunk's MFMAs), and the
// 32 x 32 x 16 BF16 MFMA, whose operands each serve 32 rows or columns.
//
// Contract and epilogues as in gemm.h.  Summation order: K in chunks of 64
// in increasing order, each chunk by the MFMA's fixed order; fixed by the
// tile id, which the container records.
#include "gemm.h"

namespace edpc {

constexpr int kWideThreads = 512;  // 8 waves
constexpr int kWideBK = 64;
constexpr int kWideLds = kWideBK + 8;  // LDS row stride (bf16): 144 bytes

// LDS element offset of the 16-byte chunk `chunk` (8 k values) of tile row
// `row` (rows of 144 bytes).  gfx950's LDS serves a 16-byte access 16 lanes
// at a time over 64 four-byte banks, so a pass is conflict-free when its 16
// lanes hit 16 distinct 16-byte bank groups; the row stride is 9 groups.
// * Tiles staged K-major: no swizzle.  MFMA operand reads (16 consecutive
//   rows at one chunk: 9 r mod 16) and the staging stores (kmajor_row: rows
//   r and r + 8, 8 chunks each, 8 groups apart) are both conflict-free.
// * Tiles staged from the other layout (8 x 8 blocks transposed in
//   registers, SWZ = 4): chunks XOR-swizzled by the row's group of 16.  That
//   is constant over the 16 rows an MFMA read pass takes and spreads the
//   transposed stores (16 lanes: one chunk of 16 row blocks of 8, i.e. 8
//   groups of 16 rows) over all 16 bank groups.
// * The same when both operands come from the other layout (the weight
//   gradients, SWZ = 3): XOR by the row's group of 8, 2-way conflicted on a
//   64-bank LDS, since the 16-row swizzle changes with the fragment index
//   and there the extra address registers spill.
template <int SWZ>
__device__ __forceinline__ int wide_lds_off(int row, int chunk) {
  if constexpr (SWZ == 0) return row * kWideLds + 8 * chunk;
  return row * kWideLds + 8 * (chunk ^ ((row >> SWZ) & 7));
}

// Tile row of 16-byte vector v in the K-major staging (chunk v & 7): lanes
// 8q .. 8q + 7 take one row's 8 chunks, and the two rows of a 16-lane pass
// are 8 apart.
__device__ __forceinline__ int kmajor_row(int v) {
  return 16 * (v >> 7) + ((v >> 4) & 7) + 8 * ((v >> 3) & 1);
}

// Global -> registers -> LDS staging of one [ROWS x 64] operand tile, stored
// in LDS as [ROWS][kWideLds] (k contiguous).
//   KMAJOR: src[row * ld + k], moved as 16-byte vectors of 8 k;
//   else:   src[k * ld + row], moved as 8 x 8 blocks transposed in registers.
// Tile row i maps to global row base0 + i (i < half) or base1 + i - half
// (K-major only: the two branch matrices of the gated product), valid below
// lim0 / lim1.
template <int ROWS, bool KMAJOR, int SWZ = 0>
struct WideStage {
  static_assert(kWideBK == 64 && ROWS % 16 == 0, "8 chunks a row, rows in groups of 16");
  static constexpr int NV = ROWS * kWideBK / 8;                     // 16-byte vectors
  static constexpr int NBLK = (ROWS / 8) * (kWideBK / 8);           // 8 x 8 blocks
  static constexpr int VPT = (NV + kWideThreads - 1) / kWideThreads;
  static constexpr int BPT = (NBLK + kWideThreads - 1) / kWideThreads;
  static constexpr int NREG = KMAJOR ? VPT : 8 * BPT;
  uint4 r[NREG];

  __device__ __forceinline__ void load(const bf16_t* __restrict__ src, int ld, int base0, int lim0,
                                       int half, int base1, int lim1, int k0, int K) {
    if constexpr (KMAJOR) {
#pragma unroll
      for (int p = 0; p < VPT; ++p) {
        const int v = threadIdx.x + p * kWideThreads;
        const int i = kmajor_row(v), kq = v & 7;
        const int gk = k0 + kq * 8;
        const bool second = i >= half;
        const int grow = second ? base1 + (i - half) : base0 + i;
        const int lim = second ? lim1 : lim0;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (v < NV && grow < lim && gk < K) val = ld_global16(src + (size_t)grow * ld + gk);
        r[p] = val;
      }
    } else {
#pragma unroll
      for (int p = 0; p < BPT; ++p) {
        const int b = threadIdx.x + p * kWideThreads;
        const int kb = b / (ROWS / 8), rb = b % (ROWS / 8);
        const int grow = base0 + rb * 8;  // 8 contiguous rows (lim0 is a multiple of 8)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int gk = k0 + kb * 8 + q;
          uint4 val = make_uint4(0, 0, 0, 0);
          if (b < NBLK && grow < lim0 && gk < K) val = ld_global16(src + (size_t)gk * ld + grow);
          r[8 * p + q] = val;
        }
      }
    }
  }

  __device__ __forceinline__ void store(bf16_t* lds) const {
    if constexpr (KMAJOR) {
#pragma unroll
      for (int p = 0; p < VPT; ++p) {
        const int v = threadIdx.x + p * kWideThreads;
        if (v >= NV) continue;
        *(uint4*)(lds + wide_lds_off<0>(kmajor_row(v), v & 7)) = r[p];
      }
    } else {
#pragma unroll
      for (int p = 0; p < BPT; ++p) {
        const int b = threadIdx.x + p * kWideThreads;
        if (b >= NBLK) continue;
        const int kb = b / (ROWS / 8), rb = b % (ROWS / 8);
        // r[8p + q] holds k = kb*8 + q for rows rb*8 .. rb*8 + 7
        const uint32_t* w = (const uint32_t*)&r[8 * p];
#pragma unroll
        for (int j = 0; j < 8; ++j) {  // row rb*8 + j gets its 8 k values
          const int q2 = j >> 1;
          const uint32_t sel = (j & 1) ? 0x07060302u : 0x05040100u;
          uint32_t o[4];
#pragma unroll
          for (int t = 0; t < 4; ++t)
            o[t] = __builtin_amdgcn_perm(w[4 * (2 * t + 1) + q2], w[4 * (2 * t) + q2], sel);
          *(uint4*)(lds + wide_lds_off<SWZ>(rb * 8 + j, kb)) = make_uint4(o[0], o[1], o[2], o[3]);
        }
      }
    }
  }
};

// Tile of BM x BN outputs over 8 waves arranged WM x WN; each wave owns
// (BM / WM) x (BN / WN) outputs as TM x TN blocks of 32 x 32.  GATE: the
// tile's columns are BN / 2 outputs of each of two branch products, and a
// wave's two column blocks are the same outputs of the two branches.
template <int BM_, int BN_, int WM_, bool GATE_>
struct WideTile {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = 8 / WM_;
  static constexpr int TM = BM / WM / 32, TN = BN / WN / 32;
  static constexpr bool GATE = GATE_;
  static_assert(!GATE || TN == 2, "gated tiles give each wave one block per branch");
  static constexpr int LDS_A = BM * kWideLds, LDS_B = BN * kWideLds;  // bf16 elements
  static constexpr int SMEM = 2 * (LDS_A + LDS_B) * 2;                  // bytes, two stages
  // tile-local column (B row) of block tn of wave wn
  __device__ static int col_block(int wn, int tn) {
    return GATE ? tn * (BN / 2) + wn * 32 : wn * (BN / WN) + tn * 32;
  }
};

template <class T, bool AK, bool BKM>
struct WideCompute {
  typedef f32x16 Acc;
  // LDS placement of each operand (see wide_lds_off)
  static constexpr int SWA = AK ? 0 : (BKM ? 4 : 3);
  static constexpr int SWB = BKM ? 0 : (AK ? 4 : 3);
  Acc acc[T::TM][T::TN];

  // A rows [m0, m0 + BM) valid below M; B rows as WideStage; k in [kb, K)
  // in chunks of 64 from kb.
  __device__ __forceinline__ void run(const bf16_t* A, int lda, int m0, int M, const bf16_t* B,
                                      int ldb, int b0, int blim0, int bhalf, int b1, int blim1,
                                      int kb, int K, char* smem) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave / T::WN, wn = wave % T::WN;
#pragma unroll
    for (int i = 0; i < T::TM; ++i)
#pragma unroll
      for (int j = 0; j < T::TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    bf16_t* lds = (bf16_t*)smem;
    auto lds_a = [&](int s) { return lds + s * (T::LDS_A + T::LDS_B); };
    auto lds_b = [&](int s) { return lds + s * (T::LDS_A + T::LDS_B) + T::LDS_A; };
    WideStage<T::BM, AK, SWA> sa;
    WideStage<T::BN, BKM, SWB> sb;
    const int nchunks = (K - kb + kWideBK - 1) / kWideBK;
    sa.load(A, lda, m0, M, T::BM, 0, 0, kb, K);
    sb.load(B, ldb, b0, blim0, bhalf, b1, blim1, kb, K);
    sa.store(lds_a(0));
    sb.store(lds_b(0));
    __syncthreads();
    // operand rows of this lane: 32 rows per block, chunk half by lane / 32
    const int lrow = lane & 31, lhalf = lane >> 5;
    for (int c = 0; c < nchunks; ++c) {
      const bool more = c + 1 < nchunks;
      if (more) {
        sa.load(A, lda, m0, M, T::BM, 0, 0, kb + (c + 1) * kWideBK, K);
        sb.load(B, ldb, b0, blim0, bhalf, b1, blim1, kb + (c + 1) * kWideBK, K);
      }
      const bf16_t* la = lds_a(c & 1);
      const bf16_t* lb = lds_b(c & 1);
#pragma unroll
      for (int kk = 0; kk < kWideBK; kk += 16) {
        bf16x8 fa[T::TM], fb[T::TN];
        const int ch = kk / 8 + lhalf;
#pragma unroll
        for (int i = 0; i < T::TM; ++i)
          fa[i] = __builtin_bit_cast(
              bf16x8, *(const uint4*)(la + wide_lds_off<SWA>(wm * (T::BM / T::WM) + i * 32 + lrow, ch)));
#pragma unroll
        for (int j = 0; j < T::TN; ++j)
          fb[j] = __builtin_bit_cast(
              bf16x8, *(const uint4*)(lb + wide_lds_off<SWB>(T::col_block(wn, j) + lrow, ch)));
#pragma unroll
        for (int i = 0; i < T::TM; ++i)
#pragma unroll
          for (int j = 0; j < T::TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
      }
      if (more) {
        sa.store(lds_a((c + 1) & 1));
        sb.store(lds_b((c + 1) & 1));
      }
      __syncthreads();
    }
  }
};

__device__ __forceinline__ int wacc_row(int r, int lane) {
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

__device__ __forceinline__ float4 ld4(const float* p) {
  return __builtin_bit_cast(float4, ld_global16(p));
}
__device__ __forceinline__ void st4(float* p, float4 v) {
  st_global16(p, __builtin_bit_cast(uint4, v));
}
__device__ __forceinline__ void st4bf(bf16_t* p, float4 v) {
  typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
  const u32x2 u = {(uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16),
                   (uint32_t)f2bf(v.z) | ((uint32_t)f2bf(v.w) << 16)};
  *(__attribute__((address_space(1))) u32x2*)p = u;
}

// Epilogue through LDS.  The accumulators of half the tile's rows go to LDS
// as FP32 [BM / 2][BN + 4] (the MFMA layout gives each lane single values
// scattered over rows), then every thread walks that half tile four columns
// at a time, so that the bias / residual / branch-value reads and the
// output writes are 16-byte accesses that fill whole cache lines.  With one
// work-group per CU nothing else hides the latency of those reads, so each
// thread issues the reads of EB items before it uses any of them, the first
// batch before the accumulators go through LDS.
// EPI_WGRAD_OUT: dw = acc (ld = N), used by the weight-gradient kernel.
constexpr int EPI_WGRAD_OUT = 16;
// EPI_GATE_BWD with the branch count nb (1..3) fixed at compile time, so that
// the branch values of an item stay in registers (indexed by a runtime count
// they would live in scratch memory).
constexpr int epi_gate_bwd(int nb) { return 32 + nb; }
constexpr int gate_bwd_branches(int epi) { return epi > 32 && epi <= 35 ? epi - 32 : 0; }

template <int EPI>
struct EpiPre {  // global operands of one item (four columns of one row)
  static constexpr int NB = gate_bwd_branches(EPI);
  static constexpr int N = NB > 0 ? NB : (EPI == EPI_STORE ? 1 : 0);
  static constexpr int EB = NB > 0 ? 4 : 8;  // items per batch
  float4 v[N > 0 ? N : 1];
};

template <class T, int EPI>
__device__ __forceinline__ void wide_epilogue(const typename WideCompute<T, true, true>::Acc (&acc)[T::TM][T::TN],
                                              const GemmArgs& g, float* dw, int m0, int n0, int M,
                                              int N, char* smem, int tid) {
  constexpr int HR = T::BM / 2, LDE = T::BN + 4;
  float* lds = (float*)smem;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / T::WN, wn = wave % T::WN;
  constexpr int WROWS = T::BM / T::WM;  // rows per wave
  // output columns of the tile handled per half-tile row (gated: per branch)
  constexpr int COLS = T::GATE ? T::BN / 2 : T::BN;
  constexpr int ITEMS = HR * COLS / 4;
  static_assert(kWideThreads % (COLS / 4) == 0, "a thread keeps its columns");
  constexpr int EB = EpiPre<EPI>::EB;
  constexpr int NB = EpiPre<EPI>::NB;  // gated backward: branch count
  // a thread's items all lie in the same four columns
  const int c = 4 * (tid % (COLS / 4));
  const int n = n0 + c;
  const bool col_ok = n < N;
  float4 bias0 = make_float4(0.f, 0.f, 0.f, 0.f), bias1 = bias0;
  if constexpr (EPI == EPI_STORE) {
    if (g.bias && col_ok) bias0 = ld4(g.bias + n);
  } else if constexpr (EPI == EPI_GATE_FWD) {
    if (col_ok) {
      bias0 = ld4(g.bias + n);
      bias1 = ld4(g.bias + g.bias_branch_stride + n);
    }
  }
  auto row_of = [&](int it) { return it / (COLS / 4); };
  // global operands of item `it` of half h
  auto fetch = [&](int h, int it, EpiPre<EPI>& p) {
    const int m = m0 + h * HR + row_of(it);
    if (it >= ITEMS || m >= M || !col_ok) return;
    if constexpr (EPI == EPI_STORE) {
      if (g.resid) p.v[0] = ld4(g.resid + (size_t)m * g.ld_resid + n);
    } else if constexpr (NB > 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
        p.v[b] = ld4(g.aux + (size_t)m * g.ld_aux + b * g.aux_branch + n);
    }
  };
  // result of item `it` of half h from the LDS half tile and its operands
  auto finish = [&](int h, int it, const EpiPre<EPI>& p) {
    const int row = row_of(it);
    const int m = m0 + h * HR + row;
    if (it >= ITEMS || m >= M || !col_ok) return;
    const float4 v = *(const float4*)&lds[row * LDE + c];
    if constexpr (EPI == EPI_WGRAD_OUT) {
      st4(dw + (size_t)m * N + n, v);
    } else if constexpr (EPI == EPI_STORE) {
      float4 o = make_float4(v.x + bias0.x, v.y + bias0.y, v.z + bias0.z, v.w + bias0.w);
      if (g.resid) {
        const float4 q = p.v[0];
        o.x += q.x; o.y += q.y; o.z += q.z; o.w += q.w;
      }
      if (g.out32) st4(g.out32 + (size_t)m * g.ld_out32 + n, o);
      if (g.out16) st4bf(g.out16 + (size_t)m * g.ld_out16 + n, o);
    } else if constexpr (EPI == EPI_GATE_FWD) {
      // a_b = acc_b + bias_b (Eq. 10); aux keeps both; out = GeLU(a_0 a_1) (Eqs. 11-12)
      const float4 w1 = *(const float4*)&lds[row * LDE + T::BN / 2 + c];
      const float4 a0 = make_float4(v.x + bias0.x, v.y + bias0.y, v.z + bias0.z, v.w + bias0.w);
      const float4 a1 = make_float4(w1.x + bias1.x, w1.y + bias1.y, w1.z + bias1.z, w1.w + bias1.w);
      st4(g.aux + (size_t)m * g.ld_aux + n, a0);
      st4(g.aux + (size_t)m * g.ld_aux + g.aux_branch + n, a1);
      const float4 o = make_float4(gelu_f(a0.x * a1.x), gelu_f(a0.y * a1.y),
                                   gelu_f(a0.z * a1.z), gelu_f(a0.w * a1.w));
      if (g.out32) st4(g.out32 + (size_t)m * g.ld_out32 + n, o);
      if (g.out16) st4bf(g.out16 + (size_t)m * g.ld_out16 + n, o);
    } else {  // gated backward: dP = acc * GeLU'(prod a); dX_b = dP * prod_{c != b} a_c
      static_assert(NB > 0, "unknown epilogue");
      const float* av = (const float*)p.v;
      const float* vv = (const float*)&v;
      float o[NB][4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float prod = av[e];
#pragma unroll
        for (int b = 1; b < NB; ++b) prod *= av[4 * b + e];
        const float dp = vv[e] * gelu_grad_f(prod);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          float x = dp;
#pragma unroll
          for (int cc = 0; cc < NB; ++cc)
            if (cc != b) x *= av[4 * cc + e];
          o[b][e] = x;
        }
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float4 ob = make_float4(o[b][0], o[b][1], o[b][2], o[b][3]);
        if (g.out32) st4(g.out32 + (size_t)m * g.ld_out32 + b * g.aux_branch + n, ob);
        if (g.out16) st4bf(g.out16 + (size_t)m * g.ld_out16 + b * g.aux_branch + n, ob);
      }
    }
  };
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    EpiPre<EPI> pre[EB];
    // first batch of operand reads in flight before the half goes through LDS
#pragma unroll
    for (int e = 0; e < EB; ++e) fetch(h, tid + e * kWideThreads, pre[e]);
    __syncthreads();  // the K loop (or the previous half) is done with LDS
    if (wm * WROWS >= h * HR && wm * WROWS < (h + 1) * HR) {
#pragma unroll
      for (int i = 0; i < T::TM; ++i)
#pragma unroll
        for (int j = 0; j < T::TN; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = wm * WROWS - h * HR + i * 32 + wacc_row(r, lane);
            lds[row * LDE + T::col_block(wn, j) + (lane & 31)] = acc[i][j][r];
          }
    }
    __syncthreads();
    for (int b0 = 0; b0 < ITEMS; b0 += EB * kWideThreads) {
      if (b0 > 0) {
#pragma unroll
        for (int e = 0; e < EB; ++e) fetch(h, b0 + tid + e * kWideThreads, pre[e]);
      }
#pragma unroll
      for (int e = 0; e < EB; ++e) finish(h, b0 + tid + e * kWideThreads, pre[e]);
    }
  }
}

template <class T, bool AK, bool BKM, int EPI>
__global__ void __launch_bounds__(kWideThreads) gemm_wide_kernel(GemmArgs g) {
  extern __shared__ __align__(16) char smem[];
  const int M = g.m_rows ? g.st->rows : g.M;
  const int K = g.k_rows ? g.st->rows : g.K;
  const int N = g.N;
  const int tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int tx = tile % gridDim.x, ty = tile / gridDim.x;
  const int m0 = ty * T::BM;
  if (m0 >= M) return;
  WideCompute<T, AK, BKM> wc;
  int n0;  // first output column of the tile (per branch for gated tiles)
  if constexpr (T::GATE) {
    n0 = tx * (T::BN / 2);
    const int bro = (int)(g.b_branch_stride / g.ldb);  // rows between the branch matrices
    wc.run((const bf16_t*)g.A, g.lda, m0, M, (const bf16_t*)g.B, g.ldb, n0, N, T::BN / 2,
           bro + n0, bro + N, 0, K, smem);
  } else {
    n0 = tx * T::BN;
    wc.run((const bf16_t*)g.A, g.lda, m0, M, (const bf16_t*)g.B, g.ldb, n0, N, T::BN, 0, 0, 0, K,
           smem);
  }
  wide_epilogue<T, EPI>(wc.acc, g, nullptr, m0, n0, M, N, smem, threadIdx.x);
}

// Problem and output origin of tile `tile` of a grouped weight-gradient table.
template <class T>
__device__ __forceinline__ WgradProblem wgrad_tile(const WgradProblem* __restrict__ probs,
                                                   int n_probs, int tile, int* m0, int* n0) {
  int p = 0;
  while (p + 1 < n_probs && tile >= probs[p + 1].tile_begin) ++p;
  const WgradProblem pr = probs[p];
  const int t = tile - pr.tile_begin;
  *m0 = (t / pr.tiles_n) * T::BM;
  *n0 = (t % pr.tiles_n) * T::BN;
  return pr;
}

// Weight gradients dW = dOut^T In over grouped problems (K = active rows).
template <class T>
__global__ void __launch_bounds__(kWideThreads) wgrad_wide_kernel(const WgradProblem* __restrict__ probs,
                                                                  int n_probs, const StepState* st) {
  extern __shared__ __align__(16) char smem[];
  int m0, n0;
  const WgradProblem pr = wgrad_tile<T>(probs, n_probs, xcd_tile(blockIdx.x, gridDim.x), &m0, &n0);
  const int K = st->rows;
  WideCompute<T, false, false> wc;
  wc.run((const bf16_t*)pr.dout, pr.M, m0, pr.M, (const bf16_t*)pr.in, pr.N, n0, pr.N, T::BN, 0,
         0, 0, K, smem);
  GemmArgs unused;
  wide_epilogue<T, EPI_WGRAD_OUT>(wc.acc, unused, pr.dw, m0, n0, pr.M, pr.N, smem, threadIdx.x);
}

// The thread index behind an empty asm statement.  Values the epilogue
// derives from it are then computed where they are used: taken from
// threadIdx.x directly, the compiler hoists them out of the split kernel's
// loop over tiles, keeps them live across the K loop, and spills them.
__device__ __forceinline__ int opaque_thread_index() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// The same products balanced over the CUs, for tables with at least as many
// tiles as CUs, where one work-group per tile leaves most CUs idle in the
// last, short round of tiles (measured slower than one work-group per tile
// for smaller tables, where the parts cost more than the shorter K loops
// save).  The K chunks of all tiles, in tile order, form kWgradRanges equal
// ranges, one per work-group (XCD x takes a contiguous band of ranges, so
// neighbouring tiles share its L2).  A tile summed whole by one range is
// written directly, with wgrad_wide_kernel's summation order.  A tile cut
// by range boundaries is summed in parts: range w writes the part it starts
// inside a tile (or that lies inside one) to scratch slot 2w + 1, and the
// part it ends inside a tile to slot 2w; wgrad_fixup_kernel adds a cut
// tile's parts in K order.
template <class T>
__global__ void __launch_bounds__(kWideThreads) wgrad_wide_split_kernel(
    const WgradProblem* __restrict__ probs, int n_probs, const StepState* st, int total_tiles,
    float* __restrict__ part) {
  extern __shared__ __align__(16) char smem[];
  const int K = st->rows;
  const long long nck = (K + kWideBK - 1) / kWideBK;
  if (nck == 0) return;  // no rows: nothing to sum (the fixup returns too)
  const long long U = (long long)total_tiles * nck;
  const int w = xcd_tile(blockIdx.x, kWgradRanges);  // this work-group's range
  const long long u0 = (long long)w * U / kWgradRanges;
  const long long u1 = (long long)(w + 1) * U / kWgradRanges;
  // The range's segments (one per tile it touches) run with the first one
  // last: every later segment starts at K chunk 0, and with equal range
  // lengths the work-groups then stay within a few K chunks of each other,
  // so tiles that share an operand panel read it from L2 together (in range
  // order, the work-groups of an XCD sit at scattered K offsets and each
  // streams its panels from HBM).  Each segment is summed as before.
  const long long first_end = min(u1, (u0 / nck + 1) * nck);
  long long v = first_end;
  bool first_done = u0 >= first_end;
  GemmArgs unused;
  for (;;) {
    long long a, b;
    if (v < u1) {
      a = v;
      b = min(u1, (v / nck + 1) * nck);
      v = b;
    } else if (!first_done) {
      a = u0;
      b = first_end;
      first_done = true;
    } else {
      break;
    }
    const int tile = (int)(a / nck);
    const long long c0 = a % nck, c1 = c0 + (b - a);
    int m0, n0;
    const WgradProblem pr = wgrad_tile<T>(probs, n_probs, tile, &m0, &n0);
    WideCompute<T, false, false> wc;
    wc.run((const bf16_t*)pr.dout, pr.M, m0, pr.M, (const bf16_t*)pr.in, pr.N, n0, pr.N, T::BN,
           0, 0, (int)(c0 * kWideBK), (int)min((long long)K, c1 * kWideBK), smem);
    // a whole tile goes to dW, a part to its slot ([BM][BN], origin 0)
    const bool whole = c0 == 0 && c1 == nck;
    const long long slot = c0 != 0 ? 2LL * w + 1 : 2LL * w;
    float* dst = whole ? pr.dw : part + slot * (T::BM * T::BN);
    wide_epilogue<T, EPI_WGRAD_OUT>(wc.acc, unused, dst, whole ? m0 : 0, whole ? n0 : 0,
                                    whole ? pr.M : T::BM, whole ? pr.N : T::BN, smem,
                                    opaque_thread_index());
    __syncthreads();  // the epilogue's LDS before the next tile's staging
  }
}

// dW of every cut tile: its parts added in K order (ranges wa .. wb, empty
// ranges skipped).  One work-group per tile; uncut tiles return at once.
template <class T>
__global__ void __launch_bounds__(256) wgrad_fixup_kernel(const WgradProblem* __restrict__ probs,
                                                          int n_probs, const StepState* st,
                                                          int total_tiles,
                                                          const float* __restrict__ part) {
  const int t = blockIdx.x;
  const long long nck = (st->rows + kWideBK - 1) / kWideBK;
  if (nck == 0) return;  // no rows: the split kernel wrote nothing
  const long long U = (long long)total_tiles * nck;
  // the range holding chunk u: the last w with floor(w U / R) <= u
  auto range_of = [&](long long u) { return (int)(((u + 1) * kWgradRanges + U - 1) / U - 1); };
  const int wa = range_of((long long)t * nck), wb = range_of((long long)t * nck + nck - 1);
  if (wa == wb) return;  // summed whole by range wa
  int m0, n0;
  const WgradProblem pr = wgrad_tile<T>(probs, n_probs, t, &m0, &n0);
  constexpr int TE = T::BM * T::BN;
  for (int e = threadIdx.x; e < TE / 4; e += 256) {
    const int i = (4 * e) / T::BN, j = (4 * e) % T::BN;
    const int m = m0 + i, n = n0 + j;
    if (m >= pr.M || n >= pr.N) continue;  // N is a multiple of 4
    float4 a = ld4(part + (size_t)(2 * wa) * TE + 4 * e);
    for (int r = wa + 1; r <= wb; ++r) {
      if ((long long)r * U / kWgradRanges == (long long)(r + 1) * U / kWgradRanges) continue;
      const float4 b = ld4(part + (size_t)(2 * r + 1) * TE + 4 * e);
      a = make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
    }
    st4(pr.dw + (size_t)m * pr.N + n, a);
  }
}

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------
template <class T, bool AK, bool BKM, int EPI>
static hipError_t launch_wide_one(const GemmArgs& g, int grid_m_max, hipStream_t s) {
  const int cols = T::GATE ? T::BN / 2 : T::BN;
  dim3 grid((g.N + cols - 1) / cols, (grid_m_max + T::BM - 1) / T::BM);
  if (grid.x == 0 || grid.y == 0) return hipSuccess;
  static_assert(T::SMEM <= 160 * 1024, "tile does not fit in LDS");
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)gemm_wide_kernel<T, AK, BKM, EPI>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, T::SMEM);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((gemm_wide_kernel<T, AK, BKM, EPI>), grid, dim3(kWideThreads), T::SMEM, s, g);
  return hipGetLastError();
}

template <int BM, int BN, int WM>
static hipError_t launch_wide_t(bool ak, bool bk, EpiKind epi, int nb, const GemmArgs& g, int gm,
                                hipStream_t s) {
  typedef WideTile<BM, BN, WM, false> P;
  typedef WideTile<BM, BN, WM, true> G;
  if (ak && bk) {
    if (epi == EPI_STORE) return launch_wide_one<P, true, true, EPI_STORE>(g, gm, s);
    if (epi == EPI_GATE_FWD && nb == 2) return launch_wide_one<G, true, true, EPI_GATE_FWD>(g, gm, s);
  } else if (ak && !bk) {
    if (epi == EPI_STORE) return launch_wide_one<P, true, false, EPI_STORE>(g, gm, s);
    if (epi == EPI_GATE_BWD) {
      // one B matrix (W_o); the branch count k travels in bias_branch_stride
      switch (g.bias_branch_stride) {
        case 1: return launch_wide_one<P, true, false, epi_gate_bwd(1)>(g, gm, s);
        case 2: return launch_wide_one<P, true, false, epi_gate_bwd(2)>(g, gm, s);
        case 3: return launch_wide_one<P, true, false, epi_gate_bwd(3)>(g, gm, s);
        default: return hipErrorInvalidValue;
      }
    }
  }
  return hipErrorInvalidValue;
}

bool wide_tile_supported(int tile, bool bf16, EpiKind epi, int nb) {
  if (tile < TILE_W128x128) return true;
  if (!bf16) return false;
  return !(epi == EPI_GATE_FWD && nb != 2);
}

hipError_t launch_gemm_wide(int tile, bool a_kmajor, bool b_kmajor, EpiKind epi, int nb,
                            const GemmArgs& g, int grid_m_max, hipStream_t s) {
  switch (tile) {
    case TILE_W128x128: return launch_wide_t<128, 128, 4>(a_kmajor, b_kmajor, epi, nb, g, grid_m_max, s);
    case TILE_W256x128: return launch_wide_t<256, 128, 4>(a_kmajor, b_kmajor, epi, nb, g, grid_m_max, s);
    case TILE_W128x256: return launch_wide_t<128, 256, 2>(a_kmajor, b_kmajor, epi, nb, g, grid_m_max, s);
    case TILE_W256x256: return launch_wide_t<256, 256, 2>(a_kmajor, b_kmajor, epi, nb, g, grid_m_max, s);
  }
  return hipErrorInvalidValue;
}

template <class T>
static hipError_t launch_wgrad_wide_t(const WgradProblem* d_probs, int n_probs, int total_tiles,
                                      const StepState* st, float* part, hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)wgrad_wide_kernel<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, T::SMEM);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)wgrad_wide_split_kernel<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, T::SMEM);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (part && total_tiles >= kWgradRanges) {
    hipLaunchKernelGGL((wgrad_wide_split_kernel<T>), dim3(kWgradRanges), dim3(kWideThreads), T::SMEM,
                       s, d_probs, n_probs, st, total_tiles, part);
    hipLaunchKernelGGL((wgrad_fixup_kernel<T>), dim3(total_tiles), dim3(256), 0, s, d_probs,
                       n_probs, st, total_tiles, (const float*)part);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((wgrad_wide_kernel<T>), dim3(total_tiles), dim3(kWideThreads), T::SMEM, s,
                     d_probs, n_probs, st);
  return hipGetLastError();
}

hipError_t launch_wgrad_wide(int tile, const WgradProblem* d_probs, int n_probs, int total_tiles,
                             const StepState* st, float* part, hipStream_t s) {
  switch (tile) {
    case TILE_W128x128: return launch_wgrad_wide_t<WideTile<128, 128, 4, false>>(d_probs, n_probs, total_tiles, st, part, s);
    case TILE_W256x128: return launch_wgrad_wide_t<WideTile<256, 128, 4, false>>(d_probs, n_probs, total_tiles, st, part, s);
    case TILE_W128x256: return launch_wgrad_wide_t<WideTile<128, 256, 2, false>>(d_probs, n_probs, total_tiles, st, part, s);
    case TILE_W256x256: return launch_wgrad_wide_t<WideTile<256, 256, 2, false>>(d_probs, n_probs, total_tiles, st, part, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace edpc
