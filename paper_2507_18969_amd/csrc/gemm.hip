// MFMA matrix products for gfx950; see gemm.h for the contract.
#include "gemm.h"

namespace edpc {

// 4 waves of 64, arranged 2 x 2 over the tile; also the element count of an
// element-range Adam item (kAdamVecItem), which takes one thread an element
constexpr int kThreads = 256;

template <bool BF, int MB>
struct Mfma;

template <>
struct Mfma<false, 32> {  // v_mfma_f32_32x32x2_f32
  static constexpr int KSTEP = 2;
  static constexpr int NACC = 16;
  typedef f32x16 Acc;
  typedef float Frag;
  __device__ static Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<false, 16> {  // v_mfma_f32_16x16x4_f32
  static constexpr int KSTEP = 4;
  static constexpr int NACC = 4;
  typedef f32x4 Acc;
  typedef float Frag;
  __device__ static Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<true, 32> {  // v_mfma_f32_32x32x16_bf16
  static constexpr int KSTEP = 16;
  static constexpr int NACC = 16;
  typedef f32x16 Acc;
  typedef bf16x8 Frag;
  __device__ static Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<true, 16> {  // v_mfma_f32_16x16x32_bf16
  static constexpr int KSTEP = 32;
  static constexpr int NACC = 4;
  typedef f32x4 Acc;
  typedef bf16x8 Frag;
  __device__ static Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// Row / column of accumulator register r of this lane inside an MB x MB block.
template <int MB>
__device__ __forceinline__ int acc_row(int r, int lane) {
  if constexpr (MB == 32) return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
  else return 4 * (lane >> 4) + r;
}
template <int MB>
__device__ __forceinline__ int acc_col(int lane) {
  return lane & (MB - 1);
}

// ---------------------------------------------------------------------------
// Operand tile staging.  LDS layout: FP32 tiles are stored k-major
// [BK][ROWS + 4]; BF16 tiles row-major [ROWS][BK + 8] so that one lane reads
// its 8 consecutive k values with a single 16-byte access.  A BF16 operand
// stored row-contiguous in memory (k slowest) is moved in 8 x 8 blocks that
// each thread transposes in registers, so LDS still gets 16-byte stores.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void transpose8x8_bf16(const uint4* in, uint4* out) {
  // in[i] holds 8 bf16 of row i (columns 0..7); out[j] gets column j (rows 0..7)
  const uint32_t* w = (const uint32_t*)in;  // w[4 * i + q] = (col 2q, col 2q+1) of row i
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

// 8 x 8 block b of a row-contiguous BF16 operand tile with 16 chunks of 8 k
// (BK = 128): row block rb, chunk kb.  The 16 lanes of an LDS store pass take
// 2 adjacent row blocks x 8 chunks: a 272-byte row is 17 16-byte bank groups,
// so the two row blocks start 8 groups apart and the 16 stores fill all 16
// groups of gfx950's 64-bank LDS (one row block x 16 chunks would fill 2).  A
// wave covers 8 row blocks x 8 chunks (ROWS >= 64; 4 x 16 at ROWS = 32), so
// each global load reads whole 128-byte lines (half lines at ROWS = 32, as
// before).
template <int ROWS>
__device__ __forceinline__ void blk_of(int b, int& rb, int& kb) {
  constexpr int U4 = ROWS / 16 < 4 ? ROWS / 16 : 4;  // row-block pairs a wave covers
  const int g = b >> 4, u = (g % U4) + U4 * (g / (2 * U4)), v = (g / U4) & 1;
  rb = 2 * u + ((b >> 3) & 1);
  kb = 8 * v + (b & 7);
}

// FP32 tiles hold an operand k-major in LDS, [BK][ROWS + PAD].  An MFMA
// operand read takes MB consecutive rows at each of 64 / MB k values, and
// gfx950's LDS has 64 four-byte banks, so the read is conflict-free when the
// row stride is MB (mod 64): the k groups land on disjoint banks.  Operands
// staged from the row-contiguous layout are stored as 16-byte row chunks,
// conflict-free at any stride, and take that stride.  K-major operands are
// transposed into LDS by 4-byte stores, for which a stride of 4 (mod 64)
// spreads a wave's stores best; they keep PAD = 4.
constexpr int fp32_lds_pad(bool kmajor, int rows, int mb) {
  return kmajor ? 4 : ((mb - rows % 64) % 64 + 64) % 64;
}

template <bool BF, int ROWS, int BK, int PAD = 4>
struct Stage {
  static constexpr int VEC = BF ? 8 : 4;                 // elements per 16-byte vector
  static constexpr int NVEC = ROWS * BK / VEC;           // vectors per tile
  static constexpr int PER_THREAD = (NVEC + kThreads - 1) / kThreads;
  static constexpr int NBLK = (ROWS / 8) * (BK / 8);     // 8 x 8 blocks (BF16, row-contiguous)
  static_assert(!BF || (BK == 128 && ROWS % 16 == 0), "blk_of: 16 chunks, row blocks in pairs");
  static constexpr int BLK_PER_THREAD = (NBLK + kThreads - 1) / kThreads;
  static constexpr int NREG = PER_THREAD > 8 * BLK_PER_THREAD ? PER_THREAD : 8 * BLK_PER_THREAD;
  static constexpr int STRIDE = BF ? (BK + 8) : (ROWS + PAD);  // LDS row stride (elements)
  static constexpr int LDS_ELEMS = BF ? ROWS * (BK + 8) : BK * (ROWS + PAD);
  static_assert(BF || (ROWS + PAD) % 4 == 0, "16-byte aligned FP32 rows");
  uint4 reg[NREG];

  // Global -> registers.  kmajor: src[row * ld + k]; else src[k * ld + row].
  template <bool KMAJOR>
  __device__ __forceinline__ void load(const void* srcv, int ld, int row0, int rows_valid,
                                       int k0, int K) {
    const char* src = (const char*)srcv;
    const int esz = BF ? 2 : 4;
    if constexpr (BF && !KMAJOR) {
#pragma unroll
      for (int p = 0; p < BLK_PER_THREAD; ++p) {
        const int b = threadIdx.x + p * kThreads;
        int rb, kb;
        blk_of<ROWS>(b, rb, kb);
        const int gr = row0 + rb * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int gk = k0 + kb * 8 + i;
          reg[8 * p + i] = ld_global16_or_zero(src + ((long long)gk * ld + gr) * esz,
                                               b < NBLK && gr < rows_valid && gk < K);
        }
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < PER_THREAD; ++p) {
      const int v = threadIdx.x + p * kThreads;
      if constexpr (KMAJOR) {
        const int row = v / (BK / VEC), kq = v % (BK / VEC);
        const int gr = row0 + row, gk = k0 + kq * VEC;
        reg[p] = ld_global16_or_zero(src + ((long long)gr * ld + gk) * esz,
                                     v < NVEC && gr < rows_valid && gk < K);
      } else {
        const int k = v / (ROWS / VEC), rq = v % (ROWS / VEC);
        const int gr = row0 + rq * VEC, gk = k0 + k;
        reg[p] = ld_global16_or_zero(src + ((long long)gk * ld + gr) * esz,
                                     v < NVEC && gr < rows_valid && gk < K);
      }
    }
  }

  template <bool KMAJOR>
  __device__ __forceinline__ void store(void* ldsv) {
    if constexpr (BF && !KMAJOR) {
      bf16_t* lds = (bf16_t*)ldsv;
#pragma unroll
      for (int p = 0; p < BLK_PER_THREAD; ++p) {
        const int b = threadIdx.x + p * kThreads;
        if (b >= NBLK) continue;
        int rb, kb;
        blk_of<ROWS>(b, rb, kb);
        uint4 t[8];
        transpose8x8_bf16(&reg[8 * p], t);
#pragma unroll
        for (int j = 0; j < 8; ++j) *(uint4*)(lds + (rb * 8 + j) * STRIDE + kb * 8) = t[j];
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < PER_THREAD; ++p) {
      const int v = threadIdx.x + p * kThreads;
      if (v >= NVEC) continue;
      if constexpr (!BF) {
        float* lds = (float*)ldsv;
        const float* f = (const float*)&reg[p];
        if constexpr (KMAJOR) {
          const int row = v / (BK / VEC), kq = v % (BK / VEC);
#pragma unroll
          for (int j = 0; j < 4; ++j) lds[(kq * 4 + j) * STRIDE + row] = f[j];
        } else {
          const int k = v / (ROWS / VEC), rq = v % (ROWS / VEC);
          *(uint4*)(lds + k * STRIDE + rq * 4) = reg[p];
        }
      } else {
        bf16_t* lds = (bf16_t*)ldsv;
        const int row = v / (BK / VEC), kq = v % (BK / VEC);
        *(uint4*)(lds + row * STRIDE + kq * 8) = reg[p];
      }
    }
  }
};

template <bool BF, int MB, int BK>
__device__ __forceinline__ typename Mfma<BF, MB>::Frag frag_read(const void* ldsv, int stride,
                                                                 int row_base, int kk, int lane) {
  if constexpr (!BF) {
    const float* lds = (const float*)ldsv;
    const int r = lane % MB, k = lane / MB;
    return lds[(kk + k) * stride + row_base + r];
  } else {
    const bf16_t* lds = (const bf16_t*)ldsv;
    const int r = lane % MB, kg = lane / MB;
    uint4 u = *(const uint4*)(lds + (row_base + r) * stride + kk + 8 * kg);
    return __builtin_bit_cast(bf16x8, u);
  }
}

template <int BM_, int BN_, int MB_, int TM_, int TN_>
struct TileCfg {
  static constexpr int BM = BM_, BN = BN_, MB = MB_, TM = TM_, TN = TN_;
};

// One output tile (m0, n0) of C = A * B_i for i < NB.
template <bool BF, class T, bool AK, bool BKM, int NB>
struct TileCompute {
  static constexpr int BK = BF ? 128 : 64;
  static constexpr int MB = T::MB, TM = T::TM, TN = T::TN;
  typedef Mfma<BF, MB> Op;
  typedef Stage<BF, T::BM, BK, fp32_lds_pad(AK, T::BM, T::MB)> SA;
  typedef Stage<BF, T::BN, BK, fp32_lds_pad(BKM, T::BN, T::MB)> SB;
  // two register stages unless that would hold more than 16 vectors a thread
  static constexpr int ST = (SA::NREG + NB * SB::NREG) <= 16 ? 2 : 1;
  typename Op::Acc acc[NB][TM][TN];

  __device__ __forceinline__ void run(const void* A, int lda, const void* B, int ldb,
                                      long long bstride, int M, int N, int K, int m0, int n0,
                                      char* smem) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    void* lds_a = smem;
    char* lds_b = smem + SA::LDS_ELEMS * (BF ? 2 : 4);
    const int esz = BF ? 2 : 4;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < Op::NACC; ++r) acc[b][i][j][r] = 0.0f;

    // ST register stages: tiles k0 .. k0 + (ST-1)*BK are in flight together
    SA sa[ST];
    SB sb[ST][NB];
#pragma unroll
    for (int q = 0; q < ST; ++q) {
      if (q * BK < K) {
        sa[q].template load<AK>(A, lda, m0, M, q * BK, K);
#pragma unroll
        for (int b = 0; b < NB; ++b)
          sb[q][b].template load<BKM>((const char*)B + b * bstride * esz, ldb, n0, N, q * BK, K);
      }
    }
    for (int k0 = 0; k0 < K; k0 += ST * BK) {
#pragma unroll
      for (int q = 0; q < ST; ++q) {
        const int kq = k0 + q * BK;
        if (kq < K) {
          __syncthreads();
          sa[q].template store<AK>(lds_a);
#pragma unroll
          for (int b = 0; b < NB; ++b)
            sb[q][b].template store<BKM>(lds_b + b * SB::LDS_ELEMS * esz);
          __syncthreads();
          if (kq + ST * BK < K) {
            sa[q].template load<AK>(A, lda, m0, M, kq + ST * BK, K);
#pragma unroll
            for (int b = 0; b < NB; ++b)
              sb[q][b].template load<BKM>((const char*)B + b * bstride * esz, ldb, n0, N,
                                          kq + ST * BK, K);
          }
          // keep the loads' consumers (the transposes of the next stores)
          // below the products, so that the loads stay in flight under them
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int kk = 0; kk < BK; kk += Op::KSTEP) {
            typename Op::Frag fa[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i)
              fa[i] = frag_read<BF, MB, BK>(lds_a, SA::STRIDE, (wm * TM + i) * MB, kk, lane);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
#pragma unroll
              for (int j = 0; j < TN; ++j) {
                typename Op::Frag fb = frag_read<BF, MB, BK>(lds_b + b * SB::LDS_ELEMS * esz,
                                                             SB::STRIDE, (wn * TN + j) * MB, kk, lane);
#pragma unroll
                for (int i = 0; i < TM; ++i) acc[b][i][j] = Op::mma(fa[i], fb, acc[b][i][j]);
              }
            }
          }
        }
      }
    }
  }

  static constexpr int smem_bytes() {
    return (SA::LDS_ELEMS + NB * SB::LDS_ELEMS) * (BF ? 2 : 4);
  }
};

template <bool BF, class T, bool AK, bool BKM, int EPI, int NB>
__global__ void __launch_bounds__(kThreads) gemm_kernel(GemmArgs g) {
  typedef TileCompute<BF, T, AK, BKM, NB> TC;
  extern __shared__ __align__(16) char smem[];
  const int M = g.m_rows ? g.st->rows : g.M;
  const int K = g.k_rows ? g.st->rows : g.K;
  const int N = g.N;
  const int tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int m0 = (tile / gridDim.x) * T::BM, n0 = (tile % gridDim.x) * T::BN;
  if (m0 >= M) return;
  TC tc;
  tc.run(g.A, g.lda, g.B, g.ldb, g.b_branch_stride, M, N, K, m0, n0, smem);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int i = 0; i < T::TM; ++i)
#pragma unroll
    for (int j = 0; j < T::TN; ++j)
#pragma unroll
      for (int r = 0; r < TC::Op::NACC; ++r) {
        const int m = m0 + (wm * T::TM + i) * T::MB + acc_row<T::MB>(r, lane);
        const int n = n0 + (wn * T::TN + j) * T::MB + acc_col<T::MB>(lane);
        if (m >= M || n >= N) continue;
        if constexpr (EPI == EPI_STORE) {
          float v = tc.acc[0][i][j][r];
          if (g.bias) v += g.bias[n];
          if (g.resid) v += g.resid[(long long)m * g.ld_resid + n];
          if (g.out32) g.out32[(long long)m * g.ld_out32 + n] = v;
          if (g.out16) g.out16[(long long)m * g.ld_out16 + n] = f2bf(v);
        } else if constexpr (EPI == EPI_GATE_FWD) {
          float prod = 1.0f;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const float a = tc.acc[b][i][j][r] + g.bias[b * g.bias_branch_stride + n];
            g.aux[(long long)m * g.ld_aux + b * g.aux_branch + n] = a;
            prod = (b == 0) ? a : prod * a;
          }
          const float v = gelu_f(prod);
          if (g.out32) g.out32[(long long)m * g.ld_out32 + n] = v;
          if (g.out16) g.out16[(long long)m * g.ld_out16 + n] = f2bf(v);
        } else {  // EPI_GATE_BWD: branch count in bias_branch_stride
          const int nbr = g.bias_branch_stride;
          float a[3];
          float prod = 1.0f;
          for (int b = 0; b < nbr; ++b) {
            a[b] = g.aux[(long long)m * g.ld_aux + b * g.aux_branch + n];
            prod = (b == 0) ? a[b] : prod * a[b];
          }
          const float dp = tc.acc[0][i][j][r] * gelu_grad_f(prod);
          for (int b = 0; b < nbr; ++b) {
            float o = dp;
            for (int c = 0; c < nbr; ++c)
              if (c != b) o *= a[c];
            if (g.out32) g.out32[(long long)m * g.ld_out32 + b * g.aux_branch + n] = o;
            if (g.out16) g.out16[(long long)m * g.ld_out16 + b * g.aux_branch + n] = f2bf(o);
          }
        }
      }
}

// LDS of the Adam epilogue: the FP32 gradient tile, then its BF16 copy.
template <class T>
struct WgradAdamLds {
  static constexpr int LDG = T::BN + 4, LDT = T::BN + 8;
  static constexpr int BYTES = T::BM * LDG * 4 + T::BM * LDT * 2;
};

template <bool BF, class T, bool ADAM>
__global__ void __launch_bounds__(kThreads) wgrad_kernel(const WgradProblem* __restrict__ probs,
                                                         int n_probs, const StepState* st,
                                                         WgradAdam ad) {
  typedef TileCompute<BF, T, false, false, 1> TC;
  extern __shared__ __align__(16) char smem[];
  if constexpr (ADAM) {
    if ((int)blockIdx.x >= ad.tiles) {  // an element-range Adam item
      const int it = blockIdx.x - ad.tiles;
      int j = 0;
      while (j + 1 < ad.n_ejobs && it >= ad.ejobs[j + 1].item_begin) ++j;
      const AdamJob jb = ad.ejobs[j];
      adam_elements(st, jb, it - jb.item_begin, ad.p, ad.g, ad.m, ad.v, ad.ac, ad.ac.lr / st->bc1,
                    1.0f / st->bc2);
      return;
    }
  }
  const int tile = xcd_tile(blockIdx.x, ADAM ? ad.tiles : (int)gridDim.x);
  int p = 0;
  while (p + 1 < n_probs && tile >= probs[p + 1].tile_begin) ++p;
  const WgradProblem pr = probs[p];
  const int t = tile - pr.tile_begin;
  const int m0 = (t / pr.tiles_n) * T::BM, n0 = (t % pr.tiles_n) * T::BN;
  const int K = st->rows;
  TC tc;
  tc.run(pr.dout, pr.M, pr.in, pr.N, 0, pr.M, pr.N, K, m0, n0, smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  if constexpr (!ADAM) {
#pragma unroll
    for (int i = 0; i < T::TM; ++i)
#pragma unroll
      for (int j = 0; j < T::TN; ++j)
#pragma unroll
        for (int r = 0; r < TC::Op::NACC; ++r) {
          const int m = m0 + (wm * T::TM + i) * T::MB + acc_row<T::MB>(r, lane);
          const int n = n0 + (wn * T::TN + j) * T::MB + acc_col<T::MB>(lane);
          if (m < pr.M && n < pr.N) gl(pr.dw)[(long long)m * pr.N + n] = tc.acc[0][i][j][r];
        }
  } else {
    // The tile's sum over rows is complete: Adam on its parameters.  Each
    // thread takes items of 8 consecutive columns of a row (16-byte
    // accesses; the nt fragment copy straight from registers).  The loads of
    // up to 4 items are issued together, the first group before the gradient
    // is staged through LDS; the nn copy is read back transposed from a BF16
    // tile.
    typedef WgradAdamLds<T> LD;
    constexpr int CH = T::BN / 8;
    constexpr int ITEMS = T::BM * CH;
    constexpr int PER = (ITEMS + kThreads - 1) / kThreads;
    constexpr int GR = PER < 4 ? PER : 4;
    static_assert(PER % GR == 0, "item groups");
    float* sG = (float*)smem;
    bf16_t* sT = (bf16_t*)(smem + T::BM * LD::LDG * 4);
    const float lr_bc = ad.ac.lr / st->bc1;
    const float inv_bc2 = 1.0f / st->bc2;
    const size_t base = (size_t)(pr.dw - ad.g);  // element offset of the matrix
#pragma unroll
    for (int q0 = 0; q0 < PER; q0 += GR) {
      float P[GR][8], Mo[GR][8], V[GR][8];
      size_t o[GR];
      bool ok[GR];
      int rl[GR], cl[GR];
#pragma unroll
      for (int k = 0; k < GR; ++k) {
        const int idx = (int)threadIdx.x + (q0 + k) * kThreads;
        rl[k] = idx / CH;
        cl[k] = 8 * (idx - rl[k] * CH);
        ok[k] = idx < ITEMS && m0 + rl[k] < pr.M && n0 + cl[k] < pr.N;
        // an item outside the matrix loads its element 0 and stores nothing
        o[k] = ok[k] ? (size_t)(m0 + rl[k]) * pr.N + n0 + cl[k] : 0;
        adam8_load(ad.p + base + o[k], ad.m + base + o[k], ad.v + base + o[k], P[k], Mo[k], V[k]);
      }
      if (q0 == 0) {
        __syncthreads();  // every wave's last operand reads are done
#pragma unroll
        for (int i = 0; i < T::TM; ++i)
#pragma unroll
          for (int j = 0; j < T::TN; ++j)
#pragma unroll
            for (int r = 0; r < TC::Op::NACC; ++r) {
              const int ml = (wm * T::TM + i) * T::MB + acc_row<T::MB>(r, lane);
              const int nl = (wn * T::TN + j) * T::MB + acc_col<T::MB>(lane);
              sG[ml * LD::LDG + nl] = tc.acc[0][i][j][r];
            }
        __syncthreads();
      }
#pragma unroll
      for (int k = 0; k < GR; ++k) {
        if (!ok[k]) continue;
        float gv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) gv[e] = sG[rl[k] * LD::LDG + cl[k] + e];
        float4* gp = (float4*)(pr.dw + o[k]);
        gp[0] = make_float4(gv[0], gv[1], gv[2], gv[3]);
        gp[1] = make_float4(gv[4], gv[5], gv[6], gv[7]);
        adam8_math(P[k], Mo[k], V[k], gv, lr_bc, inv_bc2, ad.ac);
        adam8_store(ad.p + base + o[k], ad.m + base + o[k], ad.v + base + o[k], P[k], Mo[k], V[k]);
        const uint4 pk = pack_bf16x8(P[k]);
        const int row = m0 + rl[k], col = n0 + cl[k];
        // nt fragment (nb = row/16, kb = col/32), lane = row%16 + 16*((col%32)/8)
        st_global16(pr.nt + ((size_t)(row >> 4) * (pr.N / 32) + (col >> 5)) * 64 + (row & 15) +
                        16 * ((col & 31) >> 3),
                    pk);
        *(uint4*)&sT[rl[k] * LD::LDT + cl[k]] = pk;
      }
    }
    __syncthreads();
    // nn fragment (nb = col/16, kb = row/32), lane = col%16 + 16*((row%32)/8):
    // 8 consecutive rows of one column
    for (int idx = threadIdx.x; idx < (T::BM / 8) * T::BN; idx += kThreads) {
      const int rb = idx / T::BN, cl = idx - rb * T::BN;
      const int row = m0 + 8 * rb, col = n0 + cl;
      if (row >= pr.M || col >= pr.N) continue;
      uint32_t w[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        w[k] = (uint32_t)sT[(8 * rb + 2 * k) * LD::LDT + cl] |
               ((uint32_t)sT[(8 * rb + 2 * k + 1) * LD::LDT + cl] << 16);
      st_global16(pr.nn + ((size_t)(col >> 4) * (pr.M / 32) + (row >> 5)) * 64 + (col & 15) +
                      16 * ((row & 31) >> 3),
                  make_uint4(w[0], w[1], w[2], w[3]));
    }
  }
}

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------
typedef TileCfg<32, 32, 16, 1, 1> T32x32;
typedef TileCfg<64, 32, 16, 2, 1> T64x32;
typedef TileCfg<32, 64, 16, 1, 2> T32x64;
typedef TileCfg<64, 64, 32, 1, 1> T64x64;
typedef TileCfg<128, 64, 32, 2, 1> T128x64;
typedef TileCfg<64, 128, 32, 1, 2> T64x128;
typedef TileCfg<128, 128, 32, 2, 2> T128x128;

template <bool BF, class T, bool AK, bool BKM, int EPI, int NB>
static hipError_t launch_one(const GemmArgs& g, int grid_m_max, hipStream_t s) {
  typedef TileCompute<BF, T, AK, BKM, NB> TC;
  dim3 grid((g.N + T::BN - 1) / T::BN, (grid_m_max + T::BM - 1) / T::BM);
  if (grid.x == 0 || grid.y == 0) return hipSuccess;
  constexpr int smem = TC::smem_bytes();
  static_assert(smem <= 160 * 1024, "tile does not fit in LDS");
  if constexpr (smem > 64 * 1024) {
    static bool done = false;
    if (!done) {
      hipError_t e = hipFuncSetAttribute((const void*)gemm_kernel<BF, T, AK, BKM, EPI, NB>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, smem);
      if (e != hipSuccess) return e;
      done = true;
    }
  }
  hipLaunchKernelGGL((gemm_kernel<BF, T, AK, BKM, EPI, NB>), grid, dim3(kThreads), smem, s, g);
  return hipGetLastError();
}

template <bool BF, class T>
static hipError_t launch_t(bool ak, bool bk, EpiKind epi, int nb, const GemmArgs& g, int gm,
                           hipStream_t s) {
  if (ak && bk) {  // forward dense layers
    if (epi == EPI_STORE) return launch_one<BF, T, true, true, EPI_STORE, 1>(g, gm, s);
    if (epi == EPI_GATE_FWD) {
      if (nb == 1) return launch_one<BF, T, true, true, EPI_GATE_FWD, 1>(g, gm, s);
      if (nb == 2) return launch_one<BF, T, true, true, EPI_GATE_FWD, 2>(g, gm, s);
      if (nb == 3) return launch_one<BF, T, true, true, EPI_GATE_FWD, 3>(g, gm, s);
    }
  } else if (ak && !bk) {  // adjoint of the input
    if (epi == EPI_STORE) return launch_one<BF, T, true, false, EPI_STORE, 1>(g, gm, s);
    if (epi == EPI_GATE_BWD) return launch_one<BF, T, true, false, EPI_GATE_BWD, 1>(g, gm, s);
  }
  return hipErrorInvalidValue;
}

template <bool BF>
static hipError_t launch_p(int tile, bool ak, bool bk, EpiKind epi, int nb, const GemmArgs& g,
                           int gm, hipStream_t s) {
  switch (tile) {
    case TILE_32x32: return launch_t<BF, T32x32>(ak, bk, epi, nb, g, gm, s);
    case TILE_64x32: return launch_t<BF, T64x32>(ak, bk, epi, nb, g, gm, s);
    case TILE_32x64: return launch_t<BF, T32x64>(ak, bk, epi, nb, g, gm, s);
    case TILE_64x64: return launch_t<BF, T64x64>(ak, bk, epi, nb, g, gm, s);
    case TILE_128x64: return launch_t<BF, T128x64>(ak, bk, epi, nb, g, gm, s);
    case TILE_64x128: return launch_t<BF, T64x128>(ak, bk, epi, nb, g, gm, s);
    case TILE_128x128: return launch_t<BF, T128x128>(ak, bk, epi, nb, g, gm, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm(int tile, bool bf16, bool a_kmajor, bool b_kmajor, EpiKind epi, int nb,
                       const GemmArgs& g, int grid_m_max, hipStream_t s) {
  if (tile >= TILE_W128x128) {
    if (!wide_tile_supported(tile, bf16, epi, nb)) return hipErrorInvalidValue;
    return launch_gemm_wide(tile, a_kmajor, b_kmajor, epi, nb, g, grid_m_max, s);
  }
  return bf16 ? launch_p<true>(tile, a_kmajor, b_kmajor, epi, nb, g, grid_m_max, s)
              : launch_p<false>(tile, a_kmajor, b_kmajor, epi, nb, g, grid_m_max, s);
}

template <bool BF, class T>
static hipError_t launch_w(const WgradProblem* d_probs, int n_probs, int total_tiles,
                           const StepState* st, hipStream_t s) {
  typedef TileCompute<BF, T, false, false, 1> TC;
  if (total_tiles == 0) return hipSuccess;
  constexpr int smem = TC::smem_bytes();
  static_assert(smem <= 160 * 1024, "tile does not fit in LDS");
  if constexpr (smem > 64 * 1024) {
    static bool done = false;
    if (!done) {
      hipError_t e = hipFuncSetAttribute((const void*)wgrad_kernel<BF, T, false>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, smem);
      if (e != hipSuccess) return e;
      done = true;
    }
  }
  hipLaunchKernelGGL((wgrad_kernel<BF, T, false>), dim3(total_tiles), dim3(kThreads), smem, s,
                     d_probs, n_probs, st, WgradAdam{});
  return hipGetLastError();
}

template <class T>
static hipError_t launch_wa(const WgradProblem* d_probs, int n_probs, int wgs,
                            const StepState* st, const WgradAdam& ad, hipStream_t s) {
  typedef TileCompute<true, T, false, false, 1> TC;
  if (wgs == 0) return hipSuccess;
  constexpr int smem = TC::smem_bytes() > WgradAdamLds<T>::BYTES ? TC::smem_bytes()
                                                                  : WgradAdamLds<T>::BYTES;
  static_assert(smem <= 160 * 1024, "tile does not fit in LDS");
  static_assert(T::BM % 32 == 0 && T::BN % 8 == 0, "Adam epilogue tile shape");
  if constexpr (smem > 64 * 1024) {
    static bool done = false;
    if (!done) {
      hipError_t e = hipFuncSetAttribute((const void*)wgrad_kernel<true, T, true>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, smem);
      if (e != hipSuccess) return e;
      done = true;
    }
  }
  hipLaunchKernelGGL((wgrad_kernel<true, T, true>), dim3(wgs), dim3(kThreads), smem, s, d_probs,
                     n_probs, st, ad);
  return hipGetLastError();
}

hipError_t launch_wgrad_adam(int tile, const WgradProblem* p, int n, int tt, int elem_items,
                             const StepState* st, const WgradAdam& ad_in, hipStream_t s) {
  WgradAdam ad = ad_in;
  ad.tiles = tt;
  const int wgs = tt + elem_items;
  switch (tile) {
    case TILE_32x32: return launch_wa<T32x32>(p, n, wgs, st, ad, s);
    case TILE_64x32: return launch_wa<T64x32>(p, n, wgs, st, ad, s);
    case TILE_32x64: return launch_wa<T32x64>(p, n, wgs, st, ad, s);
    case TILE_64x64: return launch_wa<T64x64>(p, n, wgs, st, ad, s);
    case TILE_128x64: return launch_wa<T128x64>(p, n, wgs, st, ad, s);
    case TILE_64x128: return launch_wa<T64x128>(p, n, wgs, st, ad, s);
    case TILE_128x128: return launch_wa<T128x128>(p, n, wgs, st, ad, s);
  }
  return hipErrorInvalidValue;
}

template <bool BF>
static hipError_t launch_wp(int tile, const WgradProblem* p, int n, int tt, const StepState* st,
                            hipStream_t s) {
  switch (tile) {
    case TILE_32x32: return launch_w<BF, T32x32>(p, n, tt, st, s);
    case TILE_64x32: return launch_w<BF, T64x32>(p, n, tt, st, s);
    case TILE_32x64: return launch_w<BF, T32x64>(p, n, tt, st, s);
    case TILE_64x64: return launch_w<BF, T64x64>(p, n, tt, st, s);
    case TILE_128x64: return launch_w<BF, T128x64>(p, n, tt, st, s);
    case TILE_64x128: return launch_w<BF, T64x128>(p, n, tt, st, s);
    case TILE_128x128: return launch_w<BF, T128x128>(p, n, tt, st, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_wgrad(int tile, bool bf16, const WgradProblem* d_probs, int n_probs,
                        int total_tiles, const StepState* st, float* part, hipStream_t s) {
  if (tile >= TILE_W128x128) {
    if (!bf16) return hipErrorInvalidValue;
    return launch_wgrad_wide(tile, d_probs, n_probs, total_tiles, st, part, s);
  }
  return bf16 ? launch_wp<true>(tile, d_probs, n_probs, total_tiles, st, s)
              : launch_wp<false>(tile, d_probs, n_probs, total_tiles, st, s);
}

}  // namespace edpc
