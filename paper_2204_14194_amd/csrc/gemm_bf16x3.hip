// Split-BF16 ("BF16x3") variant of the NT GEMM of gemm.hip, for the
// precision path of the table generation (eq. 16) and of the initial
// projections (eq. 12).  Every float32 operand x is stored as two bfloat16
// numbers, hi = bf16(x) and lo = bf16(x - hi); the product a b is formed as
// lo_a hi_b + hi_a lo_b + hi_a hi_b on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16) with float32 accumulation.  The dropped term
// lo_a lo_b is below 2^-16 relative.
//
// MFMA 16x16x32 bf16 mapping (lane l): A row m = l % 16 and B column
// n = l % 16, each lane supplying 8 consecutive contraction steps starting at
// 8 (l / 16); the result layout equals the 16x16x4 f32 one:
// D[4 (l / 16) + e][l % 16].
#include "se_internal.h"

namespace sefase {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int hBK = 32;      // contraction steps per stage
constexpr int hPad = 8;      // bf16 elements of row padding (16 bytes)

__device__ inline int xcd_remap_h(int id, int ntiles) {
  if ((ntiles & 7) != 0) return id;
  const int per = ntiles >> 3;
  return (id & 7) * per + (id >> 3);
}

template <int ROWS>
struct TileRegs {
  static constexpr int NQ = ROWS * hBK / 8 / 256;   // 16-byte chunks per thread
  uint4 hi[NQ > 0 ? NQ : 1], lo[NQ > 0 ? NQ : 1];
};

template <int ROWS, bool VEC>
__device__ inline void load_h(const uint16_t* __restrict__ shi, const uint16_t* __restrict__ slo,
                              int ld, int row0, int nrows, int k0, int P, TileRegs<ROWS>& t) {
#pragma unroll
  for (int q = 0; q < TileRegs<ROWS>::NQ; ++q) {
    const int idx = threadIdx.x + 256 * q;
    const int r = idx / (hBK / 8);
    const int c = (idx % (hBK / 8)) * 8;
    const int gr = row0 + r, gk = k0 + c;
    uint4 vh = make_uint4(0, 0, 0, 0), vl = make_uint4(0, 0, 0, 0);
    if (gr < nrows) {
      const size_t o = (size_t)gr * ld + gk;
      if (VEC && gk + 7 < P) {
        vh = *reinterpret_cast<const uint4*>(shi + o);
        vl = *reinterpret_cast<const uint4*>(slo + o);
      } else {
        uint16_t eh[8], el[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          eh[e] = (gk + e < P) ? shi[o + e] : (uint16_t)0;
          el[e] = (gk + e < P) ? slo[o + e] : (uint16_t)0;
        }
        vh = make_uint4(eh[0] | (eh[1] << 16), eh[2] | (eh[3] << 16), eh[4] | (eh[5] << 16),
                        eh[6] | (eh[7] << 16));
        vl = make_uint4(el[0] | (el[1] << 16), el[2] | (el[3] << 16), el[4] | (el[5] << 16),
                        el[6] | (el[7] << 16));
      }
    }
    t.hi[q] = vh;
    t.lo[q] = vl;
  }
}

template <int ROWS>
__device__ inline void store_h(uint16_t (*lhi)[hBK + hPad], uint16_t (*llo)[hBK + hPad],
                               const TileRegs<ROWS>& t) {
#pragma unroll
  for (int q = 0; q < TileRegs<ROWS>::NQ; ++q) {
    const int idx = threadIdx.x + 256 * q;
    const int r = idx / (hBK / 8);
    const int c = (idx % (hBK / 8)) * 8;
    *reinterpret_cast<uint4*>(&lhi[r][c]) = t.hi[q];
    *reinterpret_cast<uint4*>(&llo[r][c]) = t.lo[q];
  }
}

template <int BM, int BN, bool VEC, bool SYRK>
__global__ __launch_bounds__(256) void k_gemm_nt_bf16x3(
    const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo, int lda,
    const uint16_t* __restrict__ Bhi, const uint16_t* __restrict__ Blo, int ldb,
    float* __restrict__ C, int ldc, int Mr, int Nc, int Nst, int P, int tiles_n, int ntiles) {
  constexpr int SI = BM / 32, SJ = BN / 32;
  __shared__ __attribute__((aligned(16))) uint16_t Ash[2][BM][hBK + hPad];
  __shared__ __attribute__((aligned(16))) uint16_t Asl[2][BM][hBK + hPad];
  __shared__ __attribute__((aligned(16))) uint16_t Bsh[2][BN][hBK + hPad];
  __shared__ __attribute__((aligned(16))) uint16_t Bsl[2][BN][hBK + hPad];

  const int tile = xcd_remap_h(blockIdx.x, ntiles);
  int bi, bj;
  if (SYRK) {
    bi = (int)((sqrtf(8.0f * (float)tile + 1.0f) - 1.0f) * 0.5f);
    while ((bi + 1) * (bi + 2) / 2 <= tile) ++bi;
    while (bi * (bi + 1) / 2 > tile) --bi;
    bj = tile - bi * (bi + 1) / 2;
  } else {
    bi = tile / tiles_n;
    bj = tile - bi * tiles_n;
  }
  const int m0 = bi * BM, n0 = bj * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int lr = lane & 15, lq = lane >> 4;

  floatx4 acc[SI][SJ];
#pragma unroll
  for (int i = 0; i < SI; ++i)
#pragma unroll
    for (int j = 0; j < SJ; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  TileRegs<BM> ra;
  TileRegs<BN> rb;
  const int nk = (P + hBK - 1) / hBK;
  load_h<BM, VEC>(Ahi, Alo, lda, m0, Mr, 0, P, ra);
  load_h<BN, VEC>(Bhi, Blo, ldb, n0, Nc, 0, P, rb);
  store_h<BM>(Ash[0], Asl[0], ra);
  store_h<BN>(Bsh[0], Bsl[0], rb);
  __syncthreads();

  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      load_h<BM, VEC>(Ahi, Alo, lda, m0, Mr, (kt + 1) * hBK, P, ra);
      load_h<BN, VEC>(Bhi, Blo, ldb, n0, Nc, (kt + 1) * hBK, P, rb);
    }
    bf16x8 fah[SI], fal[SI], fbh[SJ], fbl[SJ];
#pragma unroll
    for (int i = 0; i < SI; ++i) {
      const int r = wr * (BM / 2) + 16 * i + lr;
      fah[i] = *reinterpret_cast<const bf16x8*>(&Ash[cur][r][8 * lq]);
      fal[i] = *reinterpret_cast<const bf16x8*>(&Asl[cur][r][8 * lq]);
    }
#pragma unroll
    for (int j = 0; j < SJ; ++j) {
      const int r = wc * (BN / 2) + 16 * j + lr;
      fbh[j] = *reinterpret_cast<const bf16x8*>(&Bsh[cur][r][8 * lq]);
      fbl[j] = *reinterpret_cast<const bf16x8*>(&Bsl[cur][r][8 * lq]);
    }
#pragma unroll
    for (int i = 0; i < SI; ++i)
#pragma unroll
      for (int j = 0; j < SJ; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal[i], fbh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbh[j], acc[i][j], 0, 0, 0);
      }
    if (kt + 1 < nk) {
      store_h<BM>(Ash[cur ^ 1], Asl[cur ^ 1], ra);
      store_h<BN>(Bsh[cur ^ 1], Bsl[cur ^ 1], rb);
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < SI; ++i)
#pragma unroll
    for (int j = 0; j < SJ; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = m0 + wr * (BM / 2) + 16 * i + 4 * lq + e;
        const int c = n0 + wc * (BN / 2) + 16 * j + lr;
        const float v = acc[i][j][e];
        if (SYRK) {
          if (r < Mr && c < Nc && r >= c) {
            C[(size_t)r * ldc + c] = v;
            if (r > c) C[(size_t)c * ldc + r] = v;
          }
        } else {
          if (r < Mr && c < Nst) C[(size_t)r * ldc + c] = v;
        }
      }
}

template <int BM, bool SYRK>
static se_status launch_h(const uint16_t* Ahi, const uint16_t* Alo, int lda, const uint16_t* Bhi,
                          const uint16_t* Blo, int ldb, float* C, int ldc, int Mr, int Nc,
                          int Nst, int P, bool vec, hipStream_t s) {
  int ntiles, tiles_n;
  if (SYRK) {
    const int nb = (Mr + BM - 1) / BM;
    ntiles = nb * (nb + 1) / 2;
    tiles_n = nb;
  } else {
    tiles_n = (Nst + BM - 1) / BM;
    ntiles = ((Mr + BM - 1) / BM) * tiles_n;
  }
  if (ntiles <= 0) return SE_OK;
  if (vec)
    hipLaunchKernelGGL((k_gemm_nt_bf16x3<BM, BM, true, SYRK>), dim3(ntiles), dim3(256), 0, s, Ahi,
                       Alo, lda, Bhi, Blo, ldb, C, ldc, Mr, Nc, Nst, P, tiles_n, ntiles);
  else
    hipLaunchKernelGGL((k_gemm_nt_bf16x3<BM, BM, false, SYRK>), dim3(ntiles), dim3(256), 0, s,
                       Ahi, Alo, lda, Bhi, Blo, ldb, C, ldc, Mr, Nc, Nst, P, tiles_n, ntiles);
  return check_launch("gemm_nt_bf16x3");
}

se_status gemm_nt_bf16x3(const uint16_t* Ahi, const uint16_t* Alo, int lda, const uint16_t* Bhi,
                         const uint16_t* Blo, int ldb, float* C, int ldc, int Mr, int Nc, int Nst,
                         int P, bool syrk, hipStream_t s) {
  const uintptr_t al = reinterpret_cast<uintptr_t>(Ahi) | reinterpret_cast<uintptr_t>(Alo) |
                       reinterpret_cast<uintptr_t>(Bhi) | reinterpret_cast<uintptr_t>(Blo);
  const bool vec = (lda % 8 == 0) && (ldb % 8 == 0) && (al % 16 == 0);
  long long big;
  if (syrk) {
    const long long nb = (Mr + 127) / 128;
    big = nb * (nb + 1) / 2;
  } else {
    big = (long long)((Mr + 127) / 128) * ((Nst + 127) / 128);
  }
  if (big >= 512)
    return syrk ? launch_h<128, true>(Ahi, Alo, lda, Bhi, Blo, ldb, C, ldc, Mr, Nc, Nst, P, vec, s)
                : launch_h<128, false>(Ahi, Alo, lda, Bhi, Blo, ldb, C, ldc, Mr, Nc, Nst, P, vec, s);
  return syrk ? launch_h<64, true>(Ahi, Alo, lda, Bhi, Blo, ldb, C, ldc, Mr, Nc, Nst, P, vec, s)
              : launch_h<64, false>(Ahi, Alo, lda, Bhi, Blo, ldb, C, ldc, Mr, Nc, Nst, P, vec, s);
}

}  // namespace sefase
