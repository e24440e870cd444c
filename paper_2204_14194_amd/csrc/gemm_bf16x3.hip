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
// 8 (l / 16) for both operands; the result layout equals the 16x16x4 f32
// one: D[4 (l / 16) + e][l % 16].
//
// Tiling, clamped row reads, the contraction tail and the three store modes
// follow gemm.hip.
#include "se_internal.h"

namespace sefase {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int hBK = 32;      // contraction steps per stage
constexpr int hPad = 8;      // bf16 elements of row padding (16 bytes)

enum StoreModeH { hStoreRowMajor = 0, hStoreTransposed = 1, hStoreSymmetric = 2 };

__device__ inline int xcd_remap_h(int id, int ntiles) {
  if ((ntiles & 7) != 0) return id;
  const int per = ntiles >> 3;
  return (id & 7) * per + (id >> 3);
}

template <int ROWS>
struct TileRegs {
  static constexpr int NQ = ROWS * hBK / 8 / 256;   // 16-byte chunks per thread
  uint4 hi[NQ], lo[NQ];
};

__device__ inline uint4 pack8(const uint16_t (&e)[8]) {
  return make_uint4(e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16),
                    e[4] | ((uint32_t)e[5] << 16), e[6] | ((uint32_t)e[7] << 16));
}

template <int ROWS, bool VEC, bool KTAIL>
__device__ inline void load_h(const uint16_t* __restrict__ shi, const uint16_t* __restrict__ slo,
                              int ld, int row0, int nrows, int k0, int P, TileRegs<ROWS>& t) {
#pragma unroll
  for (int q = 0; q < TileRegs<ROWS>::NQ; ++q) {
    const int idx = threadIdx.x + 256 * q;
    const int r = idx / (hBK / 8);
    const int c = (idx % (hBK / 8)) * 8;
    int gr = row0 + r;
    gr = gr < nrows ? gr : nrows - 1;
    const int gk = k0 + c;
    const size_t o = (size_t)gr * ld + gk;
    if (VEC && !KTAIL) {
      t.hi[q] = *reinterpret_cast<const uint4*>(shi + o);
      t.lo[q] = *reinterpret_cast<const uint4*>(slo + o);
    } else {
      uint16_t eh[8], el[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool ok = !KTAIL || gk + e < P;
        eh[e] = ok ? shi[o + e] : (uint16_t)0;
        el[e] = ok ? slo[o + e] : (uint16_t)0;
      }
      t.hi[q] = pack8(eh);
      t.lo[q] = pack8(el);
    }
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

template <int BM, int BN, bool VEC, int MODE>
__global__ __launch_bounds__(256) void k_gemm_nt_bf16x3(
    const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo, int lda,
    const uint16_t* __restrict__ Bhi, const uint16_t* __restrict__ Blo, int ldb,
    float* __restrict__ C, int ldc, int Ma, int Nb, int Mst, int Nst, int P, int tiles_n,
    int ntiles, const int32_t* __restrict__ nb_dev, const int32_t* __restrict__ cmap) {
  constexpr int SI = BM / 32, SJ = BN / 32;
  __shared__ __attribute__((aligned(16))) uint16_t Ash[2][BM][hBK + hPad];
  __shared__ __attribute__((aligned(16))) uint16_t Asl[2][BM][hBK + hPad];
  __shared__ __attribute__((aligned(16))) uint16_t Bsh[2][BN][hBK + hPad];
  __shared__ __attribute__((aligned(16))) uint16_t Bsl[2][BN][hBK + hPad];

  const int tile = xcd_remap_h(blockIdx.x, ntiles);
  int bi, bj;
  if (MODE == hStoreSymmetric) {
    bi = (int)((sqrtf(8.0f * (float)tile + 1.0f) - 1.0f) * 0.5f);
    while ((bi + 1) * (bi + 2) / 2 <= tile) ++bi;
    while (bi * (bi + 1) / 2 > tile) --bi;
    bj = tile - bi * (bi + 1) / 2;
  } else {
    bi = tile / tiles_n;
    bj = tile - bi * tiles_n;
  }
  const int m0 = bi * BM, n0 = bj * BN;
  // rows formed on demand: block count on the device, mapped destinations
  if (MODE == hStoreTransposed && nb_dev) {
    Nb = min(Nb, *nb_dev);
    if (n0 >= Nb) return;                     // uniform over the workgroup
  }
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
  const bool ragged = (P % hBK) != 0;
  if (nk == 1 && ragged) {
    load_h<BM, VEC, true>(Ahi, Alo, lda, m0, Ma, 0, P, ra);
    load_h<BN, VEC, true>(Bhi, Blo, ldb, n0, Nb, 0, P, rb);
  } else {
    load_h<BM, VEC, false>(Ahi, Alo, lda, m0, Ma, 0, P, ra);
    load_h<BN, VEC, false>(Bhi, Blo, ldb, n0, Nb, 0, P, rb);
  }
  store_h<BM>(Ash[0], Asl[0], ra);
  store_h<BN>(Bsh[0], Bsl[0], rb);
  __syncthreads();

  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      const int k1 = (kt + 1) * hBK;
      if (kt + 2 == nk && ragged) {
        load_h<BM, VEC, true>(Ahi, Alo, lda, m0, Ma, k1, P, ra);
        load_h<BN, VEC, true>(Bhi, Blo, ldb, n0, Nb, k1, P, rb);
      } else {
        load_h<BM, VEC, false>(Ahi, Alo, lda, m0, Ma, k1, P, ra);
        load_h<BN, VEC, false>(Bhi, Blo, ldb, n0, Nb, k1, P, rb);
      }
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
    // blocked summation: this stage's products into fresh accumulators
    floatx4 part[SI][SJ];
#pragma unroll
    for (int i = 0; i < SI; ++i)
#pragma unroll
      for (int j = 0; j < SJ; ++j)
        part[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal[i], fbh[j],
                                                             floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < SI; ++i)
#pragma unroll
      for (int j = 0; j < SJ; ++j)
        part[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbl[j], part[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < SI; ++i)
#pragma unroll
      for (int j = 0; j < SJ; ++j)
        part[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbh[j], part[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < SI; ++i)
#pragma unroll
      for (int j = 0; j < SJ; ++j) acc[i][j] += part[i][j];
    if (kt + 1 < nk) {
      store_h<BM>(Ash[cur ^ 1], Asl[cur ^ 1], ra);
      store_h<BN>(Bsh[cur ^ 1], Bsl[cur ^ 1], rb);
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < SI; ++i)
#pragma unroll
    for (int j = 0; j < SJ; ++j) {
      const int r0 = m0 + wr * (BM / 2) + 16 * i + 4 * lq;
      const int c = n0 + wc * (BN / 2) + 16 * j + lr;
      if (MODE == hStoreTransposed) {
        if (c < Nst && c < Nb) {
          float4 v;
          v.x = r0 + 0 < Ma ? acc[i][j][0] : 0.0f;
          v.y = r0 + 1 < Ma ? acc[i][j][1] : 0.0f;
          v.z = r0 + 2 < Ma ? acc[i][j][2] : 0.0f;
          v.w = r0 + 3 < Ma ? acc[i][j][3] : 0.0f;
          float* dst = C + (size_t)(cmap ? cmap[c] : c) * ldc + r0;
          if ((ldc & 3) == 0 && (reinterpret_cast<uintptr_t>(C) & 15) == 0 && r0 + 3 < Mst) {
            *reinterpret_cast<float4*>(dst) = v;
          } else {
            if (r0 + 0 < Mst) dst[0] = v.x;
            if (r0 + 1 < Mst) dst[1] = v.y;
            if (r0 + 2 < Mst) dst[2] = v.z;
            if (r0 + 3 < Mst) dst[3] = v.w;
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + e;
          const float v = acc[i][j][e];
          if (MODE == hStoreSymmetric) {
            if (bi == bj && r < Ma && c < Nb && r >= c) {   // diagonal tile
              C[(size_t)r * ldc + c] = v;
              if (r > c) C[(size_t)c * ldc + r] = v;
            } else if (bi != bj && r < Ma && c < Nb) {
              C[(size_t)r * ldc + c] = v;                   // mirror below, as float4
            }
          } else {
            if (r < Mst && c < Nst) C[(size_t)r * ldc + c] = (r < Ma && c < Nb) ? v : 0.0f;
          }
        }
        if (MODE == hStoreSymmetric && bi != bj && c < Nb) {
          // off-diagonal tile: rows r0..r0+3 of column c are one row segment of
          // the mirrored tile
          float* dst = C + (size_t)(cmap ? cmap[c] : c) * ldc + r0;
          if ((ldc & 3) == 0 && r0 + 3 < Ma) {
            *reinterpret_cast<float4*>(dst) =
                make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (r0 + e < Ma) dst[e] = acc[i][j][e];
          }
        }
      }
    }
}

template <int BM, int MODE>
static se_status launch_h(const uint16_t* Ahi, const uint16_t* Alo, int lda, const uint16_t* Bhi,
                          const uint16_t* Blo, int ldb, float* C, int ldc, int Ma, int Nb,
                          int Mst, int Nst, int P, bool vec, hipStream_t s,
                          const int32_t* nb_dev = nullptr, const int32_t* cmap = nullptr) {
  int ntiles, tiles_n;
  if (MODE == hStoreSymmetric) {
    const int nb = (Ma + BM - 1) / BM;
    ntiles = nb * (nb + 1) / 2;
    tiles_n = nb;
  } else {
    tiles_n = (Nst + BM - 1) / BM;
    ntiles = ((Mst + BM - 1) / BM) * tiles_n;
  }
  if (ntiles <= 0 || P <= 0) return SE_OK;
  if (vec)
    hipLaunchKernelGGL((k_gemm_nt_bf16x3<BM, BM, true, MODE>), dim3(ntiles), dim3(256), 0, s, Ahi,
                       Alo, lda, Bhi, Blo, ldb, C, ldc, Ma, Nb, Mst, Nst, P, tiles_n, ntiles, nb_dev,
                       cmap);
  else
    hipLaunchKernelGGL((k_gemm_nt_bf16x3<BM, BM, false, MODE>), dim3(ntiles), dim3(256), 0, s,
                       Ahi, Alo, lda, Bhi, Blo, ldb, C, ldc, Ma, Nb, Mst, Nst, P, tiles_n, ntiles, nb_dev,
                       cmap);
  return check_launch("gemm_nt_bf16x3");
}

template <int MODE>
static se_status dispatch_h(const uint16_t* Ahi, const uint16_t* Alo, int lda, const uint16_t* Bhi,
                            const uint16_t* Blo, int ldb, float* C, int ldc, int Ma, int Nb,
                            int Mst, int Nst, int P, hipStream_t s, int tile = 0,
                            const int32_t* nb_dev = nullptr, const int32_t* cmap = nullptr) {
  const uintptr_t al = reinterpret_cast<uintptr_t>(Ahi) | reinterpret_cast<uintptr_t>(Alo) |
                       reinterpret_cast<uintptr_t>(Bhi) | reinterpret_cast<uintptr_t>(Blo);
  const bool vec = (lda % 8 == 0) && (ldb % 8 == 0) && (al % 16 == 0);
  long long big;
  if (MODE == hStoreSymmetric) {
    const long long nb = (Ma + 127) / 128;
    big = nb * (nb + 1) / 2;
  } else {
    big = (long long)((Mst + 127) / 128) * ((Nst + 127) / 128);
  }
  if (tile <= 0) tile = big >= 512 ? 128 : 64;
  if (tile == 128)
    return launch_h<128, MODE>(Ahi, Alo, lda, Bhi, Blo, ldb, C, ldc, Ma, Nb, Mst, Nst, P, vec, s,
                               nb_dev, cmap);
  return launch_h<64, MODE>(Ahi, Alo, lda, Bhi, Blo, ldb, C, ldc, Ma, Nb, Mst, Nst, P, vec, s,
                            nb_dev, cmap);
}

se_status gemm_syrk_bf16x3(const uint16_t* Yhi, const uint16_t* Ylo, int ldy, int K, int P,
                           float* G, int ldg, hipStream_t s) {
  return dispatch_h<hStoreSymmetric>(Yhi, Ylo, ldy, Yhi, Ylo, ldy, G, ldg, K, K, K, K, P, s);
}

se_status gemm_project_bf16x3(const uint16_t* Yhi, const uint16_t* Ylo, int ldy, int K,
                              const uint16_t* Xhi, const uint16_t* Xlo, int ldx, int n_blk, int P,
                              float* R, int ldr, hipStream_t s, bool pad) {
  return dispatch_h<hStoreTransposed>(Yhi, Ylo, ldy, Xhi, Xlo, ldx, R, ldr, K, n_blk,
                                      pad ? ldr : K, n_blk, P, s);
}

se_status gemm_rows_bf16x3(const uint16_t* Yhi, const uint16_t* Ylo, int ldy, int K,
                           const uint16_t* Xhi, const uint16_t* Xlo, int ldx, int n_max,
                           const int32_t* n_dev, const int32_t* cmap, int P, float* rows, int ldr,
                           int tile, hipStream_t s) {
  return dispatch_h<hStoreTransposed>(Yhi, Ylo, ldy, Xhi, Xlo, ldx, rows, ldr, K, n_max, K, n_max,
                                      P, s, tile, n_dev, cmap);
}

}  // namespace sefase
