// Matrix-core GEMM for the two dense contractions of the method:
//   * table generation (Algorithm 2, eq. 16): G = Y Y^T over the area pixels,
//     lower-triangle tiles only, each stored twice (G is symmetric, so only
//     (|D|^2 + |D|)/2 scalar products are needed);
//   * initial projections (eq. 12) of a batch of blocks: R = X Y^T.
// C[r][c] = sum_p A[r][p] B[c][p]; both operands row-major with the
// contraction index p contiguous ("NT").
//
// FP32 path: v_mfma_f32_16x16x4_f32.  A 256-thread workgroup (4 waves, 2x2)
// owns a BM x BN output tile; each wave a (BM/2) x (BN/2) sub-tile made of
// 16x16 MFMA tiles.  Operand tiles of BK = 32 contraction steps are staged
// through LDS, double-buffered (one barrier per step).  A lane feeds the MFMA
// a float4 along p: four consecutive MFMAs consume its x, y, z, w components,
// which only permutes the order of the contraction, identically for A and B.
//
// MFMA 16x16x4 f32 operand/result mapping (lane l, 0..63):
//   A[m][k]: m = l % 16, k = l / 16        B[k][n]: n = l % 16, k = l / 16
//   D[m][n] (4 floats e = 0..3): m = 4 (l / 16) + e, n = l % 16
#include "se_internal.h"

namespace sefase {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kBK = 32;
constexpr int kPad = 4;

// Map the linear workgroup id to a tile so that the 8 XCDs (which receive
// workgroups round-robin) each work on a contiguous range of tiles.
__device__ inline int xcd_remap(int id, int ntiles) {
  if ((ntiles & 7) != 0) return id;
  const int per = ntiles >> 3;
  return (id & 7) * per + (id >> 3);
}

template <int ROWS, bool VEC>
__device__ inline void load_tile(const float* __restrict__ src, int ld, int row0, int nrows,
                                 int k0, int P, float4 (&reg)[ROWS * kBK / 4 / 256]) {
  constexpr int NQ = ROWS * kBK / 4 / 256;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int idx = threadIdx.x + 256 * q;
    const int r = idx / (kBK / 4);
    const int c = (idx % (kBK / 4)) * 4;
    const int gr = row0 + r;
    const int gk = k0 + c;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gr < nrows) {
      const float* p = src + (size_t)gr * ld + gk;
      if (VEC && gk + 3 < P) {
        v = *reinterpret_cast<const float4*>(p);
      } else {
        if (gk + 0 < P) v.x = p[0];
        if (gk + 1 < P) v.y = p[1];
        if (gk + 2 < P) v.z = p[2];
        if (gk + 3 < P) v.w = p[3];
      }
    }
    reg[q] = v;
  }
}

template <int ROWS>
__device__ inline void store_tile(float (*lds)[kBK + kPad], const float4 (&reg)[ROWS * kBK / 4 / 256]) {
  constexpr int NQ = ROWS * kBK / 4 / 256;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int idx = threadIdx.x + 256 * q;
    const int r = idx / (kBK / 4);
    const int c = (idx % (kBK / 4)) * 4;
    *reinterpret_cast<float4*>(&lds[r][c]) = reg[q];
  }
}

template <int BM, int BN, bool VEC, bool SYRK>
__global__ __launch_bounds__(256) void k_gemm_nt_f32(const float* __restrict__ A, int lda,
                                                     const float* __restrict__ B, int ldb,
                                                     float* __restrict__ C, int ldc, int Mr, int Nc,
                                                     int Nst, int P, int tiles_n, int ntiles) {
  constexpr int SI = BM / 32, SJ = BN / 32;   // 16x16 MFMA tiles per wave
  __shared__ __attribute__((aligned(16))) float As[2][BM][kBK + kPad];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN][kBK + kPad];

  const int tile = xcd_remap(blockIdx.x, ntiles);
  int bi, bj;
  if (SYRK) {
    // tile -> (bi, bj), bj <= bi, row-major over the lower triangle
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

  float4 ra[BM * kBK / 4 / 256], rb[BN * kBK / 4 / 256];
  const int nk = (P + kBK - 1) / kBK;
  load_tile<BM, VEC>(A, lda, m0, Mr, 0, P, ra);
  load_tile<BN, VEC>(B, ldb, n0, Nc, 0, P, rb);
  store_tile<BM>(As[0], ra);
  store_tile<BN>(Bs[0], rb);
  __syncthreads();

  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      load_tile<BM, VEC>(A, lda, m0, Mr, (kt + 1) * kBK, P, ra);
      load_tile<BN, VEC>(B, ldb, n0, Nc, (kt + 1) * kBK, P, rb);
    }
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 16) {
      float4 fa[SI], fb[SJ];
#pragma unroll
      for (int i = 0; i < SI; ++i)
        fa[i] = *reinterpret_cast<const float4*>(&As[cur][wr * (BM / 2) + 16 * i + lr][kk + 4 * lq]);
#pragma unroll
      for (int j = 0; j < SJ; ++j)
        fb[j] = *reinterpret_cast<const float4*>(&Bs[cur][wc * (BN / 2) + 16 * j + lr][kk + 4 * lq]);
#pragma unroll
      for (int i = 0; i < SI; ++i)
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].x, fb[j].x, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].y, fb[j].y, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].z, fb[j].z, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].w, fb[j].w, acc[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) {
      store_tile<BM>(As[cur ^ 1], ra);
      store_tile<BN>(Bs[cur ^ 1], rb);
    }
    __syncthreads();
  }

  // epilogue
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

template <int BM, int BN, bool SYRK>
static se_status launch_f32(const float* A, int lda, const float* B, int ldb, float* C, int ldc,
                            int Mr, int Nc, int Nst, int P, bool vec, hipStream_t s) {
  int ntiles, tiles_n;
  if (SYRK) {
    const int nb = (Mr + BM - 1) / BM;
    ntiles = nb * (nb + 1) / 2;
    tiles_n = nb;
  } else {
    tiles_n = (Nst + BN - 1) / BN;
    ntiles = ((Mr + BM - 1) / BM) * tiles_n;
  }
  if (ntiles <= 0) return SE_OK;
  if (vec)
    hipLaunchKernelGGL((k_gemm_nt_f32<BM, BN, true, SYRK>), dim3(ntiles), dim3(256), 0, s, A, lda,
                       B, ldb, C, ldc, Mr, Nc, Nst, P, tiles_n, ntiles);
  else
    hipLaunchKernelGGL((k_gemm_nt_f32<BM, BN, false, SYRK>), dim3(ntiles), dim3(256), 0, s, A,
                       lda, B, ldb, C, ldc, Mr, Nc, Nst, P, tiles_n, ntiles);
  return check_launch("gemm_nt_f32");
}

se_status gemm_nt_f32(const float* A, int lda, const float* B, int ldb, float* C, int ldc, int Mr,
                      int Nc, int Nst, int P, bool syrk, int tile, hipStream_t s) {
  const bool vec = (lda % 4 == 0) && (ldb % 4 == 0) &&
                   ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) % 16 == 0);
  if (tile <= 0) {
    // enough tiles to give every compute unit work with the larger tile?
    long long big;
    if (syrk) {
      const long long nb = (Mr + 127) / 128;
      big = nb * (nb + 1) / 2;
    } else {
      big = (long long)((Mr + 127) / 128) * ((Nst + 127) / 128);
    }
    tile = big >= 512 ? 128 : 64;
  }
  if (tile == 128)
    return syrk ? launch_f32<128, 128, true>(A, lda, B, ldb, C, ldc, Mr, Nc, Nst, P, vec, s)
                : launch_f32<128, 128, false>(A, lda, B, ldb, C, ldc, Mr, Nc, Nst, P, vec, s);
  return syrk ? launch_f32<64, 64, true>(A, lda, B, ldb, C, ldc, Mr, Nc, Nst, P, vec, s)
              : launch_f32<64, 64, false>(A, lda, B, ldb, C, ldc, Mr, Nc, Nst, P, vec, s);
}

}  // namespace sefase
