// Matrix-core GEMM for the two dense contractions of the method:
//   * table generation (Algorithm 2, eq. 16): G = Y Y^T over the area pixels,
//     lower-triangle tiles only, each stored twice (G is symmetric, so only
//     (|D|^2 + |D|)/2 scalar products are needed);
//   * initial projections (eq. 12) of a batch of blocks: R = X Y^T, computed
//     as Y X^T and stored transposed so every lane writes float4 rows.
// S[r][c] = sum_p A[r][p] B[c][p]; both operands row-major with the
// contraction index p contiguous ("NT").
//
// FP32 path: v_mfma_f32_16x16x4_f32.  A 256-thread workgroup (4 waves, 2x2)
// owns a BM x BN tile of S; each wave a (BM/2) x (BN/2) sub-tile made of
// 16x16 MFMA tiles.  Operand tiles of BK = 32 contraction steps are staged
// through LDS, double-buffered (one barrier per step).  A lane feeds the MFMA
// a float4 along p: four consecutive MFMA rounds consume its x, y, z, w
// components, which only permutes the order of the contraction, identically
// for A and B.  Rows beyond the valid range are read clamped to the last
// valid row (they only feed outputs that are never stored), so the main loop
// has no per-lane branches; only the last contraction tile checks p < P.
//
// MFMA 16x16x4 f32 operand/result mapping (lane l, 0..63):
//   A[m][k]: m = l % 16, k = l / 16        B[k][n]: n = l % 16, k = l / 16
//   D[m][n] (4 floats e = 0..3): m = 4 (l / 16) + e, n = l % 16
#include <algorithm>

#include "se_internal.h"

namespace sefase {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kBK = 32;
constexpr int kPad = 4;

enum StoreMode { kStoreRowMajor = 0, kStoreTransposed = 1, kStoreSymmetric = 2 };

// Map the linear workgroup id to a tile so that the 8 XCDs (which receive
// workgroups round-robin) each work on a contiguous range of tiles.
__device__ inline int xcd_remap(int id, int ntiles) {
  if ((ntiles & 7) != 0) return id;
  const int per = ntiles >> 3;
  return (id & 7) * per + (id >> 3);
}

template <int ROWS, bool VEC, bool KTAIL>
__device__ inline void load_tile(const float* __restrict__ src, int ld, int row0, int nrows,
                                 int k0, int P, float4 (&reg)[ROWS * kBK / 4 / 256]) {
  constexpr int NQ = ROWS * kBK / 4 / 256;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int idx = threadIdx.x + 256 * q;
    const int r = idx / (kBK / 4);
    const int c = (idx % (kBK / 4)) * 4;
    int gr = row0 + r;
    gr = gr < nrows ? gr : nrows - 1;
    const int gk = k0 + c;
    const float* p = src + (size_t)gr * ld + gk;
    float4 v;
    if (!KTAIL) {
      if (VEC) {
        v = *reinterpret_cast<const float4*>(p);
      } else {
        v = make_float4(p[0], p[1], p[2], p[3]);
      }
    } else {
      v.x = gk + 0 < P ? p[0] : 0.0f;
      v.y = gk + 1 < P ? p[1] : 0.0f;
      v.z = gk + 2 < P ? p[2] : 0.0f;
      v.w = gk + 3 < P ? p[3] : 0.0f;
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

// S = A B^T for a BM x BN tile.
//   Ma, Nb : valid rows of A and of B
//   Mst, Nst : extent of S that is stored; S entries with r >= Ma or c >= Nb
//              inside it are stored as 0
//   MODE kStoreRowMajor   : C[r][c] = S[r][c]
//        kStoreTransposed : C[c][r] = S[r][c]
//        kStoreSymmetric  : A == B; only tiles with bj <= bi run; C[r][c] and
//                           C[c][r] = S[r][c] for r >= c
template <int BM, int BN, bool VEC, int MODE>
__global__ __launch_bounds__(256) void k_gemm_nt_f32(const float* __restrict__ A, int lda,
                                                     const float* __restrict__ B, int ldb,
                                                     float* __restrict__ C, int ldc, int Ma, int Nb,
                                                     int Mst, int Nst, int P, int tiles_n,
                                                     int ntiles, int kchunk, size_t cstride,
                                                     const int32_t* __restrict__ nb_dev,
                                                     const int32_t* __restrict__ cmap) {
  constexpr int SI = BM / 32, SJ = BN / 32;   // 16x16 MFMA tiles per wave
  // split contraction: slice z covers p in [z kchunk, (z + 1) kchunk) and
  // writes its partial S to C + z cstride
  {
    const int kz = blockIdx.y;
    A += (size_t)kz * kchunk;
    B += (size_t)kz * kchunk;
    C += (size_t)kz * cstride;
    P = min(kchunk, P - kz * kchunk);
  }
  __shared__ __attribute__((aligned(16))) float As[2][BM][kBK + kPad];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN][kBK + kPad];

  const int tile = xcd_remap(blockIdx.x, ntiles);
  int bi, bj;
  if (MODE == kStoreSymmetric) {
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
  // rows formed on demand (transposed store): the valid blocks are counted
  // on the device, and tiles past the count have nothing to do
  if (MODE == kStoreTransposed && nb_dev) {
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

  float4 ra[BM * kBK / 4 / 256], rb[BN * kBK / 4 / 256];
  const int nk = (P + kBK - 1) / kBK;
  const bool ragged = (P % kBK) != 0;
  if (nk == 1 && ragged) {
    load_tile<BM, VEC, true>(A, lda, m0, Ma, 0, P, ra);
    load_tile<BN, VEC, true>(B, ldb, n0, Nb, 0, P, rb);
  } else {
    load_tile<BM, VEC, false>(A, lda, m0, Ma, 0, P, ra);
    load_tile<BN, VEC, false>(B, ldb, n0, Nb, 0, P, rb);
  }
  store_tile<BM>(As[0], ra);
  store_tile<BN>(Bs[0], rb);
  __syncthreads();

  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      const int k1 = (kt + 1) * kBK;
      if (kt + 2 == nk && ragged) {
        load_tile<BM, VEC, true>(A, lda, m0, Ma, k1, P, ra);
        load_tile<BN, VEC, true>(B, ldb, n0, Nb, k1, P, rb);
      } else {
        load_tile<BM, VEC, false>(A, lda, m0, Ma, k1, P, ra);
        load_tile<BN, VEC, false>(B, ldb, n0, Nb, k1, P, rb);
      }
    }
    // this stage's 32 products go to fresh accumulators and are then added to
    // the running sums (blocked summation keeps the FP32 rounding error
    // growing with the number of stages instead of the number of pixels)
    floatx4 part[SI][SJ];
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
        for (int j = 0; j < SJ; ++j)
          part[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(
              fa[i].x, fb[j].x, kk == 0 ? floatx4{0.f, 0.f, 0.f, 0.f} : part[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < SI; ++i)
#pragma unroll
        for (int j = 0; j < SJ; ++j)
          part[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].y, fb[j].y, part[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < SI; ++i)
#pragma unroll
        for (int j = 0; j < SJ; ++j)
          part[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].z, fb[j].z, part[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < SI; ++i)
#pragma unroll
        for (int j = 0; j < SJ; ++j)
          part[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].w, fb[j].w, part[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < SI; ++i)
#pragma unroll
      for (int j = 0; j < SJ; ++j) acc[i][j] += part[i][j];
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
    for (int j = 0; j < SJ; ++j) {
      const int r0 = m0 + wr * (BM / 2) + 16 * i + 4 * lq;   // rows r0 .. r0+3
      const int c = n0 + wc * (BN / 2) + 16 * j + lr;
      if (MODE == kStoreTransposed) {
        if (c < Nst && c < Nb) {
          float4 v;
          v.x = r0 + 0 < Ma ? acc[i][j][0] : 0.0f;
          v.y = r0 + 1 < Ma ? acc[i][j][1] : 0.0f;
          v.z = r0 + 2 < Ma ? acc[i][j][2] : 0.0f;
          v.w = r0 + 3 < Ma ? acc[i][j][3] : 0.0f;
          float* dst = C + (size_t)(cmap ? cmap[c] : c) * ldc + r0;
          if (VEC && r0 + 3 < Mst) {
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
          if (MODE == kStoreSymmetric) {
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
        if (MODE == kStoreSymmetric && bi != bj && c < Nb) {
          // off-diagonal tile: rows r0..r0+3 of column c are one row segment of
          // the mirrored tile
          float* dst = C + (size_t)c * ldc + r0;
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

// C[c][r] = sum_z W[z][c][r] for c < rows, r < cols (the partial products of
// a split contraction, summed in a fixed order)
template <bool VEC>
__global__ __launch_bounds__(256) void k_splitk_sum(const float* __restrict__ W, int ldw,
                                                    size_t wstride, int S,
                                                    float* __restrict__ C, int ldc, int rows,
                                                    int cols, const int32_t* __restrict__ nb_dev,
                                                    const int32_t* __restrict__ cmap) {
  const int c = blockIdx.y;
  const int r = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
  if (nb_dev) rows = min(rows, *nb_dev);
  if (c >= rows || r >= cols) return;
  const float* w = W + (size_t)c * ldw + r;
  float* dst = C + (size_t)(cmap ? cmap[c] : c) * ldc + r;
  if (VEC && r + 3 < cols) {
    float4 v = *reinterpret_cast<const float4*>(w);
    for (int z = 1; z < S; ++z) {
      const float4 u = *reinterpret_cast<const float4*>(w + (size_t)z * wstride);
      v.x += u.x;
      v.y += u.y;
      v.z += u.z;
      v.w += u.w;
    }
    *reinterpret_cast<float4*>(dst) = v;
  } else {
    for (int e = 0; e < 4 && r + e < cols; ++e) {
      float v = w[e];
      for (int z = 1; z < S; ++z) v += w[(size_t)z * wstride + e];
      dst[e] = v;
    }
  }
}

// Slices of a split contraction for a transposed product of 64 x 64 tiles:
// enough workgroups to give every compute unit several, each slice at least
// 8 stages of kBK.  Returns 1 (no split) when the tiles alone fill the chip.
static int splitk_slices(int Mst, int Nst, int P) {
  const long long tiles = (long long)((Mst + 63) / 64) * ((Nst + 63) / 64);
  const int nk = (P + kBK - 1) / kBK;
  if (tiles <= 0 || tiles >= 512) return 1;
  int S = (int)((768 + tiles - 1) / tiles);
  S = std::min(S, std::min(8, nk / 8));
  if (S < 2) return 1;
  const int per = (nk + S - 1) / S;    // stages per slice
  return (nk + per - 1) / per;
}

static inline int ldw_of(int Mst) { return (Mst + 3) & ~3; }

// Slices of a contraction over P samples fixed by P alone (each at least 16
// stages of kBK, at most 8): a product split this way sums every entry in an
// order that does not depend on how many blocks share the product.
static int shape_slices(int P) {
  const int nk = (P + kBK - 1) / kBK;
  return std::max(1, std::min(8, nk / 16));
}

size_t gemm_invariant_floats(int Mst, int Nst, int P) {
  const int S = shape_slices(P);
  return S > 1 ? (size_t)S * Nst * ldw_of(Mst) : 0;
}

size_t gemm_splitk_floats(int Mst, int Nst_max, int P) {
  // the largest S * Nst * ldw over every block count up to Nst_max
  size_t best = 0;
  for (int tn = 1; 64 * (tn - 1) < Nst_max; ++tn) {
    const int Nst = std::min(64 * tn, Nst_max);
    const int S = splitk_slices(Mst, Nst, P);
    if (S > 1) best = std::max(best, (size_t)S * Nst * ldw_of(Mst));
  }
  return best;
}

template <int BM, int BN, int MODE>
static se_status launch_f32(const float* A, int lda, const float* B, int ldb, float* C, int ldc,
                            int Ma, int Nb, int Mst, int Nst, int P, bool vec, hipStream_t s,
                            int S = 1, int kchunk = 0, size_t cstride = 0,
                            const int32_t* nb_dev = nullptr, const int32_t* cmap = nullptr) {
  int ntiles, tiles_n;
  if (MODE == kStoreSymmetric) {
    const int nb = (Ma + BM - 1) / BM;
    ntiles = nb * (nb + 1) / 2;
    tiles_n = nb;
  } else {
    tiles_n = (Nst + BN - 1) / BN;
    ntiles = ((Mst + BM - 1) / BM) * tiles_n;
  }
  if (ntiles <= 0 || P <= 0) return SE_OK;
  if (S <= 1) kchunk = P;
  if (vec)
    hipLaunchKernelGGL((k_gemm_nt_f32<BM, BN, true, MODE>), dim3(ntiles, S), dim3(256), 0, s, A,
                       lda, B, ldb, C, ldc, Ma, Nb, Mst, Nst, P, tiles_n, ntiles, kchunk, cstride, nb_dev,
                       cmap);
  else
    hipLaunchKernelGGL((k_gemm_nt_f32<BM, BN, false, MODE>), dim3(ntiles, S), dim3(256), 0, s, A,
                       lda, B, ldb, C, ldc, Ma, Nb, Mst, Nst, P, tiles_n, ntiles, kchunk, cstride, nb_dev,
                       cmap);
  return check_launch("gemm_nt_f32");
}

// Rows formed on demand: the valid block count read on the device (nb_dev)
// and each output row placed at its own destination row (cmap).
struct RowMap {
  const int32_t* nb_dev = nullptr;
  const int32_t* cmap = nullptr;
};

// Tiles of BM x BN with the contraction split over slices (partial products
// in ws, summed in slice order) when `split` asks for it and ws holds them,
// else unsplit.
template <int BM, int BN, int MODE>
static se_status launch_tiles(const float* A, int lda, const float* B, int ldb, float* C, int ldc,
                              int Ma, int Nb, int Mst, int Nst, int P, bool vec, hipStream_t s,
                              float* ws, size_t ws_floats, int split, const RowMap& map) {
  if (MODE == kStoreTransposed && ws && vec && Mst > 0 && Nst > 0 && split != 0 && split != 1) {
    // few tiles: split the contraction over slices that write partial
    // products to the workspace, then sum them in slice order
    const int nk = (P + kBK - 1) / kBK;
    const int S = split < 0 ? splitk_slices(Mst, Nst, P) : std::min(split, nk);
    const int ldw = ldw_of(Mst);
    const size_t wstride = (size_t)Nst * ldw;
    if (S > 1 && (size_t)S * wstride <= ws_floats &&
        reinterpret_cast<uintptr_t>(ws) % 16 == 0) {
      const int kchunk = ((nk + S - 1) / S) * kBK;
      const int Sr = (nk + kchunk / kBK - 1) / (kchunk / kBK);   // slices that hold stages
      se_status st = launch_f32<BM, BN, MODE>(A, lda, B, ldb, ws, ldw, Ma, Nb, Mst, Nst, P, true,
                                              s, Sr, kchunk, wstride, map.nb_dev, nullptr);
      if (st) return st;
      const dim3 grid((unsigned)((Mst + 1023) / 1024), (unsigned)Nst);
      hipLaunchKernelGGL(k_splitk_sum<true>, grid, dim3(256), 0, s, ws, ldw, wstride, Sr, C, ldc,
                         Nst, Mst, map.nb_dev, map.cmap);
      return check_launch("splitk_sum");
    }
  }
  return launch_f32<BM, BN, MODE>(A, lda, B, ldb, C, ldc, Ma, Nb, Mst, Nst, P, vec, s, 1, 0, 0,
                                  map.nb_dev, map.cmap);
}

// tile: 0 = automatic, 64, 128, or kTile128x64 (128 atoms x 64 blocks, for
// products with few blocks).  split: -1 = automatic (slices when the
// tiles alone leave the chip idle and the workspace holds the partials),
// 0 or 1 = none, S = S slices (64-wide tiles only; falls back to none when
// the workspace is too small), kSplitShape = the slices of shape_slices(P)
// whatever the number of blocks (an error when the workspace cannot hold
// them: the caller relies on the fixed order).
template <int MODE>
static se_status dispatch_f32(const float* A, int lda, const float* B, int ldb, float* C, int ldc,
                              int Ma, int Nb, int Mst, int Nst, int P, int tile, hipStream_t s,
                              float* ws = nullptr, size_t ws_floats = 0, int split = -1,
                              RowMap map = RowMap{}) {
  const bool vec = (lda % 4 == 0) && (ldb % 4 == 0) && (ldc % 4 == 0) &&
                   ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) |
                     reinterpret_cast<uintptr_t>(C)) % 16 == 0);
  if (tile <= 0) {
    // the larger tile only when it still gives every compute unit work
    long long big;
    if (MODE == kStoreSymmetric) {
      const long long nb = (Ma + 127) / 128;
      big = nb * (nb + 1) / 2;
    } else {
      big = (long long)((Mst + 127) / 128) * ((Nst + 127) / 128);
    }
    tile = big >= 512 ? 128 : 64;
  }
  if (split == kSplitShape) {
    split = shape_slices(P);
    if (split > 1) {
      const size_t need = (size_t)split * Nst * ldw_of(Mst);
      if (MODE != kStoreTransposed || !vec || !ws || ws_floats < need ||
          reinterpret_cast<uintptr_t>(ws) % 16 != 0)
        return fail(SE_ENOMEM, "the fixed split of an invariant product needs %zu floats of "
                               "workspace and aligned operands", need);
      tile = 64;
    }
  }
  if (tile == 128)
    return launch_f32<128, 128, MODE>(A, lda, B, ldb, C, ldc, Ma, Nb, Mst, Nst, P, vec, s, 1, 0,
                                      0, map.nb_dev, map.cmap);
  if (MODE == kStoreTransposed && tile == kTile128x64)
    return launch_tiles<128, 64, MODE>(A, lda, B, ldb, C, ldc, Ma, Nb, Mst, Nst, P, vec, s, ws,
                                       ws_floats, split, map);
  return launch_tiles<64, 64, MODE>(A, lda, B, ldb, C, ldc, Ma, Nb, Mst, Nst, P, vec, s, ws,
                                    ws_floats, split, map);
}

se_status gemm_syrk_f32(const float* Y, int ldy, int K, int P, float* G, int ldg, hipStream_t s) {
  return dispatch_f32<kStoreSymmetric>(Y, ldy, Y, ldy, G, ldg, K, K, K, K, P, 0, s);
}

se_status gemm_project_f32(const float* Y, int ldy, int K, const float* X, int ldx, int n_blk,
                           int P, float* R, int ldr, int tile, hipStream_t s, bool pad, float* ws,
                           size_t ws_floats, int split) {
  // S = Y X^T (atoms x blocks), stored transposed: R[b][k]; atoms K .. ldr-1 as 0
  return dispatch_f32<kStoreTransposed>(Y, ldy, X, ldx, R, ldr, K, n_blk, pad ? ldr : K, n_blk, P,
                                        tile, s, ws, ws_floats, split);
}

size_t gemm_rows_splitk_floats(int K, int n_max, int P, int split) {
  if (split == 0 || split == 1) return 0;
  if (split == kSplitShape) return gemm_invariant_floats(K, n_max, P);
  if (split < 0) return gemm_splitk_floats(K, n_max, P);
  return (size_t)split * n_max * ldw_of(K);
}

se_status gemm_rows_f32(const float* Y, int ldy, int K, const float* X, int ldx, int n_max,
                        const int32_t* n_dev, const int32_t* cmap, int P, float* rows, int ldr,
                        int tile, int split, hipStream_t s, float* ws, size_t ws_floats) {
  RowMap map;
  map.nb_dev = n_dev;
  map.cmap = cmap;
  return dispatch_f32<kStoreTransposed>(Y, ldy, X, ldx, rows, ldr, K, n_max, K, n_max, P, tile, s,
                                        ws, ws_floats, split, map);
}

}  // namespace sefase
