// Transform parts of a dictionary (Section VI): when a range of atoms holds
// the separable 2-D atoms of a discrete transform, the weighted scalar
// products of a vector v with those atoms are the transform coefficients of
// the weighted vector w v (eq. 21-23).  For an M x N area the 2-D transform
// is A X B^T with the 1-D transform matrices A (M x M) and B (N x N): two
// small matrix products per block, M N (M + N) multiply-adds instead of the
// K M N of a product with the dictionary.
//
// 1-D matrices (built in LDS by every workgroup, from the definitions):
//   DCT-II:  A[k][m] = alpha_k cos(pi (2m+1) k / 2M), alpha_0 = 1/sqrt(M),
//            alpha_k = sqrt(2/M); row M/2 takes its exact values +-1/sqrt(M)
//   WHT:     A[k][m] = (-1)^popcount(k & m) / sqrt(M), natural order
#include "se_internal.h"

namespace sefase {

constexpr int kTxThreads = 256;

// cos(pi j / 2n) for j < 4n, in FP64 (the DCT entries are rounded once, from
// FP64, like the atoms they must reproduce)
__device__ void build_cos_table(int n, double* ct) {
  for (int j = threadIdx.x; j < 4 * n; j += blockDim.x) ct[j] = cospi((double)j / (double)(2 * n));
}

// entry (k, m) of the n-point 1-D transform of `kind`; ct from build_cos_table
__device__ inline float basis_1d(int kind, int n, int k, int m, const double* ct) {
  const double inv = 1.0 / sqrt((double)n);
  if (kind == SE_PART_WHT2) return (float)((__popc(k & m) & 1) ? -inv : inv);
  if (k == 0) return (float)inv;
  if (2 * k == n) return (float)(((m & 3) == 0 || (m & 3) == 3) ? inv : -inv);
  return (float)(sqrt(2.0 / (double)n) * ct[((2 * m + 1) * k) % (4 * n)]);
}

// ---------------------------------------------------------------------------
// Verification of a declared part against phi: every atom k of the part,
// every pixel (m, n), |phi[first + k][m N + n] - A[k1][m] B[k2][n]| <= tol.
__global__ __launch_bounds__(kTxThreads) void k_check_part(const float* __restrict__ phi, int M,
                                                          int N, int kind, int first, float tol,
                                                          int* __restrict__ flag) {
  extern __shared__ double smd[];
  double* ctM = smd;              // 4M
  double* ctN = ctM + 4 * M;      // 4N
  float* A = reinterpret_cast<float*>(ctN + 4 * N);   // M x M
  float* Bm = A + M * M;                               // N x N
  build_cos_table(M, ctM);
  build_cos_table(N, ctN);
  __syncthreads();
  for (int i = threadIdx.x; i < M * M; i += blockDim.x) A[i] = basis_1d(kind, M, i / M, i % M, ctM);
  for (int i = threadIdx.x; i < N * N; i += blockDim.x) Bm[i] = basis_1d(kind, N, i / N, i % N, ctN);
  __syncthreads();
  const int P = M * N;
  int bad = 0;
  for (int k = blockIdx.x; k < P; k += gridDim.x) {
    const int k1 = k / N, k2 = k - k1 * N;
    const float* row = phi + (size_t)(first + k) * P;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
      const int m = p / N, n = p - m * N;
      if (fabsf(row[p] - A[k1 * M + m] * Bm[k2 * N + n]) > tol) bad = 1;
    }
  }
  if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Shared layout of the separable transform in LDS (floats):
//   A  : Mp x lda   rows k1 of the vertical transform (rows >= M zero)
//   Bt : N  x Np    Bt[n][k2] = B[k2][n] (columns >= N zero)
//   X  : Mp x ldx   the weighted vector as an M x N image (rows >= M zero)
//   Y1 : Mp x Np    X B^T
// Mp, Np = M, N rounded up to even; lda = M + 1, ldx = N + 1 (odd strides,
// so the rows a wave reads at once fall in different banks).
struct TxLayout {
  int M, N, Mp, Np, lda, ldx;
  int oA, oBt, oX, oY1, nfloat;   // offsets per part (A, Bt) and shared (X, Y1)
  __host__ __device__ TxLayout(int M_, int N_, int parts) : M(M_), N(N_) {
    Mp = (M + 1) & ~1;
    Np = (N + 1) & ~1;
    lda = M + 1;
    ldx = N + 1;
    const int szA = (Mp * lda + 3) & ~3, szB = (N * Np + 3) & ~3;
    oA = 0;
    oBt = parts * szA;
    oX = oBt + parts * szB;
    oY1 = oX + ((Mp * ldx + 3) & ~3);
    nfloat = oY1 + Mp * Np;
  }
  __host__ __device__ int szA() const { return (Mp * lda + 3) & ~3; }
  __host__ __device__ int szB() const { return (N * Np + 3) & ~3; }
  // bytes: the floats, then the two FP64 cosine tables
  __host__ __device__ size_t bytes() const {
    return (((size_t)nfloat * 4 + 7) & ~(size_t)7) + (size_t)4 * (M + N) * 8;
  }
};

// Build A and Bt of one part (all threads; ends synchronised).
__device__ void build_part(const TxLayout& L, int kind, float* A, float* Bt, double* ctM,
                           double* ctN) {
  build_cos_table(L.M, ctM);
  build_cos_table(L.N, ctN);
  __syncthreads();
  for (int i = threadIdx.x; i < L.Mp * L.lda; i += blockDim.x) {
    const int k = i / L.lda, m = i - k * L.lda;
    A[i] = (k < L.M && m < L.M) ? basis_1d(kind, L.M, k, m, ctM) : 0.0f;
  }
  for (int i = threadIdx.x; i < L.N * L.Np; i += blockDim.x) {
    const int n = i / L.Np, k = i - n * L.Np;
    Bt[i] = k < L.N ? basis_1d(kind, L.N, k, n, ctN) : 0.0f;
  }
  __syncthreads();
}

// Z = A X B^T for X, Y1 in LDS; calls out(k1, k2, z) for every k1 < M,
// k2 < N.  Each thread computes 2 x 2 outputs per pass.  Starts and ends
// with the caller's X complete; ends synchronised.
template <typename Out>
__device__ void separable_2d(const TxLayout& L, const float* A, const float* Bt, const float* X,
                             float* Y1, Out out) {
  const int hp = L.Np >> 1, pairs = (L.Mp >> 1) * hp;
  for (int q = threadIdx.x; q < pairs; q += blockDim.x) {
    const int mi = q / hp, m = 2 * mi, k2 = 2 * (q - mi * hp);
    const float* x0 = X + m * L.ldx;
    const float* x1 = x0 + L.ldx;
    const float* bt = Bt + k2;
    float a00 = 0.f, a01 = 0.f, a10 = 0.f, a11 = 0.f;
    for (int n = 0; n < L.N; ++n) {
      const float2 b = *reinterpret_cast<const float2*>(bt + n * L.Np);
      const float u = x0[n], v = x1[n];
      a00 = fmaf(u, b.x, a00);
      a01 = fmaf(u, b.y, a01);
      a10 = fmaf(v, b.x, a10);
      a11 = fmaf(v, b.y, a11);
    }
    *reinterpret_cast<float2*>(Y1 + m * L.Np + k2) = make_float2(a00, a01);
    *reinterpret_cast<float2*>(Y1 + (m + 1) * L.Np + k2) = make_float2(a10, a11);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < pairs; q += blockDim.x) {
    const int mi = q / hp, k1 = 2 * mi, k2 = 2 * (q - mi * hp);
    const float* r0 = A + k1 * L.lda;
    const float* r1 = r0 + L.lda;
    const float* y = Y1 + k2;
    float z00 = 0.f, z01 = 0.f, z10 = 0.f, z11 = 0.f;
    for (int m = 0; m < L.M; ++m) {
      const float2 c = *reinterpret_cast<const float2*>(y + m * L.Np);
      const float u = r0[m], v = r1[m];
      z00 = fmaf(u, c.x, z00);
      z01 = fmaf(u, c.y, z01);
      z10 = fmaf(v, c.x, z10);
      z11 = fmaf(v, c.y, z11);
    }
    if (k1 < L.M) {
      out(k1, k2, z00);
      if (k2 + 1 < L.N) out(k1, k2 + 1, z01);
    }
    if (k1 + 1 < L.M) {
      out(k1 + 1, k2, z10);
      if (k2 + 1 < L.N) out(k1 + 1, k2 + 1, z11);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Initial projections of the transform parts (eq. 12 via eq. 22), fused with
// the gather: x = w s over the block's area (0 outside the image), then per
// part R[b][first + k1 N + k2] = D_k (A x B^T)[k1][k2].  Columns K .. ldR-1
// of R are written as 0.  Workgroups loop over blocks, so the 1-D matrices
// are built once per workgroup.
struct TxArgs {
  const uint8_t* images;
  int H, W;
  const DevBlock* blk;
  int n_blk;
  int K;
  const float* sqrtw;
  const float* D;
  int n_parts;
  int kind[2], first[2];
  float* R;
  int ldR;
};

__global__ __launch_bounds__(kTxThreads) void k_project_tx(TxArgs a, TxLayout L) {
  extern __shared__ double smd[];
  float* sm = reinterpret_cast<float*>(smd);
  double* ctM = smd + (((size_t)L.nfloat * 4 + 7) >> 3);
  double* ctN = ctM + 4 * L.M;
  float* X = sm + L.oX;
  float* Y1 = sm + L.oY1;
  for (int q = 0; q < a.n_parts; ++q)
    build_part(L, a.kind[q], sm + L.oA + q * L.szA(), sm + L.oBt + q * L.szB(), ctM, ctN);
  const int M = L.M, N = L.N;
  for (int b = blockIdx.x; b < a.n_blk; b += gridDim.x) {
    const DevBlock d = a.blk[b];
    const uint8_t* img = a.images + (size_t)d.img * a.H * a.W;
    for (int p = threadIdx.x; p < L.Mp * L.ldx; p += blockDim.x) {
      const int m = p / L.ldx, n = p - m * L.ldx;
      const int y = d.y0 + m, x = d.x0 + n;
      float v = 0.0f;
      if (m < M && n < N && y >= 0 && y < a.H && x >= 0 && x < a.W) {
        const float sw = a.sqrtw[m * N + n];
        v = (sw * sw) * (float)img[(size_t)y * a.W + x];
      }
      X[p] = v;
    }
    float* Rb = a.R + (size_t)b * a.ldR;
    for (int k = a.K + threadIdx.x; k < a.ldR; k += blockDim.x) Rb[k] = 0.0f;
    __syncthreads();
    for (int q = 0; q < a.n_parts; ++q) {
      const int f = a.first[q];
      const float* Dq = a.D + f;
      float* Rq = Rb + f;
      separable_2d(L, sm + L.oA + q * L.szA(), sm + L.oBt + q * L.szB(), X, Y1,
                   [&](int k1, int k2, float z) {
                     const int k = k1 * N + k2;
                     Rq[k] = Dq[k] * z;
                   });
    }
  }
}

static int tx_grid(size_t lds, int n_blk) {
  int per_cu = (int)((160 * 1024) / (lds ? lds : 1));
  per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
  const int cap = 256 * per_cu;
  return n_blk < cap ? n_blk : cap;
}

se_status check_part(const float* phi, int M, int N, int kind, int first, int* dflag,
                     hipStream_t s) {
  const size_t lds = (size_t)4 * (M + N) * 8 + (size_t)(M * M + N * N) * 4;
  const int P = M * N;
  const int grid = P < 2048 ? P : 2048;
  hipLaunchKernelGGL(k_check_part, dim3(grid), dim3(kTxThreads), lds, s, phi, M, N, kind, first,
                     2e-6f, dflag);
  return check_launch("check_part");
}

size_t tx_lds_bytes(int M, int N, int n_parts) { return TxLayout(M, N, n_parts).bytes(); }

se_status project_tx(const se_tables* t, const uint8_t* images, int H, int W, const DevBlock* blk,
                     int n_blk, float* R, int ldR, hipStream_t s) {
  TxArgs a;
  a.images = images;
  a.H = H;
  a.W = W;
  a.blk = blk;
  a.n_blk = n_blk;
  a.K = t->K;
  a.sqrtw = t->sqrtw;
  a.D = t->D;
  a.n_parts = t->n_parts;
  for (int q = 0; q < 2; ++q) {
    a.kind[q] = q < t->n_parts ? t->parts[q].kind : 0;
    a.first[q] = q < t->n_parts ? t->parts[q].first : 0;
  }
  a.R = R;
  a.ldR = ldR;
  const TxLayout L(t->M, t->N, t->n_parts);
  const size_t lds = L.bytes();
  if (lds > 160 * 1024) return fail(SE_EINVAL, "transform of a %dx%d area exceeds LDS", t->M, t->N);
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(&k_project_tx),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return fail(SE_EHIP, "project_tx: %zu bytes of LDS refused", lds);
  hipLaunchKernelGGL(k_project_tx, dim3(tx_grid(lds, n_blk)), dim3(kTxThreads), lds, s, a, L);
  return check_launch("project_tx");
}

}  // namespace sefase
