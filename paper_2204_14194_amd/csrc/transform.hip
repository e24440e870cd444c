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
// An area of T > 1 frames is transformed as the T M x N matrix of its
// frames stacked row-wise (sample (tau, m, n) at row tau M + m): the 3-D
// separable transform is then the 2-D one with the vertical matrix the
// Kronecker product A_T (x) A_M, entry (kt M + k1, tau M + m) =
// A_T[kt][tau] A_M[k1][m] (formed in FP64, rounded once).
#include <atomic>

#include "se_internal.h"
#include "tx_device.h"

namespace sefase {

constexpr int kTxThreads = 256;

// cos(pi j / 2n) for j < 4n, in FP64 (the DCT entries are rounded once, from
// FP64, like the atoms they must reproduce)
__device__ void build_cos_table(int n, double* ct) {
  for (int j = threadIdx.x; j < 4 * n; j += blockDim.x) ct[j] = cospi((double)j / (double)(2 * n));
}

// Entry (k, m) of the n-point 1-D transform of `kind`, in FP64.  ct from
// build_cos_table; inv = 1/sqrt(n), a2 = sqrt(2/n) (FP64).
__device__ inline double basis_1d_d(int kind, int n, int k, int m, const double* ct, double inv,
                                    double a2) {
  if (kind == SE_PART_WHT2) return (__popc(k & m) & 1) ? -inv : inv;
  // the conjugate DFT matrix: phase index (k m) mod n, sin(x) = cos(x + 3 pi / 2)
  if (kind == kKindDftRe) return inv * ct[4 * ((k * m) % n)];
  if (kind == kKindDftIm) return -inv * ct[(4 * ((k * m) % n) + 3 * n) % (4 * n)];
  if (k == 0) return inv;
  if (2 * k == n) return ((m & 3) == 0 || (m & 3) == 3) ? inv : -inv;
  return a2 * ct[((2 * m + 1) * k) % (4 * n)];
}

__device__ inline float basis_1d(int kind, int n, int k, int m, const double* ct, double inv,
                                 double a2) {
  return (float)basis_1d_d(kind, n, k, m, ct, inv, a2);
}

// The vertical transform of a stack of T frames of Ms rows (M = T Ms rows
// in all): entry (k, m); the 1-D matrix itself when T = 1.  ctT, ctS:
// cosine tables of T and Ms points.
struct VertBasis {
  int T, Ms;
  const double* ctT;
  const double* ctS;
  __device__ float operator()(int kind, int k, int m) const {
    const double iS = 1.0 / sqrt((double)Ms), aS = sqrt(2.0 / (double)Ms);
    if (T == 1) return basis_1d(kind, Ms, k, m, ctS, iS, aS);
    const double iT = 1.0 / sqrt((double)T), aT = sqrt(2.0 / (double)T);
    return (float)(basis_1d_d(kind, T, k / Ms, m / Ms, ctT, iT, aT) *
                   basis_1d_d(kind, Ms, k % Ms, m % Ms, ctS, iS, aS));
  }
};

// ---------------------------------------------------------------------------
// Verification of a declared part against phi: every atom k of the part,
// every pixel (m, n), |phi[first + k][m N + n] - A[k1][m] B[k2][n]| <= tol
// (M = T Ms rows: T frames of Ms rows, A the vertical transform above).
__global__ __launch_bounds__(kTxThreads) void k_check_part(const float* __restrict__ phi, int T,
                                                          int Ms, int N, int kind, int first,
                                                          float tol, int* __restrict__ flag) {
  extern __shared__ double smd[];
  const int M = T * Ms;
  double* ctS = smd;              // 4 Ms
  double* ctN = ctS + 4 * Ms;     // 4N
  double* ctT = ctN + 4 * N;      // 4T
  float* A = reinterpret_cast<float*>(ctT + 4 * T);   // M x M
  float* Bm = A + M * M;                               // N x N
  build_cos_table(Ms, ctS);
  build_cos_table(N, ctN);
  build_cos_table(T, ctT);
  __syncthreads();
  const double iN = 1.0 / sqrt((double)N), aN = sqrt(2.0 / (double)N);
  const VertBasis vb{T, Ms, ctT, ctS};
  for (int i = threadIdx.x; i < M * M; i += blockDim.x) A[i] = vb(kind, i / M, i % M);
  for (int i = threadIdx.x; i < N * N; i += blockDim.x)
    Bm[i] = basis_1d(kind, N, i / N, i % N, ctN, iN, aN);
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

// A complex DFT part: every atom k1 N + k2 of the part against its exact
// value exp(j 2 pi q / M N) / sqrt(M N), q = (k1 m N + k2 n M) mod M N, in
// both the real (phi) and the imaginary parts (phi_im).
__global__ __launch_bounds__(kTxThreads) void k_check_dft(const float* __restrict__ phi,
                                                         const float* __restrict__ phi_im, int M,
                                                         int N, int first, float tol,
                                                         int* __restrict__ flag) {
  const int P = M * N;
  const double sc = 1.0 / sqrt((double)P);
  int bad = 0;
  for (int k = blockIdx.x; k < P; k += gridDim.x) {
    const int k1 = k / N, k2 = k - k1 * N;
    const size_t row = (size_t)(first + k) * P;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
      const int m = p / N, n = p - m * N;
      const int q = (k1 * m * N + k2 * n * M) % P;
      double sn, cs;
      sincospi(2.0 * (double)q / (double)P, &sn, &cs);
      if (fabs((double)phi[row + p] - cs * sc) > tol || fabs((double)phi_im[row + p] - sn * sc) > tol)
        bad = 1;
    }
  }
  if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// The constant operands (se_weighted_gram, once per table set): entry x of
// se_tables.tx, every workgroup computing a slice.
struct TxBuildArgs {
  int M, N, parts;
  int T, Ms;   // M = T Ms: frames of Ms rows stacked
  int kind0, kind1, first0, first1;
  const float* D;
  const float* sqrtw;
  float* tx;
};

__global__ __launch_bounds__(kTxThreads) void k_build_tx(TxBuildArgs a, TxLayout L) {
  extern __shared__ double ctab[];   // 4 Ms + 4N + 4T cosines
  double* ctS = ctab;
  double* ctN = ctS + 4 * a.Ms;
  double* ctT = ctN + 4 * a.N;
  build_cos_table(a.Ms, ctS);
  build_cos_table(a.N, ctN);
  build_cos_table(a.T, ctT);
  __syncthreads();
  const int M = a.M, N = a.N, MT = L.MT, NT = L.NT;
  const double iN = 1.0 / sqrt((double)N), aN = sqrt(2.0 / (double)N);
  const VertBasis vb{a.T, a.Ms, ctT, ctS};
  const int nA = MT * MT * 256, nB = NT * NT * 256, nD = MT * NT * 256;
  // class-order operands: two DCT-II / Walsh-Hadamard parts on areas of even
  // sides (the parity classes); otherwise that region stays 0
  const bool kinds_ok = (a.kind0 == SE_PART_DCT2 || a.kind0 == SE_PART_WHT2) &&
                        (a.kind1 == SE_PART_DCT2 || a.kind1 == SE_PART_WHT2);
  const bool cls = a.parts == 2 && kinds_ok && (a.Ms & 1) == 0 && (N & 1) == 0;
  const int HV = M / 2, HS = a.Ms / 2, HN = N / 2;
  // original stacked row of class-order row k (parity, frame, row / 2), and
  // original column of class-order column k (parity, column / 2)
  auto vrow = [&](int kind, int k) {
    const int pv = k / HV, rem = k - pv * HV, kt = rem / HS;
    return kt * a.Ms + parity_row(kind, rem - kt * HS, pv);
  };
  auto hcol = [&](int kind, int k) {
    const int ph = k / HN;
    return parity_row(kind, k - ph * HN, ph);
  };
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < L.ntotal; x += gridDim.x * blockDim.x) {
    float v = 0.0f;
    if (x < L.oBtf) {                       // Af
      const int q = x / nA, y = x - q * nA;
      const int e = y & 3, l = (y >> 2) & 63, ri = y >> 8;
      const int r = ri / MT, i = ri - r * MT;
      const int row = 16 * r + (l & 15), col = 16 * i + 4 * (l >> 4) + e;
      if (row < M && col < M) v = vb(q ? a.kind1 : a.kind0, row, col);
    } else if (x < L.oDf) {                 // Btf
      const int z = x - L.oBtf, q = z / nB, y = z - q * nB;
      const int t = y & 3, l = (y >> 2) & 63, cs = y >> 8;
      const int c = cs / NT, sq = cs - c * NT;
      const int k2 = 16 * c + (l & 15), n = 16 * sq + 4 * (l >> 4) + t;
      if (k2 < N && n < N) v = basis_1d(q ? a.kind1 : a.kind0, N, k2, n, ctN, iN, aN);
    } else if (!a.D) {                      // operands of unscaled transforms only
      break;
    } else if (x >= L.nconst) {             // class-order Ac, Bc, Dc
      if (cls) {
        if (x < L.oBc) {
          const int z = x - L.oAc, q = z / nA, y = z - q * nA;
          const int e = y & 3, l = (y >> 2) & 63, ri = y >> 8;
          const int r = ri / MT, i = ri - r * MT;
          const int row = 16 * r + (l & 15), col = 16 * i + 4 * (l >> 4) + e;
          const int kind = q ? a.kind1 : a.kind0;
          if (row < M && col < M) v = vb(kind, vrow(kind, row), col);
        } else if (x < L.oDc) {
          const int z = x - L.oBc, q = z / nB, y = z - q * nB;
          const int t = y & 3, l = (y >> 2) & 63, cs = y >> 8;
          const int c = cs / NT, sq = cs - c * NT;
          const int k2 = 16 * c + (l & 15), n = 16 * sq + 4 * (l >> 4) + t;
          const int kind = q ? a.kind1 : a.kind0;
          if (k2 < N && n < N) v = basis_1d(kind, N, hcol(kind, k2), n, ctN, iN, aN);
        } else {
          const int z = x - L.oDc, q = z / nD, y = z - q * nD;
          const int e = y & 3, l = (y >> 2) & 63, cr = y >> 8;
          const int c = cr / MT, r = cr - c * MT;
          const int k1 = 16 * r + 4 * (l >> 4) + e, k2 = 16 * c + (l & 15);
          const int kind = q ? a.kind1 : a.kind0;
          if (k1 < M && k2 < N)
            v = a.D[(q ? a.first1 : a.first0) + vrow(kind, k1) * N + hcol(kind, k2)];
        }
      }
    } else if (x < L.oWf) {                 // Df
      const int z = x - L.oDf, q = z / nD, y = z - q * nD;
      const int e = y & 3, l = (y >> 2) & 63, cr = y >> 8;
      const int c = cr / MT, r = cr - c * MT;
      const int k1 = 16 * r + 4 * (l >> 4) + e, k2 = 16 * c + (l & 15);
      if (k1 < M && k2 < N) v = a.D[(q ? a.first1 : a.first0) + k1 * N + k2];
    } else {                                // Wf
      const int y = x - L.oWf;
      const int t = y & 3, l = (y >> 2) & 63, is = y >> 8;
      const int i = is / NT, sq = is - i * NT;
      const int m = 16 * i + (l & 15), n = 16 * sq + 4 * (l >> 4) + t;
      if (m < M && n < N) {
        const float sw = a.sqrtw[m * N + n];
        v = sw * sw;
      }
    }
    a.tx[x] = v;
  }
}

template <int MT, int NT, int NP, bool STAGE, bool VOL>
__global__ __launch_bounds__((tx_max_threads<MT, NT>())) void k_project_tx(TxArgs a, TxLayout L) {
  extern __shared__ floatx4 smv[];
  float* sm = reinterpret_cast<float*>(smv);
  const int M = L.M, N = L.N;
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  float* Xf = sm + L.oXf + wave * L.wsz;
  // the first block's pixel loads and the copy of the constant operands
  // are in flight together
  int b = blockIdx.x * W + wave;
  DevBlock d = a.blk[b < a.n_blk ? b : 0];
  TxPixels<MT, NT> P;
  tx_load<MT, NT, VOL>(a, d, M, N, P);
  {
    const floatx4* src = reinterpret_cast<const floatx4*>(a.tx);
    for (int x = threadIdx.x; x < L.nconst / 4; x += blockDim.x) smv[x] = src[x];
  }
  __syncthreads();
  for (bool first = true; b < a.n_blk; b += gridDim.x * W, first = false) {
    if (!first) {
      d = a.blk[b];
      tx_load<MT, NT, VOL>(a, d, M, N, P);
    }
    floatx4 xv[MT][NT];
    tx_x_operands<MT, NT, VOL>(a, d, M, N, P, sm + L.oWf, Xf, xv);
    float* Rb = a.R + (size_t)b * a.ldR;
    for (int k = a.K + l; k < a.ldR; k += 64) Rb[k] = 0.0f;
#pragma unroll 1
    for (int q = 0; q < NP; ++q) {
      float* Rq = Rb + (q ? a.first1 : a.first0);
      const float* Af = sm + L.oAf + q * MT * MT * 256;
      const float* Btf = sm + L.oBtf + q * NT * NT * 256;
      const float* Df = sm + L.oDf + q * MT * NT * 256;
      if (STAGE) {
        // the part's output goes to this wave's LDS first and then to R as
        // whole 16-byte lanes of contiguous memory (full cache lines)
        wave_sync();   // the X operands and the previous part are read
        tx_part<MT, NT, true>(Af, Btf, Df, xv, M, N,
                              [&](int k1, int k2, float v) { Xf[k1 * L.zs + k2] = v; });
        wave_sync();
        for (int k = 4 * l; k < M * N; k += 256) {
          const int k1 = k / N, k2 = k - k1 * N;
          *reinterpret_cast<floatx4*>(Rq + k) = *reinterpret_cast<const floatx4*>(Xf + k1 * L.zs + k2);
        }
      } else {
        tx_part<MT, NT, true>(Af, Btf, Df, xv, M, N,
                              [&](int k1, int k2, float v) { Rq[k1 * N + k2] = v; });
      }
    }
    if (STAGE) wave_sync();   // the copies read before the next block's X writes
  }
}

// ---------------------------------------------------------------------------
// Initial projections of a complex DFT part (eq. 12 with conjugated atoms,
// Section VI): the weighted scalar products of the block's samples s with
// the atoms phi_(k1 N + k2) = exp(j 2 pi (k1 m / M + k2 n / N)) / sqrt(M N)
// are Z = Ac X Bc^T, X = w s, with the conjugate 1-D DFT matrices
// Ac = Ar + j Ai (M x M) and Bc = Br + j Bi (N x N).  X is real, so
//   Yr = X Br^T, Yi = X Bi^T,  Re Z = Ar Yr - Ai Yi,  Im Z = Ai Yr + Ar Yi
// -- six real products of the transform sizes, on the same fragments and
// matrix-core steps as the real transforms (the operand buffer holds Ar, Br
// as its first transform and Ai, Bi as its second; Df holds D_k once per
// transform).  Output: R[b][first + k] = D_k Re Z_k, R[b][im + first + k] =
// D_k Im Z_k.  One column tile of Z at a time.
template <int MT, int NT>
__device__ inline void dft_cols(int c, const float* Ar, const float* Ai, const float* Br,
                                const float* Bi, const float* Df, const floatx4 (&x)[MT][NT],
                                int M, int N, float* Rre, float* Rim) {
  const int l = threadIdx.x & 63;
  floatx4 yr[MT], yi[MT];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    yr[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    yi[i] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int sq = 0; sq < NT; ++sq) {
    const floatx4 br = *reinterpret_cast<const floatx4*>(Br + ((c * NT + sq) * 64 + l) * 4);
    const floatx4 bi = *reinterpret_cast<const floatx4*>(Bi + ((c * NT + sq) * 64 + l) * 4);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        yr[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[i][sq][t], br[t], yr[i], 0, 0, 0);
        yi[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[i][sq][t], bi[t], yi[i], 0, 0, 0);
      }
  }
  floatx4 zr[MT], zi[MT];
#pragma unroll
  for (int r = 0; r < MT; ++r) {
    zr[r] = floatx4{0.f, 0.f, 0.f, 0.f};
    zi[r] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    const floatx4 yn = -yi[i];
#pragma unroll
    for (int r = 0; r < MT; ++r) {
      const floatx4 ar = *reinterpret_cast<const floatx4*>(Ar + ((r * MT + i) * 64 + l) * 4);
      const floatx4 ai = *reinterpret_cast<const floatx4*>(Ai + ((r * MT + i) * 64 + l) * 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        zr[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[e], yr[i][e], zr[r], 0, 0, 0);
        zi[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[e], yr[i][e], zi[r], 0, 0, 0);
        zr[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[e], yn[e], zr[r], 0, 0, 0);
        zi[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[e], yi[i][e], zi[r], 0, 0, 0);
      }
    }
  }
  const int k2 = 16 * c + (l & 15);
#pragma unroll
  for (int r = 0; r < MT; ++r) {
    const floatx4 dv = *reinterpret_cast<const floatx4*>(Df + ((c * MT + r) * 64 + l) * 4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k1 = 16 * r + 4 * (l >> 4) + e;
      if (k1 < M && k2 < N) {
        Rre[k1 * N + k2] = dv[e] * zr[r][e];
        Rim[k1 * N + k2] = dv[e] * zi[r][e];
      }
    }
  }
}

// One wave per block, the workgroup's waves looping over blocks; each
// workgroup copies the operand buffer to LDS once (the loaders and the X
// operands of the real transforms).  Half the real transforms' workgroup
// bound: the two accumulator sets need more registers per lane.
template <int MT, int NT>
constexpr int dft_max_threads() {
  return tx_max_threads<MT, NT>() / 2;
}

template <int MT, int NT>
__global__ __launch_bounds__((dft_max_threads<MT, NT>())) void k_project_dft(TxArgs a, TxLayout L,
                                                                             int im) {
  extern __shared__ floatx4 smv[];
  float* sm = reinterpret_cast<float*>(smv);
  const int M = L.M, N = L.N;
  const int wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  float* Xf = sm + L.oXf + wave * L.wsz;
  int b = blockIdx.x * W + wave;
  DevBlock d = a.blk[b < a.n_blk ? b : 0];
  TxPixels<MT, NT> P;
  tx_load<MT, NT>(a, d, M, N, P);
  {
    const floatx4* src = reinterpret_cast<const floatx4*>(a.tx);
    for (int x = threadIdx.x; x < L.nconst / 4; x += blockDim.x) smv[x] = src[x];
  }
  __syncthreads();
  const float* Ar = sm + L.oAf;
  const float* Ai = Ar + MT * MT * 256;
  const float* Br = sm + L.oBtf;
  const float* Bi = Br + NT * NT * 256;
  const float* Df = sm + L.oDf;
  for (bool first = true; b < a.n_blk; b += gridDim.x * W, first = false) {
    if (!first) {
      d = a.blk[b];
      tx_load<MT, NT>(a, d, M, N, P);
    }
    floatx4 xv[MT][NT];
    tx_x_operands<MT, NT>(a, d, M, N, P, sm + L.oWf, Xf, xv);
    float* Rre = a.R + (size_t)b * a.ldR + a.first0;
#pragma unroll 1
    for (int c = 0; c < NT; ++c) dft_cols<MT, NT>(c, Ar, Ai, Br, Bi, Df, xv, M, N, Rre, Rre + im);
  }
}

// ---------------------------------------------------------------------------
// Rows of the per-block tables formed on demand (eq. 16, row u of C_b) for
// the transform parts: rows[b][first + k] = sum_p phi_k[p] V[b][p] with
// V[b] = w_b phi_u (M x N floats), i.e. the transform A V_b B^T.  Same
// matrix-core scheme as k_project_tx without the D scaling; the fragments of
// A and B come first in the operand buffer.
struct TxRowsArgs {
  const float* V;
  int ldV, n_blk;
  const float* tx;
  int first0, first1;
  float* rows;
  int ld;
  const int32_t* n_dev;   // optional: rows to form counted on the device (<= n_blk)
  const int32_t* out_row; // optional: destination row of V row i
};

template <int MT, int NT, int NP>
__global__ __launch_bounds__((tx_max_threads<MT, NT>())) void k_rows_tx(TxRowsArgs a, TxLayout L) {
  extern __shared__ floatx4 smv[];
  float* sm = reinterpret_cast<float*>(smv);
  {
    const floatx4* src = reinterpret_cast<const floatx4*>(a.tx);
    for (int x = threadIdx.x; x < L.oDf / 4; x += blockDim.x) smv[x] = src[x];
  }
  __syncthreads();
  const int M = L.M, N = L.N;
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  const int lr = l & 15, lc = 4 * (l >> 4);
  const bool vec = (N & 3) == 0;
  const int nb = a.n_dev ? min(a.n_blk, *a.n_dev) : a.n_blk;
  for (int b = blockIdx.x * W + wave; b < nb; b += gridDim.x * W) {
    const float* Vb = a.V + (size_t)b * a.ldV;
    // every load at clamped (valid) coordinates and issued before the
    // first use; entries outside the area are zeroed afterwards
    floatx4 xv[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const int m = 16 * i + lr;
      const float* row = Vb + (size_t)min(m, M - 1) * N;
#pragma unroll
      for (int sq = 0; sq < NT; ++sq) {
        const int n0 = 16 * sq + lc;
        if (vec) {
          xv[i][sq] = *reinterpret_cast<const floatx4*>(row + min(n0, N - 4));
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) xv[i][sq][t] = row[min(n0 + t, N - 1)];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int sq = 0; sq < NT; ++sq)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          float v = xv[i][sq][t];
          asm volatile("" : "+v"(v));   // keeps the loads above unconditional
          xv[i][sq][t] = (16 * i + lr < M && 16 * sq + lc + t < N) ? v : 0.0f;
        }
#pragma unroll 1
    for (int q = 0; q < NP; ++q) {
      float* Rq = a.rows + (size_t)(a.out_row ? a.out_row[b] : b) * a.ld + (q ? a.first1 : a.first0);
      tx_part<MT, NT, false>(sm + L.oAf + q * MT * MT * 256, sm + L.oBtf + q * NT * NT * 256,
                             nullptr, xv, M, N,
                             [&](int k1, int k2, float v) { Rq[k1 * N + k2] = v; });
    }
  }
}

// ---------------------------------------------------------------------------
// Table rows from transforms (Algorithm 2 for the transform parts, eq. 16):
// for atom k and part q, G[k][first_q + j] = D_k D_{first_q + j}
// sum_p w phi_k phi_{first_q + j} = D_k (D_q ⊙ T_q(w phi_k))_j -- the
// transform of the weighted atom, the same scheme as k_project_tx with the
// atom's FP32 values in place of the pixels.  Every atom's row is formed over
// the part columns; the rest of the table comes from the product of the
// dense atoms and a mirror pass.
struct TxGramArgs {
  const float* phi;
  int K;
  const float* tx;
  const float* D;
  int first0, first1;
  float* G;
  int ldG;
};

template <int MT, int NT, int NP>
__global__ __launch_bounds__((tx_max_threads<MT, NT>())) void k_gram_tx(TxGramArgs a, TxLayout L) {
  extern __shared__ floatx4 smv[];
  float* sm = reinterpret_cast<float*>(smv);
  {
    const floatx4* src = reinterpret_cast<const floatx4*>(a.tx);
    for (int x = threadIdx.x; x < L.nconst / 4; x += blockDim.x) smv[x] = src[x];
  }
  __syncthreads();
  const int M = L.M, N = L.N, P = M * N;
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  const int lr = l & 15, lc = 4 * (l >> 4);
  const bool vec = (N & 3) == 0;
  float* Zs = sm + L.oXf + wave * L.wsz;
  for (int k = blockIdx.x * W + wave; k < a.K; k += gridDim.x * W) {
    const float* row = a.phi + (size_t)k * P;
    // X operands w phi_k, loaded at clamped coordinates (issued before the
    // first use) and zeroed outside the area
    floatx4 xv[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const float* r = row + (size_t)min(16 * i + lr, M - 1) * N;
#pragma unroll
      for (int sq = 0; sq < NT; ++sq) {
        const int n0 = 16 * sq + lc;
        if (vec) {
          xv[i][sq] = *reinterpret_cast<const floatx4*>(r + min(n0, N - 4));
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) xv[i][sq][t] = r[min(n0 + t, N - 1)];
        }
      }
    }
    const float Dk = a.D[k];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int sq = 0; sq < NT; ++sq) {
        const floatx4 w = *reinterpret_cast<const floatx4*>(sm + L.oWf + ((i * NT + sq) * 64 + l) * 4);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          float v = xv[i][sq][t];
          asm volatile("" : "+v"(v));   // keeps the loads above unconditional
          xv[i][sq][t] = (16 * i + lr < M && 16 * sq + lc + t < N) ? w[t] * v : 0.0f;
        }
      }
    float* Gk = a.G + (size_t)k * a.ldG;
#pragma unroll 1
    for (int q = 0; q < NP; ++q) {
      float* Gq = Gk + (q ? a.first1 : a.first0);
      const float* Af = sm + L.oAf + q * MT * MT * 256;
      const float* Btf = sm + L.oBtf + q * NT * NT * 256;
      const float* Df = sm + L.oDf + q * MT * NT * 256;
      if (L.zs > 0) {   // staged: the row segment is written as whole lines
        wave_sync();
        tx_part<MT, NT, true>(Af, Btf, Df, xv, M, N,
                              [&](int k1, int k2, float v) { Zs[k1 * L.zs + k2] = Dk * v; });
        wave_sync();
        for (int j = 4 * l; j < P; j += 256) {
          const int k1 = j / N, k2 = j - k1 * N;
          *reinterpret_cast<floatx4*>(Gq + j) = *reinterpret_cast<const floatx4*>(Zs + k1 * L.zs + k2);
        }
      } else {
        tx_part<MT, NT, true>(Af, Btf, Df, xv, M, N,
                              [&](int k1, int k2, float v) { Gq[k1 * N + k2] = Dk * v; });
      }
    }
    wave_sync();
  }
}

// The entries no transform row produced, and exact symmetry: for rows r of
// a part, G[r][c] = G[c][r] where column c is a dense atom (the dense row c
// holds the value over its part columns) or a part atom with c > r (the
// lower triangle's value).  Dense x dense entries come from the product of
// the dense atoms.  32 x 32 tiles, transposed through LDS.
__global__ __launch_bounds__(256) void k_gram_mirror(float* __restrict__ G, int ldG, int K, int p0,
                                                     int q0, int P) {
  __shared__ float tile[32][33];
  const int rb = blockIdx.y * 32, cb = blockIdx.x * 32;
  auto in_part = [&](int i) { return (i >= p0 && i < p0 + P) || (i >= q0 && i < q0 + P); };
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {   // source G[c][r]: rows cb.., columns rb..
    const int c = cb + y, r = rb + tx;
    tile[y][tx] = (c < K && r < K) ? G[(size_t)c * ldG + r] : 0.0f;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int r = rb + y, c = cb + tx;
    if (r < K && c < K && in_part(r) && (!in_part(c) || c > r))
      G[(size_t)r * ldG + c] = tile[tx][y];
  }
}

se_status check_part(const float* phi, int T, int Ms, int N, int kind, int first, int* dflag,
                     hipStream_t s) {
  const int M = T * Ms;
  const size_t lds = (size_t)4 * (Ms + N + T) * 8 + (size_t)(M * M + N * N) * 4;
  const int P = M * N;
  const int grid = P < 2048 ? P : 2048;
  hipLaunchKernelGGL(k_check_part, dim3(grid), dim3(kTxThreads), lds, s, phi, T, Ms, N, kind,
                     first, 2e-6f, dflag);
  return check_launch("check_part");
}

se_status check_dft_part(const float* phi, const float* phi_im, int M, int N, int first,
                         int* dflag, hipStream_t s) {
  const int P = M * N;
  const int grid = P < 2048 ? P : 2048;
  hipLaunchKernelGGL(k_check_dft, dim3(grid), dim3(kTxThreads), 0, s, phi, phi_im, M, N, first,
                     2e-6f, dflag);
  return check_launch("check_dft_part");
}

size_t tx_const_bytes(int M, int N, int n_parts) {
  if (M < 1 || N < 1 || M > 64 || N > 64 || n_parts < 1 || n_parts > 2) return 0;
  return (size_t)TxLayout(M, N, n_parts, 0).ntotal * 4;
}

se_status build_tx(const se_tables* t, hipStream_t s) {
  TxBuildArgs a;
  a.T = area_frames(t->T);
  a.Ms = t->M;
  a.M = tx_rows(t);
  a.N = t->N;
  a.parts = tx_layout_parts(t->n_parts, t->parts);
  a.kind0 = t->parts[0].kind;
  a.first0 = t->parts[0].first;
  a.kind1 = t->n_parts > 1 ? t->parts[1].kind : 0;
  a.first1 = t->n_parts > 1 ? t->parts[1].first : 0;
  if (a.kind0 == SE_PART_DFT2) {
    // the real and the imaginary 1-D matrices as the two transforms, both
    // scaled by the part's D
    a.kind0 = kKindDftRe;
    a.kind1 = kKindDftIm;
    a.first1 = a.first0;
  }
  a.D = t->D;
  a.sqrtw = t->sqrtw;
  a.tx = t->tx;
  const TxLayout L(a.M, t->N, a.parts, 0);
  const int grid = (L.ntotal + kTxThreads - 1) / kTxThreads;
  hipLaunchKernelGGL(k_build_tx, dim3(grid), dim3(kTxThreads),
                     (size_t)4 * (a.Ms + a.N + a.T) * 8, s, a, L);
  return check_launch("build_tx");
}

se_status build_tx_basis(const se_basis* b, float* tx, hipStream_t s) {
  TxBuildArgs a;
  a.T = 1;    // rows on demand: two-dimensional areas
  a.Ms = b->M;
  a.M = b->M;
  a.N = b->N;
  a.parts = b->n_parts;
  a.kind0 = b->parts[0].kind;
  a.first0 = b->parts[0].first;
  a.kind1 = b->n_parts > 1 ? b->parts[1].kind : 0;
  a.first1 = b->n_parts > 1 ? b->parts[1].first : 0;
  a.D = nullptr;
  a.sqrtw = nullptr;
  a.tx = tx;
  const TxLayout L(b->M, b->N, b->n_parts, 0);
  const int grid = (L.oDf + kTxThreads - 1) / kTxThreads;
  hipLaunchKernelGGL(k_build_tx, dim3(grid), dim3(kTxThreads),
                     (size_t)4 * (a.Ms + a.N + a.T) * 8, s, a, L);
  return check_launch("build_tx_basis");
}

template <int MT, int NT, int NP>
static se_status launch_gram(const TxGramArgs& a, const TxLayout& L, int grid, size_t lds,
                             hipStream_t s) {
  static std::atomic<uint64_t> raised{0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev > 63)
    return fail(SE_EHIP, "gram_tx: no current device");
  if (lds > 64 * 1024 && !(raised.load() & (1ull << dev))) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram_tx<MT, NT, NP>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
      return fail(SE_EHIP, "gram_tx: %zu bytes of LDS refused", lds);
    raised.fetch_or(1ull << dev);
  }
  hipLaunchKernelGGL((k_gram_tx<MT, NT, NP>), dim3(grid), dim3(64 * L.waves), lds, s, a, L);
  return check_launch("gram_tx");
}

template <int MT, int NT>
static se_status launch_gram_np(const TxGramArgs& a, const TxLayout& L, int grid, size_t lds,
                                hipStream_t s) {
  return L.parts == 2 ? launch_gram<MT, NT, 2>(a, L, grid, lds, s)
                      : launch_gram<MT, NT, 1>(a, L, grid, lds, s);
}

static int tx_waves(int M, int N, int n_parts, int n_blk);

se_status gram_tx(const se_tables* t, hipStream_t s) {
  TxGramArgs a;
  a.phi = t->phi;
  a.K = t->K;
  a.tx = t->tx;
  a.D = t->D;
  a.first0 = t->parts[0].first;
  a.first1 = t->n_parts > 1 ? t->parts[1].first : 0;
  a.G = t->G;
  a.ldG = t->ldG;
  const int Mv = tx_rows(t);
  const int waves = tx_waves(Mv, t->N, t->n_parts, t->K);
  if (waves == 0) return fail(SE_EINVAL, "transform of a %dx%d area exceeds LDS", Mv, t->N);
  const bool stage = (t->N & 3) == 0 && (a.first0 & 3) == 0 && (a.first1 & 3) == 0 &&
                     (t->ldG & 3) == 0 &&
                     TxLayout(Mv, t->N, t->n_parts, waves, true).bytes() <= 160 * 1024;
  const TxLayout L(Mv, t->N, t->n_parts, waves, stage);
  const size_t lds = L.bytes();
  const int per_cu = (int)std::min<size_t>(4, (160 * 1024) / lds);
  const int grid = std::max(1, std::min((t->K + waves - 1) / waves, 256 * per_cu));
  se_status st = SE_OK;
  switch (L.MT * 10 + L.NT) {
#define SE_TX_CASE(mt, nt)                                \
  case mt * 10 + nt:                                      \
    st = launch_gram_np<mt, nt>(a, L, grid, lds, s); \
    break;
    SE_TX_CASE(1, 1) SE_TX_CASE(1, 2) SE_TX_CASE(1, 3) SE_TX_CASE(1, 4)
    SE_TX_CASE(2, 1) SE_TX_CASE(2, 2) SE_TX_CASE(2, 3) SE_TX_CASE(2, 4)
    SE_TX_CASE(3, 1) SE_TX_CASE(3, 2) SE_TX_CASE(3, 3) SE_TX_CASE(3, 4)
    SE_TX_CASE(4, 1) SE_TX_CASE(4, 2) SE_TX_CASE(4, 3) SE_TX_CASE(4, 4)
#undef SE_TX_CASE
    default: return fail(SE_EINVAL, "transform parts need M, N <= 64");
  }
  return st;
}

se_status gram_mirror(const se_tables* t, hipStream_t s) {
  const int P = area_samples(t);
  const int p0 = t->parts[0].first;
  const int q0 = t->n_parts > 1 ? t->parts[1].first : p0;
  const int nb = (t->K + 31) / 32;
  hipLaunchKernelGGL(k_gram_mirror, dim3(nb, nb), dim3(256), 0, s, t->G, t->ldG, t->K, p0, q0, P);
  return check_launch("gram_mirror");
}

// Waves per workgroup: the kernel's workgroup bound, fewer when that leaves
// compute units without a workgroup or exceeds the LDS.
static int tx_waves(int M, int N, int n_parts, int n_blk) {
  const int MT = (M + 15) / 16, NT = (N + 15) / 16;
  int w = (MT >= 3 || MT * NT >= 6) ? 4 : 16;
  while (w > 1 && (long long)w * 256 > n_blk) w /= 2;
  while (w >= 1 && TxLayout(M, N, n_parts, w).bytes() > 160 * 1024) w /= 2;
  return w;
}

size_t tx_lds_bytes(int M, int N, int n_parts) {
  const int w = tx_waves(M, N, n_parts, 1 << 30);
  return w ? TxLayout(M, N, n_parts, w).bytes() : 0;
}

template <int MT, int NT, int NP, bool STAGE, bool VOL>
static se_status launch_tx(const TxArgs& a, const TxLayout& L, int grid, size_t lds,
                           hipStream_t s) {
  // the LDS limit is raised once per device and instantiation, so that the
  // launches of a caller's stream capture contain no attribute call
  static std::atomic<uint64_t> raised{0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev > 63)
    return fail(SE_EHIP, "project_tx: no current device");
  if (lds > 64 * 1024 && !(raised.load() & (1ull << dev))) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_project_tx<MT, NT, NP, STAGE, VOL>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
      return fail(SE_EHIP, "project_tx: %zu bytes of LDS refused", lds);
    raised.fetch_or(1ull << dev);
  }
  hipLaunchKernelGGL((k_project_tx<MT, NT, NP, STAGE, VOL>), dim3(grid), dim3(64 * L.waves), lds, s,
                     a, L);
  return check_launch("project_tx");
}

template <int MT, int NT, bool VOL>
static se_status launch_tx_vol(const TxArgs& a, const TxLayout& L, int grid, size_t lds,
                               hipStream_t s) {
  if (L.zs > 0)
    return L.parts == 2 ? launch_tx<MT, NT, 2, true, VOL>(a, L, grid, lds, s)
                        : launch_tx<MT, NT, 1, true, VOL>(a, L, grid, lds, s);
  return L.parts == 2 ? launch_tx<MT, NT, 2, false, VOL>(a, L, grid, lds, s)
                      : launch_tx<MT, NT, 1, false, VOL>(a, L, grid, lds, s);
}

// areas of several frames take the loaders that stack the frames
template <int MT, int NT>
static se_status launch_tx_np(const TxArgs& a, const TxLayout& L, int grid, size_t lds,
                              hipStream_t s, bool vol) {
  return vol ? launch_tx_vol<MT, NT, true>(a, L, grid, lds, s)
             : launch_tx_vol<MT, NT, false>(a, L, grid, lds, s);
}

template <int MT, int NT, int NP>
static se_status launch_rows(const TxRowsArgs& a, const TxLayout& L, int grid, size_t lds,
                             hipStream_t s) {
  static std::atomic<uint64_t> raised{0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev > 63)
    return fail(SE_EHIP, "rows_tx: no current device");
  if (lds > 64 * 1024 && !(raised.load() & (1ull << dev))) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rows_tx<MT, NT, NP>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
      return fail(SE_EHIP, "rows_tx: %zu bytes of LDS refused", lds);
    raised.fetch_or(1ull << dev);
  }
  hipLaunchKernelGGL((k_rows_tx<MT, NT, NP>), dim3(grid), dim3(64 * L.waves), lds, s, a, L);
  return check_launch("rows_tx");
}

template <int MT, int NT>
static se_status launch_rows_np(const TxRowsArgs& a, const TxLayout& L, int grid, size_t lds,
                                hipStream_t s) {
  return L.parts == 2 ? launch_rows<MT, NT, 2>(a, L, grid, lds, s)
                      : launch_rows<MT, NT, 1>(a, L, grid, lds, s);
}

se_status rows_tx(const se_basis* b, const float* tx, const float* V, int ldV, int n_blk,
                  float* rows, int ld, hipStream_t s, const int32_t* n_dev,
                  const int32_t* out_row) {
  if (n_blk <= 0) return SE_OK;
  if (b->n_parts < 1 || b->n_parts > 2) return fail(SE_EINVAL, "no transform part declared");
  TxRowsArgs a;
  a.V = V;
  a.ldV = ldV;
  a.n_blk = n_blk;
  a.tx = tx;
  a.first0 = b->parts[0].first;
  a.first1 = b->n_parts > 1 ? b->parts[1].first : 0;
  a.rows = rows;
  a.ld = ld;
  a.n_dev = n_dev;
  a.out_row = out_row;
  const int MT = (b->M + 15) / 16, NT = (b->N + 15) / 16;
  int waves = (MT >= 3 || MT * NT >= 6) ? 4 : 16;
  while (waves > 1 && (long long)waves * 256 > n_blk) waves /= 2;
  const TxLayout L(b->M, b->N, b->n_parts, waves);
  const size_t lds = (size_t)L.oDf * 4;
  const int per_cu = (int)std::min<size_t>(4, (160 * 1024) / lds);
  const int grid = std::max(1, std::min((n_blk + waves - 1) / waves, 256 * per_cu));
  switch (MT * 10 + NT) {
#define SE_TX_CASE(mt, nt) \
  case mt * 10 + nt:       \
    return launch_rows_np<mt, nt>(a, L, grid, lds, s);
    SE_TX_CASE(1, 1) SE_TX_CASE(1, 2) SE_TX_CASE(1, 3) SE_TX_CASE(1, 4)
    SE_TX_CASE(2, 1) SE_TX_CASE(2, 2) SE_TX_CASE(2, 3) SE_TX_CASE(2, 4)
    SE_TX_CASE(3, 1) SE_TX_CASE(3, 2) SE_TX_CASE(3, 3) SE_TX_CASE(3, 4)
    SE_TX_CASE(4, 1) SE_TX_CASE(4, 2) SE_TX_CASE(4, 3) SE_TX_CASE(4, 4)
#undef SE_TX_CASE
    default: return fail(SE_EINVAL, "transform parts need M, N <= 64");
  }
}

se_status project_tx(const se_tables* t, const uint8_t* images, int H, int W, const DevBlock* blk,
                     int n_blk, float* R, int ldR, hipStream_t s) {
  if (t->n_parts < 1 || t->n_parts > 2) return fail(SE_EINVAL, "no transform part declared");
  TxArgs a;
  a.images = images;
  a.H = H;
  a.W = W;
  a.blk = blk;
  a.n_blk = n_blk;
  a.K = t->K;
  a.tx = t->tx;
  a.first0 = t->parts[0].first;
  a.first1 = t->n_parts > 1 ? t->parts[1].first : 0;
  a.R = R;
  a.ldR = ldR;
  const bool vol = area_frames(t->T) > 1;
  a.fs = 0;
  if (vol)
    while ((1 << a.fs) < t->M) ++a.fs;   // rows per frame: a power of two (checked)
  const int Mv = tx_rows(t);
  const int waves = tx_waves(Mv, t->N, t->n_parts, n_blk);
  if (waves == 0) return fail(SE_EINVAL, "transform of a %dx%d area exceeds LDS", Mv, t->N);
  // staged (coalesced) output when rows of four floats stay aligned and the
  // staging area fits beside the operands
  bool stage = (t->N & 3) == 0 && (a.first0 & 3) == 0 && (a.first1 & 3) == 0 && (ldR & 3) == 0 &&
               TxLayout(Mv, t->N, t->n_parts, waves, true).bytes() <= 160 * 1024;
  const TxLayout L(Mv, t->N, t->n_parts, waves, stage);
  const size_t lds = L.bytes();
  // about one block per wave, at most four workgroups per compute unit
  const int per_cu = (int)std::min<size_t>(4, (160 * 1024) / lds);
  const int grid = std::max(1, std::min((n_blk + waves - 1) / waves, 256 * per_cu));
  switch (L.MT * 10 + L.NT) {
#define SE_TX_CASE(mt, nt) \
  case mt * 10 + nt:       \
    return launch_tx_np<mt, nt>(a, L, grid, lds, s, vol);
    SE_TX_CASE(1, 1) SE_TX_CASE(1, 2) SE_TX_CASE(1, 3) SE_TX_CASE(1, 4)
    SE_TX_CASE(2, 1) SE_TX_CASE(2, 2) SE_TX_CASE(2, 3) SE_TX_CASE(2, 4)
    SE_TX_CASE(3, 1) SE_TX_CASE(3, 2) SE_TX_CASE(3, 3) SE_TX_CASE(3, 4)
    SE_TX_CASE(4, 1) SE_TX_CASE(4, 2) SE_TX_CASE(4, 3) SE_TX_CASE(4, 4)
#undef SE_TX_CASE
    default: return fail(SE_EINVAL, "transform parts need M, N <= 64");
  }
}

template <int MT, int NT>
static se_status launch_dft(const TxArgs& a, const TxLayout& L, int grid, size_t lds, int im,
                            hipStream_t s) {
  static std::atomic<uint64_t> raised{0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev > 63)
    return fail(SE_EHIP, "project_dft: no current device");
  if (lds > 64 * 1024 && !(raised.load() & (1ull << dev))) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_project_dft<MT, NT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
      return fail(SE_EHIP, "project_dft: %zu bytes of LDS refused", lds);
    raised.fetch_or(1ull << dev);
  }
  hipLaunchKernelGGL((k_project_dft<MT, NT>), dim3(grid), dim3(64 * L.waves), lds, s, a, L, im);
  return check_launch("project_dft");
}

se_status project_dft(const se_tables* t, const uint8_t* images, int H, int W,
                      const DevBlock* blk, int n_blk, float* R, int ldR, int im, hipStream_t s) {
  if (t->n_parts != 1 || t->parts[0].kind != SE_PART_DFT2 || area_frames(t->T) != 1)
    return fail(SE_EINVAL, "no DFT part declared");
  if (n_blk <= 0) return SE_OK;
  TxArgs a;
  a.images = images;
  a.H = H;
  a.W = W;
  a.blk = blk;
  a.n_blk = n_blk;
  a.K = t->K;
  a.tx = t->tx;
  a.first0 = t->parts[0].first;
  a.first1 = a.first0;
  a.R = R;
  a.ldR = ldR;
  a.fs = 0;
  int waves = tx_waves(t->M, t->N, 2, n_blk);
  if (waves == 0) return fail(SE_EINVAL, "transform of a %dx%d area exceeds LDS", t->M, t->N);
  const int MT = (t->M + 15) / 16, NT = (t->N + 15) / 16;
  waves = std::min(waves, (MT >= 3 || MT * NT >= 6) ? 2 : 8);   // dft_max_threads / 64
  const TxLayout L(t->M, t->N, 2, waves);
  const size_t lds = L.bytes();
  const int per_cu = (int)std::min<size_t>(4, (160 * 1024) / lds);
  const int grid = std::max(1, std::min((n_blk + waves - 1) / waves, 256 * per_cu));
  switch (L.MT * 10 + L.NT) {
#define SE_TX_CASE(mt, nt) \
  case mt * 10 + nt:       \
    return launch_dft<mt, nt>(a, L, grid, lds, im, s);
    SE_TX_CASE(1, 1) SE_TX_CASE(1, 2) SE_TX_CASE(1, 3) SE_TX_CASE(1, 4)
    SE_TX_CASE(2, 1) SE_TX_CASE(2, 2) SE_TX_CASE(2, 3) SE_TX_CASE(2, 4)
    SE_TX_CASE(3, 1) SE_TX_CASE(3, 2) SE_TX_CASE(3, 3) SE_TX_CASE(3, 4)
    SE_TX_CASE(4, 1) SE_TX_CASE(4, 2) SE_TX_CASE(4, 3) SE_TX_CASE(4, 4)
#undef SE_TX_CASE
    default: return fail(SE_EINVAL, "transform parts need M, N <= 64");
  }
}

}  // namespace sefase
