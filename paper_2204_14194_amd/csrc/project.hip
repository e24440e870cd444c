// Inputs of the initial weighted scalar products (eq. 12):
//   X[b][p] = sqrt(w_p) s_b[p]  -- the block's area cut out of the 8-bit
//   image (of T consecutive frames, sample (tau, m, n) at (tau M + m) N + n),
//   weighted; pixels outside the image contribute 0.  With
//   Y[k][p] = D_k sqrt(w_p) phi_k[p] the products R = X Y^T are the
//   R_k^(0) of eq. 12 in units of D_k.
// plus the matrix-vector form of the same product for one block (the plain
// per-block path).
#include "bf16.h"
#include "se_internal.h"

namespace sefase {

__global__ void k_gather(const uint8_t* __restrict__ images, int H, int W,
                         const DevBlock* __restrict__ blk, int n_blk, int T, int M, int N,
                         const float* __restrict__ sqrtw, float* __restrict__ X, int ldX) {
  const int b = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int S = M * N, P = T * S;
  if (b >= n_blk || p >= P) return;
  const DevBlock d = blk[b];
  const int tau = p / S, q = p - tau * S;
  const int m = q / N, n = q - m * N;
  const int y = d.y0 + m, x = d.x0 + n;
  float v = 0.0f;
  if (y >= 0 && y < H && x >= 0 && x < W)
    v = sqrtw[p] * (float)images[(size_t)(d.img + tau) * H * W + (size_t)y * W + x];
  X[(size_t)b * ldX + p] = v;
}

void launch_gather(const uint8_t* images, int H, int W, const DevBlock* blk, int n_blk, int T,
                   int M, int N, const float* sqrtw, float* X, int ldX, hipStream_t s) {
  const int P = T * M * N;
  hipLaunchKernelGGL(k_gather, dim3((P + 255) / 256, n_blk), dim3(256), 0, s, images, H, W, blk,
                     n_blk, T, M, N, sqrtw, X, ldX);
}

__global__ void k_gather_split(const uint8_t* __restrict__ images, int H, int W,
                               const DevBlock* __restrict__ blk, int n_blk, int T, int M, int N,
                               const float* __restrict__ sqrtw, uint16_t* __restrict__ Xhi,
                               uint16_t* __restrict__ Xlo, int ldX) {
  const int b = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int S = M * N, P = T * S;
  if (b >= n_blk || p >= P) return;
  const DevBlock d = blk[b];
  const int tau = p / S, q = p - tau * S;
  const int m = q / N, n = q - m * N;
  const int y = d.y0 + m, x = d.x0 + n;
  float v = 0.0f;
  if (y >= 0 && y < H && x >= 0 && x < W)
    v = sqrtw[p] * (float)images[(size_t)(d.img + tau) * H * W + (size_t)y * W + x];
  uint16_t h, l;
  bf16_split(v, h, l);
  Xhi[(size_t)b * ldX + p] = h;
  Xlo[(size_t)b * ldX + p] = l;
}

void launch_gather_split(const uint8_t* images, int H, int W, const DevBlock* blk, int n_blk,
                         int T, int M, int N, const float* sqrtw, uint16_t* Xhi, uint16_t* Xlo,
                         int ldX, hipStream_t s) {
  const int P = T * M * N;
  hipLaunchKernelGGL(k_gather_split, dim3((P + 255) / 256, n_blk), dim3(256), 0, s, images, H, W,
                     blk, n_blk, T, M, N, sqrtw, Xhi, Xlo, ldX);
}

// r[k] = sum_p Y[k][p] x[p]; one wavefront per atom, lane-strided partial
// sums combined by a fixed butterfly.
__global__ __launch_bounds__(256) void k_gemv(const float* __restrict__ Y, int K, int P,
                                              const float* __restrict__ x, float* __restrict__ r) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= K) return;
  const float* row = Y + (size_t)k * P;
  float acc = 0.0f;
  for (int p = lane; p < P; p += 64) acc = fmaf(row[p], x[p], acc);
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) r[k] = acc;
}

void launch_gemv(const float* Y, int K, int P, const float* x, float* r, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv, dim3((K + 3) / 4), dim3(256), 0, s, Y, K, P, x, r);
}

}  // namespace sefase
