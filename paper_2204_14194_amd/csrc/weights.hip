// Weighting function of Selective Extrapolation: w = rho on the support
// area A and 0 on the loss area B (eq. 4), with the exponentially decaying
// rho = rho_hat ^ (distance to the area centre ((M-1)/2, (N-1)/2)) (eq. 5).
// Pixels outside the image or lost (in any block) are not support.  An area
// of T > 1 consecutive frames takes the distance to the centre of the
// T x M x N box, the time axis counted in frames like the two spatial axes
// in pixels; with T = 1 the temporal term is exactly 0.
#include "se_internal.h"

namespace sefase {

// One thread per (block, sample); the grid is exact, so every access is in
// bounds by construction (the frames img .. img+T-1 of every block were
// range-checked on the host).
__global__ void k_area_weights(int T, int M, int N, float log_rho,
                               const uint8_t* __restrict__ lost, int H, int W,
                               const DevBlock* __restrict__ blk, int n_blk,
                               float* __restrict__ w) {
  const int S = M * N, P = T * S;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n_blk * P) return;
  const int b = (int)(i / P);
  const int p = (int)(i - (long long)b * P);
  const int tau = p / S, q = p - tau * S;
  const int m = q / N, n = q - m * N;
  const DevBlock d = blk[b];
  const int y = d.y0 + m, x = d.x0 + n;
  float v = 0.0f;
  if (y >= 0 && y < H && x >= 0 && x < W &&
      lost[(size_t)(d.img + tau) * H * W + (size_t)y * W + x] == 0) {
    const float dt = (float)tau - 0.5f * (float)(T - 1);
    const float dy = (float)m - 0.5f * (float)(M - 1);
    const float dx = (float)n - 0.5f * (float)(N - 1);
    v = expf(log_rho * sqrtf(dt * dt + dy * dy + dx * dx));
  }
  w[i] = v;
}

void launch_area_weights(int T, int M, int N, float rho_hat, const uint8_t* lost, int H, int W,
                         const DevBlock* blk, int n_blk, float* w, hipStream_t s) {
  const long long total = (long long)n_blk * T * M * N;
  const int tpb = 256;
  const unsigned grid = (unsigned)((total + tpb - 1) / tpb);
  hipLaunchKernelGGL(k_area_weights, dim3(grid), dim3(tpb), 0, s, T, M, N, logf(rho_hat), lost,
                     H, W, blk, n_blk, w);
}

}  // namespace sefase

namespace sefase {

// Lost-pixel mask of a frame: zero it, then mark each loss rectangle
// (rects: y, x, h, w in frame coordinates, already validated).
__global__ void k_fill_u8(uint8_t* __restrict__ a, size_t n, uint8_t v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_mark_rects(uint8_t* __restrict__ mask, int H, int W,
                             const int4* __restrict__ rects, int n) {
  const int r = blockIdx.x;
  if (r >= n) return;
  const int4 q = rects[r];
  for (int i = threadIdx.x; i < q.z * q.w; i += blockDim.x) {
    const int y = q.x + i / q.w, x = q.y + i % q.w;
    if (y >= 0 && y < H && x >= 0 && x < W) mask[(size_t)y * W + x] = 1;
  }
}

void launch_lost_mask(uint8_t* mask, int H, int W, const int4* rects, int n, hipStream_t s) {
  const size_t total = (size_t)H * W;
  hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, mask,
                     total, (uint8_t)0);
  if (n > 0) hipLaunchKernelGGL(k_mark_rects, dim3(n), dim3(256), 0, s, mask, H, W, rects, n);
}

}  // namespace sefase
