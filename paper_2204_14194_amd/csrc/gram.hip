// Table generation (Algorithm 2) support kernels: the diagonal C_(k,k) of
// eq. 16, D_k = 1/sqrt(C_(k,k)) of eq. 17, and the scaled dictionary
// Y[k][p] = D_k sqrt(w_p) phi_k[p] from which both the Gram matrix
// (G = Y Y^T, computed by the GEMM in gemm.hip) and the initial projections
// (eq. 12) are formed.
#include "bf16.h"
#include "se_internal.h"

namespace sefase {

// One wavefront per atom.  Lane l sums pixels l, l+64, l+128, ... in order,
// then the 64 partials are combined by a fixed butterfly.  The order depends
// only on the pixel index, never on the atom's position, so bit-identical
// atoms get bit-identical sums.
// A complex dictionary (phi_im non-NULL) sums |phi|^2 w = (re^2 + im^2) w.
__global__ __launch_bounds__(256) void k_diag(const float* __restrict__ phi,
                                              const float* __restrict__ phi_im,
                                              const float* __restrict__ w, int K, int P,
                                              float* __restrict__ diag32,
                                              double* __restrict__ diag64) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= K) return;
  const float* row = phi + (size_t)k * P;
  float s32 = 0.0f;
  double s64 = 0.0;
  for (int p = lane; p < P; p += 64) {
    const float v = row[p];
    const float wp = w[p];
    s32 = fmaf(v * wp, v, s32);
    s64 = fma((double)v * (double)wp, (double)v, s64);
    if (phi_im) {
      const float vi = phi_im[(size_t)k * P + p];
      s32 = fmaf(vi * wp, vi, s32);
      s64 = fma((double)vi * (double)wp, (double)vi, s64);
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    s32 += __shfl_xor(s32, off);
    s64 += __shfl_xor(s64, off);
  }
  if (lane == 0) {
    diag32[k] = s32;
    diag64[k] = s64;
  }
}

// Single workgroup.  Decides FP32 vs FP64 for the diagonal (mode 0: FP64
// when min/max over positive C_kk < 1e-3 or force64), writes D_k (0 for a
// non-positive diagonal), sqrt(w) and the info word.
__global__ __launch_bounds__(1024) void k_finalize_d(const float* __restrict__ diag32,
                                                     const double* __restrict__ diag64,
                                                     const float* __restrict__ w, int K, int P,
                                                     int mode, int force64, float* __restrict__ D,
                                                     float* __restrict__ sqrtw,
                                                     int32_t* __restrict__ info) {
  __shared__ double smin[16], smax[16];
  __shared__ int use64;
  const int tid = threadIdx.x;
  double lo = 1.0e300, hi = 0.0;
  for (int k = tid; k < K; k += blockDim.x) {
    const double d = diag64[k];
    if (d > 0.0) {
      lo = fmin(lo, d);
      hi = fmax(hi, d);
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off));
    hi = fmax(hi, __shfl_xor(hi, off));
  }
  if ((tid & 63) == 0) {
    smin[tid >> 6] = lo;
    smax[tid >> 6] = hi;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 1.0e300, b = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      a = fmin(a, smin[i]);
      b = fmax(b, smax[i]);
    }
    int u;
    if (mode == 1) u = 1;
    else if (mode == 2) u = 0;
    else u = (force64 || (b > 0.0 && a / b < 1.0e-3)) ? 1 : 0;
    use64 = u;
    if (info) info[0] = u;
  }
  __syncthreads();
  const int u = use64;
  for (int k = tid; k < K; k += blockDim.x) {
    const double d = u ? diag64[k] : (double)diag32[k];
    D[k] = d > 0.0 ? (float)(1.0 / sqrt(d)) : 0.0f;
  }
  for (int p = tid; p < P; p += blockDim.x) sqrtw[p] = sqrtf(fmaxf(w[p], 0.0f));
}

// neg: the imaginary rows of a complex dictionary, Y = D sqrt(w) conj(phi)
__global__ void k_scale_y(const float* __restrict__ phi, const float* __restrict__ D,
                          const float* __restrict__ sqrtw, int K, int P, bool neg,
                          float* __restrict__ Y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)K * P) return;
  const int k = (int)(i / P);
  const int p = (int)(i - (long long)k * P);
  const float v = D[k] * (sqrtw[p] * phi[i]);
  Y[i] = neg ? -v : v;
}

// The Hermitian table of a complex dictionary from S = Z Z^T, Z = [A; B]
// the real and imaginary rows of Y = D sqrt(w) conj(phi) (2K x P):
//   G = Y Y^H:  Re G[k][l] = S[k][l] + S[K+k][K+l],
//               Im G[k][l] = S[K+k][l] - S[k][K+l].
__global__ void k_combine_c(const float* __restrict__ S, int ldS, int K,
                            float* __restrict__ G, float* __restrict__ G_im, int ldG) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (l >= K) return;
  const float* top = S + (size_t)k * ldS;
  const float* bot = S + (size_t)(K + k) * ldS;
  G[(size_t)k * ldG + l] = top[l] + bot[K + l];
  G_im[(size_t)k * ldG + l] = bot[l] - top[K + l];
}

__global__ void k_split_bf16(const float* __restrict__ x, size_t n, uint16_t* __restrict__ hi,
                             uint16_t* __restrict__ lo) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint16_t h, l;
  bf16_split(x[i], h, l);
  hi[i] = h;
  lo[i] = l;
}

__global__ void k_zero_cols(float* __restrict__ A, int rows, int c0, int ld) {
  const int w = ld - c0;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)rows * w) return;
  const int r = (int)(i / w);
  A[(size_t)r * ld + c0 + (int)(i - (long long)r * w)] = 0.0f;
}

__global__ void k_zero_range(float* __restrict__ A, int rows, int ld, int c0, int c1) {
  const int w = c1 - c0;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)rows * w) return;
  const int r = (int)(i / w);
  A[(size_t)r * ld + c0 + (int)(i - (long long)r * w)] = 0.0f;
}

void launch_zero_range(float* A, int rows, int ld, int c0, int c1, hipStream_t s) {
  const long long total = (long long)rows * (c1 - c0);
  if (total <= 0) return;
  hipLaunchKernelGGL(k_zero_range, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, A, rows,
                     ld, c0, c1);
}

void launch_zero_cols(float* A, int rows, int c0, int ld, hipStream_t s) {
  const long long total = (long long)rows * (ld - c0);
  if (total <= 0) return;
  hipLaunchKernelGGL(k_zero_cols, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, A, rows,
                     c0, ld);
}

void launch_diag(const float* phi, const float* phi_im, const float* w, int K, int P,
                 float* diag32, double* diag64, hipStream_t s) {
  hipLaunchKernelGGL(k_diag, dim3((K + 3) / 4), dim3(256), 0, s, phi, phi_im, w, K, P, diag32,
                     diag64);
}

void launch_combine_c(const float* S, int ldS, int K, float* G, float* G_im, int ldG,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_combine_c, dim3((K + 255) / 256, K), dim3(256), 0, s, S, ldS, K, G, G_im,
                     ldG);
}

void launch_finalize_d(const float* diag32, const double* diag64, const float* w, int K, int P,
                       int mode, int force64, float* D, float* sqrtw, int32_t* info,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_d, dim3(1), dim3(1024), 0, s, diag32, diag64, w, K, P, mode,
                     force64, D, sqrtw, info);
}

void launch_scale_y(const float* phi, const float* D, const float* sqrtw, int K, int P, float* Y,
                    hipStream_t s, bool neg) {
  const long long total = (long long)K * P;
  hipLaunchKernelGGL(k_scale_y, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, phi, D,
                     sqrtw, K, P, neg, Y);
}

void launch_split_bf16(const float* x, size_t n, uint16_t* hi, uint16_t* lo, hipStream_t s) {
  hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, hi,
                     lo);
}

}  // namespace sefase
