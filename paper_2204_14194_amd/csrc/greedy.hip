// The iteration loop of Fast Selective Extrapolation (Algorithm 3), one
// workgroup per lost block.
//
// State: the K weighted scalar products R_k (eq. 11) live in registers,
// VPL per lane, in units of D_k (R~_k = D_k R_k; the initial values come
// from the projection GEMM).  With the unit-diagonal table
// G[k][l] = D_k C_(k,l) D_l the three per-iteration formulas become
//   u  = argmax_k |R~_k|                       (eq. 18: |R_k| D_k = |R~_k|)
//   c  = gamma R~_u D_u                        (eq. 19: gamma R_u D_u^2)
//   R~_k -= gamma R~_u G[u][k]  for all k      (eq. 20 scaled by D_k, using
//                                               C symmetric: row u = column u)
// and the model update g += c phi_u (eq. 9) is applied to the loss pixels
// only, in registers, every iteration (the rest of g is never used).
//
// Atom ownership: lane t of the workgroup (T = 64 * WAVES lanes) holds atoms
// 4 (j T + t) + e, j < VPL/4, e < 4, so every row load is a coalesced float4
// sweep and a lane's atoms increase with (j, e).  Ties: the scan keeps the
// first maximum of a lane, the cross-lane reduction prefers the lower index,
// so exact ties go to the lowest atom index.
#include "se_internal.h"

namespace sefase {

constexpr int kQPL = 4;   // loss pixels per lane (the loss may hold <= 4 T pixels)

__device__ inline void better(float& bv, int& bi, float ov, int oi) {
  const float a = fabsf(ov), c = fabsf(bv);
  if (a > c || (a == c && oi < bi)) {
    bv = ov;
    bi = oi;
  }
}

template <int WAVES, int VPL>
__global__ __launch_bounds__(64 * WAVES) void k_greedy(GreedyArgs a) {
  constexpr int T = 64 * WAVES;
  constexpr int NJ = VPL / 4;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int b = a.blk0 + (int)blockIdx.x;
  const DevBlock d = a.blk[b];
  const int K = a.K, P = a.M * a.N;

  // ---- load R~^(0) --------------------------------------------------------
  float R[NJ][4];
  {
    const float* src = a.R0 + (size_t)blockIdx.x * a.ldR;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int idx = 4 * (j * T + t);
      if (idx + 3 < K) {
        const float4 v = *reinterpret_cast<const float4*>(src + idx);
        R[j][0] = v.x; R[j][1] = v.y; R[j][2] = v.z; R[j][3] = v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) R[j][e] = (idx + e < K) ? src[idx + e] : 0.0f;
      }
    }
  }

  // ---- loss pixels owned by this lane ----------------------------------
  const int nloss = d.lh * d.lw;
  int poff[kQPL];
  float g[kQPL];
#pragma unroll
  for (int q = 0; q < kQPL; ++q) {
    const int i = t + q * T;
    g[q] = 0.0f;
    poff[q] = -1;
    if (i < nloss) {
      const int my = i / d.lw, mx = i - my * d.lw;
      poff[q] = (d.ly + my) * a.N + d.lx + mx;
    }
  }

  __shared__ float s_val[2][WAVES];
  __shared__ int s_idx[2][WAVES];
  int par = 0;

  // local candidate of the initial state
  float bv = 0.0f;
  int bi = 0x7fffffff;
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (fabsf(R[j][e]) > fabsf(bv)) {
        bv = R[j][e];
        bi = 4 * (j * T + t) + e;
      }

  const float gamma = a.gamma;
  for (int it = 0; it < a.iters; ++it) {
    // ---- argmax over the workgroup --------------------------------------
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const float ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      better(bv, bi, ov, oi);
    }
    if (WAVES > 1) {
      if (lane == 0) {
        s_val[par][wave] = bv;
        s_idx[par][wave] = bi;
      }
      __syncthreads();
      bv = s_val[par][0];
      bi = s_idx[par][0];
#pragma unroll
      for (int w = 1; w < WAVES; ++w) better(bv, bi, s_val[par][w], s_idx[par][w]);
      par ^= 1;
    }
    int u = bi;
    float rv = bv;
    if (u == 0x7fffffff) {   // every score is zero: a no-op iteration on atom 0
      u = 0;
      rv = 0.0f;
    }
    const float tc = gamma * rv;              // coefficient of the unit-norm atom
    const float c = tc * a.D[u];              // eq. 19
    if (t == 0) {
      if (a.sel) a.sel[(size_t)b * a.iters + it] = u;
      if (a.coef) a.coef[(size_t)b * a.iters + it] = c;
    }

    // ---- stream row u of the table and the atom over the loss -------------
    const float* grow = a.G + (size_t)u * a.ldG;
    float row[NJ][4];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int idx = 4 * (j * T + t);
      if (idx + 3 < K) {
        const float4 v = *reinterpret_cast<const float4*>(grow + idx);
        row[j][0] = v.x; row[j][1] = v.y; row[j][2] = v.z; row[j][3] = v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) row[j][e] = (idx + e < K) ? grow[idx + e] : 0.0f;
      }
    }
    const float* prow = a.phi + (size_t)u * P;
#pragma unroll
    for (int q = 0; q < kQPL; ++q)
      if (poff[q] >= 0) g[q] = fmaf(c, prow[poff[q]], g[q]);   // eq. 9

    // ---- eq. 20 and the next local candidate -----------------------------
    bv = 0.0f;
    bi = 0x7fffffff;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        R[j][e] = fmaf(-tc, row[j][e], R[j][e]);
        if (fabsf(R[j][e]) > fabsf(bv)) {
          bv = R[j][e];
          bi = 4 * (j * T + t) + e;
        }
      }
  }

  // ---- replace the loss area by the model ----------------------------------
#pragma unroll
  for (int q = 0; q < kQPL; ++q) {
    const int i = t + q * T;
    if (i >= nloss) continue;
    if (a.g_loss) a.g_loss[(size_t)b * a.g_loss_ld + i] = g[q];
    const int my = i / d.lw, mx = i - my * d.lw;
    const int y = d.y0 + d.ly + my, x = d.x0 + d.lx + mx;
    if (y >= 0 && y < a.H && x >= 0 && x < a.W) {
      const float v = fminf(fmaxf(rintf(g[q]), 0.0f), 255.0f);
      a.images[(size_t)d.img * a.H * a.W + (size_t)y * a.W + x] = (uint8_t)v;
    }
  }
}

int greedy_waves_for(int K) {
  if (K <= 2048) return 1;
  if (K <= 4096) return 2;
  if (K <= 8192) return 4;
  if (K <= 16384) return 8;
  return 0;
}

se_status launch_greedy(const GreedyArgs& a, int grid, hipStream_t s) {
  if (grid <= 0) return SE_OK;
  const int K = a.K;
  if (K <= 512)
    hipLaunchKernelGGL((k_greedy<1, 8>), dim3(grid), dim3(64), 0, s, a);
  else if (K <= 1024)
    hipLaunchKernelGGL((k_greedy<1, 16>), dim3(grid), dim3(64), 0, s, a);
  else if (K <= 2048)
    hipLaunchKernelGGL((k_greedy<1, 32>), dim3(grid), dim3(64), 0, s, a);
  else if (K <= 4096)
    hipLaunchKernelGGL((k_greedy<2, 32>), dim3(grid), dim3(128), 0, s, a);
  else if (K <= 8192)
    hipLaunchKernelGGL((k_greedy<4, 32>), dim3(grid), dim3(256), 0, s, a);
  else if (K <= 16384)
    hipLaunchKernelGGL((k_greedy<8, 32>), dim3(grid), dim3(512), 0, s, a);
  else
    return fail(SE_EINVAL, "K=%d exceeds the largest loop configuration (16384)", K);
  return check_launch("greedy");
}

}  // namespace sefase
