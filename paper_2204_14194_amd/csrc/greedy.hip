// The iteration loop of Fast Selective Extrapolation (Algorithm 3), one
// workgroup per lost block, from initial projections in device memory; the
// loop itself is greedy_block (greedy_device.h).
#include "greedy_device.h"

namespace sefase {

// ONE: the launch conceals the single block a.blk0 (plain per-block form); a
// separate instantiation so profiles keep the two forms apart.  Q16: the
// rows are the fixed-point words a.Gqr.
template <int WAVES, int VPL, bool ONE, bool Q16>
__global__ __launch_bounds__(64 * WAVES) void k_greedy(GreedyArgs a) {
  constexpr int T = 64 * WAVES;
  constexpr int NJ = VPL / 4;
  const int t = threadIdx.x;
  // R~^(0), rows padded with zeros to T * VPL
  float R[NJ][4];
  const float* src = a.R0 + (size_t)blockIdx.x * a.ldR;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const float4 v = *reinterpret_cast<const float4*>(src + 4 * (j * T + t));
    R[j][0] = v.x; R[j][1] = v.y; R[j][2] = v.z; R[j][3] = v.w;
  }
  greedy_block<WAVES, VPL, false, Q16>(a, ONE ? a.blk0 : (int)blockIdx.x, R);
}

// Workgroup shapes: (waves, values per lane).  The capacity 64 * waves * vpl
// is the padded row length.
struct LoopShape {
  int waves, vpl;
};
static const LoopShape kShapes[] = {
    {1, 8}, {1, 16}, {1, 24}, {1, 32}, {2, 8}, {2, 16}, {2, 24}, {2, 32}, {4, 8}, {4, 16},
    {4, 24}, {4, 32}, {8, 8}, {8, 16}, {8, 24}, {8, 32}, {16, 24}, {16, 32},
};
// The default shape for K: the smallest capacity >= K, then the fewest waves.
// Only shapes with 24 or 32 values per lane are defaults; the others share
// their capacity with a default and are alternatives for the tuner.
static LoopShape default_shape(int K) {
  LoopShape best{0, 0};
  long long cap_best = 1LL << 40;
  for (const LoopShape& s : kShapes) {
    if (s.vpl < 24 && !(s.waves == 1)) continue;
    const long long cap = 64LL * s.waves * s.vpl;
    if (cap >= K && (cap < cap_best || (cap == cap_best && s.waves < best.waves))) {
      best = s;
      cap_best = cap;
    }
  }
  return best;
}

int greedy_waves_for(int K) { return default_shape(K).waves; }

int greedy_row_len(int K) {
  const LoopShape s = default_shape(K);
  return 64 * s.waves * s.vpl;
}

int greedy_shapes_for(int K, int* waves, int* vpl, int cap) {
  const int len = greedy_row_len(K);
  int n = 0;
  for (const LoopShape& s : kShapes)
    if (64 * s.waves * s.vpl == len && n < cap) {
      waves[n] = s.waves;
      vpl[n] = s.vpl;
      ++n;
    }
  return n;
}

template <int W, int V>
static void launch_shape(const GreedyArgs& a, int grid, hipStream_t s) {
  const bool q = a.Gqr != nullptr;
  if (grid == 1 && a.blk0 >= 0) {
    if (q)
      hipLaunchKernelGGL((k_greedy<W, V, true, true>), dim3(1), dim3(64 * W), 0, s, a);
    else
      hipLaunchKernelGGL((k_greedy<W, V, true, false>), dim3(1), dim3(64 * W), 0, s, a);
  } else if (q) {
    hipLaunchKernelGGL((k_greedy<W, V, false, true>), dim3(grid), dim3(64 * W), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_greedy<W, V, false, false>), dim3(grid), dim3(64 * W), 0, s, a);
  }
}

se_status launch_greedy(const GreedyArgs& a, int grid, hipStream_t s, int waves, int vpl) {
  if (grid <= 0) return SE_OK;
  LoopShape sh = default_shape(a.K);
  if (sh.waves == 0) return fail(SE_EINVAL, "K=%d exceeds the largest loop configuration", a.K);
  if (waves > 0) {
    if (64 * waves * vpl != 64 * sh.waves * sh.vpl)
      return fail(SE_EINVAL, "loop shape %dx%d does not match the row length of K=%d", waves,
                  vpl, a.K);
    sh = LoopShape{waves, vpl};
  }
  const int cap = 64 * sh.waves * sh.vpl;
  if (a.ldG < cap || a.ldR < cap)
    return fail(SE_EINVAL, "row strides (ldG=%d, ldR=%d) below the padded length %d", a.ldG,
                a.ldR, cap);
  switch (sh.waves * 100 + sh.vpl) {
    case 108: launch_shape<1, 8>(a, grid, s); break;
    case 116: launch_shape<1, 16>(a, grid, s); break;
    case 124: launch_shape<1, 24>(a, grid, s); break;
    case 132: launch_shape<1, 32>(a, grid, s); break;
    case 208: launch_shape<2, 8>(a, grid, s); break;
    case 216: launch_shape<2, 16>(a, grid, s); break;
    case 224: launch_shape<2, 24>(a, grid, s); break;
    case 232: launch_shape<2, 32>(a, grid, s); break;
    case 408: launch_shape<4, 8>(a, grid, s); break;
    case 416: launch_shape<4, 16>(a, grid, s); break;
    case 424: launch_shape<4, 24>(a, grid, s); break;
    case 432: launch_shape<4, 32>(a, grid, s); break;
    case 808: launch_shape<8, 8>(a, grid, s); break;
    case 816: launch_shape<8, 16>(a, grid, s); break;
    case 824: launch_shape<8, 24>(a, grid, s); break;
    case 832: launch_shape<8, 32>(a, grid, s); break;
    case 1624: launch_shape<16, 24>(a, grid, s); break;
    case 1632: launch_shape<16, 32>(a, grid, s); break;
    default: return fail(SE_EINVAL, "no loop shape for K=%d", a.K);
  }
  return check_launch("greedy");
}

}  // namespace sefase
