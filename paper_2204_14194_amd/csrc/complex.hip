// Algorithm 3 for a complex dictionary (the paper's general case, Sections
// II-III): R, the table G = D C D (Hermitian) and the coefficients are
// complex; the image is real and the real part of the model replaces the
// loss.  With the unit-diagonal table, per iteration
//   u  = argmax_k |R~_k|                        (eq. 18)
//   c  = gamma R~_u D_u                         (eq. 19)
//   R~_k -= gamma R~_u G[k][u],  G[k][u] = conj(G[u][k])   (eq. 20)
//   g  += c phi_u over the loss (real part)     (eq. 9)
// One workgroup per block.  Lane t holds atoms 4 (j T + t) + e as in the
// real loop, with separate real and imaginary registers; the rows of Re G
// and Im G are streamed as float4 sweeps.  The selection compares |R~|^2
// (same order as |R~|) as the real loop compares |R~|: a DPP wave maximum,
// a scalar scan of the one holding lane (or, for exact ties across lanes,
// 64-bit (|R~|^2, lowest index) keys), and across waves the keys through
// LDS, the winner's complex value travelling with its key.
#include "argmax.h"
#include "se_internal.h"

namespace sefase {

constexpr int kCQPL = 4;   // loss pixels per lane (the loss may hold <= 4 T pixels)

struct CplxArgs {
  const float* G_im;     // K x ldG, Im G
  const float* phi_im;   // K x M*N, Im phi
};

template <int WAVES, int VPL>
__global__ __launch_bounds__(64 * WAVES) void k_greedy_c(GreedyArgs a, CplxArgs x) {
  constexpr int T = 64 * WAVES;
  constexpr int NJ = VPL / 4;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int b = blockIdx.x;
  const DevBlock d = a.blk[b];
  const int K = a.K, P = a.P;
  const int L = a.ldR / 2;   // R row: real parts at [0, L), imaginary at [L, 2 L)

  float Rr[NJ][4], Ri[NJ][4];
  {
    const float* src = a.R0 + (size_t)b * a.ldR;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const float4 v = *reinterpret_cast<const float4*>(src + 4 * (j * T + t));
      const float4 u = *reinterpret_cast<const float4*>(src + L + 4 * (j * T + t));
      Rr[j][0] = v.x; Rr[j][1] = v.y; Rr[j][2] = v.z; Rr[j][3] = v.w;
      Ri[j][0] = u.x; Ri[j][1] = u.y; Ri[j][2] = u.z; Ri[j][3] = u.w;
    }
  }

  // loss pixels owned by this lane (lanes past the end repeat the last one)
  const int nloss = d.ld * d.lh * d.lw;
  const int nq = (nloss + T - 1) / T;
  int poff[kCQPL];
  float g[kCQPL], gc[kCQPL];
#pragma unroll
  for (int q = 0; q < kCQPL; ++q) {
    int i = t + q * T;
    i = i < nloss ? i : nloss - 1;
    poff[q] = loss_sample(d, i, a.M, a.N).off;
    g[q] = 0.0f;
    gc[q] = 0.0f;
  }

  // a block with nothing to extrapolate from (no available sample, or every
  // atom of zero weighted norm): sel = -1, coefficients and model 0, the loss
  // left as it is (as in the real loop)
  {
    bool deg = (d.geom & kBlockNoSupport) != 0;
    if (!deg) {
      bool nz = false;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) nz = nz || Rr[j][e] != 0.0f || Ri[j][e] != 0.0f;
      if (!any_in_workgroup<WAVES>(nz)) {
        bool dnz = false;
        for (int j = 0; j < NJ; ++j)
          for (int e = 0; e < 4; ++e) {
            const int k = 4 * (j * T + t) + e;
            if (k < K) dnz = dnz || a.D[k] != 0.0f;
          }
        deg = !any_in_workgroup<WAVES>(dnz);
      }
    }
    if (deg) {
      degenerate_outputs(a.sel, a.coef, 2, a.g_loss, a.g_loss_ld, a.iters, nloss, b, t, T,
                         a.n_degenerate);
      return;
    }
  }

  __shared__ uint64_t s_key[2][WAVES];
  __shared__ float s_val[2][WAVES][2];
  int par = 0;
  const float gamma = a.gamma;

  for (int it = 0; it < a.iters; ++it) {
    // ---- the wave's largest |R~|^2 and its lowest index ----------------------
    // Group maxima (4 atoms each) and the lane maximum, then the wave
    // maximum by DPP.  When one lane alone holds it, that lane's group
    // maxima and then the complex values of its first matching group are
    // read into scalar registers and scanned (lowest index first); several
    // holding lanes (exact ties) take the key reduction.
    float gm[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      float m[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) m[e] = fmaf(Rr[j][e], Rr[j][e], Ri[j][e] * Ri[j][e]);
      gm[j] = fmaxf(fmaxf(m[0], m[1]), fmaxf(m[2], m[3]));
    }
    float lm = gm[0];
#pragma unroll
    for (int j = 1; j < NJ; ++j) lm = fmaxf(lm, gm[j]);
    const float Mx = wave_max_f32(lm);
    const uint64_t holders = __builtin_amdgcn_ballot_w64(lm == Mx);
    uint64_t key = 0;                          // every score zero: atom 0, value 0
    float vre = 0.0f, vim = 0.0f;
    if (Mx != 0.0f && __builtin_popcountll(holders) == 1) {
      const int L = __builtin_ctzll(holders);
      const uint32_t Mb = __float_as_uint(Mx);
      int gsel = NJ - 1;
#pragma unroll
      for (int j = NJ - 2; j >= 0; --j)
        gsel = (uint32_t)__builtin_amdgcn_readlane(__float_as_int(gm[j]), L) == Mb ? j : gsel;
      float re[4] = {0.0f, 0.0f, 0.0f, 0.0f}, im[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if (j == gsel) {                       // uniform branch
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            re[e] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Rr[j][e]), L));
            im[e] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Ri[j][e]), L));
          }
        }
      // the same expression as the lane's own, so the winner compares equal
      int csel = 3;
#pragma unroll
      for (int e = 2; e >= 0; --e)
        csel = __float_as_uint(fmaf(re[e], re[e], im[e] * im[e])) == Mb ? e : csel;
      vre = csel == 0 ? re[0] : csel == 1 ? re[1] : csel == 2 ? re[2] : re[3];
      vim = csel == 0 ? im[0] : csel == 1 ? im[1] : csel == 2 ? im[2] : im[3];
      key = make_key(Mx, 4 * (gsel * T + wave * 64 + L) + csel);
    } else if (Mx != 0.0f) {
      // exact ties across lanes: every lane's first maximum as a key; the
      // owner of the wave's winner holds its complex value
      float bm = 0.0f, bre = 0.0f, bim = 0.0f;
      int bc = 0;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float m2 = fmaf(Rr[j][e], Rr[j][e], Ri[j][e] * Ri[j][e]);
          if (m2 > bm) {
            bm = m2;
            bre = Rr[j][e];
            bim = Ri[j][e];
            bc = 4 * j + e;
          }
        }
      const uint64_t mine = make_key(bm, 4 * ((bc >> 2) * T + t) + (bc & 3));
      key = wave_max_key((uint32_t)(mine >> 32), (uint32_t)mine);
      const int kw = 0xFFFF - (int)((uint32_t)key >> 16);
      const int owner = ((kw >> 2) % T) & 63;
      vre = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bre), owner));
      vim = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bim), owner));
    }
    if (WAVES > 1) {
      if (lane == 0) {
        s_key[par][wave] = key;
        s_val[par][wave][0] = vre;
        s_val[par][wave][1] = vim;
      }
      __syncthreads();
      int win = 0;
      key = s_key[par][0];
#pragma unroll
      for (int w = 1; w < WAVES; ++w) {
        const uint64_t o = s_key[par][w];
        if (o > key) {
          key = o;
          win = w;
        }
      }
      vre = s_val[par][win][0];
      vim = s_val[par][win][1];
      par ^= 1;
    }
    int u;
    float mag2;
    decode_key(key, K, u, mag2);
    if (mag2 == 0.0f) {
      vre = 0.0f;
      vim = 0.0f;
    }
    u = __builtin_amdgcn_readfirstlane(u);
    const float tr = gamma * __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(vre)));
    const float ti = gamma * __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(vim)));

    // ---- rows u of Re G and Im G, the atom over the loss ---------------------
    const float* pr = a.phi + (size_t)u * P;
    const float* pi = x.phi_im + (size_t)u * P;
    float pvr[kCQPL], pvi[kCQPL];
#pragma unroll
    for (int q = 0; q < kCQPL; ++q)
      if (q < nq) {
        pvr[q] = pr[poff[q]];
        pvi[q] = pi[poff[q]];
      }
    const float* gr = a.G + (size_t)u * a.ldG;
    const float* gi = x.G_im + (size_t)u * a.ldG;
    float4 rr[NJ], ri[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      rr[j] = *reinterpret_cast<const float4*>(gr + 4 * (j * T + t));
      ri[j] = *reinterpret_cast<const float4*>(gi + 4 * (j * T + t));
    }
    const float Du = a.D[u];
    const float cr = tr * Du, ci = ti * Du;      // eq. 19
    if (t == 0) {
      if (a.sel) a.sel[(size_t)b * a.iters + it] = u;
      if (a.coef) {
        a.coef[((size_t)b * a.iters + it) * 2] = cr;
        a.coef[((size_t)b * a.iters + it) * 2 + 1] = ci;
      }
    }
#pragma unroll
    for (int q = 0; q < kCQPL; ++q)
      if (q < nq) {                              // eq. 9, real part, compensated
        const float y = fmaf(cr, pvr[q], -fmaf(ci, pvi[q], gc[q]));
        const float s = g[q] + y;
        gc[q] = (s - g[q]) - y;
        g[q] = s;
        asm volatile("" ::: "memory");
      }

    // ---- eq. 20: R~_k -= (tr + j ti) (Re G[u][k] - j Im G[u][k]) --------------
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const float xr[4] = {rr[j].x, rr[j].y, rr[j].z, rr[j].w};
      const float xi[4] = {ri[j].x, ri[j].y, ri[j].z, ri[j].w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        Rr[j][e] = fmaf(-ti, xi[e], fmaf(-tr, xr[e], Rr[j][e]));
        Ri[j][e] = fmaf(tr, xi[e], fmaf(-ti, xr[e], Ri[j][e]));
      }
    }
  }

  // ---- replace the loss by the model's real part ------------------------------
#pragma unroll
  for (int q = 0; q < kCQPL; ++q) {
    const int i = t + q * T;
    if (i >= nloss) continue;
    if (a.g_loss && i < a.g_loss_ld) a.g_loss[(size_t)b * a.g_loss_ld + i] = g[q];
    const LossSample ls = loss_sample(d, i, a.M, a.N);
    if (ls.y >= 0 && ls.y < a.H && ls.x >= 0 && ls.x < a.W) {
      const float v = fminf(fmaxf(rintf(g[q]), 0.0f), 255.0f);
      a.images[(size_t)ls.frame * a.H * a.W + (size_t)ls.y * a.W + ls.x] = (uint8_t)v;
    }
  }
}

// Shapes (waves, complex atoms per lane) with the row lengths of the real
// loop, so a complex table has the same padded rows.
struct CShape {
  int waves, vpl;
};
static const CShape kCShapes[] = {{1, 8},  {1, 16}, {1, 32}, {2, 12}, {2, 16},  {4, 12},
                                  {4, 16}, {8, 12}, {8, 16}, {16, 12}, {16, 16}};

bool complex_loop_for(int K) {
  const int cap = greedy_row_len(K);
  for (const CShape& c : kCShapes)
    if (64 * c.waves * c.vpl == cap) return true;
  return false;
}

se_status launch_greedy_c(const GreedyArgs& a, const float* G_im, const float* phi_im, int grid,
                          hipStream_t s) {
  if (grid <= 0) return SE_OK;
  const int cap = greedy_row_len(a.K);
  CShape sh{0, 0};
  for (const CShape& c : kCShapes)
    if (64 * c.waves * c.vpl == cap) {
      sh = c;
      break;
    }
  if (sh.waves == 0) return fail(SE_EINVAL, "no complex loop shape for K=%d", a.K);
  if (a.ldG < cap || a.ldR < 2 * cap)
    return fail(SE_EINVAL, "row strides (ldG=%d, ldR=%d) below %d and %d", a.ldG, a.ldR, cap,
                2 * cap);
  const CplxArgs x{G_im, phi_im};
  switch (sh.waves * 100 + sh.vpl) {
#define SE_C_CASE(w, v)                                                                  \
  case w * 100 + v:                                                                      \
    hipLaunchKernelGGL((k_greedy_c<w, v>), dim3(grid), dim3(64 * w), 0, s, a, x); \
    break;
    SE_C_CASE(1, 8) SE_C_CASE(1, 16) SE_C_CASE(1, 32) SE_C_CASE(2, 12) SE_C_CASE(2, 16) SE_C_CASE(4, 12)
    SE_C_CASE(4, 16) SE_C_CASE(8, 12) SE_C_CASE(8, 16) SE_C_CASE(16, 12) SE_C_CASE(16, 16)
#undef SE_C_CASE
    default: return fail(SE_EINVAL, "no complex loop shape for K=%d", a.K);
  }
  return check_launch("greedy_c");
}

}  // namespace sefase
