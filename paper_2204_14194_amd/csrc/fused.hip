// Initial projections and the iteration loop in one launch, for tables whose
// every atom lies in a declared transform part (Section VI): each block's
// workgroup computes R~^(0) = D ⊙ T(w s) of its own area on the matrix cores
// (eq. 12 via eq. 22, the scheme of the projection kernel), stages it in LDS
// in the loop's atom order and runs Algorithm 3 from there.  R~^(0) never
// goes to device memory, and no second launch is needed.  The arithmetic of
// both stages is that of the separate kernels, so the results are the same
// bit for bit.
#include "greedy_device.h"
#include "tx_device.h"

namespace sefase {

// LDS (floats): the padded row R~^(0) of T * VPL atoms; before the projection
// writes it, the same space holds the X operands of the waves that compute a
// part (MT * NT * 256 floats each, for areas inside the image on a 16-byte
// grid).
template <int WAVES, int VPL, int MT, int NT, int NP>
constexpr int conceal_lds_floats() {
  constexpr int row = 64 * WAVES * VPL;
  constexpr int xs = (WAVES < NP ? WAVES : NP) * MT * NT * 256;
  return row > xs ? row : xs;
}

// Areas up to 32 x 32: held to four waves per SIMD (128 registers), so the
// compiler keeps the projection stage in vector registers without the
// accumulation registers it would otherwise add (four resident blocks per
// SIMD cover a 4096-block batch at once); larger areas take what they need.
// VOL: areas of several frames, read as their frames stacked (M = T rows of
// frames).  Q16: the class rows as fixed-point words.
template <int WAVES, int VPL, int MT, int NT, int NP, bool CLS, bool VOL, bool Q16>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(MT * NT <= 4 ? 4 : 1)))
void k_conceal_tx(GreedyArgs a, TxArgs x, TxLayout L) {
  constexpr int T = 64 * WAVES;
  constexpr int NJ = VPL / 4;
  extern __shared__ floatx4 smv[];
  float* Rs = reinterpret_cast<float*>(smv);
  const int t = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);   // uniform: operand addresses in SGPRs
  const int b = blockIdx.x;
  const DevBlock d = a.blk[b];
  const int M = L.M, N = L.N;

  // ---- projections: wave q computes part q (a single wave both) -----------
  const bool computes = wave < NP;
  floatx4 xv[MT][NT];
  if (computes) {
    TxPixels<MT, NT> P;
    tx_load<MT, NT, VOL>(x, d, M, N, P);
    tx_x_operands<MT, NT, VOL>(x, d, M, N, P, x.tx + L.oWf, Rs + wave * MT * NT * 256, xv);
  }
  __syncthreads();   // every X operand is in registers: the LDS becomes the row
  // class form on one frame (the launcher's areas have M = 16 MT rows, MT
  // even, and N = 16 NT columns): the vertical stage on the folded rows
  // (tx_fold_rows), and for NT even the horizontal stage on the folded
  // columns too (tx_fold_cols): a quarter of the contraction
  constexpr bool FOLD = CLS && !VOL && MT % 2 == 0;
  if constexpr (FOLD) {
    if (computes) {
      floatx4 xf[2][MT / 2][NT];
      tx_fold_rows<MT, NT>(xv, xf);
      constexpr bool HFOLD = NT % 2 == 0;
      floatx4 xh[2][2][MT / 2][HFOLD ? NT / 2 : 1];
      if constexpr (HFOLD) {
        tx_fold_cols<MT / 2, NT>(xf[0], xh[0]);
        tx_fold_cols<MT / 2, NT>(xf[1], xh[1]);
      }
      const int HV = M / 2, HN = N / 2, Kc = a.K / 4;
#pragma unroll 1
      for (int q = wave; q < NP; q += WAVES) {
        const float* Af = x.tx + L.oAc + q * MT * MT * 256;
        const float* Btf = M == N ? Af : x.tx + L.oBc + q * NT * NT * 256;
        const float* Df = x.tx + L.oDc + q * MT * NT * 256;
        const int qoff = (q ? x.first1 > x.first0 : x.first0 > x.first1) ? HV * HN : 0;
        auto out = [&](int k1, int k2, float v) {
          const int pv = k1 >= HV, ph = k2 >= HN;
          Rs[(2 * pv + ph) * Kc + qoff + (k1 - pv * HV) * HN + k2 - ph * HN] = v;
        };
        if constexpr (HFOLD)
          tx_part_hfold<MT, NT>(Af, Btf, Df, xh, out);
        else
          tx_part_fold<MT, NT>(Af, Btf, Df, xf, out);
      }
    }
  } else if (computes) {
#pragma unroll 1
    for (int q = wave; q < NP; q += WAVES) {
      // a square area of one frame transforms rows and columns with the same
      // matrix, whose two fragment orders then coincide: one copy is read
      if constexpr (CLS) {
        // the class-order operands: the transform's 2 x 2 parity quadrants
        // are the parity classes' atoms of this part in class order, so the
        // output goes straight to its class position (class c = 2 pv + ph
        // in blocks of K / 4; in a class the part with the lower first atom
        // first; in a part row-major over (frame, row / 2, column / 2))
        const float* Af = x.tx + L.oAc + q * MT * MT * 256;
        const float* Btf = M == N && !VOL ? Af : x.tx + L.oBc + q * NT * NT * 256;
        const int HV = M / 2, HN = N / 2, Kc = a.K / 4;
        const int qoff = (q ? x.first1 > x.first0 : x.first0 > x.first1) ? HV * HN : 0;
        tx_part<MT, NT, true>(Af, Btf, x.tx + L.oDc + q * MT * NT * 256, xv, M, N,
                              [&](int k1, int k2, float v) {
                                const int pv = k1 >= HV, ph = k2 >= HN;
                                Rs[(2 * pv + ph) * Kc + qoff + (k1 - pv * HV) * HN + k2 -
                                   ph * HN] = v;
                              });
      } else {
        float* Rq = Rs + (q ? x.first1 : x.first0);
        const float* Af = x.tx + L.oAf + q * MT * MT * 256;
        const float* Btf = M == N ? Af : x.tx + L.oBtf + q * NT * NT * 256;
        tx_part<MT, NT, true>(Af, Btf, x.tx + L.oDf + q * MT * NT * 256, xv, M, N,
                              [&](int k1, int k2, float v) { Rq[k1 * N + k2] = v; });
      }
    }
  }
  for (int k = a.K + t; k < T * VPL; k += T) Rs[k] = 0.0f;   // padding atoms
  __syncthreads();

  // ---- Algorithm 3 from R~^(0) ------------------------------------------------
  // (in the loop's order: atom order, or the class order the class form wrote)
  float R[NJ][4];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const floatx4 v = *reinterpret_cast<const floatx4*>(Rs + 4 * (j * T + t));
    R[j][0] = v[0]; R[j][1] = v[1]; R[j][2] = v[2]; R[j][3] = v[3];
  }
  greedy_block<WAVES, VPL, CLS, Q16>(a, b, R);
}

template <int WAVES, int VPL, int MT, int NT, int NP, bool CLS, bool VOL = false, bool Q16 = false>
static se_status launch_conceal(const GreedyArgs& a, const TxArgs& x, const TxLayout& L, int grid,
                                hipStream_t s) {
  // the class form's folded projection writes whole tiles unchecked
  if (CLS && !VOL && MT % 2 == 0 && (L.M != 16 * MT || L.N != 16 * NT))
    return fail(SE_EINVAL, "folded projection needs whole tiles (%dx%d)", L.M, L.N);
  const size_t lds = (size_t)conceal_lds_floats<WAVES, VPL, MT, NT, NP>() * 4;
  hipLaunchKernelGGL((k_conceal_tx<WAVES, VPL, MT, NT, NP, CLS, VOL, Q16>), dim3(grid),
                     dim3(64 * WAVES), lds, s, a, x, L);
  return check_launch("conceal_tx");
}

// The instantiated combinations: two parts covering every atom of 32 x 32 or
// 64 x 64 areas (K = 2048 or 8192), with every loop shape of that row length,
// and of 64 x 16 (K = 2048) -- also four frames of 16 x 16 stacked.  M is the
// transformed row count (frames x rows).
static int conceal_case(int M, int N, int n_parts) {
  if (n_parts != 2) return 0;
  if (M == N) return M == 32 ? 2 : M == 64 ? 4 : 0;
  return M == 64 && N == 16 ? 5 : 0;
}

bool conceal_tx_supported(const se_tables* t) {
  if (!t || t->n_parts < 1 || !t->tx || conceal_case(tx_rows(t), t->N, t->n_parts) == 0)
    return false;
  int lo[3], hi[3];
  return dense_ranges(t->K, area_samples(t), t->n_parts, t->parts, lo, hi) == 0;
}

se_status conceal_tx(const se_tables* t, const GreedyArgs& a, const uint8_t* images, int H, int W,
                     int n_blk, hipStream_t s, int waves, int vpl) {
  if (n_blk <= 0) return SE_OK;
  if (!conceal_tx_supported(t)) return fail(SE_EINVAL, "no fused projection for these tables");
  // class tables: the class form, at the default shape when the requested
  // one does not hold whole class sweeps
  const bool cls = t->n_classes == 4 && a.Gc && a.cls;
  if (a.Gq && !cls) return fail(SE_EINVAL, "fixed-point rows need class tables");
  if (waves <= 0 || (cls && (vpl / 4) % 4 != 0)) {
    waves = greedy_waves_for(t->K);
    vpl = greedy_row_len(t->K) / (64 * waves);
  }
  if (64 * waves * vpl != greedy_row_len(t->K) || a.ldG < 64 * waves * vpl)
    return fail(SE_EINVAL, "loop shape %dx%d does not match the row length of K=%d", waves, vpl,
                t->K);
  TxArgs x{};
  x.images = images;
  x.H = H;
  x.W = W;
  x.blk = a.blk;
  x.n_blk = n_blk;
  x.K = t->K;
  x.tx = t->tx;
  x.first0 = t->parts[0].first;
  x.first1 = t->n_parts > 1 ? t->parts[1].first : 0;
  // several frames: the loaders that stack them (rows per frame 2^fs)
  const bool vol = area_frames(t->T) > 1;
  x.fs = 0;
  if (vol)
    while ((1 << x.fs) < t->M) ++x.fs;
  const int Mv = tx_rows(t);
  const TxLayout L(Mv, t->N, t->n_parts, 0);
  const int key = conceal_case(Mv, t->N, t->n_parts) * 10000 + waves * 100 + vpl;
  if (cls && a.Gq) {
    switch (key) {
      case 20132: return launch_conceal<1, 32, 2, 2, 2, true, false, true>(a, x, L, n_blk, s);
      case 20216: return launch_conceal<2, 16, 2, 2, 2, true, false, true>(a, x, L, n_blk, s);
      case 40432: return launch_conceal<4, 32, 4, 4, 2, true, false, true>(a, x, L, n_blk, s);
      case 40816: return launch_conceal<8, 16, 4, 4, 2, true, false, true>(a, x, L, n_blk, s);
      case 50132:
        return vol ? launch_conceal<1, 32, 4, 1, 2, true, true, true>(a, x, L, n_blk, s)
                   : launch_conceal<1, 32, 4, 1, 2, true, false, true>(a, x, L, n_blk, s);
      default:
        return fail(SE_EINVAL, "no fixed-point class loop of shape %dx%d for K=%d", waves, vpl,
                    t->K);
    }
  }
  if (cls) {
    switch (key) {
      case 20132: return launch_conceal<1, 32, 2, 2, 2, true>(a, x, L, n_blk, s);
      case 20216: return launch_conceal<2, 16, 2, 2, 2, true>(a, x, L, n_blk, s);
      case 40432: return launch_conceal<4, 32, 4, 4, 2, true>(a, x, L, n_blk, s);
      case 40816: return launch_conceal<8, 16, 4, 4, 2, true>(a, x, L, n_blk, s);
      case 50132:
        return vol ? launch_conceal<1, 32, 4, 1, 2, true, true>(a, x, L, n_blk, s)
                   : launch_conceal<1, 32, 4, 1, 2, true, false>(a, x, L, n_blk, s);
      default: break;   // whole rows
    }
  }
  if (vol) {
    switch (key) {
      case 50132: return launch_conceal<1, 32, 4, 1, 2, false, true>(a, x, L, n_blk, s);
      case 50216: return launch_conceal<2, 16, 4, 1, 2, false, true>(a, x, L, n_blk, s);
      default: return fail(SE_EINVAL, "no fused loop shape %dx%d for K=%d", waves, vpl, t->K);
    }
  }
  switch (key) {
    case 20132: return launch_conceal<1, 32, 2, 2, 2, false>(a, x, L, n_blk, s);
    case 20216: return launch_conceal<2, 16, 2, 2, 2, false>(a, x, L, n_blk, s);
    case 20408: return launch_conceal<4, 8, 2, 2, 2, false>(a, x, L, n_blk, s);
    case 40432: return launch_conceal<4, 32, 4, 4, 2, false>(a, x, L, n_blk, s);
    case 40816: return launch_conceal<8, 16, 4, 4, 2, false>(a, x, L, n_blk, s);
    case 50132: return launch_conceal<1, 32, 4, 1, 2, false>(a, x, L, n_blk, s);
    case 50216: return launch_conceal<2, 16, 4, 1, 2, false>(a, x, L, n_blk, s);
    default: return fail(SE_EINVAL, "no fused loop shape %dx%d for K=%d", waves, vpl, t->K);
  }
}

}  // namespace sefase
