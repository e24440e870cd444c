// Device building blocks of the separable transforms on the matrix cores
// (Section VI, eq. 21-23), shared by the projection, table-row and fused
// kernels.
#pragma once

#include "se_internal.h"

namespace sefase {

// ---------------------------------------------------------------------------
// Separable transform on the FP32 matrix cores (v_mfma_f32_16x16x4f32).
// Areas are padded to Mp = 16 MT rows and Np = 16 NT columns (zeros); one
// wave transforms one block.  With j = l/16 the lane's group of 16:
//   stage 1   Y1 = X B^T   tile (i, c), k-steps (sq, t): the k index j
//             stands for column n = 16 sq + 4 j + t, so a lane's four
//             t-values are four adjacent pixels of one row.  A-operand
//             X[16i + l%16][n], B-operand B[16c + l%16][n]; lane l then
//             holds Y1[16i + 4j + e][16c + l%16], e < 4
//   stage 2   Z = A Y1     tile (r, c): the stage-1 registers serve as the
//             B-operands unchanged, k-step (i, e) standing for the rows
//             m = 16i + 4j + e, with the A-operand A[16r + l%16][m]; lane l
//             then holds Z[16r + 4j + e][16c + l%16]
// (both sums run in a permuted order, so nothing moves between the
// stages).  Operands are stored in fragment order -- lane l's four
// consecutive floats at (tile * 64 + l) * 4, one conflict-free
// ds_read_b128 each.  The constant operands (se_tables.tx, written once
// by se_weighted_gram, copied to LDS by every workgroup):
//   Af [part][r][i]  [l][e]  A[16r + l%16][16i + 4j + e]
//   Btf[part][c][sq] [l][t]  B[16c + l%16][16sq + 4j + t]
//   Df [part][c][r]  [l][e]  D_k of output (16r + 4j + e, 16c + l%16)
//   Wf [i][sq]       [l][t]  w of pixel (16i + l%16, 16sq + 4j + t)
// and per wave in LDS, the block's X = w s in the order of Wf (Xf).
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct TxLayout {
  int M, N, MT, NT, parts, waves;
  // offsets in floats; [0, nconst) is the copy of se_tables.tx.  Each wave
  // owns wsz floats at oXf: its X fragments, and with staging (zs > 0) one
  // part's M x N output at row stride zs.  With two parts, se_tables.tx
  // continues after nconst with the class-order operands (oAc, oBc, oDc, up
  // to ntotal): A, B and D of both parts with their rows sorted by (parity,
  // frame, row / 2), so that each 2 x 2 parity quadrant of a transform is
  // one parity class's atoms of the part in class order (read from device
  // memory by the one-launch class kernel only, never copied to LDS).
  int oAf, oBtf, oDf, oWf, nconst, oXf, zs, wsz, nfloat;
  int oAc, oBc, oDc, ntotal;
  __host__ __device__ TxLayout(int M_, int N_, int parts_, int waves_, bool stage = false)
      : M(M_), N(N_), parts(parts_), waves(waves_) {
    MT = (M + 15) / 16;
    NT = (N + 15) / 16;
    oAf = 0;
    oBtf = oAf + parts * MT * MT * 256;
    oDf = oBtf + parts * NT * NT * 256;
    oWf = oDf + parts * MT * NT * 256;
    nconst = oWf + MT * NT * 256;
    oAc = nconst;
    oBc = oAc + (parts == 2 ? 2 * MT * MT * 256 : 0);
    oDc = oBc + (parts == 2 ? 2 * NT * NT * 256 : 0);
    ntotal = oDc + (parts == 2 ? 2 * MT * NT * 256 : 0);
    oXf = nconst;
    zs = stage ? N + 4 : 0;
    wsz = MT * NT * 256 > M * zs ? MT * NT * 256 : M * zs;
    nfloat = oXf + waves * wsz;
  }
  __host__ __device__ size_t bytes() const { return (size_t)nfloat * 4; }
};

// Column tiles c0 .. c0 + CP - 1 of Z = A X B^T for one part, from the X
// operands x (registers, x[i][sq][t] as above); the CP tiles share the X and
// A operands and run as independent accumulation chains.  out(k1, k2, v)
// for every k1 < M, k2 < N of those tiles, v = D_k z when SCALE (Df read),
// else z.
template <int MT, int NT, int CP, bool SCALE, typename Out>
__device__ inline void tx_cols(int c0, const float* Af, const float* Btf, const float* Df,
                               const floatx4 (&x)[MT][NT], int M, int N, Out& out) {
  const int l = threadIdx.x & 63;
  floatx4 y[CP][MT];
#pragma unroll
  for (int cc = 0; cc < CP; ++cc)
#pragma unroll
    for (int i = 0; i < MT; ++i) y[cc][i] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int sq = 0; sq < NT; ++sq) {
    floatx4 bv[CP];
#pragma unroll
    for (int cc = 0; cc < CP; ++cc)
      bv[cc] = *reinterpret_cast<const floatx4*>(Btf + (((c0 + cc) * NT + sq) * 64 + l) * 4);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int cc = 0; cc < CP; ++cc)
#pragma unroll
        for (int i = 0; i < MT; ++i)
          y[cc][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[i][sq][t], bv[cc][t], y[cc][i], 0, 0, 0);
  }
  floatx4 z[CP][MT];
#pragma unroll
  for (int cc = 0; cc < CP; ++cc)
#pragma unroll
    for (int r = 0; r < MT; ++r) z[cc][r] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    floatx4 av[MT];
#pragma unroll
    for (int r = 0; r < MT; ++r)
      av[r] = *reinterpret_cast<const floatx4*>(Af + ((r * MT + i) * 64 + l) * 4);
    // consecutive products go to different accumulators
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int cc = 0; cc < CP; ++cc)
#pragma unroll
        for (int r = 0; r < MT; ++r)
          z[cc][r] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r][e], y[cc][i][e], z[cc][r], 0, 0, 0);
  }
#pragma unroll
  for (int cc = 0; cc < CP; ++cc) {
    const int c = c0 + cc, k2 = 16 * c + (l & 15);
#pragma unroll
    for (int r = 0; r < MT; ++r) {
      floatx4 dv = floatx4{1.f, 1.f, 1.f, 1.f};
      if (SCALE) dv = *reinterpret_cast<const floatx4*>(Df + ((c * MT + r) * 64 + l) * 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k1 = 16 * r + 4 * (l >> 4) + e;
        if (k1 < M && k2 < N) out(k1, k2, dv[e] * z[cc][r][e]);
      }
    }
  }
}

// Z = A X B^T of one part (operand fragments of that part), two column
// tiles per pass.
template <int MT, int NT, bool SCALE, typename Out>
__device__ void tx_part(const float* Af, const float* Btf, const float* Df,
                        const floatx4 (&x)[MT][NT], int M, int N, Out out) {
#pragma unroll 1
  for (int c0 = 0; c0 + 1 < NT; c0 += 2) {
    // re-read the A operands per pass instead of holding them in registers
    // across the loop: an offset the compiler cannot see through (the
    // pointer itself keeps its address space, so the reads stay LDS or
    // global loads rather than flat ones)
    int opaque = 0;
    asm volatile("" : "+s"(opaque));
    tx_cols<MT, NT, 2, SCALE>(c0, Af + opaque, Btf, Df, x, M, N, out);
  }
  if (NT & 1) tx_cols<MT, NT, 1, SCALE>(NT - 1, Af, Btf, Df, x, M, N, out);
}

// ---------------------------------------------------------------------------
// Class-order transforms with the vertical fold.  With the operand rows in
// class order (TxLayout's oAc, oBc, oDc), rows [0, M/2) of the vertical
// matrix A' are even about the area's centre (A'[k][M-1-m] = A'[k][m]) and
// rows [M/2, M) odd (= -A'[k][m]), for the DCT-II and the Walsh-Hadamard
// rows alike.  So A' X = [A'_e (X_top + X_bot~); A'_o (X_top - X_bot~)] over
// the first M/2 columns of A', X_bot~ the bottom rows of X upside down: half
// the contraction of the vertical stage.  For M = 16 MT (MT even) the mirror
// of row 16 i + r is row 16 (MT-1-i) + 15 - r: the same lane of the mirrored
// lane within its row of 16 lanes (a DPP row mirror) in register MT-1-i.
//   xf[0] = X_top + X_bot~, xf[1] = X_top - X_bot~ (MT/2 row tiles each)
template <int MT, int NT>
__device__ inline void tx_fold_rows(const floatx4 (&x)[MT][NT], floatx4 (&xf)[2][MT / 2][NT]) {
#pragma unroll
  for (int i = 0; i < MT / 2; ++i)
#pragma unroll
    for (int sq = 0; sq < NT; ++sq)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float m = __int_as_float(__builtin_amdgcn_update_dpp(
            0, __float_as_int(x[MT - 1 - i][sq][t]), 0x140 /* row_mirror */, 0xF, 0xF, false));
        xf[0][i][sq][t] = x[i][sq][t] + m;
        xf[1][i][sq][t] = x[i][sq][t] - m;
      }
}

// Stage 2 of the folded forms and the output: z = A'_pv y over the first M/2
// columns of the class-order rows of parity pv (rows pv M/2 .. pv M/2 +
// M/2 - 1), out(k1, k2, D_k z) with k1 the class-order row.  Whole tiles
// only (M = 16 MT, N = 16 NT): every output is in range.
template <int MT, int NT, int CP, typename Out>
__device__ inline void tx_fold_rows_out(int c0, int pv, const float* Af, const float* Df,
                                        const floatx4 (&y)[CP][MT / 2], Out& out) {
  constexpr int MH = MT / 2;
  const int l = threadIdx.x & 63;
  floatx4 z[CP][MH];
#pragma unroll
  for (int cc = 0; cc < CP; ++cc)
#pragma unroll
    for (int r = 0; r < MH; ++r) z[cc][r] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < MH; ++i) {
    floatx4 av[MH];
#pragma unroll
    for (int r = 0; r < MH; ++r)
      av[r] = *reinterpret_cast<const floatx4*>(Af + (((pv * MH + r) * MT + i) * 64 + l) * 4);
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int cc = 0; cc < CP; ++cc)
#pragma unroll
        for (int r = 0; r < MH; ++r)
          z[cc][r] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r][e], y[cc][i][e], z[cc][r], 0, 0, 0);
  }
#pragma unroll
  for (int cc = 0; cc < CP; ++cc) {
    const int c = c0 + cc, k2 = 16 * c + (l & 15);
#pragma unroll
    for (int r = 0; r < MH; ++r) {
      const int rr = pv * MH + r;
      const floatx4 dv = *reinterpret_cast<const floatx4*>(Df + ((c * MT + rr) * 64 + l) * 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) out(16 * rr + 4 * (l >> 4) + e, k2, dv[e] * z[cc][r][e]);
    }
  }
}

// Column tiles c0 .. c0 + CP - 1 of the class-order rows of parity pv from
// the row-folded operand x = xf[pv]: the scheme of tx_cols with MT/2 row
// tiles in both stages.
template <int MT, int NT, int CP, typename Out>
__device__ inline void tx_cols_fold(int c0, int pv, const float* Af, const float* Btf,
                                    const float* Df, const floatx4 (&x)[MT / 2][NT], Out& out) {
  constexpr int MH = MT / 2;
  const int l = threadIdx.x & 63;
  floatx4 y[CP][MH];
#pragma unroll
  for (int cc = 0; cc < CP; ++cc)
#pragma unroll
    for (int i = 0; i < MH; ++i) y[cc][i] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int sq = 0; sq < NT; ++sq) {
    floatx4 bv[CP];
#pragma unroll
    for (int cc = 0; cc < CP; ++cc)
      bv[cc] = *reinterpret_cast<const floatx4*>(Btf + (((c0 + cc) * NT + sq) * 64 + l) * 4);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int cc = 0; cc < CP; ++cc)
#pragma unroll
        for (int i = 0; i < MH; ++i)
          y[cc][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[i][sq][t], bv[cc][t], y[cc][i], 0, 0, 0);
  }
  tx_fold_rows_out<MT, NT, CP>(c0, pv, Af, Df, y, out);
}

// The horizontal fold on top: the class-order columns of B' split the same
// way (columns [0, N/2) even about the area's centre, [N/2, N) odd), so
// column tile c of the horizontal stage needs only the first N/2 columns of
// X_f +- X_f~, X_f~ the columns of X_f right to left.  Column n = 16 sq +
// 4 g + t (g = lane / 16) mirrors to 16 (NT-1-sq) + 4 (3-g) + 3-t: register
// [NT-1-sq][3-t] of lane ^ 48 (a crossbar permute, once per block).
//   xh[0] = X_f + X_f~, xh[1] = X_f - X_f~ (NT/2 column tiles each)
template <int MH, int NT>
__device__ inline void tx_fold_cols(const floatx4 (&x)[MH][NT], floatx4 (&xh)[2][MH][NT / 2]) {
  const int src = ((threadIdx.x & 63) ^ 48) * 4;
#pragma unroll
  for (int i = 0; i < MH; ++i)
#pragma unroll
    for (int sq = 0; sq < NT / 2; ++sq)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float m = __int_as_float(
            __builtin_amdgcn_ds_bpermute(src, __float_as_int(x[i][NT - 1 - sq][3 - t])));
        xh[0][i][sq][t] = x[i][sq][t] + m;
        xh[1][i][sq][t] = x[i][sq][t] - m;
      }
}

// Column tiles c0 and c0 + 1 of the class-order rows of parity pv from the
// fully folded operands of their column parities (xa for c0, xb for c0 + 1).
template <int MT, int NT, typename Out>
__device__ inline void tx_cols_hfold(int c0, int pv, const float* Af, const float* Btf,
                                     const float* Df, const floatx4 (&xa)[MT / 2][NT / 2],
                                     const floatx4 (&xb)[MT / 2][NT / 2], Out& out) {
  constexpr int MH = MT / 2;
  const int l = threadIdx.x & 63;
  floatx4 y[2][MH];
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int i = 0; i < MH; ++i) y[cc][i] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int sq = 0; sq < NT / 2; ++sq) {
    floatx4 bv[2];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc)
      bv[cc] = *reinterpret_cast<const floatx4*>(Btf + (((c0 + cc) * NT + sq) * 64 + l) * 4);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < MH; ++i) {
        y[0][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[i][sq][t], bv[0][t], y[0][i], 0, 0, 0);
        y[1][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(xb[i][sq][t], bv[1][t], y[1][i], 0, 0, 0);
      }
  }
  tx_fold_rows_out<MT, NT, 2>(c0, pv, Af, Df, y, out);
}

// One part in class order from the fully folded operands (NT even): one pass
// per pair of column tiles of one column parity, or one pass over the two
// column tiles when each parity has one.
template <int MT, int NT, typename Out>
__device__ void tx_part_hfold(const float* Af, const float* Btf, const float* Df,
                              const floatx4 (&xh)[2][2][MT / 2][NT / 2], Out out) {
  constexpr int NH = NT / 2;
  static_assert(NH == 1 || NH % 2 == 0, "pairs of column tiles");
#pragma unroll
  for (int pv = 0; pv < 2; ++pv) {
    if constexpr (NH == 1) {
      tx_cols_hfold<MT, NT>(0, pv, Af, Btf, Df, xh[pv][0], xh[pv][1], out);
    } else {
#pragma unroll
      for (int ph = 0; ph < 2; ++ph) {
#pragma unroll 1
        for (int c0 = ph * NH; c0 < ph * NH + NH; c0 += 2) {
          int opaque = 0;
          asm volatile("" : "+s"(opaque));
          tx_cols_hfold<MT, NT>(c0, pv, Af + opaque, Btf, Df, xh[pv][ph], xh[pv][ph], out);
        }
      }
    }
  }
}

// One part in class order from the folded operands: both parities, two
// column tiles per pass.
template <int MT, int NT, typename Out>
__device__ void tx_part_fold(const float* Af, const float* Btf, const float* Df,
                             const floatx4 (&xf)[2][MT / 2][NT], Out out) {
  // both parities unrolled: a register array indexed at run time would go
  // to scratch
#pragma unroll
  for (int pv = 0; pv < 2; ++pv) {
#pragma unroll 1
    for (int c0 = 0; c0 + 1 < NT; c0 += 2) {
      int opaque = 0;
      asm volatile("" : "+s"(opaque));
      tx_cols_fold<MT, NT, 2>(c0, pv, Af + opaque, Btf, Df, xf[pv], out);
    }
    if (NT & 1) tx_cols_fold<MT, NT, 1>(NT - 1, pv, Af, Btf, Df, xf[pv], out);
  }
}

// Orders this wave's LDS writes before its later reads (and reads before
// later writes).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Initial projections of the transform parts (eq. 12 via eq. 22), fused with
// the gather: x = w s over the block's area (0 outside the image), then per
// part R[b][first + k1 N + k2] = D_k (A x B^T)[k1][k2].  An area of several
// frames of 2^fs rows (the loaders' VOL form) is read as its frames stacked:
// row m of the M-row area is row m - (f << fs) of frame img + f,
// f = m >> fs.  Columns K .. ldR-1
// of R are written as 0.  One wave per block; each workgroup copies the
// constant operands to LDS once and its waves loop over blocks.
struct TxArgs {
  const uint8_t* images;
  int H, W;
  const DevBlock* blk;
  int n_blk;
  int K;
  const float* tx;
  int first0, first1;
  float* R;
  int ldR;
  int fs;   // log2 of the rows per frame (read by the VOL loaders only)
};

// Pixels of one block, as the lane holds them until they become X operands:
// whole 16-pixel row segments when the area lies inside the image on a
// 16-byte grid (one 16-byte load each), else single pixels at clamped
// coordinates.
template <int MT, int NT>
struct TxPixels {
  static constexpr int CH = (MT * NT + 3) / 4;   // row segments per lane
  bool fast;
  // single pixels: v[(i * NT + sq) * 4 + t]; segments: v[4 k .. 4 k + 3]
  uint32_t v[MT * NT * 4];
};

template <int MT, int NT, bool VOL = false>
__device__ inline void tx_load(const TxArgs& a, const DevBlock& d, int M, int N,
                               TxPixels<MT, NT>& P) {
  const int l = threadIdx.x & 63, lr = l & 15, lc = 4 * (l >> 4);
  const uint8_t* img = a.images + (size_t)d.img * a.H * a.W;
  const int Ms = VOL ? 1 << a.fs : M;   // rows per frame
  const size_t plane = (size_t)a.H * a.W;
  P.fast = (M & 15) == 0 && (N & 15) == 0 && (a.W & 15) == 0 && (d.x0 & 15) == 0 &&
           d.y0 >= 0 && d.x0 >= 0 && d.y0 + Ms <= a.H && d.x0 + N <= a.W;
  if (P.fast) {
    const int spr = N >> 4, nseg = M * spr;
#pragma unroll
    for (int k = 0; k < P.CH; ++k) {
      const int c = min(l + 64 * k, nseg - 1);
      const int m = c / spr, sg = c - m * spr;
      const int f = VOL ? m >> a.fs : 0;
      const uint4 q = *reinterpret_cast<const uint4*>(img + f * plane +
                                                      (size_t)(d.y0 + m - f * Ms) * a.W +
                                                      d.x0 + 16 * sg);
      P.v[4 * k] = q.x;
      P.v[4 * k + 1] = q.y;
      P.v[4 * k + 2] = q.z;
      P.v[4 * k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const int m = 16 * i + lr;
      const int mc = VOL ? min(m, M - 1) : m, f = VOL ? mc >> a.fs : 0;
      const uint8_t* row =
          img + f * plane + (size_t)min(max(d.y0 + mc - f * Ms, 0), a.H - 1) * a.W;
#pragma unroll
      for (int sq = 0; sq < NT; ++sq)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          P.v[(i * NT + sq) * 4 + t] = row[min(max(d.x0 + 16 * sq + lc + t, 0), a.W - 1)];
    }
  }
}

// X operands x = w s (s = 0 outside the area and the image).
template <int MT, int NT, bool VOL = false>
__device__ inline void tx_x_operands(const TxArgs& a, const DevBlock& d, int M, int N,
                                     TxPixels<MT, NT>& P, const float* Wf, float* Xf,
                                     floatx4 (&xv)[MT][NT]) {
  const int l = threadIdx.x & 63, lr = l & 15, lc = 4 * (l >> 4);
  if (P.fast) {
    // segment (row m, columns 16 sg .. 16 sg + 15) covers, for j < 4, the
    // four t-values of fragment lane (m & 15) + 16 j of tile (m >> 4, sg)
    const int spr = N >> 4, nseg = M * spr;
#pragma unroll
    for (int k = 0; k < P.CH; ++k) {
      const int c = l + 64 * k;
      if (c < nseg) {
        const int m = c / spr, sg = c - m * spr;
        const uint32_t wd[4] = {P.v[4 * k], P.v[4 * k + 1], P.v[4 * k + 2], P.v[4 * k + 3]};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int o = (((m >> 4) * NT + sg) * 64 + (m & 15) + 16 * j) * 4;
          const floatx4 w = *reinterpret_cast<const floatx4*>(Wf + o);
          floatx4 v;
          v[0] = w[0] * (float)(wd[j] & 0xFFu);
          v[1] = w[1] * (float)((wd[j] >> 8) & 0xFFu);
          v[2] = w[2] * (float)((wd[j] >> 16) & 0xFFu);
          v[3] = w[3] * (float)(wd[j] >> 24);
          *reinterpret_cast<floatx4*>(Xf + o) = v;
        }
      }
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int sq = 0; sq < NT; ++sq)
        xv[i][sq] = *reinterpret_cast<const floatx4*>(Xf + ((i * NT + sq) * 64 + l) * 4);
    wave_sync();   // read before the next block's writes
  } else {
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const int m = 16 * i + lr;
      const int y = d.y0 + (VOL ? m - ((m >> a.fs) << a.fs) : m);
      const bool row_in = m < M && y >= 0 && y < a.H;
#pragma unroll
      for (int sq = 0; sq < NT; ++sq) {
        const floatx4 w = *reinterpret_cast<const floatx4*>(Wf + ((i * NT + sq) * 64 + l) * 4);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int n = 16 * sq + lc + t, x = d.x0 + n;
          // the value is taken as used here, so its load stays
          // unconditional (not moved under the test below, which would
          // serialise the loads)
          uint32_t& pv = P.v[(i * NT + sq) * 4 + t];
          asm volatile("" : "+v"(pv));
          xv[i][sq][t] = (row_in && n < N && x >= 0 && x < a.W) ? w[t] * (float)pv : 0.0f;
        }
      }
    }
  }
}

// Workgroup size bound: 16 waves for areas up to 32 x 32 (or 16 x 64), 4
// waves above (more registers per lane for the larger tiles).
template <int MT, int NT>
constexpr int tx_max_threads() {
  return (MT >= 3 || MT * NT >= 6) ? 256 : 1024;
}

}  // namespace sefase
