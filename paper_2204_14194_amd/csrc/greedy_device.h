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
// sweep.  Rows of G and of R are padded with zeros to T * VPL columns (the
// table row stride), so no load needs a bounds check; padded atoms hold 0
// and are never candidates.
//
// Selection: the wave's largest |R~| is found from per-lane maxima with a
// DPP reduction; when one lane alone holds it, that lane's group maxima and
// then the four values of its first matching group are read into scalar
// registers and scanned for the lowest index.  When several lanes hold the maximum
// (exact ties, e.g. parallel atoms), every lane scans its atoms in index
// order and the wave reduces 64-bit keys
//     |R~| bits << 32  |  (0xFFFF - k) << 16  |  sign << 15
// so the lowest index wins.  Workgroups of several waves combine the wave
// winners' keys through LDS.
//
// Class form (CLS): R~ is held in the class order of the tables' parity
// classes (four classes of K/4 atoms, class c in the sweeps j of
// [c NJ/4, (c+1) NJ/4)), the table rows are the class rows Gc (K/4 entries),
// and eq. 20 updates only the selected atom's class -- every other entry of
// its row of D C D is 0.  The selected position maps to its original atom
// (for the model, the reported selection and D) through the class table.
// Each wave keeps the largest |R~| of each class over its values across
// iterations: only the updated class is rescanned, the class maxima are
// compared in scalar registers, and the winner is found in the winning class
// (with several waves per block, each wave's pick enters the waves'
// reduction as a key).  Inside a class positions follow the atom order, so
// the lowest position holding the maximum is its lowest atom; across classes
// they do not, so an exact tie between classes (or any tie the position
// order cannot settle: several lanes, several groups of one lane, several
// waves) is decided by class_tie_key on the original atom indices, as eq. 18
// with ties to the lowest index requires.
//
// Fixed-point rows (Q16): the rows (class rows in the class form, else whole
// rows of ldG words) are read as 16-bit words q with 14 fraction bits and
// eq. 20 becomes R~ -= (tc 2^-14) q.  The
// product tc 2^-14 q equals tc (q 2^-14) exactly (both factors' scalings are
// powers of two), so each update rounds once, as with the FP32 entries
// q 2^-14; only the table bytes change.
#pragma once

#include "argmax.h"
#include "se_internal.h"

namespace sefase {

constexpr int kQPL = 4;   // loss pixels per lane (the loss may hold <= 4 T pixels)

// Fourth word of a raw buffer resource on gfx9-family devices (32-bit data
// format; offsets are bounds-checked against the record count in bytes).
constexpr int kBufferWord3 = 0x00020000;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Largest |R~| of a lane's values in class C (sweeps C NJC .. C NJC + NJC - 1).
template <int NJ, int NJC, int C>
__device__ __forceinline__ float class_lane_max(const float (&R)[NJ][4]) {
  float m = 0.0f;
#pragma unroll
  for (int j = C * NJC; j < (C + 1) * NJC; ++j)
    m = fmaxf(m, fmaxf(fmaxf(fabsf(R[j][0]), fabsf(R[j][1])), fmaxf(fabsf(R[j][2]), fabsf(R[j][3]))));
  return m;
}

// Of four wave-uniform keys (class_winner below): the largest, mk; whether
// it is direct -- mk even (one holder) and the second largest sk below it
// (no other class at the same maximum), i.e. (sk | 1) < thr with thr = mk
// for an even mk and 0 for an odd one; dir = 1 or 0 -- and x, y of the first
// class whose key equals mk (the position and value bits of its winner).
// On the scalar unit (written out: the compiler would merge the chain of
// maxima into vector max3 forms and take the comparisons as lane masks).
__device__ __forceinline__ void select_class(const uint32_t (&k)[4], const int (&x)[4],
                                             const uint32_t (&y)[4], uint32_t& mk,
                                             uint32_t& dir, int& xo, uint32_t& yo) {
  uint32_t a, b, c, sk;
  asm("s_max_u32 %[a], %[k0], %[k1]\n\t"
      "s_min_u32 %[b], %[k0], %[k1]\n\t"
      "s_max_u32 %[c], %[k2], %[k3]\n\t"
      "s_min_u32 %[sk], %[k2], %[k3]\n\t"
      "s_max_u32 %[mk], %[a], %[c]\n\t"
      "s_min_u32 %[a], %[a], %[c]\n\t"
      "s_max_u32 %[b], %[b], %[sk]\n\t"
      "s_max_u32 %[sk], %[a], %[b]\n\t"
      "s_or_b32 %[sk], %[sk], 1\n\t"
      "s_and_b32 %[c], %[mk], 1\n\t"
      "s_add_u32 %[c], %[c], -1\n\t"
      "s_and_b32 %[c], %[c], %[mk]\n\t"
      "s_cmp_lt_u32 %[sk], %[c]\n\t"
      "s_cselect_b32 %[dir], 1, 0\n\t"
      "s_cmp_eq_u32 %[k2], %[mk]\n\t"
      "s_cselect_b32 %[xo], %[x2], %[x3]\n\t"
      "s_cselect_b32 %[yo], %[y2], %[y3]\n\t"
      "s_cmp_eq_u32 %[k1], %[mk]\n\t"
      "s_cselect_b32 %[xo], %[x1], %[xo]\n\t"
      "s_cselect_b32 %[yo], %[y1], %[yo]\n\t"
      "s_cmp_eq_u32 %[k0], %[mk]\n\t"
      "s_cselect_b32 %[xo], %[x0], %[xo]\n\t"
      "s_cselect_b32 %[yo], %[y0], %[yo]"
      : [mk] "=&s"(mk), [dir] "=&s"(dir), [xo] "=&s"(xo), [yo] "=&s"(yo), [sk] "=&s"(sk),
        [a] "=&s"(a), [b] "=&s"(b), [c] "=&s"(c)
      : [k0] "s"(k[0]), [k1] "s"(k[1]), [k2] "s"(k[2]), [k3] "s"(k[3]), [x0] "s"(x[0]),
        [x1] "s"(x[1]), [x2] "s"(x[2]), [x3] "s"(x[3]), [y0] "s"(y[0]), [y1] "s"(y[1]),
        [y2] "s"(y[2]), [y3] "s"(y[3])
      : "scc");
}

// Class form: the winner of class C among a wave's values, found when the
// class changes (once at the start, then after each update of the class),
// as wave-uniform words: key = (largest |R~| of the class over the wave, as
// float bits) << 1, plus 1 when several lanes hold it (the sign bit of |R~|
// is 0, so the shift loses nothing and keys order as the maxima, a held-by-
// several key above a held-by-one key of the same maximum); and the single
// holder's position in the class order (wpos: the wave's offset, 4 x 64 x
// its index) and signed value (float bits).  The
// holding lane's lowest position at the maximum is that lane's lowest atom of
// the class (positions follow the atom order inside a class).
template <int NJ, int NJC, int C, int T>
__device__ __forceinline__ void class_winner(const float (&R)[NJ][4], int wpos, uint32_t& key,
                                             int& pos, uint32_t& val) {
  // the lane's maximum through its sweep maxima
  float ms[NJC];
#pragma unroll
  for (int s = 0; s < NJC; ++s) {
    const float* r = R[C * NJC + s];
    ms[s] = fmaxf(fmaxf(fabsf(r[0]), fabsf(r[1])), fmaxf(fabsf(r[2]), fabsf(r[3])));
  }
  float m = ms[0];
#pragma unroll
  for (int s = 1; s < NJC; ++s) m = fmaxf(m, ms[s]);
  // value e of sweep C NJC + s has the position 4 ((C NJC + s) T + t) + e, and
  // the sweeps' positions increase with s: the lowest sweep at the maximum
  // (its four values q and base b, without the lane's 4 t) ...
  float q[4];
  int b = 4 * (C * NJC + NJC - 1) * T;
#pragma unroll
  for (int e = 0; e < 4; ++e) q[e] = R[C * NJC + NJC - 1][e];
#pragma unroll
  for (int s = NJC - 2; s >= 0; --s) {
    const bool hit = ms[s] == m;
#pragma unroll
    for (int e = 0; e < 4; ++e) q[e] = hit ? R[C * NJC + s][e] : q[e];
    b = hit ? 4 * (C * NJC + s) * T : b;
  }
  // ... then its lowest entry at the maximum
  int p = 3;
  float v = q[3];
#pragma unroll
  for (int e = 2; e >= 0; --e) {
    const bool hit = fabsf(q[e]) == m;
    p = hit ? e : p;
    v = hit ? q[e] : v;
  }
  p += b;
  const uint32_t wm = __float_as_uint(wave_max_f32(m));
  const uint64_t holders = __builtin_amdgcn_ballot_w64(__float_as_uint(m) == wm);
  // key = 2 wm + (more than one holder), as wm + wm + carry with the carry
  // from the holder count (scalar instructions: the compiler would take the
  // comparison as a lane mask)
  uint32_t cnt;
  asm("s_bcnt1_i32_b64 %[c], %[h]\n\t"
      "s_cmp_gt_u32 %[c], 1\n\t"
      "s_addc_u32 %[k], %[w], %[w]"
      : [k] "=s"(key), [c] "=&s"(cnt)
      : [h] "s"(holders), [w] "s"(wm)
      : "scc");
  const int L = (int)__builtin_ctzll(holders);
  pos = __builtin_amdgcn_readlane(p, L) + 4 * L + wpos;
  val = (uint32_t)__builtin_amdgcn_readlane(__float_as_int(v), L);
}


// Class form: the classes (bit c) of the sweeps set in a mask of sweeps
// (class c holds the sweeps c NJC .. c NJC + NJC - 1).
template <int NJ, int NJC>
__device__ __forceinline__ uint32_t class_mask(uint32_t sweeps) {
  constexpr uint32_t one = (NJC >= 32) ? 0xFFFFFFFFu : ((1u << NJC) - 1u);
  uint32_t m = 0u;
#pragma unroll
  for (int c = 0; c < 4; ++c) m |= (uint32_t)((sweeps & (one << (c * NJC))) != 0u) << c;
  return m;
}

// Exact ties of the class form: every lane's positions whose |R~| bits equal
// Mb, keyed by their original atom index (class_orig), reduced over the wave
// (eq. 18 with ties to the lowest atom index).  Rare: only bit-identical
// scores take this path, so the positions are visited in a rolled loop.
template <int NJ, int T>
__device__ __forceinline__ uint64_t class_tie_key(const float (&R)[NJ][4], uint32_t Mb,
                                                  const ClassLayout& cl, int t) {
  static_assert(NJ * 4 <= 32, "one mask bit per value of a lane");
  // (float compares with the |.| operand modifier: no operand of the mask
  // is formed ahead of the rare branch that calls this)
  const float Mf = __uint_as_float(Mb);
  uint32_t mask = 0u;
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) mask |= (fabsf(R[j][e]) == Mf ? 1u : 0u) << (4 * j + e);
  int best = -1, bo = 0x7FFFFFFF;
  for (uint32_t m = mask; m; m &= m - 1) {
    const int bit = __builtin_ctz(m);
    const int o = class_orig(cl, 4 * ((bit >> 2) * T + t) + (bit & 3));
    if (o < bo) {
      bo = o;
      best = bit;
    }
  }
  uint64_t mine = 0;
  if (best >= 0) {
    uint32_t vb = 0u;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) vb = 4 * j + e == best ? __float_as_uint(R[j][e]) : vb;
    mine = make_class_key(vb, bo, 4 * ((best >> 2) * T + t) + (best & 3));
  }
  return wave_max_key((uint32_t)(mine >> 32), (uint32_t)mine);
}

// The iterations and the paste for block b of a workgroup of WAVES waves,
// from R~^(0) in registers (lane t: atoms 4 (j T + t) + e).
template <int WAVES, int VPL, bool CLS = false, bool Q16 = false>
__device__ __forceinline__ void greedy_block(const GreedyArgs& a, int b, float (&R)[VPL / 4][4]) {
  constexpr int T = 64 * WAVES;
  constexpr int NJ = VPL / 4;
  constexpr int NJC = NJ / 4 > 0 ? NJ / 4 : 1;   // sweeps of one class (CLS)
  static_assert(!CLS || NJ % 4 == 0, "the class form needs whole sweeps per class");
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const DevBlock d = a.blk[b];
  const int K = a.K, P = a.P;

  // ---- loss pixels owned by this lane ----------------------------------
  // Lanes past the end of the loss repeat its last pixel (a valid address);
  // their sums are never written.
  const int nloss = d.ld * d.lh * d.lw;
  const int nq = (nloss + T - 1) / T;          // uniform
  int poff[kQPL];
  float g[kQPL], gc[kQPL];   // model and its compensation term (Kahan summation)
#pragma unroll
  for (int q = 0; q < kQPL; ++q) {
    int i = t + q * T;
    i = i < nloss ? i : nloss - 1;
    poff[q] = loss_sample(d, i, a.M, a.N).off;
    g[q] = 0.0f;
    gc[q] = 0.0f;
  }

  // ---- a block with nothing to extrapolate from -----------------------------
  // No available sample (marked by the host), or every atom of zero weighted
  // norm (then every D_k and every R~_k is 0): eq. 17 is undefined for all
  // atoms, no atom can be selected, and the block reports sel = -1 with its
  // loss left as it is.  D is read only when every R~ is 0.
  {
    bool deg = (d.geom & kBlockNoSupport) != 0;
    if (!deg) {
      float m = 0.0f;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) m = fmaxf(m, fabsf(R[j][e]));
      if (!any_in_workgroup<WAVES>(m != 0.0f)) {
        bool dnz = false;
        for (int j = 0; j < NJ; ++j)
          for (int e = 0; e < 4; ++e) {
            const int k = 4 * (j * T + t) + e;
            if (k < K) dnz = dnz || (CLS ? __int_as_float(a.cls[k].y) : a.D[k]) != 0.0f;
          }
        deg = !any_in_workgroup<WAVES>(dnz);
      }
    }
    if (deg) {
      degenerate_outputs(a.sel, a.coef, 1, a.g_loss, a.g_loss_ld, a.iters, nloss, b, t, T,
                         a.n_degenerate);
      return;
    }
  }

  __shared__ uint64_t s_key[2][WAVES];
  __shared__ uint64_t s_tie[WAVES];
  int par = 0;
  // gamma in a vector register (loop-invariant): gamma times a scalar value
  // is then one vector multiply (a vector instruction reads one scalar)
  float gamma;
  asm("v_mov_b32 %0, %1" : "=v"(gamma) : "s"(a.gamma));

  // each class's winner kept across iterations (class form; per wave, the
  // wave-uniform words of class_winner)
  constexpr bool INC = CLS;
  const int wpos = WAVES == 1 ? 0 : __builtin_amdgcn_readfirstlane(256 * wave);
  uint32_t ck[4] = {0u, 0u, 0u, 0u};
  int c_pos[4] = {0, 0, 0, 0};
  uint32_t c_val[4] = {0u, 0u, 0u, 0u};
  if constexpr (INC) {
    class_winner<NJ, NJC, 0, T>(R, wpos, ck[0], c_pos[0], c_val[0]);
    class_winner<NJ, NJC, 1, T>(R, wpos, ck[1], c_pos[1], c_val[1]);
    class_winner<NJ, NJC, 2, T>(R, wpos, ck[2], c_pos[2], c_val[2]);
    class_winner<NJ, NJC, 3, T>(R, wpos, ck[3], c_pos[3], c_val[3]);
  }
  // the selections and coefficients of 64 iterations, gathered in the lanes
  // of wave 0 (lane i: iteration i mod 64) and written together
  int sel_buf = 0;
  float coef_buf = 0.0f;
  // class form: buffer resources of the class rows and of the atoms (the
  // class tables exist for areas of at most 64 x 64 samples and K <= 32768,
  // so every byte offset fits 32 bits; unused by the other forms)
  const __amdgpu_buffer_rsrc_t gc_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(a.Gc), (short)0, K * (T * NJ * 4), kBufferWord3);
  const __amdgpu_buffer_rsrc_t gq_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<int16_t*>(a.Gq), (short)0, K * (T * NJ * 2), kBufferWord3);
  const __amdgpu_buffer_rsrc_t phi_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(a.phi), (short)0, K * (P * 4), kBufferWord3);
  int flush_at = min(63, a.iters - 1);

  for (int it = 0; it < a.iters; ++it) {
    int u = 0;
    float rv = 0.0f;
    uint64_t key = 0;                          // every score zero: atom 0, value 0
    bool direct = WAVES == 1;
    bool class_key = false;                    // key from class_tie_key
    if constexpr (INC) {
      // ---- the largest class maximum: its class's winner, unless it ties
      // (between classes, or between lanes of the class)
      uint32_t mk, dir, vb;
      select_class(ck, c_pos, c_val, mk, dir, u, vb);   // (u, vb taken when direct)
      rv = __uint_as_float(vb);
      if constexpr (WAVES == 1) {
        if (dir == 0u) {
          u = 0;                                // every score zero: atom 0, value 0
          rv = 0.0f;
          if (mk > 1u) {
            // exact ties across lanes or between classes: the lowest atom index
            key = class_tie_key<NJ, T>(R, mk >> 1, a.cl, t);
            direct = false;
            class_key = true;
          }
        }
      } else {
        // this wave's candidate as a key for the waves' reduction below,
        // marked for the atom-index rule when it is not direct (several
        // lanes or classes of the wave at its maximum); 0 when every value
        // of the wave is 0
        key = mk > 1u ? (make_key(rv, u) | (uint64_t)(dir == 0u)) : 0ull;
      }
    } else {
    // ---- this wave's largest |R~| and its lowest index ---------------------
    // Group maxima (4 atoms each) and the lane maximum, then the wave
    // maximum by DPP.
    float gm[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      gm[j] = fmaxf(fmaxf(fabsf(R[j][0]), fabsf(R[j][1])), fmaxf(fabsf(R[j][2]), fabsf(R[j][3])));
    float lm;
    bool two = false;   // class form: the lane's maximum lies in two classes
    if constexpr (CLS) {
      // class maxima, their largest, and their second largest (the larger
      // of the smaller of each pair and the smaller pair maximum): equal to
      // the largest exactly when two classes share it
      float cm[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        cm[c] = gm[c * NJC];
#pragma unroll
        for (int j = 1; j < NJC; ++j) cm[c] = fmaxf(cm[c], gm[c * NJC + j]);
      }
      const float m01 = fmaxf(cm[0], cm[1]), m23 = fmaxf(cm[2], cm[3]);
      lm = fmaxf(m01, m23);
      two = fmaxf(fmaxf(fminf(m01, m23), fminf(cm[0], cm[1])), fminf(cm[2], cm[3])) == lm;
    } else {
      lm = gm[0];
#pragma unroll
      for (int j = 1; j < NJ; ++j) lm = fmaxf(lm, gm[j]);
    }
    const float M = wave_max_f32(lm);
    const uint64_t holders = __builtin_amdgcn_ballot_w64(lm == M);
    if (M != 0.0f && __builtin_popcountll(holders) == 1) {
      // lane L alone holds the maximum: its group maxima, then the four
      // values of the first matching group, are read into scalar
      // registers and scanned there (lowest index first)
      const int L = __builtin_ctzll(holders);
      const uint32_t Mb = __float_as_uint(M);
      int gsel = NJ - 1;
      bool mark = false;
#pragma unroll
      for (int j = NJ - 2; j >= 0; --j)
        gsel = (uint32_t)__builtin_amdgcn_readlane(__float_as_int(gm[j]), L) == Mb ? j : gsel;
      // class form: a group at the maximum in another class of the lane
      // marks the key for the atom-index rule (positions do not follow the
      // atom order across classes)
      if constexpr (CLS) mark = ((__builtin_amdgcn_ballot_w64(two) >> L) & 1ull) != 0ull;
      uint32_t r[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if (j == gsel) {                       // uniform branch
#pragma unroll
          for (int e = 0; e < 4; ++e)
            r[e] = (uint32_t)__builtin_amdgcn_readlane(__float_as_int(R[j][e]), L);
        }
      int csel = 3;
#pragma unroll
      for (int e = 2; e >= 0; --e) csel = (r[e] & 0x7FFFFFFFu) == Mb ? e : csel;
      const uint32_t vbits = csel == 0 ? r[0] : csel == 1 ? r[1] : csel == 2 ? r[2] : r[3];
      u = 4 * (gsel * T + wave * 64 + L) + csel;
      rv = __uint_as_float(vbits);
      if (u >= K) {                            // only with nonzero padding of R
        u = 0;
        rv = 0.0f;
      }
      if (WAVES > 1) key = make_key(rv, u) | (uint64_t)mark;
    } else if (M != 0.0f) {
      // exact ties across lanes: every lane's first maximum as a key
      float bv = 0.0f;
      int c = 0;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (fabsf(R[j][e]) > fabsf(bv)) {
            bv = R[j][e];
            c = 4 * j + e;
          }
      const uint64_t mine = make_key(bv, 4 * ((c >> 2) * T + t) + (c & 3));
      key = wave_max_key((uint32_t)(mine >> 32), (uint32_t)mine);
      if constexpr (CLS) {
        // holders in two classes mark the key for the atom-index rule
        uint32_t lh = 0u;
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) lh |= (uint32_t)(fabsf(R[j][e]) == M) << j;
        const uint32_t cm = class_mask<NJ, NJC>(lh);
        int ncls = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) ncls += __builtin_amdgcn_ballot_w64((cm >> k) & 1u) != 0;
        key |= (uint64_t)(ncls > 1);
      }
      direct = false;
    }
    }
    if (WAVES > 1) {
      if (lane == 0) s_key[par][wave] = key;
      __syncthreads();
      // every group of WAVES lanes reads the waves' keys (lane i: wave
      // i mod WAVES) and reduces them by DPP; the largest key holds the
      // largest |R~| and, among waves tied on it, the lowest position
      const uint64_t o = s_key[par][lane & (WAVES - 1)];
      const uint32_t ohi = (uint32_t)(o >> 32);
      key = group_max_key<WAVES>(ohi, (uint32_t)o);
      if constexpr (CLS) {
        // class form, rare: several waves at the maximum, or a winner marked
        // for holding it in two classes -- positions do not follow the atom
        // order across classes, so the atom-index rule decides
        const uint32_t kh = (uint32_t)(key >> 32);
        const uint64_t at = __builtin_amdgcn_ballot_w64(ohi == kh) & ((1ull << WAVES) - 1ull);
        if (kh != 0u && ((at & (at - 1ull)) != 0ull || (key & 1ull) != 0ull)) {
          const uint64_t k2 = class_tie_key<NJ, T>(R, kh, a.cl, t);
          if (lane == 0) s_tie[wave] = k2;
          __syncthreads();
          const uint64_t o2 = s_tie[lane & (WAVES - 1)];
          key = group_max_key<WAVES>((uint32_t)(o2 >> 32), (uint32_t)o2);
          class_key = true;
        }
      }
      par ^= 1;
    }
    // ---- the winner (wave-uniform, kept in scalar registers) ----------------
    if (!direct) {
      if (CLS && class_key)
        decode_class_key(key, u, rv);
      else
        decode_key(key, K, u, rv);
    }
    u = __builtin_amdgcn_readfirstlane(u);
    rv = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(rv)));
    const float tc = gamma * rv;              // coefficient of the unit-norm atom
    constexpr int NR = CLS ? NJC : NJ;
    const float* grow = CLS ? a.Gc + (size_t)u * (T * NJ) : a.G + (size_t)u * a.ldG;
    float4 row[NR];
    uint2 qrow[Q16 ? NR : 1];
    if constexpr (Q16 && CLS) {
      // (buffer loads, as the FP32 class rows)
      const int so = u * (T * NJ * 2);
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        const auto q = __builtin_amdgcn_raw_buffer_load_b64(gq_rsrc, 8 * (j * T + t), so, 0);
        qrow[j] = make_uint2(q[0], q[1]);
      }
    } else if constexpr (Q16) {
      const int16_t* g16 = a.Gqr + (size_t)u * a.ldG;
#pragma unroll
      for (int j = 0; j < NR; ++j) qrow[j] = *reinterpret_cast<const uint2*>(g16 + 4 * (j * T + t));
    } else if constexpr (CLS) {
      // buffer loads: the row's byte offset is a scalar offset on a fixed
      // resource, the lane's part a loop-invariant vector offset
      // (sweep j's 16 T-byte step in the scalar offset: one vector offset for all)
      const int so = u * (T * NJ * 4);
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(gc_rsrc, 16 * t, so + 16 * j * T, 0);
        row[j] = make_float4(__uint_as_float(q.x), __uint_as_float(q.y), __uint_as_float(q.z),
                             __uint_as_float(q.w));
      }
    }
    // the selected atom's original index and D (the class form: from the
    // class table; a scalar load that does not wait behind vector loads)
    int ou = u;
    float Du = 0.0f;
    if constexpr (CLS) {
      // (an unsigned 32-bit byte offset: the load takes it as its offset
      // register, no 64-bit address is formed)
      const uint64_t cu = *(const __attribute__((address_space(4))) uint64_t*)(
          (const __attribute__((address_space(4))) char*)a.cls + ((uint32_t)u << 3));
      ou = (int)(uint32_t)cu;
      Du = __uint_as_float((uint32_t)(cu >> 32));
    }

    // ---- stream row u of the table and the atom over the loss ---------------
    // (the first pixel of every lane always exists; more pixels per lane
    // only for losses larger than the workgroup, one uniform branch)
    const float* prow = a.phi + (size_t)ou * P;
    float pv[kQPL];
    if constexpr (CLS) {                       // (buffer loads, as the rows)
      const int so = ou * (P * 4);
      pv[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(phi_rsrc, 4 * poff[0], so, 0));
      if (nq > 1) {
#pragma unroll
        for (int q = 1; q < kQPL; ++q)
          if (q < nq)
            pv[q] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(phi_rsrc, 4 * poff[q], so, 0));
      }
    } else {
      pv[0] = prow[poff[0]];
      if (nq > 1) {
#pragma unroll
        for (int q = 1; q < kQPL; ++q)
          if (q < nq) pv[q] = prow[poff[q]];
      }
    }
    if constexpr (!CLS && !Q16) {
#pragma unroll
      for (int j = 0; j < NR; ++j) row[j] = *reinterpret_cast<const float4*>(grow + 4 * (j * T + t));
    }
    // D is read-only for the whole launch: a scalar load (constant address
    // space) that does not wait behind the row's vector loads
    if constexpr (!CLS) Du = ((const __attribute__((address_space(4))) float*)a.D)[u];
    const float c = tc * Du;                  // eq. 19
    if (a.sel || a.coef) {                    // uniform test first: no lane mask work
      const int slot = it & 63;
      sel_buf = lane == slot ? ou : sel_buf;
      coef_buf = lane == slot ? c : coef_buf;
      if (it == flush_at) {                   // uniform: every 64 iterations, and the last
        const size_t at = (size_t)b * a.iters + (it - slot) + lane;
        if (wave == 0 && lane <= slot) {
          if (a.sel) a.sel[at] = sel_buf;
          if (a.coef) a.coef[at] = coef_buf;
        }
        flush_at = min(flush_at + 64, a.iters - 1);
      }
    }
    // eq. 9, compensated (the class form applies it after eq. 20: its
    // atom's loads wait for the class table and are not on the path to the
    // next selection)
    auto model_update = [&]() {
      {
        const float y = fmaf(c, pv[0], -gc[0]);
        const float s = g[0] + y;
        gc[0] = (s - g[0]) - y;
        g[0] = s;
      }
      if (nq > 1) {
#pragma unroll
        for (int q = 1; q < kQPL; ++q)
          if (q < nq) {
            const float y = fmaf(c, pv[q], -gc[q]);
            const float s = g[q] + y;
            gc[q] = (s - g[q]) - y;
            g[q] = s;
          }
      }
    };
    if constexpr (!CLS) model_update();

    // ---- eq. 20 -------------------------------------------------------------
    if constexpr (Q16) {                        // the words as exact FP32 integers
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        row[j].x = (float)(int)(int16_t)(qrow[j].x & 0xFFFFu);
        row[j].y = (float)((int)qrow[j].x >> 16);
        row[j].z = (float)(int)(int16_t)(qrow[j].y & 0xFFFFu);
        row[j].w = (float)((int)qrow[j].y >> 16);
      }
    }
    const float tr = Q16 ? tc * (1.0f / 16384.0f) : tc;   // eq. 20 factor per row entry
    if (CLS) {
      const int cu = u / (T * NJC * 4);         // the selected atom's class (uniform)
#pragma unroll
      for (int cc = 0; cc < 4; ++cc)
        if (cc == cu) {
#pragma unroll
          for (int j = 0; j < NR; ++j) {
            R[cc * NJC + j][0] = fmaf(-tr, row[j].x, R[cc * NJC + j][0]);
            R[cc * NJC + j][1] = fmaf(-tr, row[j].y, R[cc * NJC + j][1]);
            R[cc * NJC + j][2] = fmaf(-tr, row[j].z, R[cc * NJC + j][2]);
            R[cc * NJC + j][3] = fmaf(-tr, row[j].w, R[cc * NJC + j][3]);
          }
          if constexpr (INC) {                  // the class's new winner
            switch (cc) {
              case 0: class_winner<NJ, NJC, 0, T>(R, wpos, ck[0], c_pos[0], c_val[0]); break;
              case 1: class_winner<NJ, NJC, 1, T>(R, wpos, ck[1], c_pos[1], c_val[1]); break;
              case 2: class_winner<NJ, NJC, 2, T>(R, wpos, ck[2], c_pos[2], c_val[2]); break;
              default: class_winner<NJ, NJC, 3, T>(R, wpos, ck[3], c_pos[3], c_val[3]); break;
            }
          }
        }
    } else {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        R[j][0] = fmaf(-tr, row[j].x, R[j][0]);
        R[j][1] = fmaf(-tr, row[j].y, R[j][1]);
        R[j][2] = fmaf(-tr, row[j].z, R[j][2]);
        R[j][3] = fmaf(-tr, row[j].w, R[j][3]);
      }
    }
    if constexpr (CLS) model_update();
  }

  // ---- replace the loss area by the model ----------------------------------
#pragma unroll
  for (int q = 0; q < kQPL; ++q) {
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


}  // namespace sefase
