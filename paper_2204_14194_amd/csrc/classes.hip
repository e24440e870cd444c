// Parity classes of a dictionary of DCT-II and Walsh-Hadamard atoms under a
// mirror-symmetric weight pattern (eq. 16).  A 1-D DCT-II row k is even
// about the centre of its M points for even k and odd for odd k; a
// Walsh-Hadamard row k in natural order is even or odd as popcount(k) is
// even or odd (reversing the point index complements its bits).  A 2-D atom
// is the product of a vertical and a horizontal row, so it is even or odd
// in each axis.  When w[m][n] = w[M-1-m][n] = w[m][N-1-n], the weighted
// scalar product of two atoms that differ in either parity is a sum whose
// terms cancel in mirrored pairs: C_(k,l) = 0.  The table is then block
// diagonal in the four classes (vertical parity, horizontal parity), and
// the recursion of eq. 20 changes R only inside the selected atom's class.
//
// Class order: class c = 2 pv + ph; in a class the two parts in the order of
// their first atoms; in a part the atoms (k1, k2) of the class by
// (k1 / 2, k2 / 2), row-major.  Each part contributes M N / 4 atoms to each
// class (M, N even: k = 2 i and k = 2 i + 1 always differ in parity).
//
// Areas of T frames: the mirrors act on the rows and columns of every frame
// (the time axis is left alone), so a 3-D atom (kt, k1, k2) takes the
// parities of k1 and k2, the weights must be mirror-symmetric within every
// frame, and a part's atoms of a class are ordered by (kt, k1 / 2, k2 / 2).
//
// The class rows may also be written as 16-bit fixed-point words (14
// fraction bits), the table form Section III suggests for a loop without
// division; the loop then streams half the bytes.
#include "se_internal.h"

namespace sefase {

// flag = 1 if the weight pattern is not mirror-symmetric in the rows and
// columns of every frame (bit for bit)
__global__ void k_sym_check(const float* __restrict__ w, int T, int M, int N,
                            int* __restrict__ flag) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= T * M * N) return;
  const int f = p / (M * N), q = p - f * M * N;
  const int m = q / N, n = q - m * N;
  const float* wf = w + (size_t)f * M * N;
  const uint32_t v = __float_as_uint(wf[q]);
  if (v != __float_as_uint(wf[(M - 1 - m) * N + n]) || v != __float_as_uint(wf[m * N + N - 1 - n]))
    atomicOr(flag, 1);
}

// Gc[p][i] = G[orig(p)][orig(c(p) Kc + i)], cls[p] = (orig(p), D_orig(p)).
// One workgroup per class-order row.
__global__ __launch_bounds__(256) void k_build_classes(ClassLayout L, const float* __restrict__ G,
                                                       int ldG, const float* __restrict__ D,
                                                       float* __restrict__ Gc, int ldGc,
                                                       int2* __restrict__ cls) {
  const int p = blockIdx.x;
  if (p >= L.K) return;
  const int o = class_orig(L, p);
  const int base = (p / L.Kc) * L.Kc;
  const float* row = G + (size_t)o * ldG;
  for (int i = threadIdx.x; i < L.Kc; i += blockDim.x)
    Gc[(size_t)p * ldGc + i] = row[class_orig(L, base + i)];
  if (threadIdx.x == 0) cls[p] = make_int2(o, __float_as_int(D[o]));
}

// The static conditions of the class tables (the weight symmetry is
// checked on the device).
bool classes_possible(const se_tables* t) {
  if (!t->Gc || !t->cls || t->n_parts != 2 || t->phi_im) return false;
  if ((t->M & 1) || (t->N & 1) || t->K % 1024 || t->K != greedy_row_len(t->K)) return false;
  int lo[3], hi[3];
  return dense_ranges(t->K, area_samples(t), t->n_parts, t->parts, lo, hi) == 0;
}

void launch_sym_check(const float* w, int T, int M, int N, int* flag, hipStream_t s) {
  const int P = T * M * N;
  hipLaunchKernelGGL(k_sym_check, dim3((P + 255) / 256), dim3(256), 0, s, w, T, M, N, flag);
}

ClassLayout class_layout(const se_tables* t) {
  ClassLayout L;
  L.T = area_frames(t->T);
  L.M = t->M;
  L.N = t->N;
  L.K = t->K;
  L.Kc = t->K / 4;
  const bool swap = t->parts[1].first < t->parts[0].first;
  const se_part& lo = t->parts[swap ? 1 : 0];
  const se_part& hi = t->parts[swap ? 0 : 1];
  L.first_lo = lo.first;
  L.kind_lo = lo.kind;
  L.first_hi = hi.first;
  L.kind_hi = hi.kind;
  return L;
}

se_status build_classes(se_tables* t, hipStream_t s) {
  const ClassLayout L = class_layout(t);
  hipLaunchKernelGGL(k_build_classes, dim3(t->K), dim3(256), 0, s, L, t->G, t->ldG, t->D, t->Gc,
                     L.Kc, reinterpret_cast<int2*>(t->cls));
  return check_launch("build_classes");
}

// Fixed-point words of the class rows: q = round(Gc 2^14), to nearest with
// ties to even.  Scaling by a power of two is exact in FP32, so the only
// rounding is the one to the word; unit-diagonal entries (|Gc| <= 1) never
// leave the 16-bit range, the bound below only keeps a corrupt table finite.
__global__ void k_quantise_rows(const float4* __restrict__ Gc, size_t n4, short4* __restrict__ Gq) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n4) return;
  const float4 v = Gc[i];
  auto word = [](float x) {
    return (short)fminf(fmaxf(rintf(x * 16384.0f), -32768.0f), 32767.0f);
  };
  Gq[i] = make_short4(word(v.x), word(v.y), word(v.z), word(v.w));
}

se_status quantise_classes(se_tables* t, hipStream_t s) {
  const size_t n4 = (size_t)t->K * (t->K / 4) / 4;
  hipLaunchKernelGGL(k_quantise_rows, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(t->Gc), n4, reinterpret_cast<short4*>(t->Gq));
  return check_launch("quantise_rows");
}

se_status quantise_rows(se_tables* t, hipStream_t s) {
  const size_t n4 = (size_t)t->K * t->ldG / 4;
  hipLaunchKernelGGL(k_quantise_rows, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(t->G), n4,
                     reinterpret_cast<short4*>(t->Gq_rows));
  return check_launch("quantise_rows");
}

}  // namespace sefase
