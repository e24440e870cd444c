// Internal declarations shared by the HIP translation units of libsefase.
// Device code targets gfx950 (CDNA4) only: 64-lane wavefronts, MFMA matrix
// cores, 160 KiB of LDS per compute unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/se.h"

namespace sefase {

// ---------------------------------------------------------------------------
// error reporting (thread-local message, see se_last_error)
// ---------------------------------------------------------------------------
se_status fail(se_status code, const char* fmt, ...);
se_status check_launch(const char* what);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Carves 256-byte aligned sub-buffers out of a caller's workspace (with a
// NULL base it only measures).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* p) : base(static_cast<char*>(p)) {}
  template <class T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
};

// Device copy of one block descriptor (same layout as se_block), validated
// on the host by se_blocks_upload (which also writes ld >= 1).
using DevBlock = se_block;

// frames per area of a dictionary or table set (0 is read as 1)
inline int area_frames(int T) { return T < 1 ? 1 : T; }

// DevBlock.geom of the device copy: flags set when the descriptors are
// uploaded (the caller's tag is not kept).
constexpr int kBlockNoSupport = 1;   // no available sample in the area

// A block whose area holds no available sample: the area lies wholly outside
// the frames' H x W, or its loss box covers every frame of the area and
// every one of its samples inside H x W.  Eq. 17 is then undefined for every
// atom (every weighted norm is 0), so nothing can be extrapolated.
__host__ __device__ inline bool block_without_support(const se_block& b, int H, int W, int T,
                                                      int M, int N) {
  const int y0 = b.y0 > 0 ? b.y0 : 0, y1 = b.y0 + M < H ? b.y0 + M : H;
  const int x0 = b.x0 > 0 ? b.x0 : 0, x1 = b.x0 + N < W ? b.x0 + N : W;
  if (y1 <= y0 || x1 <= x0) return true;
  const int ld = b.ld < 1 ? 1 : b.ld;
  if (b.lt > 0 || b.lt + ld < T) return false;
  return b.y0 + b.ly <= y0 && b.y0 + b.ly + b.lh >= y1 && b.x0 + b.lx <= x0 &&
         b.x0 + b.lx + b.lw >= x1;
}
// samples per area of a table set: T M N
inline int area_samples(const se_tables* t) { return area_frames(t->T) * t->M * t->N; }
// rows of the area as transformed: the T frames of M rows stacked (T M)
inline int tx_rows(const se_tables* t) { return area_frames(t->T) * t->M; }

// Loss sample i of a block (i < ld lh lw, frames, then rows, then columns):
// its index in the area's sample vector (T x M x N, (tau M + m) N + n), and
// its frame and position in the batch of images.
struct LossSample {
  int off, frame, y, x;
};
__device__ __forceinline__ LossSample loss_sample(const DevBlock& d, int i, int M, int N) {
  const int plane = d.lh * d.lw;
  const int mt = i / plane, r = i - mt * plane;
  const int my = r / d.lw, mx = r - my * d.lw;
  return LossSample{((d.lt + mt) * M + d.ly + my) * N + d.lx + mx, d.img + d.lt + mt,
                    d.y0 + d.ly + my, d.x0 + d.lx + mx};
}

// Class order of parity-class tables (classes.hip writes them): class
// c = 2 pv + ph in blocks of Kc = K / 4 positions; in a class the two parts
// in the order of their first atoms; in a part the atoms (kt, k1, k2) of the
// class by (kt, k1 / 2, k2 / 2), row-major.
struct ClassLayout {
  int T, M, N, K, Kc;
  int first_lo, kind_lo, first_hi, kind_hi;
};

// the row (2 i or 2 i + 1) of a 1-D transform of `kind` with parity `par`
// (a Walsh-Hadamard row k in natural order has the parity of popcount(k))
__device__ inline int parity_row(int kind, int i, int par) {
  const int even = 2 * i;
  const int p_even = kind == SE_PART_WHT2 ? (__popc(even) & 1) : 0;
  return even + (p_even ^ par);
}

// original atom index of position p of the class order (increasing with p
// inside each class, not across classes)
__device__ inline int class_orig(const ClassLayout& L, int p) {
  const int c = p / L.Kc, r = p - c * L.Kc;
  const int F = L.M * L.N / 4, Q = L.T * F, h = L.N / 2;
  const int q = r / Q, s = r - q * Q;
  const int kind = q ? L.kind_hi : L.kind_lo, first = q ? L.first_hi : L.first_lo;
  const int kt = s / F, f = s - kt * F;
  const int i1 = f / h, i2 = f - i1 * h;
  return first + (kt * L.M + parity_row(kind, i1, c >> 1)) * L.N + parity_row(kind, i2, c & 1);
}

// Predicate over a workgroup of WAVES waves (uniform result).
template <int WAVES>
__device__ __forceinline__ bool any_in_workgroup(bool p) {
  if constexpr (WAVES == 1) return __builtin_amdgcn_ballot_w64(p) != 0;
  else return __syncthreads_or(p) != 0;
}

// The outputs of a block with nothing to extrapolate from: every selection
// -1, every coefficient and model value 0; its loss is not touched.  T
// threads of the workgroup, thread t.
__device__ inline void degenerate_outputs(int32_t* sel, float* coef, int n_coef, float* g_loss,
                                          int g_loss_ld, int iters, int nloss, int b, int t,
                                          int T, int32_t* counter) {
  for (int i = t; i < iters; i += T)
    if (sel) sel[(size_t)b * iters + i] = -1;
  for (int i = t; i < n_coef * iters; i += T)
    if (coef) coef[(size_t)b * n_coef * iters + i] = 0.0f;
  const int ng = nloss < g_loss_ld ? nloss : g_loss_ld;
  for (int i = t; i < ng; i += T)
    if (g_loss) g_loss[(size_t)b * g_loss_ld + i] = 0.0f;
  if (counter && t == 0) atomicAdd(counter, 1);
}

// ---------------------------------------------------------------------------
// kernel launchers (defined in the .hip files)
// ---------------------------------------------------------------------------

// weights.hip -- eq. 4 / eq. 5 per block (T x M x N samples)
void launch_area_weights(int T, int M, int N, float rho_hat, const uint8_t* lost,
                         int H, int W, const DevBlock* blk, int n_blk,
                         float* w, hipStream_t s);

// lost-pixel mask of one H x W frame from loss rectangles (y, x, h, w)
void launch_lost_mask(uint8_t* mask, int H, int W, const int4* rects, int n, hipStream_t s);

// gram.hip -- Algorithm 2 support kernels
// diag32/diag64: C_kk summed in fp32 and fp64 with one fixed order
// (phi_im: imaginary parts of a complex dictionary, or NULL).
void launch_diag(const float* phi, const float* phi_im, const float* w, int K, int P,
                 float* diag32, double* diag64, hipStream_t s);
// Re G and Im G of a complex dictionary from the 2K x 2K product S of the
// stacked real and imaginary rows of Y.
void launch_combine_c(const float* S, int ldS, int K, float* G, float* G_im, int ldG,
                      hipStream_t s);
// D_k from the diagonal (mode 0 auto, 1 fp64, 2 fp32), sqrt(w), info word.
void launch_finalize_d(const float* diag32, const double* diag64,
                       const float* w, int K, int P, int mode, int force64,
                       float* D, float* sqrtw, int32_t* info, hipStream_t s);
// Y[k][p] = D_k sqrt(w_p) phi[k][p] (negated with neg)
void launch_scale_y(const float* phi, const float* D, const float* sqrtw,
                    int K, int P, float* Y, hipStream_t s, bool neg = false);
// zero columns [c0, ld) of a rows x ld matrix
void launch_zero_cols(float* A, int rows, int c0, int ld, hipStream_t s);
// split x = hi + lo into two bf16 arrays (precision path)
void launch_split_bf16(const float* x, size_t n, uint16_t* hi, uint16_t* lo,
                       hipStream_t s);

// gemm.hip -- FP32 matrix-core products over the area pixels
// G = Y Y^T (lower-triangle tiles, mirrored); G is K x ldg.
se_status gemm_syrk_f32(const float* Y, int ldy, int K, int P, float* G, int ldg,
                        hipStream_t s);
// R[b][k] = sum_p X[b][p] Y[k][p] for k < K, and 0 for K <= k < ldr when
// pad (else those columns are left alone).  tile: 0 = automatic, 64 or 128.
// split: -1 automatic (by the tile count; needs ws), 1 none, kSplitShape
// the slices fixed by P alone (SE_INVARIANT: the same order for any batch;
// SE_ENOMEM when ws cannot hold gemm_invariant_floats).
constexpr int kSplitShape = -2;
constexpr int kTile128x64 = 12864;   // tile code: 128 atoms x 64 blocks
se_status gemm_project_f32(const float* Y, int ldy, int K, const float* X, int ldx,
                           int n_blk, int P, float* R, int ldr, int tile, hipStream_t s,
                           bool pad = true, float* ws = nullptr, size_t ws_floats = 0,
                           int split = -1);
// partial products of the fixed (kSplitShape) split of a product with Mst
// stored atoms, Nst blocks and P samples (0 when it does not split)
size_t gemm_invariant_floats(int Mst, int Nst, int P);
// workspace (floats) that lets gemm_project_f32 split the contraction of a
// product with Mst stored atoms, up to Nst_max blocks and P pixels; 0 when it
// never splits.  Without it (or with less) the product runs unsplit.
size_t gemm_splitk_floats(int Mst, int Nst_max, int P);
// Rows formed on demand: rows[cmap[i]][k] = sum_p X[i][p] Y[k][p] for k < K
// and i < min(n_max, *n_dev) (n_dev on the device, read by the kernels, so
// the launch shape depends on n_max only); columns from K on are left alone.
// tile: 0 = automatic, 64 or 128; split: -1 automatic, 0/1 none, S slices of
// the contraction (partials in ws, gemm_rows_splitk_floats of it).
se_status gemm_rows_f32(const float* Y, int ldy, int K, const float* X, int ldx, int n_max,
                        const int32_t* n_dev, const int32_t* cmap, int P, float* rows, int ldr,
                        int tile, int split, hipStream_t s, float* ws, size_t ws_floats);
size_t gemm_rows_splitk_floats(int K, int n_max, int P, int split);
// gemm_bf16x3.hip -- the same two products from split-bf16 operands
se_status gemm_syrk_bf16x3(const uint16_t* Yhi, const uint16_t* Ylo, int ldy, int K, int P,
                           float* G, int ldg, hipStream_t s);
se_status gemm_project_bf16x3(const uint16_t* Yhi, const uint16_t* Ylo, int ldy, int K,
                              const uint16_t* Xhi, const uint16_t* Xlo, int ldx, int n_blk, int P,
                              float* R, int ldr, hipStream_t s, bool pad = true);
se_status gemm_rows_bf16x3(const uint16_t* Yhi, const uint16_t* Ylo, int ldy, int K,
                           const uint16_t* Xhi, const uint16_t* Xlo, int ldx, int n_max,
                           const int32_t* n_dev, const int32_t* cmap, int P, float* rows, int ldr,
                           int tile, hipStream_t s);

// project.hip -- X[b][p] = sqrt(w_p) s_b[p] and the per-block GEMV
void launch_gather(const uint8_t* images, int H, int W, const DevBlock* blk,
                   int n_blk, int T, int M, int N, const float* sqrtw, float* X,
                   int ldX, hipStream_t s);
void launch_gemv(const float* Y, int K, int P, const float* x, float* r,
                 hipStream_t s);
// the same gather, written as split bf16 pairs (precision path)
void launch_gather_split(const uint8_t* images, int H, int W, const DevBlock* blk,
                         int n_blk, int T, int M, int N, const float* sqrtw, uint16_t* Xhi,
                         uint16_t* Xlo, int ldX, hipStream_t s);

// transform.hip -- declared transform parts of a dictionary (Section VI)
// 1-D matrices of a complex DFT part in the operand buffer (internal kinds,
// beside the SE_PART_* kinds): Ar = cos(2 pi k m / n) / sqrt(n) and
// Ai = -sin(2 pi k m / n) / sqrt(n), the conjugate DFT matrix Ar + j Ai
constexpr int kKindDftRe = 16, kKindDftIm = 17;
// transforms whose operands the buffer holds: a DFT part takes two
inline int tx_layout_parts(int n_parts, const se_part* parts) {
  return n_parts == 1 && parts[0].kind == SE_PART_DFT2 ? 2 : n_parts;
}
// sets *dflag (device) to 1 if an atom of the part differs from its definition
// (T frames of Ms rows stacked: the vertical transform is A_T (x) A_Ms)
se_status check_part(const float* phi, int T, int Ms, int N, int kind, int first, int* dflag,
                     hipStream_t s);
// the same for a complex DFT part (real parts phi, imaginary parts phi_im)
se_status check_dft_part(const float* phi, const float* phi_im, int M, int N, int first,
                         int* dflag, hipStream_t s);
// complex tables with a DFT part: R[b][first + k] (real parts) and
// R[b][im + first + k] (imaginary parts) of eq. 12 for the part's atoms; no
// other column is written
se_status project_dft(const se_tables* t, const uint8_t* images, int H, int W,
                      const DevBlock* blk, int n_blk, float* R, int ldR, int im, hipStream_t s);
// R[b][first + k] of every part of t, and 0 in columns K .. ldR-1
se_status project_tx(const se_tables* t, const uint8_t* images, int H, int W,
                     const DevBlock* blk, int n_blk, float* R, int ldR, hipStream_t s);
size_t tx_lds_bytes(int M, int N, int n_parts);
// bytes of se_tables.tx (0 for an unsupported shape); build_tx writes it
// from t->D and t->sqrtw
size_t tx_const_bytes(int M, int N, int n_parts);
se_status build_tx(const se_tables* t, hipStream_t s);
// table rows of every atom over the part columns (transforms of w phi_k),
// then the mirror pass that completes the parts' rows and exact symmetry
se_status gram_tx(const se_tables* t, hipStream_t s);
se_status gram_mirror(const se_tables* t, hipStream_t s);
// the A and B operands alone (for unscaled transforms) into tx
se_status build_tx_basis(const se_basis* b, float* tx, hipStream_t s);
// rows[b][first + k] = transform k of V[b] (M x N), for the parts of b
// (n_dev, out_row: optional, the row count on the device, at most n_blk, and
// the destination row of each V row)
se_status rows_tx(const se_basis* b, const float* tx, const float* V, int ldV, int n_blk,
                  float* rows, int ld, hipStream_t s, const int32_t* n_dev = nullptr,
                  const int32_t* out_row = nullptr);
// abi.cpp -- the host-side checks of a basis' part declaration; the atom
// ranges outside the parts
se_status check_basis_parts(const se_basis* b);
// (P: samples per atom, the length of a part)
int dense_ranges(int K, int P, int n_parts, const se_part* parts, int lo[3], int hi[3]);

// greedy.hip -- the iteration loop of Algorithm 3
struct GreedyArgs {
  const float* R0;     // n_blk x ldR initial projections (units of D_k)
  int ldR;
  const float* G;      // K x ldG unit-diagonal Gram
  int ldG;
  const float* D;      // K
  const float* phi;    // K x P
  int K, M, N;
  int P;               // samples per atom: T M N (M N for a two-dimensional area)
  const DevBlock* blk; // n_blk
  int n_blk;
  int blk0;            // plain form: the one block of this launch; -1 when batched
  uint8_t* images;
  int H, W;
  float gamma;
  int iters;
  int32_t* sel;        // optional
  float* coef;         // optional
  float* g_loss;       // optional
  int g_loss_ld;
  // class tables (the one-launch route of tables with n_classes = 4):
  // rows of K/4 entries by position in the class order, and per position
  // (original atom index, D bits)
  const float* Gc;
  const int2* cls;
  // fixed-point class rows (Q1.14 words of Gc); non-NULL selects them
  const int16_t* Gq;   // fixed-point class rows (class form), or NULL
  const int16_t* Gqr;  // fixed-point whole rows, ldG words each (whole-row form), or NULL
  // the class order (exact ties between classes are decided by atom index)
  ClassLayout cl;
  // optional device counter of blocks with nothing to extrapolate from
  int32_t* n_degenerate;
};
// ondemand.hip -- per-block weights, rows of C_b formed on demand
struct OnDemandPlan {
  int K, M, N, n_blk;
  const float* phi;     // K x P
  const float* w;       // caller-order blocks x P weights
  uint8_t* images;
  int H, W;
  const DevBlock* blk;  // n_blk, sorted by decreasing iteration count
  const int32_t* orig;  // sorted position -> caller index
  const int* active;    // host: active[nu] = blocks with more than nu iterations
  int iters_max;
  float gamma;
  // device workspace
  float* phi2;          // K x P (phi squared)
  bool phi2_ready;      // phi2 already holds it (a prepared dictionary)
  float* X;             // n_blk x ldV
  float* V;             // n_blk x ldV (compact rows of the requested table rows)
  int ldV;
  float* R;             // n_blk x ld
  float* D;             // n_blk x ld
  float* rows;          // n_blk x (slots + 1) x ld: the cache of table rows
  int slots;            // cached rows per block (row `slots` of a block: not cached)
  int32_t* ibuf;        // 4 + 2 n_blk (+ n_blk K when slots > 0) ints cleared per run:
                        // the request counters, rows in use, deg, the atom -> row map
  int32_t* cur;         // n_blk
  int32_t* cmap;        // n_blk
  int ld;               // multiple of 1024
  int row_tile[3], row_split[3];   // per dense range of the row products
  const se_basis* basis;  // transform parts (rows formed as transforms)
  const float* tx;        // their A and B operands (when n_parts > 0)
  float* splitk;        // partial products of split contractions
  size_t splitk_floats;
  bool invariant;       // the fixed split of SE_INVARIANT for every product
  // split-BF16 operands of the per-iteration dense row products (NULL: FP32)
  uint16_t* phi_hi;     // K x P
  uint16_t* phi_lo;
  bool split_ready;     // phi_hi / phi_lo already hold the split dictionary
  uint16_t* Vhi;        // n_blk x ldV
  uint16_t* Vlo;
  float* st;            // n_blk x 2
  float* g;             // n_blk x ldg, followed by gc (n_blk x ldg)
  float* gc;
  int ldg;
  // outputs (optional)
  int32_t* sel;
  float* coef;
  float* g_loss;
  int g_loss_ld;
  int32_t* deg;           // n_blk (inside ibuf): blocks with nothing to extrapolate from
  int32_t* n_degenerate;  // optional device counter of those blocks
};
se_status ondemand_run(const OnDemandPlan& pl, hipStream_t s);
// out = phi squared, elementwise (n floats)
void launch_square(const float* phi, size_t n, float* out, hipStream_t s);

// classes.hip -- parity classes of DCT / Walsh-Hadamard tables under a
// mirror-symmetric weight pattern
bool classes_possible(const se_tables* t);
// flag (device) = 1 if w is not mirror-symmetric in the rows and columns of
// every frame
void launch_sym_check(const float* w, int T, int M, int N, int* flag, hipStream_t s);
// the class order of t's class tables
ClassLayout class_layout(const se_tables* t);
// t->Gc and t->cls from t->G and t->D
se_status build_classes(se_tables* t, hipStream_t s);
// t->Gq = round(t->Gc 2^14) (16-bit words, 14 fraction bits)
se_status quantise_classes(se_tables* t, hipStream_t s);
// t->Gq_rows = round(t->G 2^14), every row of ldG entries
se_status quantise_rows(se_tables* t, hipStream_t s);

// fused.hip -- projections of transform parts and the loop in one launch
bool conceal_tx_supported(const se_tables* t);
se_status conceal_tx(const se_tables* t, const GreedyArgs& a, const uint8_t* images, int H, int W,
                     int n_blk, hipStream_t s, int waves, int vpl);

// complex.hip -- the loop for complex dictionaries (R rows: real | imaginary)
bool complex_loop_for(int K);
se_status launch_greedy_c(const GreedyArgs& a, const float* G_im, const float* phi_im, int grid,
                          hipStream_t s);
// zero columns [c0, c1) of rows x ld
void launch_zero_range(float* A, int rows, int ld, int c0, int c1, hipStream_t s);

int greedy_waves_for(int K);   // 0 if K is too large
int greedy_row_len(int K);     // padded row length (table row stride minimum)
// loop shapes (waves, values per lane) with the row length of K; returns count
int greedy_shapes_for(int K, int* waves, int* vpl, int cap);
// waves = 0: the tuned or default shape for K
se_status launch_greedy(const GreedyArgs& a, int grid, hipStream_t s, int waves, int vpl);

// tune.cpp -- choices recorded by the autotuner (or imported), per K and
// batch size; 0 when nothing is recorded
struct TuneChoice {
  int loop_waves = 0, loop_vpl = 0, proj_tile = 0;
};
TuneChoice tune_lookup(int K, int P, int n_blk);
// rows on demand: the row products' tile (0 automatic, 64, 128, kTile128x64)
// and split (-1 automatic, 1 none, 2/4/8 slices) for Kd dense atoms of P pixels
struct RowTune {
  int tile = 0, split = -1;
};
RowTune tune_lookup_rows(int Kd, int P, int n_blk);
// plans of rows on demand, for the tuner (abi.cpp)
int ondemand_plan_dense(const se_od_plan* p, int kd[3], int* P);
int ondemand_plan_blocks(const se_od_plan* p);
void ondemand_plan_set_rows(se_od_plan* p, int tile, int split);

}  // namespace sefase
