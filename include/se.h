/*
 * se.h -- C ABI of libsefase: Fast Selective Extrapolation (FaSE) on AMD
 * Instinct MI355X (gfx950).
 *
 * The calls follow the paper's statement of the problem (J. Seiler and
 * A. Kaup, "A Fast Algorithm for Selective Signal Extrapolation with
 * Arbitrary Basis Functions"):
 *
 *   se_area_weights        -- the weighting function w (eq. 4) with the
 *                             isotropic decay rho (eq. 5), per block
 *   se_volume_weights      -- the same over T x M x N areas of consecutive
 *                             frames (the three-dimensional model of the
 *                             paper's closing section)
 *   se_weighted_gram       -- table generation, Algorithm 2 (eq. 16, 17)
 *   se_extrapolate_batch   -- model generation, Algorithm 3 (eq. 12, 18-20,
 *                             model update eq. 9, replacement of the loss
 *                             area), batched over many blocks that share one
 *                             set of tables
 *   se_extrapolate_plain   -- the same result, one block at a time
 *                             (three launches per block); the baseline form
 *
 * Conventions shared by every call
 *   * Real-valued signals and atoms (Section III: for real data the
 *     conjugations drop out).  Arithmetic is float32 unless a precision
 *     argument says otherwise.
 *   * An atom is a vector over the M x N extrapolation area, pixel (m, n) at
 *     index m*N + n.  A dictionary is K atoms, row-major K x (M*N).
 *   * Video: an area may span T consecutive frames (se_basis.T); an atom is
 *     then a vector over T x M x N samples, sample (tau, m, n) at index
 *     (tau*M + m)*N + n, and the batch of images is read as frames.  T = 1
 *     (or 0) is the two-dimensional case every statement below describes.
 *   * Pointers documented "device" point to GPU memory the CALLER allocates
 *     and owns (e.g. torch tensors); pointers documented "host" point to
 *     host memory read during the call only.  The library never frees
 *     caller memory and never keeps a pointer after a call returns.
 *   * Every call is asynchronous on `stream` (a hipStream_t passed as void*,
 *     NULL = the null stream) unless it says otherwise.  Argument errors are
 *     detected on the host before anything is launched and return SE_EINVAL
 *     synchronously; a failed launch returns SE_EHIP.  In both cases
 *     se_last_error() describes the problem.
 *   * Scratch memory ("ws") is device memory supplied by the caller; the
 *     matching *_ws_bytes() call gives the size needed.  No call allocates
 *     device memory.
 *   * Blocks with nothing to extrapolate from: when every atom has a zero
 *     weighted norm over a block's area (eq. 17 is undefined for all of
 *     them), no atom can be selected.  Such a block reports sel = -1 in
 *     every iteration, coefficients and model 0, and its loss is left as it
 *     is; the other blocks of the call are concealed as usual.  Blocks whose
 *     area holds no available sample by their geometry (the area wholly
 *     outside the frames, or the loss covering every sample of the area
 *     inside them) are found on the host: the concealment calls (and
 *     se_blocks_upload) then return SE_ENUMERIC after launching everything
 *     else, with the outputs written.  Blocks found only on the device
 *     (every D_k = 0 for their weights, e.g. an area covered by other
 *     losses) are reported through sel = -1 alone, since the calls do not
 *     wait for the device; the server reports both kinds in the request's
 *     status.
 */
#ifndef SEFASE_SE_H
#define SEFASE_SE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t se_status;
#define SE_OK 0
#define SE_EINVAL (-1)    /* invalid argument (host-side check)            */
#define SE_ENOMEM (-2)    /* workspace or budget too small                 */
#define SE_EHIP (-3)      /* a HIP runtime call or kernel launch failed    */
#define SE_EAGAIN (-4)    /* result not ready yet (serving)                */
#define SE_EBUSY (-5)     /* queue full (serving)                          */
#define SE_ENUMERIC (-6)  /* blocks with nothing to extrapolate from      */
#define SE_ECANCELED (-7) /* request cancelled / server shut down         */

typedef enum { SE_FP32 = 0, SE_BF16X3 = 1 } se_precision;

/* Diagonal flags of se_weighted_gram (how C_(k,k) of eq. 16 is summed). */
#define SE_DIAG_AUTO 0u        /* FP64 if precision is BF16X3 or the area is
                                  ill-conditioned (min/max C_kk < 1e-3 over
                                  atoms with C_kk > 0), else FP32          */
#define SE_DIAG_FP64 1u        /* always FP64                              */
#define SE_DIAG_FP32 2u        /* always FP32                              */

/* Known structure of a range of atoms (Section VI): rows first ..
 * first + M*N - 1 of phi are the separable 2-D atoms of a discrete
 * transform, atom k1*N + k2 = row k1 of the vertical 1-D transform times row
 * k2 of the horizontal one.  For such atoms the weighted scalar products of
 * a vector are that transform's coefficients of the weighted vector
 * (eq. 21-23), which the library then computes as a separable transform
 * instead of a product with the dictionary.
 *   SE_PART_DCT2: orthonormal DCT-II rows, alpha_k cos(pi (2m+1) k / 2M)
 *   SE_PART_WHT2: Walsh-Hadamard rows in natural (Sylvester) order,
 *                 (-1)^popcount(m & k) / sqrt(M); M and N powers of two
 * Parts need M, N <= 64; se_weighted_gram checks every declared atom
 * against phi (|difference| <= 2e-6) and fails with SE_EINVAL otherwise.
 * For areas of T > 1 frames a part holds the separable 3-D atoms: the same
 * 1-D transform along frames, rows and columns, atom (kt*M + k1)*N + k2 =
 * row kt of the T-point transform times row k1 of the M-point one times row
 * k2 of the N-point one (powers of two T, M, N for Walsh-Hadamard); the
 * library transforms the frames stacked as a T*M x N area, so T*M <= 64,
 * and M must be a power of two. */
#define SE_PART_DCT2 1
#define SE_PART_WHT2 2
/* SE_PART_DFT2: complex 2-D DFT atoms (Section VI's complex case), atom
 * k1*N + k2 = exp(j 2 pi (k1 m / M + k2 n / N)) / sqrt(M N) at pixel (m, n),
 * real parts in phi and imaginary parts in phi_im.  Declared only on a
 * complex dictionary, as its one part, on two-dimensional areas (any M, N
 * <= 64).  The weighted scalar products with these atoms are the 2-D DFT
 * of the weighted block, computed as two small complex matrix products per
 * block (the initial projections of eq. 12); the tables (Algorithm 2) are
 * still the product of all atoms.  Verified like the real kinds, against
 * the exact phases (k1 m N + k2 n M) mod M N. */
#define SE_PART_DFT2 3
typedef struct {
  int32_t kind, first;
} se_part;

/* A dictionary (Section II: phi_k[m, n], k in the dictionary D).
 * phi: device, K x (M*N) float32, row-major.  n_parts (0..2) declared
 * transform ranges, non-overlapping; every other atom is dense.
 * phi_im: NULL for a real dictionary; for a complex one (the paper's general
 * case, e.g. 2-D DFT atoms) the imaginary parts, device K x (M*N) float32,
 * with phi holding the real parts.  Complex dictionaries take FP32 tables,
 * declare at most one transform part (of kind SE_PART_DFT2; no other kind),
 * and are concealed by the batched calls
 * (se_extrapolate_batch, se_project/se_iterate, se_extrapolate_device);
 * the other calls refuse them (SE_EINVAL).
 * T: frames per area (0 or 1: a two-dimensional area).  With T > 1 the
 * atoms are K x (T*M*N) (sample (tau, m, n) at (tau*M + m)*N + n), and
 * the dictionary is concealed by the batched calls, se_project/se_iterate,
 * se_extrapolate_device and se_extrapolate_plain; rows on demand and the
 * server refuse it, and it must be real (phi_im NULL). */
typedef struct {
  int32_t M, N, K;
  const float* phi;
  int32_t n_parts;
  se_part parts[2];
  const float* phi_im;
  int32_t T;
} se_basis;

/* One lost block and its extrapolation area L = A u B (Section II, Fig. 2).
 * img      : index of the image in the batch of images
 * y0, x0   : top-left corner of the M x N area in image coordinates; the
 *            area may extend past the image border (those pixels are not
 *            support: weight 0)
 * ly, lx   : top-left corner of the loss rectangle B relative to the area
 * lh, lw   : loss rectangle size; B must lie inside the area
 * geom     : caller's tag of the weight pattern (not interpreted by the
 *            batch calls, which take one table set for all blocks)
 * lt, ld   : for areas of T > 1 frames: img is the area's first frame (the
 *            frames img .. img+T-1 of the batch must exist), and the loss
 *            is the box of frames lt .. lt+ld-1 of the area (inside it)
 *            times the rectangle above.  ld = 0 is read as 1, so a
 *            two-dimensional caller may leave both fields 0.            */
typedef struct {
  int32_t img, y0, x0, ly, lx, lh, lw, geom;
  int32_t lt, ld;
} se_block;

/* Tables for one weight pattern (Algorithm 2), as written by
 * se_weighted_gram.  All pointers device, allocated by the caller:
 *   G    : K x ldG float32, ldG >= se_table_ld(K), a multiple of 4,
 *          16-byte aligned.  G[k][l] = D_k C_(k,l) D_l, the weighted Gram of
 *          eq. 16 expressed for the atoms scaled to unit weighted norm (so
 *          G[k][k] = 1 for every atom with C_kk > 0).  Exactly symmetric.
 *          Columns K .. ldG-1 are written as 0 (the loop streams padded
 *          rows).
 *   D    : K float32, D_k = 1/sqrt(C_(k,k)) (eq. 17); 0 for an atom whose
 *          weighted norm is 0 (it can never be selected).
 *   Y    : K x (M*N) float32, Y[k][p] = D_k sqrt(w[p]) phi_k[p]; the
 *          initial projections of eq. 12 are Y (sqrt(w) s), in units of
 *          D_k.
 *   sqrtw: M*N float32, sqrt(w).
 *   phi  : the dictionary itself (read by the model update).
 *   info : optional (may be NULL) device int32: 1 if the diagonal was
 *          summed in FP64, 0 if in FP32.
 *   precision : set by se_weighted_gram; the initial projections of blocks
 *          using these tables are computed in the same precision.
 *   n_parts, parts : the dictionary's verified transform ranges; the
 *          projections of those atoms are computed as transforms.
 *   tx   : se_tables_tx_bytes(M, N, n_parts) bytes, 16-byte aligned;
 *          required (non-NULL) when the dictionary declares transform
 *          parts: se_weighted_gram writes the operands of those transforms
 *          there (the 1-D transform matrices, D and w, in the order the
 *          matrix cores read them).  Unused without parts (may be NULL).
 *   Yhi, Ylo : K x (M*N) bfloat16 bit patterns, Y = Yhi + Ylo (hi = bf16(Y),
 *          lo = bf16(Y - hi)); required (non-NULL) for SE_BF16X3, unused
 *          for SE_FP32.
 * A complex dictionary (se_basis.phi_im) makes the tables complex:
 *   G, G_im : real and imaginary parts of the Hermitian D C D (eq. 16 with
 *          the conjugated atom, Algorithm 2's mirror C_(l,k) = conj C_(k,l));
 *          G_im K x ldG float32, 16-byte aligned, columns K .. ldG-1 0.
 *   Y    : 2K x (M*N): rows 0..K-1 the real and rows K..2K-1 the imaginary
 *          parts of D_k sqrt(w) conj(phi_k), so eq. 12 is Y (sqrt(w) s).
 *   phi_im : copied from the dictionary.
 * For a real dictionary G_im and phi_im are NULL (G_im is not written).
 * Class tables (optional; Gc and cls may be NULL): when every atom lies in
 * the two declared transform parts of an area with even M and N, K equals
 * se_table_ld(K) and is a multiple of 1024, and the weight pattern is
 * mirror-symmetric in the rows and columns of every frame (w[m][n] =
 * w[M-1-m][n] = w[m][N-1-n], bit for bit), every DCT-II and Walsh-Hadamard
 * atom is even or odd about the area's centre in each of those axes, so
 * C_(k,l) of eq. 16 is 0 whenever k and l differ in either parity: the
 * atoms fall into four classes of Kc = K/4 and eq. 20 changes only the
 * selected atom's class.  se_weighted_gram then writes, in class order
 * (class 2 pv + ph for the vertical and horizontal parities; in a class the
 * parts in the order of their first atoms, each by (k1/2, k2/2), or by
 * (kt, k1/2, k2/2) for areas of several frames):
 *   Gc   : K x (K/4) float32, 16-byte aligned: row p holds the entries of
 *          G between the p-th atom of the class order and the atoms of its
 *          own class, in class order;
 *   cls  : K pairs of int32 (original atom index, D_k as float bits), by
 *          position in the class order;
 * and sets n_classes = 4 (else 0, and Gc, cls are not written).  The
 * one-launch route (se_extrapolate_device and se_extrapolate_batch for
 * all-transform tables) then streams a quarter of a row per iteration;
 * selections are reported as original atom indices.
 * Fixed-point class rows (optional; Gq may be NULL): Section III notes
 * that the loop of Algorithm 3 needs no division, so its tables suit
 * fixed-point words, and leaves their bit depth open.  When Gq is non-NULL
 * and class tables are written, se_weighted_gram also writes
 *   Gq   : K x (K/4) int16, 16-byte aligned: Gc in signed 16-bit words with
 *          14 fraction bits, Gq = round(Gc * 2^14) to nearest, ties to even
 *          (|Gc| <= 1, so no word saturates and the diagonal 1 is exact);
 * a loop called with SE_ROWS_Q14 then streams these words (a quarter of
 * the class rows' bytes) and updates R with Gq * 2^-14 in FP32.
 * Fixed-point whole rows (optional; Gq_rows may be NULL): for a real
 * dictionary, when Gq_rows is non-NULL se_weighted_gram also writes
 *   Gq_rows : K x ldG int16, 16-byte aligned: G in the same words,
 *          round(G * 2^14) to nearest, ties to even (|G| <= 1; columns K ..
 *          ldG-1 hold 0);
 * the loop over whole rows (the route of tables without the one-launch
 * form, se_iterate and se_extrapolate_plain) called with SE_ROWS_Q14 then
 * streams these words (half the bytes of a row of G). */
typedef struct {
  int32_t M, N, K, ldG;
  float* G;
  float* D;
  float* Y;
  float* sqrtw;
  const float* phi;
  int32_t* info;
  int32_t precision;
  uint16_t* Yhi;
  uint16_t* Ylo;
  int32_t n_parts;       /* copied from the dictionary by se_weighted_gram */
  se_part parts[2];
  float* tx;
  float* G_im;
  const float* phi_im;   /* copied from the dictionary by se_weighted_gram */
  int32_t T;             /* frames per area, copied (0 read as 1)          */
  float* Gc;             /* class tables (may be NULL, see above)          */
  int32_t* cls;
  int32_t n_classes;     /* written by se_weighted_gram: 4 or 0            */
  int16_t* Gq;           /* fixed-point class rows (may be NULL, see above) */
  int16_t* Gq_rows;      /* fixed-point whole rows (may be NULL, see above) */
} se_tables;

/* Model-generation parameters: gamma of eq. 8 (0 < gamma <= 1), the
 * iteration count I, and flags:
 *   SE_ROWS_Q14 : the loop reads fixed-point words instead of FP32 table
 *                 entries (eq. 20 with the entries quantised as described
 *                 for se_tables; R, D, the coefficients and the model stay
 *                 FP32): the class rows Gq on the one-launch route
 *                 (se_extrapolate_batch and se_extrapolate_device on tables
 *                 with n_classes = 4 and Gq written), the whole rows
 *                 Gq_rows on the loop over whole rows (those calls on
 *                 tables without the one-launch form, se_iterate and
 *                 se_extrapolate_plain, on real tables with Gq_rows
 *                 written).  Every other case, and rows on demand, return
 *                 SE_EINVAL. */
#define SE_ROWS_Q14 1u
/*   SE_ROWS_BF16X3 : rows on demand only (se_extrapolate_ondemand): the
 *                 per-iteration products of the dictionary's dense atoms
 *                 (those outside declared transform parts) with w_b phi_u
 *                 take split-BF16 operands, as SE_BF16X3 tables do (three
 *                 BF16 matrix-core products, FP32 accumulation, the dropped
 *                 lo*lo term below 2^-16 relative); the diagonals, the
 *                 initial projections and the loop stay FP32.  Every other
 *                 call returns SE_EINVAL for it. */
#define SE_ROWS_BF16X3 2u
/*   SE_INVARIANT : every FP32 matrix product of the call (the initial
 *                 projections of eq. 12 and, on demand, the diagonals and
 *                 table rows) splits its contraction into a number of
 *                 slices fixed by the number of samples per atom (one slice
 *                 per 16 stages of 32 samples, at most 8), summed in slice
 *                 order, whatever the number of blocks.  Without it the
 *                 split follows the number of blocks (few blocks: more
 *                 slices, to fill the GPU), which changes the order of the
 *                 FP32 sums; with it each block's result is the same
 *                 whichever other blocks share the call (the server sets it
 *                 for the batches it forms from several requests).  The
 *                 workspace sizes of every call include room for it.
 *                 Accepted by every call that takes se_params. */
#define SE_INVARIANT 4u
typedef struct {
  float gamma;
  int32_t iters;
  uint32_t flags; /* 0, or SE_ROWS_Q14 or SE_ROWS_BF16X3, each with or
                     without SE_INVARIANT */
} se_params;

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                              */
/* ------------------------------------------------------------------------ */

/* Text of the last error on the calling thread ("" if none). */
const char* se_last_error(void);
/* Library version as 10000*major + 100*minor + patch. */
int32_t se_version(void);
/* Minimum row stride (in floats) of the table G and of projection buffers
 * for a dictionary of K atoms: K rounded up to the padded row length of the
 * iteration loop's workgroup shape (64 * waves * values per lane).  0 if K
 * is below 1 or above 32768, the largest supported dictionary. */
int32_t se_table_ld(int32_t K);
/* Size of the transform operand buffer se_tables.tx for an M x N area with
 * n_parts declared transform parts; 0 if n_parts is 0 or out of range, or
 * M or N outside 1..64.  For areas of T frames pass T*M as M (the frames
 * are transformed stacked).  Any n_parts of 1 or 2 gets room for the
 * operands of two transforms (a SE_PART_DFT2 part takes the cosine and the
 * sine matrices) and for a second copy of them with the rows in parity-class
 * order (read by the one-launch loop on parity-class rows). */
size_t se_tables_tx_bytes(int32_t M, int32_t N, int32_t n_parts);

/* ------------------------------------------------------------------------ */
/* Weighting function: eq. 4 and eq. 5                                      */
/* ------------------------------------------------------------------------ */

/* w_b[m*N+n] = rho_hat ^ sqrt((m-(M-1)/2)^2 + (n-(N-1)/2)^2) for every
 * pixel of block b's area that lies inside the image and is not lost, and
 * 0 elsewhere (eq. 4: the loss and every unavailable pixel are masked).
 * Frames whose rows are stored with a pitch larger than their width are
 * passed with W = the pitch and their padding columns marked lost in this
 * mask: the padding then has weight 0, as samples outside the frame do, so
 * every result equals the unpadded frame's and the padding is never
 * written (the server computes its own weights and takes unpadded frames).
 *   lost    : device uint8, n_img images of H x W (row pitch W, image
 *             stride H*W); nonzero = lost pixel
 *   blocks  : host, n_blk descriptors (only img, y0, x0 are read)
 *   w       : device, n_blk x (M*N) float32 output
 *   ws      : device scratch of se_area_weights_ws_bytes(n_blk) bytes
 * Errors: SE_EINVAL for M, N < 1, rho_hat outside (0, 1], img out of range,
 * ws too small. */
size_t se_area_weights_ws_bytes(int32_t n_blk);
se_status se_area_weights(int32_t M, int32_t N, float rho_hat,
                          const uint8_t* lost, int32_t n_img, int32_t H,
                          int32_t W, const se_block* blocks, int32_t n_blk,
                          float* w, void* ws, size_t ws_bytes, void* stream);

/* The weighting function over a T x M x N area of consecutive frames (the
 * three-dimensional model of the paper's closing section, built like the
 * two-dimensional one): w_b[(tau*M + m)*N + n] =
 *   rho_hat ^ sqrt((tau-(T-1)/2)^2 + (m-(M-1)/2)^2 + (n-(N-1)/2)^2)
 * for every sample of frame img+tau that lies inside the frame and is not
 * lost, 0 elsewhere.  `lost` and the batch are n_img frames of H x W;
 * every block's frames img .. img+T-1 must exist (SE_EINVAL otherwise).
 * Only img, y0, x0 are read.  T = 1 gives se_area_weights exactly.  Other
 * arguments and errors as for se_area_weights (T < 1 is SE_EINVAL). */
se_status se_volume_weights(int32_t T, int32_t M, int32_t N, float rho_hat,
                            const uint8_t* lost, int32_t n_img, int32_t H,
                            int32_t W, const se_block* blocks, int32_t n_blk,
                            float* w, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Table generation: Algorithm 2, eq. 16, eq. 17                            */
/* ------------------------------------------------------------------------ */

/* Builds the tables of one weight pattern w (device, M*N float32, w >= 0)
 * for dictionary b into *t (whose buffers and ldG the caller has set; M, N,
 * K, phi and precision are filled in).  The diagonal C_kk is summed first
 * (FP32 or FP64 per `flags`), then D, then Y, then the lower triangle of
 * G = Y Y^T on the matrix cores (FP32 MFMA for SE_FP32; for SE_BF16X3, Y is
 * split into t->Yhi + t->Ylo and the products hi*hi + hi*lo + lo*hi are
 * accumulated in FP32 on the BF16 matrix cores), mirrored to the upper
 * triangle -- Algorithm 2 computes (|D|^2 + |D|)/2 products and mirrors the
 * rest.  With declared transform parts the call first verifies them and
 * synchronises `stream` once to read the verdict; it then writes t->tx,
 * and when the atoms outside the parts form at most one range starting at
 * a multiple of 4, forms every row over the part columns as the transform
 * of the weighted atom, D_k (D o T(w phi_k)) (eq. 21-23 applied to eq. 16,
 * FP32 matrix cores in both precisions), takes the product above for the
 * dense atoms only, and mirrors the rest, so G stays exactly symmetric.
 * ws: device scratch of se_weighted_gram_ws_bytes(b, prec) bytes.
 * Errors: SE_EINVAL for a NULL pointer, K < 1, ldG < K or not a multiple
 * of 4, an unknown precision or flag, ws too small. */
size_t se_weighted_gram_ws_bytes(const se_basis* b, se_precision prec);
se_status se_weighted_gram(const se_basis* b, const float* w,
                           se_precision prec, uint32_t flags, se_tables* t,
                           void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Model generation: Algorithm 3                                            */
/* ------------------------------------------------------------------------ */

/* Conceals n_blk lost blocks that share the tables t (one weight pattern:
 * the caller guarantees every block's available pixels match the w the
 * tables were built from).  Per block:
 *   R^(0) = initial weighted projections (eq. 12), for all blocks at once as
 *           one matrix product on the matrix cores;
 *   I times: u = argmax_k |R_k| D_k (eq. 18; exact ties go to the lowest
 *           k, also on the class route, where positions do not follow the
 *           atom order across classes), c = gamma R_u D_u^2 (eq. 19),
 *           g += c phi_u over the loss
 *           (eq. 9), R_k -= c C_(k,u) for all k (eq. 20);
 *   the loss rectangle of `images` is replaced by clip(rint(g), 0, 255)
 *           (round half to even).
 * Arguments:
 *   images  : device uint8, n_img images H x W (row pitch W, image stride
 *             H*W); read on the support, written on each loss (in place)
 *   blocks  : host, n_blk descriptors; every loss rectangle (box, for
 *             areas of several frames) must lie inside its area and hold at
 *             most 256*waves pixels (waves = the
 *             workgroup size of the loop for K: 1 for K <= 2048, 2 for
 *             K <= 4096, 4 for K <= 8192, 8 for K <= 16384, 16 above; so 256
 *             pixels are always accepted); losses of different blocks must
 *             not share a pixel inside the frames (SE_EINVAL otherwise)
 *   sel     : optional device int32 n_blk x iters, selected atom per
 *             iteration (NULL to skip)
 *   coef    : optional device float32 n_blk x iters, coefficient c per
 *             iteration (NULL to skip); for complex tables n_blk x iters
 *             pairs (real, imaginary part)
 *   g_loss  : optional device float32 n_blk x g_loss_ld, the model over the
 *             loss before rounding, row-major lh x lw (ld x lh x lw for a
 *             loss over several frames) (NULL to skip)
 *   ws      : device scratch of se_extrapolate_batch_ws_bytes() bytes
 * Errors: SE_EINVAL for bad descriptors or parameters (nothing launched),
 * SE_ENOMEM for ws too small, SE_EHIP for launch failures, SE_ENUMERIC
 * (everything launched, outputs written) when some blocks have no available
 * sample (see the conventions above). */
size_t se_extrapolate_batch_ws_bytes(const se_tables* t, int32_t n_blk);
se_status se_extrapolate_batch(const se_tables* t, uint8_t* images,
                               int32_t n_img, int32_t H, int32_t W,
                               const se_block* blocks, int32_t n_blk,
                               se_params prm, int32_t* sel, float* coef,
                               float* g_loss, int32_t g_loss_ld, void* ws,
                               size_t ws_bytes, void* stream);

/* The two stages of se_extrapolate_batch, for callers that keep block
 * descriptors on the device (graph capture, serving) or time the stages.
 *
 * se_blocks_upload: validates n_blk host descriptors exactly as
 *   se_extrapolate_batch does and copies them to dev_blocks (device, n_blk
 *   se_block, caller-owned) on `stream`; *max_loss (host, may be NULL)
 *   receives the largest loss size in pixels.  The other two calls accept
 *   only descriptors that went through this validation.
 * se_project: the initial weighted scalar products of eq. 12 for every
 *   block, R[b][k] = D_k R_k^(0) (device float32, n_blk rows of stride ldR,
 *   a multiple of 4, 16-byte aligned), as one matrix product on
 *   the matrix cores (FP32, or split BF16 when t->precision is SE_BF16X3);
 *   columns K .. ldR-1 are written as 0.  ldR >=
 *   se_table_ld(K).  ws: se_project_ws_bytes(t, n_blk) bytes.
 *   For complex tables a row of R holds the real parts at [0, ldR/2) and
 *   the imaginary parts at [ldR/2, ldR); ldR >= 2 se_table_ld(K), a
 *   multiple of 8.
 * se_iterate: the iteration loop (eq. 18, 19, 9, 20) from R and the
 *   replacement of every loss in `images`; R is read only.  Outputs as for
 *   se_extrapolate_batch; g_loss rows hold g_loss_ld values (a longer loss
 *   is truncated in g_loss, never in the image).
 * se_extrapolate_batch(...) == se_blocks_upload + se_project + se_iterate. */
se_status se_blocks_upload(const se_tables* t, int32_t n_img, int32_t H,
                           int32_t W, const se_block* blocks, int32_t n_blk,
                           se_block* dev_blocks, int32_t* max_loss,
                           void* stream);
size_t se_project_ws_bytes(const se_tables* t, int32_t n_blk);
se_status se_project(const se_tables* t, const uint8_t* images, int32_t n_img,
                     int32_t H, int32_t W, const se_block* dev_blocks,
                     int32_t n_blk, float* R, int32_t ldR, void* ws,
                     size_t ws_bytes, void* stream);
se_status se_iterate(const se_tables* t, const float* R, int32_t ldR,
                     uint8_t* images, int32_t n_img, int32_t H, int32_t W,
                     const se_block* dev_blocks, int32_t n_blk, se_params prm,
                     int32_t* sel, float* coef, float* g_loss,
                     int32_t g_loss_ld, void* stream);

/* se_project followed by se_iterate, for descriptors already on the device
 * (se_blocks_upload), with the same results bit for bit.  When every atom of
 * t lies in its declared transform parts (Section VI) -- two parts covering
 * the dictionary of a 32 x 32 or 64 x 64 area -- each block's workgroup
 * computes its own initial projections as transforms on the matrix cores
 * and keeps them in LDS for the loop (eq. 12 via eq. 22, then eq. 18-20):
 * one launch, no R in device memory, and se_extrapolate_device_ws_bytes is
 * 0.  Otherwise R and the projection workspace come from ws
 * (se_extrapolate_device_ws_bytes(t, n_blk) bytes).  se_extrapolate_batch
 * takes the same single-launch route for such tables.
 * Arguments and errors as for se_iterate (plus SE_ENOMEM when ws is needed
 * and too small). */
size_t se_extrapolate_device_ws_bytes(const se_tables* t, int32_t n_blk);
se_status se_extrapolate_device(const se_tables* t, uint8_t* images,
                                int32_t n_img, int32_t H, int32_t W,
                                const se_block* dev_blocks, int32_t n_blk,
                                se_params prm, int32_t* sel, float* coef,
                                float* g_loss, int32_t g_loss_ld, void* ws,
                                size_t ws_bytes, void* stream);

/* Same contract and results as se_extrapolate_batch, executed one block at
 * a time: per block one gather launch, one matrix-vector launch for R^(0)
 * and one single-workgroup launch of the iteration loop.  This is the
 * "plain per-block" baseline the batched form is measured against.  The
 * workspace is se_extrapolate_batch_ws_bytes(t, n_blk) (only part of it is
 * used). */
se_status se_extrapolate_plain(const se_tables* t, uint8_t* images,
                               int32_t n_img, int32_t H, int32_t W,
                               const se_block* blocks, int32_t n_blk,
                               se_params prm, int32_t* sel, float* coef,
                               float* g_loss, int32_t g_loss_ld, void* ws,
                               size_t ws_bytes, void* stream);

/* se_extrapolate_batch without a workspace argument, for callers that
 * cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Same contract, route
 * and results (bit for bit) as se_extrapolate_batch; the scratch memory is
 * a static device array of the library, SE_STATIC_SCRATCH_BYTES bytes on
 * every GPU the library's code is loaded on, held until the process ends.
 * Its device address is looked up on the first call on each device (the
 * device of `stream`; the current device for the null stream); the call
 * itself allocates no device memory and calls no allocating routine.
 *   Scratch needed: 256-byte aligned pieces of n_blk * 40 bytes of
 *   descriptors and, unless every atom lies in the two declared transform
 *   parts of a 32 x 32, 64 x 64 or 64 x 16 area (the one-launch route),
 *   n_blk rows of R (se_table_ld(K) floats, twice that for a complex
 *   dictionary) and the projection workspace (n_blk * M*N floats, plus the
 *   partial products of a split contraction for small batches).  A batch
 *   that needs more than SE_STATIC_SCRATCH_BYTES returns SE_ENOMEM and
 *   launches nothing.
 *   Sharing: every call on one GPU uses that GPU's one array, and nothing
 *   in it has to start at zero (each call writes every byte it reads).
 *   Calls that overlap in time on one GPU (on different streams or from
 *   different threads) race on the array: serialise them, e.g. on one
 *   stream.
 * Other arguments and errors as for se_extrapolate_batch. */
#define SE_STATIC_SCRATCH_BYTES ((size_t)16 << 20)
se_status se_extrapolate_batch_static(const se_tables* t, uint8_t* images,
                                      int32_t n_img, int32_t H, int32_t W,
                                      const se_block* blocks, int32_t n_blk,
                                      se_params prm, int32_t* sel, float* coef,
                                      float* g_loss, int32_t g_loss_ld,
                                      void* stream);

/* ------------------------------------------------------------------------ */
/* Autotuning of the batched path                                           */
/* ------------------------------------------------------------------------ */

/* Choices of the batched path for one (K, M*N, batch-size bucket): the
 * workgroup shape of the iteration loop (waves x values per lane; every
 * candidate has the padded row length se_table_ld(K), so tables stay
 * valid) and the projection GEMM's tile (64 or 128). */
typedef struct {
  int32_t loop_waves, loop_vpl, proj_tile;
  float loop_ms, proj_ms;   /* best measured times */
} se_tune_result;

/* Times every loop shape and projection tile on the caller's batch (the
 * arguments of se_project / se_iterate; images are rewritten with the same
 * values), `reps` runs each after one warm-up, synchronising on `stream`,
 * and records the fastest; later batched calls with the same K, area and
 * batch-size bucket (power of two) use it.  Process-wide, thread-safe. */
se_status se_autotune_batch(const se_tables* t, uint8_t* images, int32_t n_img,
                            int32_t H, int32_t W, const se_block* dev_blocks,
                            int32_t n_blk, se_params prm, float* R,
                            int32_t ldR, void* ws, size_t ws_bytes,
                            int32_t reps, void* stream, se_tune_result* out);
/* The records as text, one "K MN bucket waves vpl tile" line per entry of
 * the batched path and one "rows Kd MN bucket tile split" line per entry of
 * se_autotune_ondemand;
 * returns the length (without the terminating 0) and writes at most cap-1
 * characters plus a terminating 0 into buf (may be NULL). */
int32_t se_tune_export(char* buf, int32_t cap);
/* Adds records from such text; SE_EINVAL for a malformed or out-of-range
 * line (records before it are kept). */
se_status se_tune_import(const char* text);
/* Forgets every record (defaults apply again). */
void se_tune_clear(void);

/* ------------------------------------------------------------------------ */
/* Model generation when every block has its own weighting function         */
/* ------------------------------------------------------------------------ */

/* Conceals n_blk blocks whose weights differ (other losses or the image
 * border inside their areas), so no table can be shared: the paper notes
 * that C and D then have to be adapted to each weighting function.  Only
 * the table rows the loop reads are formed: per iteration, the rows
 * C_b[u_b][:] of every still-iterating block are one matrix product of the
 * dictionary with the vectors w_b * phi_{u_b} (FP32 MFMA), as are the
 * per-block diagonals C_b[k][k] (giving D_b) and the initial projections.
 * Rows of declared transform parts (Section VI) are instead the separable
 * transforms of w_b * phi_{u_b} on the matrix cores; the declaration is
 * verified against phi first, which synchronises `stream` once.
 * Selection, coefficients, model update and paste are those of
 * se_extrapolate_batch, so both calls give the same result for the same
 * weights (up to FP32 rounding).
 *   b       : dictionary (device phi)
 *   w       : device float32 n_blk x (M*N), block i's weights in row i (as
 *             written by se_area_weights)
 *   iters   : host, optional per-block iteration counts (NULL: prm.iters
 *             for every block)
 *   sel, coef : optional device outputs of n_blk rows with stride
 *             max(iteration counts); entries past a block's own count are
 *             left unchanged
 *   g_loss  : optional, as for se_extrapolate_batch
 *   ws      : se_extrapolate_ondemand_ws_bytes(b, n_blk, max_loss) bytes,
 *             max_loss = the largest lh*lw of the blocks (the size includes
 *             the split-BF16 copies that SE_ROWS_BF16X3 uses)
 *   prm.flags : 0 or SE_ROWS_BF16X3
 * Errors as for se_extrapolate_batch; the loss size is not limited. */
size_t se_extrapolate_ondemand_ws_bytes(const se_basis* b, int32_t n_blk,
                                        int32_t max_loss);
se_status se_extrapolate_ondemand(const se_basis* b, const float* w,
                                  uint8_t* images, int32_t n_img, int32_t H,
                                  int32_t W, const se_block* blocks,
                                  int32_t n_blk, se_params prm,
                                  const int32_t* iters, int32_t* sel,
                                  float* coef, float* g_loss,
                                  int32_t g_loss_ld, void* ws, size_t ws_bytes,
                                  void* stream);

/* The same computation split into a preparation per dictionary, a plan per
 * batch and runs of a plan, for callers that conceal many batches with one
 * dictionary, or capture the work in a HIP graph.
 *
 * Prepared dictionary (se_ondemand_prepare): the declared transform parts
 * are verified against phi once, here (the call synchronises `stream`),
 * and phi squared (the per-block diagonals C_b[k][k] of eq. 16 are its
 * products with w_b), the transform operands and, with SE_ROWS_BF16X3 in
 * flags, the split-BF16 dictionary are formed and kept on the device,
 * allocated by the library (freed by se_ondemand_release).  The dictionary
 * keeps a copy of *b and reads phi through it: phi must stay valid and
 * unchanged while the dictionary is used.  Errors: SE_EINVAL as for
 * se_extrapolate_ondemand's basis checks or an unknown flag (only
 * SE_ROWS_BF16X3 is known), SE_ENOMEM if the device memory cannot be
 * allocated, SE_EHIP; nothing is returned in *out then.
 *
 * Plan (se_ondemand_plan_create): the block checks, the order of the
 * blocks by decreasing iteration count and the device copies of their
 * descriptors (copied here, then the call synchronises `stream`), for
 * images of n_img x H x W.  The plan keeps pointers into `ws` and the
 * dictionary: both must outlive it.  prm.flags: 0, SE_ROWS_BF16X3 (the
 * dictionary must have been prepared with it) and SE_INVARIANT, as for
 * se_extrapolate_ondemand.
 *   row_slots : table rows cached per block.  A block that selects an atom
 *             whose row it has cached reuses that row (eq. 16's row of an
 *             atom depends only on the block's weights), so only the rows
 *             of atoms new to a block are formed; the first row_slots
 *             distinct atoms of a block are cached and later new ones are
 *             formed on every selection.  0 forms every row on use, as
 *             se_extrapolate_ondemand does; the largest iteration count
 *             caches every row (values above it, or above K, act as it).
 *             Results do not depend on row_slots: a cached row holds the
 *             values the product would form again.
 *   ws      : device, se_ondemand_plan_ws_bytes(d, n_blk, max_loss,
 *             row_slots) bytes (max_loss as for se_extrapolate_ondemand);
 *             the cache takes n_blk * (row_slots + 1) rows of K rounded
 *             up to a multiple of 1024 floats, and with row_slots > 0 a
 *             map of n_blk * K int32.
 * se_ondemand_plan_info returns the plan's block count (-1 for NULL) and
 * writes, where not NULL, its largest iteration count (the stride of sel
 * and coef), largest loss (the least g_loss_ld) and rows cached per block.
 *
 * Run (se_ondemand_run): conceals the plan's blocks, with results as
 * se_extrapolate_ondemand's for the same blocks, weights w, images,
 * prm and iteration counts (outputs as described there).  A run only
 * launches kernels on `stream`, with launch shapes fixed by the plan: no
 * copy, no memory fill through the runtime, no allocation, no
 * synchronisation, so it can be captured in a HIP graph and replayed (each
 * replay recomputes everything from w and the images).  Runs of one plan
 * share its workspace: runs that overlap in time (on different streams)
 * race; serialise them.  Returns SE_ENUMERIC, after completing the work,
 * if some blocks have no available sample, as se_extrapolate_ondemand.
 *
 * se_autotune_ondemand times the row products' tile (64 x 64, 128 x 128, or
 * 128 atoms x 64 blocks, code 12864) and split of the contraction (1, 2, 4
 * or 8 slices, or the automatic rule) on runs
 * of the plan (`reps` each after a warm-up, synchronising `stream`;
 * images are rewritten with the same values, sel/coef/g_loss not written),
 * records the fastest per (dense atoms, M*N, block-count bucket) for
 * later plans, and sets it in this plan.  A split other than none changes
 * the order of the FP32 sums (results stay within the FP32 rounding of the
 * products); SE_INVARIANT plans never split.  SE_EINVAL if the plan has
 * no dense atoms (every row a transform) or no blocks.
 *
 * se_ondemand_extrapolate: se_extrapolate_ondemand on a prepared dictionary
 * (same arguments and results, bit for bit; b replaced by d, and row_slots
 * as for a plan): no verification, no phi squared, no synchronisation; the
 * descriptors are staged from host memory as by the other calls.  ws:
 * se_ondemand_plan_ws_bytes(d, n_blk, max_loss, row_slots) bytes. */
typedef struct se_od_dict se_od_dict;
typedef struct se_od_plan se_od_plan;
se_status se_ondemand_prepare(const se_basis* b, uint32_t flags, se_od_dict** out,
                              void* stream);
void se_ondemand_release(se_od_dict* d);
size_t se_ondemand_plan_ws_bytes(const se_od_dict* d, int32_t n_blk, int32_t max_loss,
                                 int32_t row_slots);
se_status se_ondemand_plan_create(const se_od_dict* d, int32_t n_img, int32_t H, int32_t W,
                                  const se_block* blocks, int32_t n_blk, se_params prm,
                                  const int32_t* iters, int32_t row_slots, void* ws,
                                  size_t ws_bytes, void* stream, se_od_plan** out);
int32_t se_ondemand_plan_info(const se_od_plan* p, int32_t* iters_max, int32_t* max_loss,
                              int32_t* row_slots);
se_status se_ondemand_run(const se_od_plan* p, const float* w, uint8_t* images, int32_t* sel,
                          float* coef, float* g_loss, int32_t g_loss_ld, void* stream);
void se_ondemand_plan_release(se_od_plan* p);
se_status se_ondemand_extrapolate(const se_od_dict* d, const float* w, uint8_t* images,
                                  int32_t n_img, int32_t H, int32_t W, const se_block* blocks,
                                  int32_t n_blk, se_params prm, const int32_t* iters,
                                  int32_t* sel, float* coef, float* g_loss, int32_t g_loss_ld,
                                  int32_t row_slots, void* ws, size_t ws_bytes, void* stream);
typedef struct {
  int32_t row_tile, row_split;  /* 0 / -1: the automatic rules */
  float run_ms;                 /* best measured run time */
} se_tune_rows_result;
se_status se_autotune_ondemand(se_od_plan* p, const float* w, uint8_t* images, int32_t reps,
                               void* stream, se_tune_rows_result* out);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of concealment requests                      */
/* ------------------------------------------------------------------------ */

/* A server conceals lost blocks of whole frames submitted over time.  The
 * paper's tables depend only on the weighting pattern, so they are computed
 * ahead of use for the patterns that occur and kept (Section III); the
 * server builds them on first use and keeps them in a device cache, limited
 * by an HBM budget.  A block whose area lies inside the frame and holds no
 * other loss has the isolated pattern of its (dictionary, loss rectangle)
 * and uses the cached tables; every other block has its own weights and
 * takes the on-demand path of se_extrapolate_ondemand.
 *
 * Requests are admitted as frame slots free up; each admitted frame is
 * copied into a slot, and all admitted frames not yet launched are batched
 * together (blocks of every frame grouped by pattern) and launched on one
 * of several streams, so a batch launched while earlier batches still run
 * overlaps with them on the device.  Results do not depend on which other
 * requests share a batch.  Completion times are taken on the host
 * (CLOCK_MONOTONIC, ns). */

typedef struct se_server se_server;

typedef struct {
  int32_t device;            /* HIP device ordinal                             */
  int32_t frame_H, frame_W;  /* frame size served (every request must match)   */
  int32_t max_slots;         /* frames in flight on the device (>= 1)          */
  int32_t max_queue;         /* frames waiting for a slot (>= 1)               */
  int32_t n_streams;         /* streams batches are spread over (1 .. 8)       */
  float rho_hat;             /* decay of eq. 5, (0, 1]                         */
  size_t hbm_budget_bytes;   /* device memory for slots, tables and scratch    */
} se_serve_config;

/* One lost rectangle of a frame; its extrapolation area is the basis set's
 * M x N window centred on the loss (offset (M-h)/2, (N-w)/2). */
typedef struct {
  int32_t y, x, h, w;        /* loss rectangle in frame coordinates            */
  int32_t basis;             /* index of the basis set (see se_serve_create)   */
} se_loss;

typedef struct {
  uint8_t* frame;            /* device uint8 H x W; the losses are replaced in
                                place when the request completes; the caller
                                must not touch it until then                  */
  int32_t H, W;
  const se_loss* losses;     /* host, copied during submit                    */
  int32_t n_losses;
  se_params prm;             /* gamma and iteration count for every block;
                                flags must be 0                                  */
} se_request;

typedef struct {
  se_status status;          /* SE_OK, or the error the request ended with    */
  int32_t n_blocks, n_isolated, n_ondemand;
  uint64_t t_submit_ns, t_admit_ns, t_done_ns;
} se_result;

typedef struct {
  uint64_t submitted, completed, batches;
  uint64_t table_hits, table_builds, table_evictions, degraded_blocks;
  size_t bytes_tables, bytes_slots, bytes_scratch;
} se_serve_stats;

/* Creates a server (allocates its slots and streams on `device`).  sets:
 * host array of n_sets dictionaries (device phi, owned by the caller, must
 * outlive the server).  Errors: SE_EINVAL for bad sizes, SE_ENOMEM if the
 * slots alone exceed the budget, SE_EHIP for runtime failures. */
se_status se_serve_create(const se_serve_config* cfg, const se_basis* sets,
                          int32_t n_sets, se_server** out);
/* Queues a request; never blocks.  SE_EBUSY when the queue is full,
 * SE_EINVAL for a bad request (frame size, loss outside the frame, unknown
 * basis, loss larger than the basis area, overlapping losses),
 * SE_ECANCELED after destroy began.  *ticket identifies the request. */
se_status se_serve_submit(se_server* s, const se_request* r, uint64_t* ticket);
/* SE_EAGAIN while the request is queued or running; SE_OK once done, with
 * *out filled and the ticket released; SE_EINVAL for an unknown ticket. */
se_status se_serve_poll(se_server* s, uint64_t ticket, se_result* out);
/* Blocks until the request is done, then as se_serve_poll. */
se_status se_serve_wait(se_server* s, uint64_t ticket, se_result* out);
se_status se_serve_stats_get(se_server* s, se_serve_stats* out);
/* Finishes every admitted and queued request, then frees the server. */
se_status se_serve_destroy(se_server* s);

#ifdef __cplusplus
}
#endif
#endif /* SEFASE_SE_H */
